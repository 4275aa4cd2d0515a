// Host-only driver of the library's OGIP reader for the sanitizer build
// (AddressSanitizer and UndefinedBehaviorSanitizer, no GPU): reads one ARF
// or RMF file through the C entry points and prints the status and a
// checksum of what was read.  api_fail is the library's error hook; here it
// prints the message.
#include <cstdio>
#include <vector>

#include "../../include/ppm.h"

namespace ppm {
int api_fail(int code, const char *msg)
{
    std::printf("error %d: %s\n", code, msg);
    return code;
}
}  // namespace ppm

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    const bool arf = argv[1][0] == 'a';
    int32_t ne = 0, nc = 0;
    int st = arf ? ppm_arf_read(argv[2], &ne, nullptr, nullptr, nullptr)
                 : ppm_rmf_read(argv[2], &ne, &nc, nullptr, nullptr, nullptr, nullptr, nullptr);
    double sum = 0.0;
    if (st == PPM_OK) {
        std::vector<double> lo(ne), hi(ne), a(arf ? ne : (size_t)ne * nc), cl(nc), ch(nc);
        st = arf ? ppm_arf_read(argv[2], &ne, lo.data(), hi.data(), a.data())
                 : ppm_rmf_read(argv[2], &ne, &nc, lo.data(), hi.data(), a.data(), cl.data(), ch.data());
        for (double v : a) sum += v;
        for (double v : lo) sum += v;
    }
    std::printf("status %d n_energy %d n_chan %d sum %.17g\n", st, (int)ne, (int)nc, sum);
    return 0;
}
