// Instrument pipeline of Sect. 2.8.4 on the host: OGIP ARF and RMF files
// (FITS binary tables) read into plain arrays, the down-sampling matrix DS
// from the fine response energies to the model energy grid, the combined
// response RSP = DS (A R), and the absorption cross-section from a
// transmission table at a reference column.  FITS layout per the FITS
// standard (2880-byte blocks of 80-character cards, big-endian binary
// tables, variable-length arrays in the heap); OGIP column conventions per
// the OGIP calibration memo CAL/GEN/92-002.
//
// Every size, offset and count taken from a file is checked before use:
// header sizes against the file length (with overflow-checked products),
// variable-length array descriptors against the table's heap, and integer
// columns read as floating point for finiteness and range before they are
// converted.  No exception leaves the C entry points.

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/ppm.h"
#include "ppm_status.h"

using namespace ppm;

namespace {

struct Column {
    std::string name;
    char type = 0;        // B I J K E D (fixed) ; P / Q descriptor with element type `ptype`
    char ptype = 0;
    long repeat = 1;
    long offset = 0;      // byte offset within a row
};

struct Hdu {
    std::map<std::string, std::string> keys;
    long data_start = 0;  // file offset of the data unit
    long naxis1 = 0, naxis2 = 0, theap = 0;
    long heap_end = 0;    // end of the heap, from the data start (NAXIS1 NAXIS2 + PCOUNT)
    std::vector<Column> cols;
};

// a * b and a + b for non-negative operands, false on overflow
bool mul_ok(long a, long b, long &out)
{
    return a >= 0 && b >= 0 && !__builtin_mul_overflow(a, b, &out);
}

bool add_ok(long a, long b, long &out)
{
    return a >= 0 && b >= 0 && !__builtin_add_overflow(a, b, &out);
}

// a value read from a file as an integer: finite and within [lo, hi]
bool to_long(double x, long lo, long hi, long &out)
{
    if (!std::isfinite(x) || x < (double)lo || x > (double)hi) return false;
    out = (long)x;
    return true;
}

std::string trim(const std::string &s)
{
    size_t a = s.find_first_not_of(' '), b = s.find_last_not_of(' ');
    return a == std::string::npos ? std::string() : s.substr(a, b - a + 1);
}

// keyword value: quoted strings without quotes and trailing blanks; numbers as text
std::string card_value(const char *card)
{
    std::string v(card + 10, 70);
    v = trim(v);
    if (!v.empty() && v[0] == '\'') {
        std::string out;
        for (size_t i = 1; i < v.size(); ++i) {
            if (v[i] == '\'') {
                if (i + 1 < v.size() && v[i + 1] == '\'') {
                    out += '\'';
                    ++i;
                    continue;
                }
                break;
            }
            out += v[i];
        }
        return trim(out);
    }
    size_t slash = v.find('/');
    return trim(slash == std::string::npos ? v : v.substr(0, slash));
}

long key_long(const Hdu &h, const std::string &k, long dflt)
{
    auto it = h.keys.find(k);
    return it == h.keys.end() ? dflt : std::strtol(it->second.c_str(), nullptr, 10);
}

long type_bytes(char t)
{
    switch (t) {
    case 'L': case 'B': case 'A': return 1;
    case 'I': return 2;
    case 'J': case 'E': return 4;
    case 'K': case 'D': case 'C': case 'P': return 8;
    case 'M': case 'Q': return 16;
    default: return 0;
    }
}

bool parse_tform(const std::string &tf, Column &c)
{
    size_t i = 0;
    long r = 0;
    bool digits = false;
    while (i < tf.size() && tf[i] >= '0' && tf[i] <= '9') {
        r = r * 10 + (tf[i] - '0');
        if (r > (1L << 31)) return false;   // beyond any table row this reader accepts
        ++i;
        digits = true;
    }
    if (i >= tf.size()) return false;
    c.repeat = digits ? r : 1;
    c.type = tf[i++];
    if (c.type == 'P' || c.type == 'Q') {
        if (i >= tf.size()) return false;
        c.ptype = tf[i];
    }
    return type_bytes(c.type) > 0 || c.type == 'X';
}

long column_bytes(const Column &c)
{
    if (c.type == 'X') return (c.repeat + 7) / 8;
    return c.repeat * type_bytes(c.type);
}

bool read_hdus(FILE *f, std::vector<Hdu> &out)
{
    char block[2880];
    long pos = 0;
    if (std::fseek(f, 0, SEEK_END) != 0) return false;
    const long fsize = std::ftell(f);
    if (fsize < 0 || std::fseek(f, 0, SEEK_SET) != 0) return false;
    while (true) {
        Hdu h;
        bool end = false, any = false;
        while (!end) {
            if (std::fread(block, 1, 2880, f) != 2880) return any ? false : !out.empty();
            any = true;
            pos += 2880;
            for (int k = 0; k < 36; ++k) {
                const char *card = block + 80 * k;
                std::string name = trim(std::string(card, 8));
                if (name == "END") {
                    end = true;
                    break;
                }
                if (card[8] == '=' && !name.empty()) h.keys[name] = card_value(card);
            }
        }
        h.data_start = pos;
        const long bitpix = key_long(h, "BITPIX", 8);
        if (bitpix != 8 && bitpix != 16 && bitpix != 32 && bitpix != 64 && bitpix != -32 && bitpix != -64)
            return false;
        const long naxis = key_long(h, "NAXIS", 0);
        if (naxis < 0 || naxis > 999) return false;
        long n = naxis > 0 ? 1 : 0;
        for (long a = 1; a <= naxis; ++a)
            if (!mul_ok(n, key_long(h, "NAXIS" + std::to_string(a), 0), n)) return false;
        const long pcount = key_long(h, "PCOUNT", 0), gcount = key_long(h, "GCOUNT", 1);
        long bytes = 0;
        if (!add_ok(pcount, n, bytes) || !mul_ok(bytes, gcount, bytes) || !mul_ok(bytes, std::labs(bitpix) / 8, bytes))
            return false;
        if (bytes > fsize - pos) return false;                    // the data unit lies inside the file
        h.naxis1 = key_long(h, "NAXIS1", 0);
        h.naxis2 = key_long(h, "NAXIS2", 0);
        auto xt = h.keys.find("XTENSION");
        if (xt != h.keys.end() && xt->second == "BINTABLE") {
            long table = 0;
            if (bitpix != 8 || naxis != 2 || !mul_ok(h.naxis1, h.naxis2, table) || !add_ok(table, pcount, h.heap_end))
                return false;
            h.theap = key_long(h, "THEAP", table);
            if (h.theap < table || h.theap > h.heap_end) return false;
            const long nf = key_long(h, "TFIELDS", 0);
            if (nf < 0 || nf > 999) return false;
            long off = 0;
            for (long j = 1; j <= nf; ++j) {
                Column c;
                c.name = h.keys["TTYPE" + std::to_string(j)];
                if (!parse_tform(h.keys["TFORM" + std::to_string(j)], c)) return false;
                c.offset = off;
                if (!add_ok(off, column_bytes(c), off) || off > h.naxis1) return false;
                h.cols.push_back(c);
            }
            if (off != h.naxis1) return false;
        }
        out.push_back(h);
        long padded = (bytes + 2879) / 2880 * 2880;
        if (padded > fsize - pos) padded = fsize - pos;           // a last unit without its final padding
        if (std::fseek(f, padded, SEEK_CUR) != 0) return false;
        pos += padded;
        int ch = std::fgetc(f);
        if (ch == EOF) return true;
        std::ungetc(ch, f);
    }
}

// big-endian signed integer of a heap descriptor ('J' or 'K')
int64_t be_int(const unsigned char *p, char t)
{
    uint64_t u = 0;
    const long n = type_bytes(t);
    for (long i = 0; i < n; ++i) u = (u << 8) | p[i];
    return t == 'J' ? (int64_t)(int32_t)(uint32_t)u : (int64_t)u;
}

double be_value(const unsigned char *p, char t)
{
    uint64_t u = 0;
    const long n = type_bytes(t);
    for (long i = 0; i < n; ++i) u = (u << 8) | p[i];
    switch (t) {
    case 'B': return (double)(uint8_t)u;
    case 'I': return (double)(int16_t)(uint16_t)u;
    case 'J': return (double)(int32_t)(uint32_t)u;
    case 'K': return (double)(int64_t)u;
    case 'E': {
        uint32_t w = (uint32_t)u;
        float x;
        std::memcpy(&x, &w, 4);
        return (double)x;
    }
    case 'D': {
        double x;
        std::memcpy(&x, &u, 8);
        return x;
    }
    default: return NAN;
    }
}

const Column *find_col(const Hdu &h, const char *name)
{
    for (const Column &c : h.cols)
        if (c.name == name) return &c;
    return nullptr;
}

// values of column c in row r (fixed repeat, or a variable-length array in the heap)
bool cell(FILE *f, const Hdu &h, const Column &c, long r, std::vector<double> &v)
{
    v.clear();
    if (r < 0 || r >= h.naxis2) return false;
    std::vector<unsigned char> buf(column_bytes(c));
    if (std::fseek(f, h.data_start + r * h.naxis1 + c.offset, SEEK_SET) != 0) return false;
    if (std::fread(buf.data(), 1, buf.size(), f) != buf.size()) return false;
    if (c.type == 'P' || c.type == 'Q') {
        const char dt = c.type == 'P' ? 'J' : 'K';
        const long db = type_bytes(dt);
        if ((long)buf.size() < 2 * db) return false;
        const int64_t cnt = be_int(buf.data(), dt), off = be_int(buf.data() + db, dt);
        const long eb = type_bytes(c.ptype);
        // the array lies inside the heap: theap + off + cnt eb <= heap_end
        long nb = 0, beg = 0, end = 0;
        if (eb == 0 || cnt < 0 || off < 0 || cnt > LONG_MAX || off > LONG_MAX || !mul_ok((long)cnt, eb, nb)
            || !add_ok(h.theap, (long)off, beg) || !add_ok(beg, nb, end) || end > h.heap_end)
            return false;
        std::vector<unsigned char> heap(nb);
        if (cnt) {
            if (std::fseek(f, h.data_start + beg, SEEK_SET) != 0) return false;
            if (std::fread(heap.data(), 1, heap.size(), f) != heap.size()) return false;
        }
        for (long i = 0; i < cnt; ++i) v.push_back(be_value(heap.data() + i * eb, c.ptype));
        return true;
    }
    const long eb = type_bytes(c.type);
    for (long i = 0; i < c.repeat; ++i) v.push_back(be_value(buf.data() + i * eb, c.type));
    return true;
}

const Hdu *find_ext(const std::vector<Hdu> &hdus, const char *a, const char *b = nullptr)
{
    for (const Hdu &h : hdus) {
        auto it = h.keys.find("EXTNAME");
        if (it == h.keys.end()) continue;
        if (it->second == a || (b && it->second == b)) return &h;
    }
    return nullptr;
}

struct File {
    FILE *f = nullptr;
    explicit File(const char *p) : f(std::fopen(p, "rb")) {}
    ~File()
    {
        if (f) std::fclose(f);
    }
};

}  // namespace

namespace {

// The C entry points run their bodies through guarded(): an exception (a
// failed allocation) becomes an error status instead of leaving C code.
template <class F>
int guarded(const char *who, F &&body)
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return api_fail(PPM_ERR_ALLOC, who);
    } catch (...) {
        return api_fail(PPM_ERR_ARG, who);
    }
}

int arf_read(const char *path, int32_t *n_energy, double *e_lo, double *e_hi, double *area);
int rmf_read(const char *path, int32_t *n_energy, int32_t *n_chan, double *e_lo, double *e_hi, double *matrix,
             double *ch_lo, double *ch_hi);
int response_build(int32_t n_model, const double *e_model, int32_t n_fine, const double *e_lo, const double *e_hi,
                   const double *area, int32_t n_chan, const double *matrix, double *rsp);

}  // namespace

extern "C" {

int ppm_arf_read(const char *path, int32_t *n_energy, double *e_lo, double *e_hi, double *area)
{
    return guarded("ppm_arf_read: out of memory or internal error",
                   [&] { return arf_read(path, n_energy, e_lo, e_hi, area); });
}

int ppm_rmf_read(const char *path, int32_t *n_energy, int32_t *n_chan, double *e_lo, double *e_hi, double *matrix,
                 double *ch_lo, double *ch_hi)
{
    return guarded("ppm_rmf_read: out of memory or internal error",
                   [&] { return rmf_read(path, n_energy, n_chan, e_lo, e_hi, matrix, ch_lo, ch_hi); });
}

int ppm_response_build(int32_t n_model, const double *e_model, int32_t n_fine, const double *e_lo, const double *e_hi,
                       const double *area, int32_t n_chan, const double *matrix, double *rsp)
{
    return guarded("ppm_response_build: out of memory or internal error", [&] {
        return response_build(n_model, e_model, n_fine, e_lo, e_hi, area, n_chan, matrix, rsp);
    });
}

}  // extern "C"

namespace {

int arf_read(const char *path, int32_t *n_energy, double *e_lo, double *e_hi, double *area)
{
    if (!path || !n_energy) return api_fail(PPM_ERR_ARG, "ppm_arf_read: null argument");
    File fh(path);
    if (!fh.f) return api_fail(PPM_ERR_ARG, "ppm_arf_read: cannot open file");
    std::vector<Hdu> hdus;
    if (!read_hdus(fh.f, hdus)) return api_fail(PPM_ERR_ARG, "ppm_arf_read: not a readable FITS file");
    const Hdu *h = find_ext(hdus, "SPECRESP");
    if (!h) return api_fail(PPM_ERR_ARG, "ppm_arf_read: no SPECRESP extension");
    const Column *clo = find_col(*h, "ENERG_LO"), *chi = find_col(*h, "ENERG_HI"), *ca = find_col(*h, "SPECRESP");
    if (!clo || !chi || !ca) return api_fail(PPM_ERR_ARG, "ppm_arf_read: missing ENERG_LO, ENERG_HI or SPECRESP");
    if (h->naxis2 > INT32_MAX) return api_fail(PPM_ERR_ARG, "ppm_arf_read: too many rows");
    *n_energy = (int32_t)h->naxis2;
    if (!e_lo && !e_hi && !area) return PPM_OK;
    std::vector<double> v;
    for (long r = 0; r < h->naxis2; ++r) {
        if (e_lo) {
            if (!cell(fh.f, *h, *clo, r, v) || v.empty()) return api_fail(PPM_ERR_ARG, "ppm_arf_read: bad row");
            e_lo[r] = v[0];
        }
        if (e_hi) {
            if (!cell(fh.f, *h, *chi, r, v) || v.empty()) return api_fail(PPM_ERR_ARG, "ppm_arf_read: bad row");
            e_hi[r] = v[0];
        }
        if (area) {
            if (!cell(fh.f, *h, *ca, r, v) || v.empty()) return api_fail(PPM_ERR_ARG, "ppm_arf_read: bad row");
            area[r] = v[0];
        }
    }
    return PPM_OK;
}

int rmf_read(const char *path, int32_t *n_energy, int32_t *n_chan, double *e_lo, double *e_hi, double *matrix,
             double *ch_lo, double *ch_hi)
{
    if (!path || !n_energy || !n_chan) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: null argument");
    File fh(path);
    if (!fh.f) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: cannot open file");
    std::vector<Hdu> hdus;
    if (!read_hdus(fh.f, hdus)) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: not a readable FITS file");
    const Hdu *h = find_ext(hdus, "MATRIX", "SPECRESP MATRIX");
    if (!h) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: no MATRIX extension");
    const Column *clo = find_col(*h, "ENERG_LO"), *chi = find_col(*h, "ENERG_HI"), *cng = find_col(*h, "N_GRP");
    const Column *cfc = find_col(*h, "F_CHAN"), *cnc = find_col(*h, "N_CHAN"), *cm = find_col(*h, "MATRIX");
    if (!clo || !chi || !cng || !cfc || !cnc || !cm) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: missing a column");
    const Hdu *eb = find_ext(hdus, "EBOUNDS");
    // first channel number: TLMIN of F_CHAN (1 when absent)
    long fcol = 1;
    for (size_t j = 0; j < h->cols.size(); ++j)
        if (&h->cols[j] == cfc) fcol = (long)j + 1;
    const long tlmin = key_long(*h, "TLMIN" + std::to_string(fcol), 1);
    long nch = key_long(*h, "DETCHANS", eb ? eb->naxis2 : 0);
    if (nch <= 0) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: channel count unknown (DETCHANS / EBOUNDS)");
    if (nch > INT32_MAX || h->naxis2 > INT32_MAX) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: too many rows");
    if (tlmin < INT32_MIN || tlmin > INT32_MAX) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: bad TLMIN");
    *n_energy = (int32_t)h->naxis2;
    *n_chan = (int32_t)nch;
    if (!matrix && !e_lo && !e_hi && !ch_lo && !ch_hi) return PPM_OK;
    std::vector<double> v, fc, ncv, mv;
    for (long r = 0; r < h->naxis2; ++r) {
        if (!cell(fh.f, *h, *clo, r, v) || v.empty()) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: bad row");
        if (e_lo) e_lo[r] = v[0];
        if (!cell(fh.f, *h, *chi, r, v) || v.empty()) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: bad row");
        if (e_hi) e_hi[r] = v[0];
        if (!matrix) continue;
        double *row = matrix + (size_t)r * nch;
        for (long c = 0; c < nch; ++c) row[c] = 0.0;
        long ng = 0;
        if (!cell(fh.f, *h, *cng, r, v) || v.empty() || !to_long(v[0], 0, INT32_MAX, ng))
            return api_fail(PPM_ERR_ARG, "ppm_rmf_read: bad N_GRP");
        if (!cell(fh.f, *h, *cfc, r, fc) || !cell(fh.f, *h, *cnc, r, ncv) || !cell(fh.f, *h, *cm, r, mv))
            return api_fail(PPM_ERR_ARG, "ppm_rmf_read: bad group arrays");
        if ((long)fc.size() < ng || (long)ncv.size() < ng) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: short groups");
        long k = 0;
        for (long g = 0; g < ng; ++g) {
            long f0 = 0, n = 0;
            if (!to_long(fc[g], INT32_MIN, INT32_MAX, f0) || !to_long(ncv[g], 0, INT32_MAX, n))
                return api_fail(PPM_ERR_ARG, "ppm_rmf_read: bad F_CHAN or N_CHAN");
            const long c0 = f0 - tlmin;
            if (c0 < 0 || c0 + n > nch || k + n > (long)mv.size())
                return api_fail(PPM_ERR_ARG, "ppm_rmf_read: group outside the channel range");
            for (long i = 0; i < n; ++i) row[c0 + i] = mv[k + i];
            k += n;
        }
    }
    if ((ch_lo || ch_hi) && eb) {
        const Column *cc = find_col(*eb, "CHANNEL"), *cmin = find_col(*eb, "E_MIN"), *cmax = find_col(*eb, "E_MAX");
        if (!cc || !cmin || !cmax) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: EBOUNDS columns missing");
        for (long r = 0; r < eb->naxis2; ++r) {
            long chv = 0;
            if (!cell(fh.f, *eb, *cc, r, v) || v.empty() || !to_long(v[0], INT32_MIN, INT32_MAX, chv))
                return api_fail(PPM_ERR_ARG, "ppm_rmf_read: bad EBOUNDS");
            const long ch = chv - tlmin;
            if (ch < 0 || ch >= nch) continue;
            if (!cell(fh.f, *eb, *cmin, r, v) || v.empty()) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: bad EBOUNDS");
            if (ch_lo) ch_lo[ch] = v[0];
            if (!cell(fh.f, *eb, *cmax, r, v) || v.empty()) return api_fail(PPM_ERR_ARG, "ppm_rmf_read: bad EBOUNDS");
            if (ch_hi) ch_hi[ch] = v[0];
        }
    }
    return PPM_OK;
}

int response_build(int32_t n_model, const double *e_model, int32_t n_fine, const double *e_lo, const double *e_hi,
                   const double *area, int32_t n_chan, const double *matrix, double *rsp)
{
    if (n_model < 2 || n_fine < 1 || n_chan < 1 || !e_model || !e_lo || !e_hi || !matrix || !rsp)
        return api_fail(PPM_ERR_ARG, "ppm_response_build: bad arguments");
    for (int i = 1; i < n_model; ++i)
        if (!(e_model[i] > e_model[i - 1])) return api_fail(PPM_ERR_ARG, "model energies must increase");
    for (int e = 0; e < n_fine; ++e)
        if (!(e_hi[e] >= e_lo[e])) return api_fail(PPM_ERR_ARG, "fine bins need e_hi >= e_lo");
    std::memset(rsp, 0, sizeof(double) * (size_t)n_model * n_chan);
    const int last = n_model - 1;
    std::vector<std::pair<int, double>> ds;   // (model index, DS entry) of one fine bin
    for (int e = 0; e < n_fine; ++e) {
        const double lo = e_lo[e], hi = e_hi[e];
        ds.clear();
        // below the grid the first hat is 1, above it the last
        if (lo < e_model[0]) ds.push_back({0, std::fmin(hi, e_model[0]) - lo});
        if (hi > e_model[last]) ds.push_back({last, hi - std::fmax(lo, e_model[last])});
        // interval [E_j, E_{j+1}] overlapping [lo, hi]: the two hats are linear there
        int j = 0;
        while (j < last && e_model[j + 1] <= lo) ++j;
        for (; j < last && e_model[j] < hi; ++j) {
            const double a = std::fmax(lo, e_model[j]), b = std::fmin(hi, e_model[j + 1]);
            if (!(b > a)) continue;
            const double h = e_model[j + 1] - e_model[j], mid = 0.5 * (a + b);
            ds.push_back({j, (b - a) * (e_model[j + 1] - mid) / h});
            ds.push_back({j + 1, (b - a) * (mid - e_model[j]) / h});
        }
        const double ae = area ? area[e] : 1.0;
        const double *row = matrix + (size_t)e * n_chan;
        for (const auto &d : ds) {
            const double w = d.second * ae;
            double *out = rsp + (size_t)d.first * n_chan;
            for (int c = 0; c < n_chan; ++c) out[c] += w * row[c];
        }
    }
    return PPM_OK;
}

}  // namespace

extern "C" {

int ppm_sigma_from_table(int32_t n_tab, const double *e_tab, const double *att_tab, double nh_ref, int32_t n,
                         const double *e, double *sigma)
{
    if (n_tab < 2 || !e_tab || !att_tab || n < 1 || !e || !sigma || !(nh_ref > 0.0))
        return api_fail(PPM_ERR_ARG, "ppm_sigma_from_table: bad arguments");
    for (int i = 0; i < n_tab; ++i) {
        if (i && !(e_tab[i] > e_tab[i - 1])) return api_fail(PPM_ERR_ARG, "table energies must increase");
        if (!(att_tab[i] > 0.0 && att_tab[i] <= 1.0)) return api_fail(PPM_ERR_ARG, "transmissions must lie in (0, 1]");
    }
    for (int k = 0; k < n; ++k) {
        const double x = e[k];
        double t;
        if (x <= e_tab[0]) {
            t = att_tab[0];
        } else if (x >= e_tab[n_tab - 1]) {
            t = att_tab[n_tab - 1];
        } else {
            int lo = 0, hi = n_tab - 1;
            while (hi - lo > 1) {
                const int mid = (lo + hi) / 2;
                if (e_tab[mid] <= x) lo = mid; else hi = mid;
            }
            const double w = (x - e_tab[lo]) / (e_tab[lo + 1] - e_tab[lo]);
            t = att_tab[lo] + w * (att_tab[lo + 1] - att_tab[lo]);
        }
        sigma[k] = -std::log(t) / nh_ref;
    }
    return PPM_OK;
}

}  // extern "C"
