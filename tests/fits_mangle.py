"""Malformed variants of valid OGIP test files (test helper): each damages
one field that the reader takes from the file (header sizes, heap
descriptors, integer columns stored as floats), for the tests that check
such files are reported as errors and read nothing out of bounds."""
from __future__ import annotations

import numpy as np

from fits_writer import bintable, primary


def hdus(raw: bytes):
    """(header start, data start, keys) per HDU of a file written by fits_writer."""
    out, pos = [], 0
    while pos < len(raw):
        keys, start = {}, pos
        while True:
            block = raw[pos:pos + 2880]
            pos += 2880
            cards = [block[i:i + 80].decode("ascii") for i in range(0, 2880, 80)]
            end = False
            for c in cards:
                if c.startswith("END"):
                    end = True
                    break
                if c[8] == "=":
                    keys[c[:8].strip()] = (c[10:].split("/")[0].strip().strip("'").strip())
            if end:
                break
        n = int(keys.get("NAXIS1", 0)) * int(keys.get("NAXIS2", 0)) + int(keys.get("PCOUNT", 0))
        out.append((start, pos, keys))
        pos += (n + 2879) // 2880 * 2880
    return out


def set_card(raw: bytes, key: str, value: str) -> bytes:
    """Replace the value of the first header card `key` (right-justified)."""
    i = raw.index(key.ljust(8).encode() + b"= ")
    card = (key.ljust(8) + "= " + value.rjust(20)).ljust(80).encode()
    return raw[:i] + card + raw[i + 80:]


def set_descriptor(raw: bytes, extname: str, col_offset: int, row: int, count: int, offset: int) -> bytes:
    """Overwrite the (count, offset) heap descriptor of a 'P' column."""
    for _, ds, keys in hdus(raw):
        if keys.get("EXTNAME") == extname:
            p = ds + row * int(keys["NAXIS1"]) + col_offset
            b = bytearray(raw)
            b[p:p + 8] = np.array([count, offset], dtype=">i4").tobytes()
            return bytes(b)
    raise KeyError(extname)


def rmf_with_float_columns(path, n_grp_value, f_chan_value, channel_value=1.0):
    """A two-row RMF whose N_GRP, F_CHAN and CHANNEL columns are floats
    (allowed by FITS), holding the given (possibly non-finite or huge) values."""
    cols = [("ENERG_LO", "1E", [0.1, 0.2]), ("ENERG_HI", "1E", [0.2, 0.3]), ("N_GRP", "1E", [n_grp_value, 1.0]),
            ("F_CHAN", "1E", [f_chan_value, 1.0]), ("N_CHAN", "1E", [2.0, 2.0]), ("MATRIX", "2E", [[0.5, 0.5]] * 2)]
    eb = [("CHANNEL", "1E", [channel_value, 2.0, 3.0]), ("E_MIN", "1E", [0.1, 0.2, 0.3]), ("E_MAX", "1E", [0.2, 0.3, 0.4])]
    with open(path, "wb") as f:
        f.write(primary() + bintable("MATRIX", cols, 2, keys=[("DETCHANS", 3)])
                + bintable("EBOUNDS", eb, 3, keys=[("DETCHANS", 3)]))


def malformed_rmfs(valid: bytes):
    """(name, bytes) of damaged copies of a variable-length RMF written by
    fits_writer.write_rmf (MATRIX descriptor at byte 26 of a row)."""
    _, ds, keys = [h for h in hdus(valid) if h[2].get("EXTNAME") == "MATRIX"][0]
    pcount = int(keys["PCOUNT"])
    out = [
        ("truncated", valid[:ds + 100]),
        ("huge_count", set_descriptor(valid, "MATRIX", 26, 0, 0x7FFFFFFF, 0)),
        ("negative_count", set_descriptor(valid, "MATRIX", 26, 1, -5, 0)),
        ("offset_past_heap", set_descriptor(valid, "MATRIX", 26, 2, 4, pcount)),
        ("negative_offset", set_descriptor(valid, "MATRIX", 26, 3, 4, -64)),
        ("naxis2_huge", set_card(valid, "NAXIS2", "999999999999999")),
        ("pcount_huge", set_card(valid, "PCOUNT", "9223372036854775807")),
        ("naxis1_negative", set_card(valid, "NAXIS1", "-26")),
        ("bad_bitpix", set_card(valid, "BITPIX", "7")),
    ]
    b = bytearray(valid)
    i = bytes(b).index(b"TFORM6  = ")
    b[i:i + 80] = ("TFORM6  = " + "'99999999999999E'".rjust(20)).ljust(80).encode()
    out.append(("tform_repeat_huge", bytes(b)))
    return out
