"""Minimal FITS binary-table writer for the OGIP file tests (test helper).

Writes a primary HDU without data and BINTABLE extensions per the FITS
standard: 80-character header cards in 2880-byte blocks, big-endian
row-major tables, variable-length arrays (TFORM 'P') as (count, offset)
descriptors into the heap that follows the table.  Enough for OGIP ARF
(SPECRESP), RMF (MATRIX, EBOUNDS) test files; not a general FITS library.
"""
from __future__ import annotations

import numpy as np

_BE = {"E": ">f4", "D": ">f8", "I": ">i2", "J": ">i4", "K": ">i8", "B": "u1"}


def _card(key, value=None, comment=""):
    if value is None:
        s = key.ljust(8)
    elif isinstance(value, bool):
        s = key.ljust(8) + "= " + ("T" if value else "F").rjust(20)
    elif isinstance(value, str):
        s = key.ljust(8) + "= " + ("'" + value.replace("'", "''").ljust(8) + "'").ljust(20)
    elif isinstance(value, (int, np.integer)):
        s = key.ljust(8) + "= " + str(int(value)).rjust(20)
    else:
        s = key.ljust(8) + "= " + repr(float(value)).upper().rjust(20)
    if comment:
        s += " / " + comment
    assert len(s) <= 80, s
    return s.ljust(80)


def _block(cards):
    text = "".join(cards) + "END".ljust(80)
    pad = (-len(text)) % 2880
    return (text + " " * pad).encode("ascii")


def _pad_data(b):
    return b + b"\0" * ((-len(b)) % 2880)


def primary():
    return _block([_card("SIMPLE", True), _card("BITPIX", 8), _card("NAXIS", 0), _card("EXTEND", True)])


def bintable(extname, columns, nrows, keys=()):
    """columns: list of (name, tform, rows) where rows[r] is a scalar or a
    sequence; tform like '1E', '3J' (fixed) or 'PE(n)' (variable length)."""
    widths, parts = [], []
    heap = bytearray()
    rows_bytes = [bytearray() for _ in range(nrows)]
    for name, tform, vals in columns:
        if tform.startswith("P"):
            t = tform[1]
            for r in range(nrows):
                a = np.asarray(vals[r], dtype=_BE[t]).ravel()
                rows_bytes[r] += np.array([a.size, len(heap)], dtype=">i4").tobytes()
                heap += a.tobytes()
        else:
            n = int(tform[:-1]) if len(tform) > 1 else 1
            t = tform[-1]
            for r in range(nrows):
                a = np.asarray(vals[r], dtype=_BE[t]).ravel()
                assert a.size == n, (name, a.size, n)
                rows_bytes[r] += a.tobytes()
    naxis1 = len(rows_bytes[0]) if nrows else 0
    assert all(len(rb) == naxis1 for rb in rows_bytes)
    cards = [_card("XTENSION", "BINTABLE"), _card("BITPIX", 8), _card("NAXIS", 2), _card("NAXIS1", naxis1),
             _card("NAXIS2", nrows), _card("PCOUNT", len(heap)), _card("GCOUNT", 1),
             _card("TFIELDS", len(columns))]
    for j, (name, tform, _) in enumerate(columns, start=1):
        cards += [_card("TTYPE%d" % j, name), _card("TFORM%d" % j, tform)]
    cards.append(_card("EXTNAME", extname))
    cards += [_card(k, v) for k, v in keys]
    data = b"".join(bytes(rb) for rb in rows_bytes) + bytes(heap)
    return _block(cards) + _pad_data(data)


def write_arf(path, e_lo, e_hi, area, tform="E"):
    n = len(e_lo)
    cols = [("ENERG_LO", "1" + tform, e_lo), ("ENERG_HI", "1" + tform, e_hi), ("SPECRESP", "1" + tform, area)]
    with open(path, "wb") as f:
        f.write(primary() + bintable("SPECRESP", cols, n, keys=[("HDUCLASS", "OGIP"), ("HDUCLAS1", "RESPONSE")]))


def write_rmf(path, e_lo, e_hi, matrix, ch_lo, ch_hi, tlmin=1, variable=True, extname="MATRIX"):
    """matrix [n_energy, n_chan] dense; channel groups are the runs of
    nonzero entries of each row."""
    m = np.asarray(matrix, dtype=np.float32)
    ne, nc = m.shape
    ngrp, fch, nch, vals = [], [], [], []
    for r in range(ne):
        nz = m[r] != 0
        runs, c = [], 0
        while c < nc:
            if nz[c]:
                s = c
                while c < nc and nz[c]:
                    c += 1
                runs.append((s, c - s))
            else:
                c += 1
        ngrp.append(len(runs))
        fch.append([s + tlmin for s, _ in runs])
        nch.append([k for _, k in runs])
        vals.append(np.concatenate([m[r, s:s + k] for s, k in runs]) if runs else np.zeros(0, np.float32))
    if variable:
        gmax, vmax = max(max(ngrp), 1), max(max(len(v) for v in vals), 1)
        cols = [("ENERG_LO", "1E", e_lo), ("ENERG_HI", "1E", e_hi), ("N_GRP", "1I", ngrp),
                ("F_CHAN", "PJ(%d)" % gmax, fch), ("N_CHAN", "PJ(%d)" % gmax, nch), ("MATRIX", "PE(%d)" % vmax, vals)]
    else:
        gmax, vmax = max(max(ngrp), 1), max(max(len(v) for v in vals), 1)

        def padded(rows, n, dt):
            return [np.concatenate([np.asarray(x, dtype=dt), np.zeros(n - len(x), dtype=dt)]) for x in rows]
        cols = [("ENERG_LO", "1E", e_lo), ("ENERG_HI", "1E", e_hi), ("N_GRP", "1I", ngrp),
                ("F_CHAN", "%dI" % gmax, padded(fch, gmax, np.int16)), ("N_CHAN", "%dI" % gmax, padded(nch, gmax, np.int16)),
                ("MATRIX", "%dE" % vmax, padded(vals, vmax, np.float32))]
    keys = [("HDUCLASS", "OGIP"), ("HDUCLAS1", "RESPONSE"), ("HDUCLAS2", "RSP_MATRIX"), ("DETCHANS", nc),
            ("TLMIN4", tlmin), ("TLMAX4", tlmin + nc - 1)]
    eb = [("CHANNEL", "1J", list(range(tlmin, tlmin + nc))), ("E_MIN", "1E", ch_lo), ("E_MAX", "1E", ch_hi)]
    with open(path, "wb") as f:
        f.write(primary() + bintable(extname, cols, ne, keys=keys)
                + bintable("EBOUNDS", eb, nc, keys=[("HDUCLASS", "OGIP"), ("DETCHANS", nc), ("TLMIN1", tlmin)]))
