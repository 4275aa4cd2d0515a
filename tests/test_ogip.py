"""Host-side instrument pipeline of the library (Sect. 2.8.4) against the
oracle (``oracle/instrument.py``), no GPU needed.

* OGIP files: synthetic ARF and RMF files written by ``tests/fits_writer.py``
  (variable-length and fixed-width matrix columns, first channel 0 or 1,
  4- and 8-byte floats) read back by ``ppm_arf_read`` / ``ppm_rmf_read``
  exactly (the written float32 values);
* ``ppm_response_build`` equals the oracle's DS (A R) to 1e-13 relative,
  on fine bins that straddle, lie inside and lie beyond the model grid;
* ``ppm_sigma_from_table`` equals the oracle's -ln(Interp)/N_ref;
* unreadable input is reported, not crashed on.
"""
import os

import numpy as np
import pytest

from fits_writer import write_arf, write_rmf
from oracle import instrument as I


@pytest.fixture(scope="module")
def ppm():
    import paper_2510_07764_amd as m
    return m


def synthetic_instrument(n_fine=150, n_chan=90, seed=3):
    rng = np.random.default_rng(seed)
    edges = np.geomspace(0.1, 4.0, n_fine + 1)
    lo, hi = edges[:-1], edges[1:]
    area = (300 + 200 * np.exp(-((np.log(0.5 * (lo + hi)) - 0.4) / 0.7) ** 2)) * rng.uniform(0.95, 1.05, n_fine)
    ch_edges = np.linspace(0.05, 4.5, n_chan + 1)
    cen = 0.5 * (ch_edges[:-1] + ch_edges[1:])
    m = np.zeros((n_fine, n_chan))
    for e in range(n_fine):
        ec = 0.5 * (lo[e] + hi[e])
        w = np.exp(-0.5 * ((cen - ec) / (0.04 + 0.03 * np.sqrt(ec))) ** 2)
        w[w < 1e-4] = 0.0                      # sparse rows: channel groups
        if e % 17 == 0:
            w[:3] = 0.01                         # a second, detached group
        m[e] = w / max(w.sum(), 1e-30) * 0.9
    m[5] = 0.0                                   # a row with no group at all
    return lo, hi, area, m, ch_edges[:-1], ch_edges[1:]


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("tform", ["E", "D"])
def test_arf_round_trip(ppm, tmp_path, tform):
    lo, hi, area, _, _, _ = synthetic_instrument()
    p = os.path.join(tmp_path, "t.arf")
    write_arf(p, lo, hi, area, tform=tform)
    rlo, rhi, ra = ppm.read_arf(p)
    cast = f32 if tform == "E" else (lambda a: np.asarray(a, dtype=np.float64))
    assert np.array_equal(rlo, cast(lo)) and np.array_equal(rhi, cast(hi)) and np.array_equal(ra, cast(area))


@pytest.mark.parametrize("variable,tlmin,extname", [(True, 1, "MATRIX"), (True, 0, "SPECRESP MATRIX"),
                                                    (False, 1, "MATRIX"), (False, 0, "MATRIX")])
def test_rmf_round_trip(ppm, tmp_path, variable, tlmin, extname):
    lo, hi, _, m, cl, ch = synthetic_instrument()
    p = os.path.join(tmp_path, "t.rmf")
    write_rmf(p, lo, hi, m, cl, ch, tlmin=tlmin, variable=variable, extname=extname)
    rlo, rhi, rm, rcl, rch = ppm.read_rmf(p)
    assert rm.shape == m.shape
    assert np.array_equal(rm, f32(m))
    assert np.array_equal(rlo, f32(lo)) and np.array_equal(rhi, f32(hi))
    assert np.array_equal(rcl, f32(cl)) and np.array_equal(rch, f32(ch))


def test_response_build_against_oracle(ppm):
    lo, hi, area, m, _, _ = synthetic_instrument()
    em = np.geomspace(0.2, 3.0, 64)              # fine bins reach beyond both ends
    got = ppm.build_response(em, lo, hi, area, m)
    ref = I.response(em, lo, hi, area, m)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    # without an ARF the response is DS R
    g1, r1 = ppm.build_response(em, lo, hi, None, m), I.response(em, lo, hi, np.ones(lo.size), m)
    assert np.max(np.abs(g1 - r1)) <= 1e-13 * np.max(np.abs(r1))


def test_files_to_response(ppm, tmp_path):
    """ARF and RMF files -> RSP, against the oracle on the values the files hold."""
    lo, hi, area, m, cl, ch = synthetic_instrument(n_fine=80, n_chan=40, seed=9)
    pa, pr = os.path.join(tmp_path, "x.arf"), os.path.join(tmp_path, "x.rmf")
    write_arf(pa, lo, hi, area)
    write_rmf(pr, lo, hi, m, cl, ch)
    alo, ahi, a = ppm.read_arf(pa)
    rlo, rhi, rm, _, _ = ppm.read_rmf(pr)
    assert np.array_equal(alo, rlo) and np.array_equal(ahi, rhi)
    em = np.geomspace(0.2, 3.0, 48)
    got = ppm.build_response(em, rlo, rhi, a, rm)
    ref = I.response(em, f32(lo), f32(hi), f32(area), f32(m))
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_sigma_from_table(ppm):
    e_tab = np.geomspace(0.08, 12.0, 300)
    nref = 4e18
    att = np.exp(-nref * 2.4e-22 * e_tab ** -2.6 * (1 + 0.1 * np.sin(3 * e_tab)))
    em = np.concatenate([[0.05], np.geomspace(0.2, 3.0, 40), [20.0]])
    got = ppm.sigma_from_table(e_tab, att, nref, em)
    ref = I.sigma_from_table(e_tab, att, nref, em)
    assert np.allclose(got, ref, rtol=1e-13, atol=0)


def test_unreadable_input_is_reported(ppm, tmp_path):
    with pytest.raises(ppm.PPMError, match="cannot open"):
        ppm.read_arf(os.path.join(tmp_path, "missing.arf"))
    p = os.path.join(tmp_path, "junk.fits")
    with open(p, "wb") as f:
        f.write(b"not a fits file" * 10)
    with pytest.raises(ppm.PPMError):
        ppm.read_rmf(p)
    lo, hi, area, _, _, _ = synthetic_instrument(n_fine=10)
    pa = os.path.join(tmp_path, "y.arf")
    write_arf(pa, lo, hi, area)
    with pytest.raises(ppm.PPMError, match="MATRIX"):
        ppm.read_rmf(pa)
    with pytest.raises(ppm.PPMError, match="increase"):
        ppm.build_response([1.0, 0.5], lo, hi, area, np.ones((10, 3)))


def test_malformed_files_are_reported(ppm, tmp_path):
    """Damaged header sizes, heap descriptors outside the heap, and integer
    columns holding non-finite or out-of-range floats: an error each, no
    read outside the file or the arrays (the sanitizer build runs the same
    files, tests/test_sanitizers.py)."""
    from fits_mangle import malformed_rmfs, rmf_with_float_columns
    lo, hi, _, m, cl, ch = synthetic_instrument(n_fine=12, n_chan=10)
    p = os.path.join(tmp_path, "ok.rmf")
    write_rmf(p, lo, hi, m, cl, ch)
    valid = open(p, "rb").read()
    for name, raw in malformed_rmfs(valid):
        q = os.path.join(tmp_path, name + ".rmf")
        with open(q, "wb") as f:
            f.write(raw)
        with pytest.raises(ppm.PPMError):
            ppm.read_rmf(q)
    q = os.path.join(tmp_path, "float_ok.rmf")
    rmf_with_float_columns(q, 1.0, 1.0)
    _, _, rm, _, _ = ppm.read_rmf(q)
    assert np.array_equal(rm, [[0.5, 0.5, 0.0], [0.5, 0.5, 0.0]])
    for n_grp, f_chan, channel in [(float("nan"), 1.0, 1.0), (1e30, 1.0, 1.0), (-1.0, 1.0, 1.0),
                                   (1.0, float("nan"), 1.0), (1.0, 1e30, 1.0), (1.0, 1.0, float("inf"))]:
        q = os.path.join(tmp_path, "float_bad.rmf")
        rmf_with_float_columns(q, n_grp, f_chan, channel)
        with pytest.raises(ppm.PPMError):
            ppm.read_rmf(q)
