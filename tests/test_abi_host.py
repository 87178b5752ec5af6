"""C-ABI checks that need no GPU: the library loads, exports every function
include/rrcal.h declares, and its host-only calls agree with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2005_03060_amd as rrc
from paper_2005_03060_amd import _lib
from oracle import geometry as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rrcal.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rrc_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = rrc.load_library()
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == names


def test_strerror_and_defaults():
    lib = rrc.load_library()
    assert lib.rrc_strerror(0) == b"ok"
    assert b"degeneracies" in lib.rrc_strerror(-2)
    o = rrc.default_opts()
    assert o["max_gn"] >= 1 and o["fp64_steps"] >= 1 and o["init_mode"] == 0


@pytest.mark.parametrize("n", [4, 8, 12, 16, 24, 32])
def test_selection_matches_oracle(n):
    types, npairs = rrc.select_subset(n)
    ref = G.select_subset_square(n)
    assert types == [tuple(t) for t in ref]
    pairs, _ = G.group_pairs(G.square_positions(n), ref)
    assert npairs == len(pairs)


@pytest.mark.parametrize("base", [2.0, 10.0])
def test_selection_other_log_bases(base):
    for n in [8, 16]:
        types, _ = rrc.select_subset(n, 1.0, base)
        assert types == [tuple(t) for t in G.select_subset_square(n, 1.0, base)]


def test_degeneracy_count_matches_oracle():
    rng = np.random.default_rng(0)
    for trial in range(25):
        n = int(rng.integers(3, 8))
        allt, _ = G.square_types(n)
        k = int(rng.integers(1, min(8, len(allt)) + 1))
        sel = [allt[i] for i in sorted(rng.choice(len(allt), k, replace=False))]
        assert rrc.degeneracy_count(n, sel) == G.nullity(G.square_positions(n), sel), (n, sel)


def test_plan_errors():
    with pytest.raises(rrc.RRCError) as e:
        rrc.Plan(6, [(1, 0), (0, 1)], 1, 16)            # bipartite: 5 degeneracies
    assert e.value.code == _lib.RRC_EDEGEN
    with pytest.raises(rrc.RRCError) as e:
        rrc.Plan(6, [(1, 0), (7, 0)], 1, 16)            # |dx| >= n
    assert e.value.code == _lib.RRC_EINVAL
    with pytest.raises(rrc.RRCError) as e:
        rrc.Plan(6, [(1, 0), (1, 0), (0, 1)], 1, 16)    # duplicate type
    assert e.value.code == _lib.RRC_EINVAL
    with pytest.raises(rrc.RRCError) as e:
        rrc.Plan(6, [(-1, 0), (0, 1), (1, 1)], 1, 16)   # not canonical
    assert e.value.code == _lib.RRC_EINVAL
    with pytest.raises(rrc.RRCError) as e:               # firstcal needs (1,0) and (0,1)
        rrc.Plan(6, [(1, 1), (-1, 1), (2, 0), (0, 2), (1, 0)], 1, 16)
    assert e.value.code == _lib.RRC_EINVAL
    p = rrc.Plan(6, [(1, 1), (-1, 1), (2, 0), (0, 2), (1, 0)], 1, 16, init_mode="gains")
    assert p.n_pairs == 25 + 25 + 24 + 24 + 30
    with pytest.raises(rrc.RRCError):
        rrc.Plan(65, [(1, 0)], 1, 16)
    with pytest.raises(rrc.RRCError):
        rrc.Plan(8, [(1, 0), (0, 1), (1, 1)], 0, 16)
    with pytest.raises(rrc.RRCError) as e:               # no samples
        rrc.Plan(8, [(1, 0), (0, 1), (1, 1)], 1, 0)
    assert e.value.code == _lib.RRC_EINVAL


def test_smallest_grids():
    # 2 x 2: every type set leaves more than the four degeneracies, so the
    # selection refuses it; 3 x 3 with one sample is the smallest plan
    with pytest.raises(rrc.RRCError) as e:
        rrc.select_subset(2)
    assert e.value.code == _lib.RRC_EDEGEN
    types, npairs = rrc.select_subset(3)
    p = rrc.Plan(3, types, 1, 1)
    assert p.info["n_pairs"] == npairs and p.info["dof"] == npairs - 9 - len(types) + 2
    # 4-bit samples are staged as whole 32-bit words of four antennas
    with pytest.raises(rrc.RRCError) as e:
        rrc.Plan(3, types, 1, 1, dtype="ci4")
    assert e.value.code == _lib.RRC_ENOTIMPL
    rrc.Plan(4, rrc.select_subset(4)[0], 1, 1, dtype="ci4")


def test_plan_info_sizes():
    for n, t in [(8, 256), (16, 1024), (32, 2048), (64, 4096)]:
        types, npairs = rrc.select_subset(n)
        p = rrc.Plan(n, types, 4, t, dtype="ci4" if n == 64 else "c64")
        assert p.info["n_ant"] == n * n and p.info["n_lags"] == 2 * n * (n - 1)
        assert p.info["n_pairs"] == npairs
        assert p.info["dof"] == npairs - n * n - len(types) + 2
        assert p.info["fft_size"] == max(16, 1 << (2 * n - 1).bit_length())
        assert p.info["workspace_bytes"] > 0


def test_raw_abi_rejects_null_pointers():
    lib = rrc.load_library()
    types, _ = rrc.select_subset(8)
    plan = rrc.Plan(8, types, 1, 64)
    h = plan._h
    assert lib.rrc_fftcorr(h, None, None, None, None, None, None) == _lib.RRC_EINVAL
    assert lib.rrc_xengine(h, None, None, None, None) == _lib.RRC_EINVAL
    assert lib.rrc_solve(h, None, None, None, None, None, None, None, None, None, None) == _lib.RRC_EINVAL
    assert lib.rrc_run(h, None, 1, None) == _lib.RRC_EINVAL
    assert lib.rrc_plan_get_info(None, None) == _lib.RRC_EINVAL
    sz = ctypes.c_size_t()
    assert lib.rrc_workspace_size(h, ctypes.byref(sz)) == 0 and sz.value == plan.info["workspace_bytes"]


@pytest.mark.parametrize("n,k,base", [(4, 4, 0.0), (6, 5, 0.0), (8, 5, 0.0), (8, 8, 0.0), (10, 7, 0.0),
                                      (12, 9, 2.0), (16, 6, 0.0)])
def test_gain_variance_matches_oracle(n, k, base):
    # eq. gaincov per antenna: the library's banded factorisation against the
    # oracle's dense pseudo-inverse with the same degeneracy projection
    from oracle import stats as OS
    allt = G.select_subset_square(n, 1.0, base if base > 1 else np.e)
    types = [tuple(t) for t in allt] if len(allt) >= k else [tuple(t) for t in G.square_types(n)[0][:k]]
    pos = G.square_positions(n)
    pairs, tix = G.group_pairs(pos, types)
    ref = OS.predicted_gain_variance(pos, pairs, tix, len(types), snr=10.0)
    got = rrc.gain_variance(n, types, 10.0)
    assert np.max(np.abs(got - ref) / ref) < 1e-9


def test_gain_variance_refuses_degenerate_selection():
    with pytest.raises(rrc.RRCError) as e:
        rrc.gain_variance(6, [(1, 0), (0, 1)], 10.0)
    assert e.value.code == _lib.RRC_EDEGEN


@pytest.mark.parametrize("n,p,base", [(4, 1.0, 0.0), (8, 1.0, 0.0), (8, 0.5, 2.0), (16, 1.0, 0.0), (32, 1.0, 0.0)])
def test_lowcad_schedule_matches_oracle(n, p, base):
    # Sec. 4 round robin: whole groups in lag order within p N log N per cycle
    from oracle import lowcad as LC
    import math
    got = rrc.lowcad_schedule(n, p, base)
    assert got == LC.schedule(n, p, base if base > 1 else math.e)


# ----------------------------------------------------------- masked lattices

@pytest.mark.parametrize("side", [2, 3, 4, 5, 11, 32])
def test_hex_mask_matches_oracle(side):
    # the hexagon on its lattice grid: 3 side (side - 1) + 1 antennas (37 at
    # side 4, 331 at side 11)
    n, m = rrc.hex_mask(side)
    n2, m2, pos = G.hex_grid(side)
    assert n == n2 and np.array_equal(m.astype(bool), m2)
    assert int(m.sum()) == 3 * side * (side - 1) + 1 == len(pos)


def test_hex_mask_refuses_grids_past_the_limit():
    with pytest.raises(rrc.RRCError) as e:
        rrc.hex_mask(33)
    assert e.value.code == _lib.RRC_ERANGE


@pytest.mark.parametrize("side,p,base", [(3, 1.0, 0.0), (4, 1.0, 0.0), (4, 0.5, 2.0), (5, 1.0, 0.0),
                                         (8, 1.0, 0.0), (11, 1.0, 0.0)])
def test_masked_selection_matches_oracle(side, p, base):
    # Sec. 5 rule on the hexagonal lattice: groups by length under the hex
    # metric, pair counts over the antennas
    import math
    n, m = rrc.hex_mask(side)
    _, _, pos = G.hex_grid(side)
    types, npairs = rrc.select_subset_masked(n, m, "hex", p, base)
    want = G.select_subset(pos, G.HEX_METRIC, p, base if base > 1 else math.e)
    assert types == [tuple(t) for t in want]
    assert npairs == len(G.group_pairs(pos, want)[0])


@pytest.mark.parametrize("side", [3, 4, 6])
def test_masked_degeneracy_count_matches_oracle(side):
    # the three nearest-neighbour directions are the minimum (Sec. 5.2),
    # two of them leave the lattice split (more null directions)
    n, m = rrc.hex_mask(side)
    _, _, pos = G.hex_grid(side)
    for types in ([(1, 0), (0, 1)], [(1, 0), (-1, 1), (0, 1)], [(1, 0), (-1, 1), (0, 1), (1, 1)],
                  [(1, 0), (-2, 1)]):
        assert rrc.degeneracy_count_masked(n, m, types) == G.nullity(pos, types), types
    assert rrc.degeneracy_count_masked(n, m, [(1, 0), (-1, 1), (0, 1)]) == (1, 3)


def test_full_mask_equals_square_grid():
    # every grid point an antenna: the square grid's selection and counts
    for n in (4, 8, 16):
        full = np.ones(n * n, dtype=np.uint8)
        assert rrc.select_subset_masked(n, full, "square") == rrc.select_subset(n)
        types, _ = rrc.select_subset(n)
        assert rrc.degeneracy_count_masked(n, full, types) == rrc.degeneracy_count(n, types)


def test_masked_plan_info_and_refusals():
    side = 4
    n, m = rrc.hex_mask(side)
    _, _, pos = G.hex_grid(side)
    types, npairs = rrc.select_subset_masked(n, m, "hex")
    plan = rrc.Plan(n, types, 3, 64, mask=m)
    assert plan.info["masked"] == 1 and plan.info["n_live"] == 37
    assert plan.n_pairs == npairs and plan.n_ant == n * n and plan.n_lags == 2 * n * (n - 1)
    assert plan.dof == npairs - 37 - len(types) + 2
    lib = rrc.load_library()
    io = _lib.RunIO()
    # the whole-path calls refuse a masked plan before touching any pointer
    assert lib.rrc_run(plan._h, None, 0, ctypes.byref(io)) == _lib.RRC_ENOTIMPL
    assert lib.rrc_run_static(plan._h, None, 0, ctypes.byref(io)) == _lib.RRC_ENOTIMPL
    tune = _lib.Tune()
    io.d_gains_in = 1
    assert lib.rrc_plan_tune(plan._h, None, ctypes.byref(io), None, ctypes.byref(tune)) == _lib.RRC_ENOTIMPL
    one = ctypes.c_void_p(8)
    assert lib.rrc_solve(plan._h, None, one, None, None, one, one, one, one, one, None) == _lib.RRC_ENOTIMPL
    assert lib.rrc_chisq_fwd(plan._h, None, one, one, one, one) == _lib.RRC_ENOTIMPL
    # omnical on a masked plan needs the workspace (its pair tables)
    assert lib.rrc_omnical(plan._h, None, one, one, 1, 0.0, 1, one, one, one, one, one, None, None) == _lib.RRC_EINVAL
    hs = (ctypes.c_void_p * 1)(plan._h)
    b = ctypes.c_void_p()
    assert lib.rrc_batch_create(ctypes.byref(b), 1, hs, 0) == _lib.RRC_ENOTIMPL
    # started from the caller's gains the whole path accepts a masked plan
    # (these calls then fail only on the missing buffers)
    pg = rrc.Plan(n, types, 3, 64, mask=m, init_mode="gains")
    assert lib.rrc_run(pg._h, None, 0, ctypes.byref(_lib.RunIO())) == _lib.RRC_EINVAL
    assert lib.rrc_solve(pg._h, None, one, one, None, one, one, one, one, one, None) == _lib.RRC_EINVAL


def test_masked_plan_errors():
    n, m = rrc.hex_mask(4)
    # a type no pair of the hexagon realises
    with pytest.raises(rrc.RRCError) as e:
        rrc.Plan(n, [(1, 0), (-1, 1), (0, 1), (6, 6)], 1, 16, mask=m)
    assert e.value.code == _lib.RRC_EINVAL
    # too few types: more than the four degeneracies
    with pytest.raises(rrc.RRCError) as e:
        rrc.Plan(n, [(1, 0), (0, 1)], 1, 16, mask=m)
    assert e.value.code == _lib.RRC_EDEGEN
    # no +y neighbour of the first antenna: the references are missing
    bad = m.copy()
    first = int(np.nonzero(bad)[0][0])
    bad[first + n] = 0
    with pytest.raises(rrc.RRCError) as e:
        rrc.Plan(n, [(1, 0), (-1, 1), (0, 1)], 1, 16, mask=bad)
    assert e.value.code == _lib.RRC_EINVAL
    # 4-bit plans on an odd grid (whole 32-bit words of samples)
    with pytest.raises(rrc.RRCError) as e:
        rrc.Plan(n, [(1, 0), (-1, 1), (0, 1)], 1, 16, dtype="ci4", mask=m)
    assert e.value.code == _lib.RRC_ENOTIMPL


def test_fft_size_choices():
    # default: the smallest of 16, 32, 48, 64, 96, 128 with M >= 2n - 1 (the
    # lags never wrap round); the next power of two is the one alternative
    for n, default, alt in ((3, 16, None), (8, 16, None), (16, 32, None), (17, 48, 64), (24, 48, 64),
                            (25, 64, None), (32, 64, None), (33, 96, 128), (40, 96, 128), (48, 96, 128),
                            (49, 128, None), (64, 128, None)):
        types, _ = rrc.select_subset(n)
        p = rrc.Plan(n, types, 1, 64)
        assert p.info["fft_size"] == default, n
        for m in (16, 32, 48, 64, 96, 128):
            if m in (default, alt):
                p.set_fft_size(m)
                assert p.info["fft_size"] == m
            else:
                with pytest.raises(rrc.RRCError) as e:
                    p.set_fft_size(m)
                assert e.value.code == _lib.RRC_EINVAL
        # the workspace holds the larger grid's partial sums
        if alt:
            ws = p.info["workspace_bytes"]
            p.set_fft_size(default)
            assert p.info["workspace_bytes"] == ws

def test_branch_orders_accepted():
    types, _ = rrc.select_subset(8)
    p = rrc.Plan(8, types, 1, 64)
    for o in ("xeng_first", "fft_first", "serial"):
        p.set_order(o)
    lib = rrc.load_library()
    assert lib.rrc_plan_set_order(p._h, 3) == _lib.RRC_EINVAL
    assert lib.rrc_plan_set_order(p._h, -1) == _lib.RRC_EINVAL
