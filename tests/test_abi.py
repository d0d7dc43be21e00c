"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and
its host-side operator builder matches the oracle's sparse operators."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "qtt.h")
LIB = os.path.join(ROOT, "paper_2507_05222_amd", "libqtt.so")


def declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"\b(qtt_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libqtt.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert "qtt_apply_mpo" in names and "qtt_fractional_step" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("alpha,order", [(0.0, "interleaved"), (0.7, "interleaved"), (0.7, "concatenated")])
def test_builder_operators_match_oracle(alpha, order):
    from oracle import fd, qttref as R
    from oracle.grid import OGrid
    from paper_2507_05222_amd import qtt as Q
    import scipy.sparse as sp
    n = 4
    cyl = Q.cylinder(n, r_out=20.0, Re=100.0, dt=1e-3, alpha=alpha, order=order)
    g = OGrid(n, n)
    S = fd.FDSolver(g, 100.0, 1e-3, alpha=alpha)
    perm = R.grid_perm(n, n, order)
    x = np.random.default_rng(0).standard_normal(4 ** n)
    jh = np.sqrt(S.ops.absJ)
    ops = {Q.OP["DX"]: S.Dx, Q.OP["DZ"]: S.Dz, Q.OP["DXP"]: S.Dx_p, Q.OP["DZP"]: S.Dz_p, Q.OP["LAP"]: S.Lap,
           Q.OP["P"]: S.P, Q.OP["WX"]: sp.diags(-S.ops.absJ) @ S.Dx, Q.OP["WZ"]: sp.diags(-S.ops.absJ) @ S.Dz,
           Q.OP["HS"]: sp.diags(jh) @ S.H @ sp.diags(1 / jh), Q.OP["JH"]: sp.diags(jh), Q.OP["JMH"]: sp.diags(1 / jh)}
    for which, A in ops.items():
        slots, bonds, cap = Q.build_host(cyl, which)
        cores = [slots.reshape(2 * n, cap, 4, cap)[k, :bonds[k], :, :bonds[k + 1]].reshape(bonds[k], 2, 2, bonds[k + 1])
                 for k in range(2 * n)]
        y = R.mpo_apply_dense(cores, x[perm])
        ref = (A @ x)[perm]
        assert np.abs(y - ref).max() < 1e-12 * np.abs(ref).max(), which
        assert max(bonds) <= 25
    b = S.bc
    c = 1e-3 / 100.0
    vecs = {Q.VEC["BX_U"]: S.bcx(b["u_wall"], b["u_out"]), Q.VEC["BZ_U"]: S.bcz(b["u_wall"], b["u_out"]),
            Q.VEC["BX_V"]: S.bcx(b["v_wall"], b["v_out"]), Q.VEC["BZ_V"]: S.bcz(b["v_wall"], b["v_out"]),
            Q.VEC["BL_U"]: c * S.bcL(b["u_wall"], b["u_out"]), Q.VEC["BL_V"]: c * S.bcL(b["v_wall"], b["v_out"]),
            Q.VEC["ABSJ"]: S.ops.absJ}
    vecs[Q.VEC["BW"]] = -S.ops.absJ * (vecs[Q.VEC["BX_U"]] + vecs[Q.VEC["BZ_V"]])
    for which, v in vecs.items():
        slots, bonds, cap = Q.build_host(cyl, which)
        cores = [slots.reshape(2 * n, cap, 2, cap)[k, :bonds[k], :, :bonds[k + 1]] for k in range(2 * n)]
        ref = v[perm]
        assert np.abs(R.tt_full(cores) - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300), which
