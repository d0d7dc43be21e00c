"""Host read-outs of the library against the oracle's (oracle/diag.py, pinned by
closed forms): the wall forces (qtt_forces_host, host FP64) on the same dense
fields, an FD step of the rotating cylinder on the 2^5 x 2^5 grid, and the
Strouhal number and lift amplitude of a lift history. No GPU."""
import ctypes

import numpy as np


def test_forces_host_matches_oracle():
    from oracle import diag, fd
    from oracle.grid import OGrid
    from paper_2507_05222_amd import qtt as Q
    from qtt_inputs import noise_fields
    n, Re, dt, alpha = 5, 100.0, 1e-3, 0.7
    g = OGrid(n, n)
    S = fd.FDSolver(g, Re, dt, alpha=alpha)
    nz = noise_fields(n, n, 1e-2, seed=3)
    u, v = 1.0 + nz[0].ravel(), nz[1].ravel()
    for _ in range(2):
        st = S.step(u, v, return_stages=True)
        u, v = st["u"], st["v"]
    p = st["p"]
    bc = fd.velocity_bc(g, alpha)
    cd_o, cl_o = diag.forces(g, u, v, p, Re, bc["u_wall"], bc["v_wall"])
    N = 2 ** n
    U, V, P = u.reshape(N, N), v.reshape(N, N), p.reshape(N, N)
    rows = np.ascontiguousarray(np.concatenate([U[0], U[1], V[0], V[1], P[0]]))
    cyl = Q.cylinder(n, 20.0, Re, dt, alpha)
    cd, cl = ctypes.c_double(0), ctypes.c_double(0)
    assert Q.lib().qtt_forces_host(ctypes.byref(cyl), rows.ctypes.data, ctypes.byref(cd), ctypes.byref(cl)) == 0
    assert abs(cd.value - cd_o) <= 1e-12 * abs(cd_o) and abs(cl.value - cl_o) <= 1e-12 * max(abs(cl_o), 1e-3), \
        (cd.value, cd_o, cl.value, cl_o)


def test_strouhal_matches_oracle():
    """The binding's Strouhal read-out against the oracle's on a lift history shaped
    like the transient cylinder's (growing, then saturating oscillation, sampled
    every 10 steps of dt = 2e-3), and against the closed form of a pure sinusoid."""
    from oracle import diag
    from paper_2507_05222_amd import diag as D
    t = 2e-3 * 10 * np.arange(1, 2001)
    env = 0.6 * (1.0 - np.exp(-t / 12.0))
    cl = 0.02 + env * np.sin(2 * np.pi * 0.192 * t + 0.3)
    st_o, amp_o = diag.strouhal(t, cl, min_periods=2)
    st, amp = D.strouhal(t, cl)
    assert abs(st - st_o) <= 1e-12 * st_o and abs(amp - amp_o) <= 1e-12 * amp_o
    assert abs(st - 0.192) < 2e-3
    st, amp = D.strouhal(t, 0.4 * np.sin(2 * np.pi * 0.2 * t))
    assert abs(st - 0.2) < 1e-5 and abs(amp - 0.4) < 1e-3


def test_strouhal_edge_cases():
    """Fewer crossings than asked for gives no Strouhal number; malformed calls are refused."""
    from paper_2507_05222_amd import diag as D, qtt as Q
    import pytest
    t = np.linspace(0.0, 1.0, 101)
    st, amp = D.strouhal(t, t, window=1.0)      # a ramp: a single upward crossing of its mean
    assert st is None and abs(amp - 0.5) < 1e-15
    with pytest.raises(Q.QttError):
        D.strouhal(t[:1], t[:1])


def test_network_input_rule():
    """qtt_ws_input_host: channels b / rms(b), Re / 200, alpha / 2 in FP32, scale rms(b);
    b = 0 has no scale and is refused."""
    from paper_2507_05222_amd import qtt as Q, warmstart as W
    import pytest
    rng = np.random.default_rng(9)
    b = rng.standard_normal((64, 64)) * 3.0
    x, r = W.ws_input(b, 150.0, 1.2)
    rms = np.sqrt(np.mean(b * b))
    assert abs(r - rms) <= 1e-14 * rms
    np.testing.assert_array_equal(x[0], (b / rms).astype(np.float32))
    assert np.all(x[1] == np.float32(0.75)) and np.all(x[2] == np.float32(0.6))
    with pytest.raises(Q.QttError, match="ENUMERIC"):
        W.ws_input(np.zeros((64, 64)), 100.0, 0.0)
