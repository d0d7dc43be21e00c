"""The recorded TT runs (written by the library on the GPU, results/) against the oracle's
FD histories of the same cases: the rotating cylinder of Sec. 4.2 (Table 2: G1, Re = 100,
rotation rate 1, chi = 40, t = 0 .. 40), also against the TT row of Table 2 for chi = 40,
and the 2^10 x 2^10 transient cylinder at Re = 200 (chi = 64, mixed path, t = 0 .. 40).
CPU only: checks the committed records, not the GPU."""
import json
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TT = os.path.join(ROOT, "results", "rotating_g1_re100_chi40_tt_forces.txt")
FD = os.path.join(ROOT, "tests", "golden", "rotating_g1_re100_forces.txt")
DT = 2e-3


def _spectral_st(t, y):
    """Frequency of the largest peak of the Hann-windowed spectrum (parabolic
    interpolation on a 16x zero-padded FFT)."""
    y = y - y.mean()
    n = len(y)
    N = 16 * n
    F = np.abs(np.fft.rfft(y * np.hanning(n), N))
    f = np.fft.rfftfreq(N, t[1] - t[0])
    i = int(np.argmax(F[1:])) + 1
    a, b, c = F[i - 1], F[i], F[i + 1]
    return f[i] + 0.5 * (a - c) / (a - 2 * b + c) * (f[1] - f[0])


def test_tt_rotating_cylinder_matches_fd_and_table2():
    tt = np.loadtxt(TT)
    fd = np.loadtxt(FD)
    last = int(tt[-1, 0])
    assert last == 20000 and np.array_equal(tt[:, 0], fd[fd[:, 0] <= last, 0])
    fd = fd[fd[:, 0] <= last]
    t = tt[:, 0] * DT
    w = t >= 0.5 * t[-1]                     # t = 20 .. 40, the same window for both
    cl_tt, cl_fd = tt[w, 2].mean(), fd[w, 2].mean()
    cd_tt, cd_fd = tt[w, 1].mean(), fd[w, 1].mean()
    st_tt, st_fd = _spectral_st(t[w], tt[w, 2]), _spectral_st(t[w], fd[w, 2])
    assert abs(cl_tt - cl_fd) <= 5e-3 * cl_fd, (cl_tt, cl_fd)
    assert abs(cd_tt - cd_fd) <= 5e-3 * cd_fd, (cd_tt, cd_fd)
    assert abs(st_tt - st_fd) <= 5e-3 * st_fd, (st_tt, st_fd)
    # Table 2, TT chi = 40 (the mean lift depends on the averaging window, so only St)
    rows = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_numbers.json")))["tt_rows"]
    st_paper = next(r["value"] for r in rows if r["case"] == "rotating_g1_re100" and r["quantity"] == "St")
    assert abs(st_tt - st_paper) <= 5e-3 * st_paper, (st_tt, st_paper)
    # the whole drag and lift histories: relative L2 differences of about 1%
    assert np.linalg.norm(tt[:, 1] - fd[:, 1]) <= 0.03 * np.linalg.norm(fd[:, 1])
    assert np.linalg.norm(tt[:, 2] - fd[:, 2]) <= 0.03 * np.linalg.norm(fd[:, 2])


def _crossings(t, y):
    """Upward zero crossings of y - mean(y), linearly interpolated."""
    y = y - y.mean()
    i = np.where((y[:-1] < 0) & (y[1:] >= 0))[0]
    return t[i] - y[i] * (t[i + 1] - t[i]) / (y[i + 1] - y[i])


def test_tt_transient_cylinder_matches_fd():
    """2^10 x 2^10, Re = 200, chi = 64, mixed path: over the last half (t = 20 .. 40) the
    Strouhal number from the lift's upward crossings, the lift amplitude and the mean drag
    agree with the oracle's FD run, and the whole histories stay within the 3e-3 band."""
    tt = np.loadtxt(os.path.join(ROOT, "results", "c3_re200_chi64_mixed_tt_forces.txt"))
    fd = np.loadtxt(os.path.join(ROOT, "tests", "golden", "c3_re200_forces.txt"))
    assert int(tt[-1, 0]) == 20000 and np.array_equal(tt[:, 0], fd[:, 0])
    t = tt[:, 0] * DT
    w = t >= 20.0
    ct, cf = _crossings(t[w], tt[w, 2]), _crossings(t[w], fd[w, 2])
    assert len(ct) == len(cf) >= 3 and np.abs(ct - cf).max() < 5e-3, (ct, cf)
    st_tt, st_fd = (len(ct) - 1) / (ct[-1] - ct[0]), (len(cf) - 1) / (cf[-1] - cf[0])
    assert abs(st_tt - st_fd) <= 1e-3 * st_fd, (st_tt, st_fd)
    amp_tt, amp_fd = np.ptp(tt[w, 2]) / 2, np.ptp(fd[w, 2]) / 2
    assert abs(amp_tt - amp_fd) <= 3e-3 * amp_fd, (amp_tt, amp_fd)
    assert abs(tt[w, 1].mean() - fd[w, 1].mean()) <= 1e-3 * fd[w, 1].mean()
    assert np.linalg.norm(tt[:, 1] - fd[:, 1]) <= 3e-3 * np.linalg.norm(fd[:, 1])
    assert np.linalg.norm(tt[:, 2] - fd[:, 2]) <= 5e-3 * np.linalg.norm(fd[:, 2])


def test_steady_re40_errors_fall_with_chi_to_the_band():
    """Steady Re = 40 cylinder, 2^8 x 2^8, 2000 steps on the FP64 path at chi = 16, 32, 48
    (results/c2_steady_re40_chi_sweep.json), scored against the FD oracle's run of the same
    steps: no run beats the best bond-chi approximation of the oracle's fields by more
    than TT-SVD's quasi-optimality factor sqrt(L - 1) (tests/golden/c2_best_approximation.txt,
    oracle only), the errors fall with chi, and at chi = 48 u, v, p and the drag are inside
    the 3e-3 band."""
    rec = json.load(open(os.path.join(ROOT, "results", "c2_steady_re40_chi_sweep.json")))
    floor = {int(r[0]): r[1:] for r in np.loadtxt(os.path.join(ROOT, "tests", "golden", "c2_best_approximation.txt"))}
    errs = {}
    for chi in (16, 32, 48):
        p = rec["runs"][str(chi)]["paths"]["fp64"]
        e = [p["eps_l2_vs_oracle"][k] for k in ("u", "v", "p")]
        errs[chi] = e
        assert all(ei >= fi / np.sqrt(15.0) for ei, fi in zip(e, floor[chi])), (chi, e, floor[chi])
    for k in range(3):
        assert errs[16][k] > errs[32][k] > errs[48][k]
    assert max(errs[48]) <= 3e-3
    assert rec["runs"]["48"]["paths"]["fp64"]["C_D_rel_err"] <= 3e-3
