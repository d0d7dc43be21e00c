"""The recorded TT run of the rotating cylinder (Sec. 4.2, Table 2: G1, Re = 100, rotation
rate 1, chi = 40, t = 0 .. 40; written by the library on the GPU, results/) against the
oracle's FD history of the same case over the same window, and against the TT row of
Table 2 for chi = 40. CPU only: checks the committed record, not the GPU."""
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
