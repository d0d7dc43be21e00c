"""Diagnostics of the flow state (Sec. 4, App. C, App. F): grid rows read out of
the QTT fields, drag and lift coefficients, Strouhal number from a lift history.
Row read-out and forces run in libqtt.so (host FP64); this module marshals."""
from __future__ import annotations

import ctypes

import numpy as np

from . import qtt as Q


def read_rows(ctx: Q.Context, m: Q.MPS, rows) -> np.ndarray:
    """Rows (0 = next to the wall) of a 2^n x 2^n field, shape (len(rows), 2^n)."""
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    N = 2 ** (m.L // 2)
    out = np.empty((len(rows), N))
    ctx.check(Q.lib().qtt_read_rows(ctx.h, ctypes.byref(m.desc()), len(rows), rows.ctypes.data, out.ctypes.data,
                                    Q._stream()))
    return out


def forces(ctx: Q.Context, cyl: Q.CCylinder, u: Q.MPS, v: Q.MPS, p: Q.MPS):
    """(C_D, C_L) of the state (App. F)."""
    ru = read_rows(ctx, u, [0, 1])
    rv = read_rows(ctx, v, [0, 1])
    rp = read_rows(ctx, p, [0])
    rows = np.ascontiguousarray(np.concatenate([ru.ravel(), rv.ravel(), rp.ravel()]))
    cd, cl = ctypes.c_double(0), ctypes.c_double(0)
    rc = Q.lib().qtt_forces_host(ctypes.byref(cyl), rows.ctypes.data, ctypes.byref(cd), ctypes.byref(cl))
    if rc != 0:
        raise Q.QttError(rc, "qtt_forces_host")
    return cd.value, cl.value


def strouhal(t, cl, window=0.5):
    """(St, lift amplitude) from upward zero crossings of C_L - mean over the last
    `window` of the history, linearly interpolated (D = U = 1); St is None with
    fewer than two crossings."""
    t = np.asarray(t, dtype=float)
    cl = np.asarray(cl, dtype=float)
    n0 = int(len(t) * (1.0 - window))
    t, y = t[n0:], cl[n0:] - cl[n0:].mean()
    up = np.nonzero((y[:-1] < 0) & (y[1:] >= 0))[0]
    tc = t[up] - y[up] * (t[up + 1] - t[up]) / (y[up + 1] - y[up])
    amp = 0.5 * (cl[n0:].max() - cl[n0:].min()) if len(cl[n0:]) else 0.0
    if len(tc) < 2:
        return None, amp
    return 1.0 / float(np.mean(np.diff(tc))), amp
