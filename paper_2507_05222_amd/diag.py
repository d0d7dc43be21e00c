"""Diagnostics of the flow state (Sec. 4, App. C, App. F): grid rows read out of
the QTT fields, drag and lift coefficients, Strouhal number from a lift history.
Row read-out and forces run in libqtt.so (host FP64); this module marshals."""
from __future__ import annotations

import ctypes

import numpy as np

from . import qtt as Q


def read_rows(ctx: Q.Context, m: Q.MPS, rows, order=0) -> np.ndarray:
    """Rows (0 = next to the wall) of a 2^n x 2^n field in bit order `order`
    (0 interleaved, 1 concatenated), shape (len(rows), 2^n)."""
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    N = 2 ** (m.L // 2)
    out = np.empty((len(rows), N))
    ctx.check(Q.lib().qtt_read_rows(ctx.h, ctypes.byref(m.desc()), len(rows), rows.ctypes.data,
                                    Q.ORDERS.get(order, order), out.ctypes.data, Q._stream()))
    return out


def forces(ctx: Q.Context, cyl: Q.CCylinder, u: Q.MPS, v: Q.MPS, p: Q.MPS):
    """(C_D, C_L) of the state (App. F)."""
    ru = read_rows(ctx, u, [0, 1], cyl.order)
    rv = read_rows(ctx, v, [0, 1], cyl.order)
    rp = read_rows(ctx, p, [0], cyl.order)
    rows = np.ascontiguousarray(np.concatenate([ru.ravel(), rv.ravel(), rp.ravel()]))
    cd, cl = ctypes.c_double(0), ctypes.c_double(0)
    rc = Q.lib().qtt_forces_host(ctypes.byref(cyl), rows.ctypes.data, ctypes.byref(cd), ctypes.byref(cl))
    if rc != 0:
        raise Q.QttError(rc, "qtt_forces_host")
    return cd.value, cl.value


def strouhal(t, cl, window=0.5, min_crossings=2):
    """(St, lift amplitude) of a lift history (qtt_strouhal_host: upward zero crossings
    of C_L - mean over the last `window` of the samples, linearly interpolated,
    D = U = 1); St is None with fewer than `min_crossings` crossings."""
    t = np.ascontiguousarray(t, dtype=np.float64)
    cl = np.ascontiguousarray(cl, dtype=np.float64)
    st, amp = ctypes.c_double(0), ctypes.c_double(0)
    rc = Q.lib().qtt_strouhal_host(t.ctypes.data, cl.ctypes.data, len(t), float(window), int(min_crossings),
                                   ctypes.byref(st), ctypes.byref(amp))
    if rc != 0:
        raise Q.QttError(rc, "qtt_strouhal_host")
    return (None if np.isnan(st.value) else st.value), amp.value
