"""ctypes binding of libqtt.so (include/qtt.h): argument marshalling only.

Device memory comes from torch (float64 / int32 CUDA tensors); every computation
runs in the HIP library. There is no fallback: if libqtt.so is missing or no GPU
is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqtt.so")

F64, F32, BF16 = 0, 1, 2
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}

OP = dict(DX=0, DZ=1, DXP=2, DZP=3, WX=4, WZ=5, HS=6, P=7, JH=8, JMH=9, LAP=10)
VEC = dict(BX_U=100, BZ_U=101, BX_V=102, BZ_V=103, BL_U=104, BL_V=105, BW=106, ABSJ=107)
TT_VEC = dict(MESH_X=200, MESH_Z=201, JAC=202)   # objects only qtt_build_tt makes
TT_OPS = ("DX", "DZ", "DXP", "DZP", "WX", "WZ", "LAP", "P")  # operators qtt_build_tt makes

ERRORS = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "ECAPACITY", -4: "ENUMERIC", -5: "ENOTCONVERGED", -6: "EHIP"}


class QttError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# C structs (mirror include/qtt.h)
# ---------------------------------------------------------------------------
class CMps(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("d", ctypes.c_int32), ("cap", ctypes.c_int32),
                ("bond", ctypes.c_void_p), ("data", ctypes.c_void_p)]


class CMpo(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("wcap", ctypes.c_int32), ("bond_host", ctypes.c_void_p),
                ("bond", ctypes.c_void_p), ("data", ctypes.c_void_p)]


class CTrunc(ctypes.Structure):
    _fields_ = [("rel_tol", ctypes.c_double), ("chi_max", ctypes.c_int32), ("fit_sweeps", ctypes.c_int32)]


class CSolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_sweeps", ctypes.c_int32), ("max_local_iters", ctypes.c_int32),
                ("local_tol", ctypes.c_double), ("contract_dt", ctypes.c_int32)]


class CSolveInfo(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("local_iters", ctypes.c_int32),
                ("residual", ctypes.c_double), ("residual0", ctypes.c_double)]


class CTerm(ctypes.Structure):
    _fields_ = [("coef", ctypes.c_double), ("M", ctypes.POINTER(CMpo)), ("x", ctypes.POINTER(CMps))]


class CFlowOps(ctypes.Structure):
    _fields_ = [(n, CMpo) for n in ("Dx", "Dz", "Dxp", "Dzp", "Wx", "Wz", "Hs", "P", "Jh", "Jmh")] + \
               [(n, CMps) for n in ("bx_u", "bz_u", "bx_v", "bz_v", "bL_u", "bL_v", "bW")]


class CFlowState(ctypes.Structure):
    _fields_ = [("u", CMps), ("v", CMps), ("p", CMps), ("id", ctypes.c_uint64)]


class CWsModel(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("out_scale", ctypes.c_double), ("re", ctypes.c_double),
                ("alpha", ctypes.c_double), ("chi", ctypes.c_int32), ("bf16", ctypes.c_int32)]


class CStepOpts(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("trunc", CTrunc), ("contract_dt", ctypes.c_int32),
                ("product_dt", ctypes.c_int32), ("helmholtz", CSolveOpts), ("poisson", CSolveOpts),
                ("warm", ctypes.POINTER(CWsModel)), ("rhs_out", ctypes.POINTER(CMps))]


class CStepInfo(ctypes.Structure):
    _fields_ = [("helm_u", CSolveInfo), ("helm_v", CSolveInfo), ("poisson", CSolveInfo),
                ("warm_used", ctypes.c_int32), ("warm_energy", ctypes.c_double), ("prev_energy", ctypes.c_double)]


ORDERS = {"interleaved": 0, "concatenated": 1}


class CCylinder(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("r_out", ctypes.c_double), ("Re", ctypes.c_double),
                ("dt", ctypes.c_double), ("alpha", ctypes.c_double), ("u_inf", ctypes.c_double),
                ("order", ctypes.c_int32)]


_lib = None


def lib():
    """Load libqtt.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, p = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER
        L.qtt_create.argtypes = [i32, p(vp)]
        L.qtt_destroy.argtypes = [vp]
        L.qtt_last_error.argtypes = [vp]
        L.qtt_last_error.restype = ctypes.c_char_p
        L.qtt_apply_mpo.argtypes = [vp, i32, p(CMpo), p(CMps), p(CMps), p(CTrunc), i32, vp]
        L.qtt_round.argtypes = [vp, i32, p(CMps), p(CTrunc), vp]
        L.qtt_add.argtypes = [vp, i32, p(ctypes.c_double), p(CMps), p(ctypes.c_double), p(CMps), p(CMps),
                              p(CTrunc), vp]
        L.qtt_dot.argtypes = [vp, i32, p(CMps), p(CMps), p(ctypes.c_double), vp]
        L.qtt_dot_mpo.argtypes = [vp, i32, p(CMps), p(CMpo), p(CMps), p(ctypes.c_double), vp]
        L.qtt_dot_noalloc.argtypes = [vp, i32, p(CMps), p(CMps), vp, vp]
        L.qtt_apply_local.argtypes = [vp, i32, p(CMpo), p(CMps), p(CMps), vp]
        L.qtt_poisson_solve.argtypes = [vp, i32, p(CMpo), p(CMps), p(CMps), p(CSolveOpts), p(CSolveInfo), vp]
        L.qtt_fractional_step.argtypes = [vp, p(CFlowOps), p(CFlowState), p(CStepOpts), p(CStepInfo), vp]
        L.qtt_fit.argtypes = [vp, i32, i32, p(CTerm), p(CMps), i32, i32, i32, i32, vp]
        L.qtt_timer_start.argtypes = [vp, i32]
        L.qtt_timer_read.argtypes = [vp, p(ctypes.c_int64), p(ctypes.c_double), p(ctypes.c_double),
                                     p(ctypes.c_double), p(ctypes.c_double)]
        L.qtt_timer_durations.argtypes = [vp, p(ctypes.c_double), ctypes.c_int64, p(ctypes.c_int64)]
        L.qtt_build_host.argtypes = [p(CCylinder), i32, ctypes.c_int32, vp, vp, p(ctypes.c_int32)]
        L.qtt_build_tt.argtypes = [vp, p(CCylinder), i32, ctypes.c_int32, vp, vp, vp, p(ctypes.c_int32), vp]
        L.qtt_tt_svd_host.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, p(CTrunc), ctypes.c_int32, vp, vp]
        L.qtt_from_dense.argtypes = [vp, vp, ctypes.c_int32, p(CTrunc), p(CMps), vp]
        L.qtt_strouhal_host.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                        p(ctypes.c_double), p(ctypes.c_double)]
        L.qtt_ws_input_host.argtypes = [vp, ctypes.c_double, ctypes.c_double, vp, p(ctypes.c_double)]
        L.qtt_ws_act_floats.argtypes = [i32]
        L.qtt_ws_act_floats.restype = ctypes.c_size_t
        L.qtt_ws_forward.argtypes = [vp, vp, vp, i32, vp, vp, i32, vp]
        L.qtt_ws_backward.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp]
        L.qtt_ws_mse.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.qtt_ws_adam_step.argtypes = [vp, vp, vp, vp, vp, i32, ctypes.c_float, vp]
        L.qtt_ws_coarse.argtypes = [vp, p(CMps), vp, vp]
        L.qtt_read_rows.argtypes = [vp, p(CMps), i32, vp, ctypes.c_int32, vp, vp]
        L.qtt_forces_host.argtypes = [p(CCylinder), vp, p(ctypes.c_double), p(ctypes.c_double)]
        _lib = L
    return _lib


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# context and containers
# ---------------------------------------------------------------------------
class Context:
    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the QTT library runs on the GPU only")
        self.device = device
        torch.cuda.set_device(device)
        h = ctypes.c_void_p()
        rc = lib().qtt_create(device, ctypes.byref(h))
        if rc != 0:
            raise QttError(rc, "qtt_create failed")
        self.h = h

    def check(self, rc):
        if rc != 0:
            raise QttError(rc, lib().qtt_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().qtt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MPS:
    """A TT-vector in slot layout on the GPU (see include/qtt.h)."""

    def __init__(self, L: int, cap: int, device="cuda", d: int = 2):
        self.L, self.cap, self.d = L, cap, d
        self.data = torch.zeros(L * cap * d * cap, dtype=torch.float64, device=device)
        b = np.ones(L + 1, dtype=np.int32)
        self.bond = torch.from_numpy(b).to(device)

    def desc(self) -> CMps:
        return CMps(self.L, self.d, self.cap, self.bond.data_ptr(), self.data.data_ptr())

    @classmethod
    def from_cores(cls, cores: Sequence[np.ndarray], cap: int, device="cuda"):
        L = len(cores)
        d = cores[0].shape[1]
        m = cls(L, cap, device, d)
        slots = np.zeros((L, cap, d, cap))
        bonds = [1]
        for k, c in enumerate(cores):
            a, dd, b = c.shape
            if a > cap or b > cap:
                raise ValueError(f"core {k} shape {c.shape} exceeds cap {cap}")
            slots[k, :a, :, :b] = c
            bonds.append(b)
        m.data.copy_(torch.from_numpy(slots.reshape(-1)))
        m.bond.copy_(torch.tensor(bonds, dtype=torch.int32))
        return m

    @classmethod
    def from_slots(cls, slots: np.ndarray, bonds: np.ndarray, cap: int, device="cuda"):
        L = len(bonds) - 1
        m = cls(L, cap, device)
        m.data.copy_(torch.from_numpy(np.ascontiguousarray(slots, dtype=np.float64).reshape(-1)))
        m.bond.copy_(torch.from_numpy(np.asarray(bonds, dtype=np.int32)))
        return m

    def bonds(self) -> np.ndarray:
        return self.bond.cpu().numpy()

    def cores(self) -> list[np.ndarray]:
        b = self.bonds()
        s = self.data.cpu().numpy().reshape(self.L, self.cap, self.d, self.cap)
        return [s[k, :b[k], :, :b[k + 1]].copy() for k in range(self.L)]

    def copy_(self, other: "MPS"):
        self.data.copy_(other.data)
        self.bond.copy_(other.bond)
        return self


class MPO:
    """A TT-matrix in slot layout on the GPU; bonds also kept on the host."""

    def __init__(self, slots: np.ndarray, bonds: np.ndarray, wcap: int, device="cuda"):
        self.L = len(bonds) - 1
        self.wcap = wcap
        self.bond_host = np.ascontiguousarray(bonds, dtype=np.int32)
        self.bond = torch.from_numpy(self.bond_host.copy()).to(device)
        self.data = torch.from_numpy(np.ascontiguousarray(slots, dtype=np.float64).reshape(-1)).to(device)

    def desc(self) -> CMpo:
        return CMpo(self.L, self.wcap, self.bond_host.ctypes.data, self.bond.data_ptr(), self.data.data_ptr())

    @classmethod
    def empty(cls, L: int, wcap: int, device="cuda"):
        return cls(np.zeros(L * wcap * 4 * wcap), np.ones(L + 1, dtype=np.int32), wcap, device)

    @classmethod
    def from_cores(cls, cores: Sequence[np.ndarray], wcap: int | None = None, device="cuda"):
        L = len(cores)
        w = max(max(c.shape[0], c.shape[3]) for c in cores)
        wcap = wcap or w
        slots = np.zeros((L, wcap, 4, wcap))
        bonds = [1]
        for k, c in enumerate(cores):
            a, _, _, b = c.shape
            slots[k, :a, :, :b] = c.reshape(a, 4, b)
            bonds.append(b)
        return cls(slots, np.array(bonds, dtype=np.int32), wcap, device)

    def cores(self) -> list[np.ndarray]:
        s = self.data.cpu().numpy().reshape(self.L, self.wcap, 4, self.wcap)
        b = self.bond_host
        return [s[k, :b[k], :, :b[k + 1]].reshape(b[k], 2, 2, b[k + 1]).copy() for k in range(self.L)]


def _arr(ctype, items):
    return (ctype * len(items))(*items)


def _trunc(tol, chi, fit=0):
    return CTrunc(float(tol), int(chi), int(fit))


# ---------------------------------------------------------------------------
# operations (names follow include/qtt.h)
# ---------------------------------------------------------------------------
def apply_mpo(ctx: Context, Ms, xs, ys, tol=0.0, chi=None, dtype="f64", fit=2, stream=None):
    chi = chi if chi is not None else ys[0].cap
    ctx.check(lib().qtt_apply_mpo(ctx.h, len(xs), _arr(CMpo, [m.desc() for m in Ms]),
                                  _arr(CMps, [x.desc() for x in xs]), _arr(CMps, [y.desc() for y in ys]),
                                  ctypes.byref(_trunc(tol, chi, fit)), DTYPES.get(dtype, dtype), _stream(stream)))


def round_(ctx: Context, xs, tol=0.0, chi=None, stream=None):
    chi = chi if chi is not None else xs[0].cap
    ctx.check(lib().qtt_round(ctx.h, len(xs), _arr(CMps, [x.desc() for x in xs]),
                              ctypes.byref(_trunc(tol, chi)), _stream(stream)))


def add(ctx: Context, a, xs, b, ys, zs, tol=0.0, chi=None, stream=None):
    chi = chi if chi is not None else zs[0].cap
    n = len(xs)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (n,)).copy()
    b = np.broadcast_to(np.asarray(b, dtype=np.float64), (n,)).copy()
    ctx.check(lib().qtt_add(ctx.h, n, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            _arr(CMps, [x.desc() for x in xs]),
                            b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            _arr(CMps, [y.desc() for y in ys]), _arr(CMps, [z.desc() for z in zs]),
                            ctypes.byref(_trunc(tol, chi)), _stream(stream)))


def dot(ctx: Context, xs, ys, stream=None) -> np.ndarray:
    out = np.zeros(len(xs))
    ctx.check(lib().qtt_dot(ctx.h, len(xs), _arr(CMps, [x.desc() for x in xs]), _arr(CMps, [y.desc() for y in ys]),
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(stream)))
    return out


def dot_noalloc(ctx: Context, xs, ys, out: torch.Tensor, stream=None) -> torch.Tensor:
    """qtt_dot_noalloc: <x_i, y_i> into the device tensor out (float64, len(xs)), stream-ordered."""
    if out.dtype != torch.float64 or not out.is_cuda or out.numel() < len(xs):
        raise QttError(-1, "dot_noalloc: out must be a float64 device tensor of len(xs) values")
    ctx.check(lib().qtt_dot_noalloc(ctx.h, len(xs), _arr(CMps, [x.desc() for x in xs]),
                                    _arr(CMps, [y.desc() for y in ys]), ctypes.c_void_p(out.data_ptr()),
                                    _stream(stream)))
    return out


def dot_mpo(ctx: Context, xs, As, ys, stream=None) -> np.ndarray:
    out = np.zeros(len(xs))
    ctx.check(lib().qtt_dot_mpo(ctx.h, len(xs), _arr(CMps, [x.desc() for x in xs]),
                                _arr(CMpo, [a.desc() for a in As]), _arr(CMps, [y.desc() for y in ys]),
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(stream)))
    return out


def apply_local(ctx: Context, Ds, xs, ys, stream=None):
    ctx.check(lib().qtt_apply_local(ctx.h, len(xs), _arr(CMpo, [d.desc() for d in Ds]),
                                    _arr(CMps, [x.desc() for x in xs]), _arr(CMps, [y.desc() for y in ys]),
                                    _stream(stream)))


def fit(ctx: Context, problems, ys, chi=None, sweeps=1, init=1, dtype="f64", stream=None):
    """y_i ~ sum_t c M x for each problem i; problems[i] = [(coef, MPO or None, MPS), ...]."""
    n = len(ys)
    nt = len(problems[0])
    chi = chi if chi is not None else ys[0].cap
    keep = []
    terms = (CTerm * (n * nt))()
    for i, prob in enumerate(problems):
        if len(prob) != nt:
            raise ValueError("every problem needs the same number of terms")
        for t, (c, M, x) in enumerate(prob):
            xd = x.desc()
            keep.append(xd)
            md = None
            if M is not None:
                md = M.desc()
                keep.append(md)
            terms[i * nt + t] = CTerm(float(c), ctypes.pointer(md) if md is not None else None, ctypes.pointer(xd))
    ctx.check(lib().qtt_fit(ctx.h, n, nt, terms, _arr(CMps, [y.desc() for y in ys]), int(chi), int(sweeps), int(init),
                            DTYPES.get(dtype, dtype), _stream(stream)))


def solve_opts(tol=1e-8, max_sweeps=10, max_local_iters=100, local_tol=1e-3, dtype="f64") -> CSolveOpts:
    return CSolveOpts(float(tol), int(max_sweeps), int(max_local_iters), float(local_tol), DTYPES.get(dtype, dtype))


def poisson_solve(ctx: Context, As, bs, xs, opts: CSolveOpts, stream=None, raise_on_nonconv=False):
    n = len(xs)
    info = (CSolveInfo * n)()
    rc = lib().qtt_poisson_solve(ctx.h, n, _arr(CMpo, [a.desc() for a in As]), _arr(CMps, [b.desc() for b in bs]),
                                 _arr(CMps, [x.desc() for x in xs]), ctypes.byref(opts), info, _stream(stream))
    if rc == -5 and not raise_on_nonconv:
        return list(info), False
    ctx.check(rc)
    return list(info), True


# ---------------------------------------------------------------------------
# host-side setup (operators, initial fields)
# ---------------------------------------------------------------------------
def cylinder(n, r_out=20.0, Re=100.0, dt=1e-3, alpha=0.0, u_inf=1.0, order="interleaved") -> CCylinder:
    return CCylinder(int(n), float(r_out), float(Re), float(dt), float(alpha), float(u_inf),
                     ORDERS.get(order, order))


def build_host(cyl: CCylinder, which: int, cap: int | None = None):
    """(slots, bonds, cap) of an operator (QTT_OP_*) or boundary vector (QTT_VEC_*)."""
    need = ctypes.c_int32(0)
    rc = lib().qtt_build_host(ctypes.byref(cyl), int(which), 0, None, None, ctypes.byref(need))
    if rc != 0:
        raise QttError(rc, "qtt_build_host (query)")
    cap = max(cap or 0, need.value)
    L = 2 * cyl.n
    d = 4 if which < 100 else 2
    slots = np.zeros(L * cap * d * cap)
    bonds = np.zeros(L + 1, dtype=np.int32)
    rc = lib().qtt_build_host(ctypes.byref(cyl), int(which), cap, slots.ctypes.data, bonds.ctypes.data, None)
    if rc != 0:
        raise QttError(rc, "qtt_build_host")
    return slots, bonds, cap


def build_tt(ctx: "Context", cyl: CCylinder, which: int, cap: int | None = None, stream=None):
    """An operator (QTT_OP_* in TT_OPS: an MPO) or a mesh field (TT_VEC: an MPS) built
    in TT format on the device by qtt_build_tt."""
    need = ctypes.c_int32(0)
    st = _stream(stream)
    ctx.check(lib().qtt_build_tt(ctx.h, ctypes.byref(cyl), int(which), 0, None, None, None, ctypes.byref(need), st))
    cap = max(cap or 0, need.value)
    L = 2 * cyl.n
    if which >= 100:
        m = MPS(L, cap)
        bh = np.zeros(L + 1, dtype=np.int32)
        ctx.check(lib().qtt_build_tt(ctx.h, ctypes.byref(cyl), int(which), cap, m.data.data_ptr(),
                                     m.bond.data_ptr(), bh.ctypes.data, None, st))
        return m
    m = MPO.empty(L, cap)
    ctx.check(lib().qtt_build_tt(ctx.h, ctypes.byref(cyl), int(which), cap, m.data.data_ptr(), m.bond.data_ptr(),
                                 m.bond_host.ctypes.data, None, st))
    return m


def build_mpo(cyl: CCylinder, which: int, device="cuda") -> MPO:
    slots, bonds, cap = build_host(cyl, which)
    return MPO(slots, bonds, cap, device)


def build_vec(cyl: CCylinder, which: int, cap: int, device="cuda") -> MPS:
    slots, bonds, c = build_host(cyl, which, cap)
    if c != cap:
        raise QttError(-3, f"vector needs cap {c} > {cap}")
    return MPS.from_slots(slots, bonds, cap, device)


def tt_svd_host(dense: np.ndarray, L: int, tol: float, chi: int, cap: int, device="cuda") -> MPS:
    dense = np.ascontiguousarray(dense, dtype=np.float64)
    slots = np.zeros(L * cap * 2 * cap)
    bonds = np.zeros(L + 1, dtype=np.int32)
    rc = lib().qtt_tt_svd_host(dense.ctypes.data, L, 2, ctypes.byref(_trunc(tol, chi)), cap, slots.ctypes.data,
                               bonds.ctypes.data)
    if rc != 0:
        raise QttError(rc, "qtt_tt_svd_host")
    return MPS.from_slots(slots, bonds, cap, device)


def from_dense(ctx: "Context", dense: np.ndarray, L: int, tol: float, chi: int, cap: int, stream=None) -> MPS:
    """qtt_from_dense: TT-SVD of a host vector of 2^L values into a new device MPS."""
    dense = np.ascontiguousarray(dense, dtype=np.float64).ravel()
    if dense.size != 2 ** L:
        raise QttError(-1, f"from_dense: {dense.size} values for L = {L}")
    out = MPS(L, cap)
    ctx.check(lib().qtt_from_dense(ctx.h, dense.ctypes.data, L, ctypes.byref(_trunc(tol, chi)),
                                   ctypes.byref(out.desc()), _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# measurement hook
# ---------------------------------------------------------------------------
KERNEL_CLASSES = {"zip_contract": 0, "zip_gram": 1, "zip_factor": 2, "zip_carry": 3, "rl_svd": 4,
                  "qr_moves": 5, "env_gemm": 6, "cg_update": 7, "env_gemm_lowp": 8,
                  "zip_mpo": 9, "cg_coop": 10}


class KernelTimer:
    """HIP-event timing of one kernel class inside the library (qtt_timer_*)."""

    def __init__(self, ctx: Context, name: str, dtype: str = "f64"):
        self.ctx, self.name, self.dtype = ctx, name, dtype
        self.kc = KERNEL_CLASSES[name]

    def start(self):
        self.ctx.check(lib().qtt_timer_start(self.ctx.h, self.kc))

    def read(self):
        n = ctypes.c_int64(0)
        ms, fl, by, ov = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        self.ctx.check(lib().qtt_timer_read(self.ctx.h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl),
                                            ctypes.byref(by), ctypes.byref(ov)))
        launches = int(n.value)
        return {"name": self.name, "dtype": self.dtype, "launches": launches, "ms": ms.value,
                "idle_bracket_ms": ov.value, "flops": fl.value, "bytes": by.value}

    def durations(self, cap: int = 4096):
        """Per-launch bracket durations (ms) of the last read, in launch order."""
        buf = (ctypes.c_double * cap)()
        n = ctypes.c_int64(0)
        self.ctx.check(lib().qtt_timer_durations(self.ctx.h, buf, cap, ctypes.byref(n)))
        return [buf[i] for i in range(n.value)]
