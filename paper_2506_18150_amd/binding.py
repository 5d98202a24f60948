"""ctypes binding of libhelrm (include/helrm.h).

Argument marshalling only: every function forwards to the C call of the same
name; device buffers are torch tensors (int64 storage holding uint64
residues), streams are torch streams.  The library must be built
(``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # loads the HIP runtime libhelrm links against

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libhelrm.so")

HELRM_OK = 0
HELRM_EINVAL, HELRM_ENOMEM, HELRM_EHIP, HELRM_ESTATE = -1, -2, -3, -4
HELRM_OP_ADD, HELRM_OP_SUB, HELRM_OP_MUL, HELRM_OP_NEG = 0, 1, 2, 3
HELRM_BASIS_Q, HELRM_BASIS_PQ = 0, 1
HELRM_CAL_BUTTERFLY, HELRM_CAL_MAD_U64, HELRM_CAL_FMA_F64 = 0, 1, 2
HELRM_NOALLOC_MAX_BYTES = 256 << 20   # static scratch of helrm_lookup_packed_noalloc (include/helrm.h)

_c_int = ctypes.c_int
_vp = ctypes.c_void_p
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i64p = ctypes.POINTER(ctypes.c_int64)


class HelrmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libhelrm error {code}: {msg}")
        self.code = code


class helrm_params(ctypes.Structure):
    _fields_ = [("log_n", _c_int), ("L", _c_int), ("K", _c_int), ("alpha", _c_int),
                ("q", _u64p), ("p", _u64p)]


class helrm_plan_desc(ctypes.Structure):
    _fields_ = [("level", _c_int), ("m", _c_int), ("n1", _c_int), ("n2", _c_int),
                ("radix", _c_int), ("n_diag", _c_int), ("diag", _i32p), ("coeffs", _i64p),
                ("sign", _c_int), ("fold_span", _c_int)]


EXPORTS = [
    "helrm_last_error", "helrm_create", "helrm_destroy", "helrm_get_psi", "helrm_load_eval_keys",
    "helrm_ntt", "helrm_intt", "helrm_automorph", "helrm_poly_op", "helrm_mul_scalar",
    "helrm_from_signed", "helrm_keyswitch_hoisted", "helrm_rescale", "helrm_plan_create",
    "helrm_plan_destroy", "helrm_plan_rotation_steps", "helrm_ptxt_ct_matvec_diag",
    "helrm_lookup_packed", "helrm_footprint", "helrm_reserve", "helrm_release_stream", "helrm_timing_enable",
    "helrm_timing_read",
    "helrm_set_tuning", "helrm_mul_relin", "helrm_add_plain", "helrm_mod_drop", "helrm_lookup_multi",
    "helrm_key_uniform", "helrm_footprint_multi", "helrm_reserve_multi", "helrm_batch_graph_create",
    "helrm_batch_graph_replay", "helrm_batch_graph_destroy", "helrm_lookup_packed_noalloc",
    "helrm_calibrate_alu", "helrm_lookup_batch", "helrm_footprint_batch", "helrm_reserve_batch",
    "helrm_batch_graph_create_mixed", "helrm_plan_fold_keys",
]

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIBPATH)
    L.helrm_last_error.restype = ctypes.c_char_p
    L.helrm_last_error.argtypes = []
    L.helrm_create.argtypes = [ctypes.POINTER(helrm_params), ctypes.POINTER(_vp)]
    L.helrm_destroy.argtypes = [_vp]
    L.helrm_get_psi.argtypes = [_vp, _c_int, _u64p]
    L.helrm_load_eval_keys.argtypes = [_vp, _u32p, _c_int, _vp, _u64p]
    L.helrm_key_uniform.argtypes = [_vp, ctypes.c_uint64, _c_int, _vp, _vp]
    L.helrm_ntt.argtypes = [_vp, _vp, _c_int, _i32p, _c_int, _vp]
    L.helrm_intt.argtypes = [_vp, _vp, _c_int, _i32p, _c_int, _vp]
    L.helrm_automorph.argtypes = [_vp, _vp, _vp, ctypes.c_uint32, _c_int, _c_int, _vp]
    L.helrm_poly_op.argtypes = [_vp, _c_int, _vp, _vp, _vp, _c_int, _i32p, _c_int, _vp]
    L.helrm_mul_scalar.argtypes = [_vp, _vp, _u64p, _vp, _c_int, _i32p, _c_int, _vp]
    L.helrm_from_signed.argtypes = [_vp, _vp, _vp, _c_int, _i32p, _c_int, _vp]
    L.helrm_keyswitch_hoisted.argtypes = [_vp, _vp, _c_int, _i32p, _c_int, _vp, _c_int, _c_int, _vp]
    L.helrm_rescale.argtypes = [_vp, _vp, _c_int, _vp, _c_int, _vp]
    L.helrm_plan_create.argtypes = [_vp, ctypes.POINTER(helrm_plan_desc), ctypes.POINTER(_vp)]
    L.helrm_plan_destroy.argtypes = [_vp]
    L.helrm_plan_rotation_steps.argtypes = [_vp, _i32p, _c_int, ctypes.POINTER(_c_int)]
    L.helrm_ptxt_ct_matvec_diag.argtypes = [_vp, _vp, _vp, _vp, _c_int, _vp]
    L.helrm_lookup_packed.argtypes = [_vp, _vp, _vp, _c_int, _vp, _vp]
    L.helrm_lookup_packed_noalloc.argtypes = [_vp, _vp, _vp, _c_int, _vp, _vp]
    L.helrm_calibrate_alu.argtypes = [_vp, _c_int, _c_int, _vp, ctypes.POINTER(ctypes.c_double)]
    L.helrm_footprint.argtypes = [_vp, _vp, _c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.helrm_reserve.argtypes = [_vp, _vp, _c_int, _vp]
    L.helrm_release_stream.argtypes = [_vp, _vp]
    L.helrm_timing_enable.argtypes = [_vp, _c_int]
    L.helrm_set_tuning.argtypes = [_vp, ctypes.c_char_p, _c_int]
    L.helrm_mul_relin.argtypes = [_vp, _vp, _vp, _c_int, _vp, _c_int, _vp]
    L.helrm_add_plain.argtypes = [_vp, _vp, _vp, _c_int, _vp, _c_int, _vp]
    L.helrm_mod_drop.argtypes = [_vp, _vp, _c_int, _vp, _c_int, _c_int, _vp]
    L.helrm_lookup_multi.argtypes = [_vp, ctypes.POINTER(_vp), _c_int, _vp, _c_int, _vp, _vp]
    L.helrm_footprint_multi.argtypes = [_vp, ctypes.POINTER(_vp), _c_int, _c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.helrm_reserve_multi.argtypes = [_vp, ctypes.POINTER(_vp), _c_int, _c_int, _vp]
    L.helrm_batch_graph_create.argtypes = [_vp, ctypes.POINTER(_vp), _c_int, _vp, _c_int, _vp, ctypes.POINTER(_vp)]
    L.helrm_batch_graph_replay.argtypes = [_vp, _vp]
    L.helrm_plan_fold_keys.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)]
    L.helrm_lookup_batch.argtypes = [_vp, ctypes.POINTER(_vp), _vp, _c_int, _vp, _vp]
    L.helrm_footprint_batch.argtypes = [_vp, ctypes.POINTER(_vp), _c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.helrm_reserve_batch.argtypes = [_vp, ctypes.POINTER(_vp), _c_int, _vp]
    L.helrm_batch_graph_create_mixed.argtypes = [_vp, ctypes.POINTER(_vp), _vp, _c_int, _vp, ctypes.POINTER(_vp)]
    L.helrm_batch_graph_destroy.argtypes = [_vp]
    L.helrm_timing_read.argtypes = [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
    for name in EXPORTS[1:]:
        getattr(L, name).restype = _c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != HELRM_OK:
        raise HelrmError(rc, lib().helrm_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_contiguous(), "tensor must be contiguous"
    assert t.element_size() == 8, "64-bit tensor expected"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _i32(v: Sequence[int]):
    a = np.ascontiguousarray(np.array(list(v), dtype=np.int32))
    return a, a.ctypes.data_as(_i32p)


class Context:
    """An helrm_ctx handle.  Methods are the C calls of the same name."""

    def __init__(self, log_n: int, q: Sequence[int], p: Sequence[int], alpha: int):
        self.q = [int(x) for x in q]
        self.p = [int(x) for x in p]
        self.log_n = log_n
        self.N = 1 << log_n
        self.L = len(self.q) - 1
        self.K = len(self.p)
        self.alpha = alpha
        self.dnum = -(-(self.L + 1) // alpha)
        qa = np.array(self.q, dtype=np.uint64)
        pa = np.array(self.p, dtype=np.uint64)
        prm = helrm_params(log_n, self.L, self.K, alpha, qa.ctypes.data_as(_u64p), pa.ctypes.data_as(_u64p))
        h = ctypes.c_void_p()
        _check(lib().helrm_create(ctypes.byref(prm), ctypes.byref(h)))
        self.h = h

    # prime index helpers
    def primes(self):
        return self.q + self.p

    def pq_index(self, level: int):
        return list(range(level + 1)) + list(range(self.L + 1, self.L + 1 + self.K))

    def close(self):
        if getattr(self, "h", None):
            _check(lib().helrm_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def helrm_get_psi(self, i: int) -> int:
        v = ctypes.c_uint64()
        _check(lib().helrm_get_psi(self.h, i, ctypes.byref(v)))
        return int(v.value)

    def helrm_load_eval_keys(self, galois: Sequence[int], keys: torch.Tensor, seeds: Optional[Sequence[int]] = None):
        g = np.ascontiguousarray(np.array(list(galois), dtype=np.uint32))
        sd = None if seeds is None else np.ascontiguousarray(np.array([int(x) for x in seeds], dtype=np.uint64))
        _check(lib().helrm_load_eval_keys(self.h, g.ctypes.data_as(_u32p), len(g), _ptr(keys),
                                          None if sd is None else sd.ctypes.data_as(_u64p)))

    def helrm_key_uniform(self, seed: int, digit: int, out, stream=None):
        _check(lib().helrm_key_uniform(self.h, int(seed), digit, _ptr(out), _stream(stream)))

    def helrm_ntt(self, data: torch.Tensor, prime_index: Sequence[int], batch: int, stream=None):
        a, pa = _i32(prime_index)
        _check(lib().helrm_ntt(self.h, _ptr(data), len(a), pa, batch, _stream(stream)))

    def helrm_intt(self, data: torch.Tensor, prime_index: Sequence[int], batch: int, stream=None):
        a, pa = _i32(prime_index)
        _check(lib().helrm_intt(self.h, _ptr(data), len(a), pa, batch, _stream(stream)))

    def helrm_automorph(self, d_in, d_out, galois: int, n_limbs: int, batch: int, stream=None):
        _check(lib().helrm_automorph(self.h, _ptr(d_in), _ptr(d_out), galois, n_limbs, batch, _stream(stream)))

    def helrm_poly_op(self, op: int, a, b, out, prime_index: Sequence[int], batch: int, stream=None):
        ia, pa = _i32(prime_index)
        _check(lib().helrm_poly_op(self.h, op, _ptr(a), _ptr(b), _ptr(out), len(ia), pa, batch, _stream(stream)))

    def helrm_mul_scalar(self, a, scalars: Sequence[int], out, prime_index: Sequence[int], batch: int,
                         stream=None):
        ia, pa = _i32(prime_index)
        sc = np.ascontiguousarray(np.array([int(s) for s in scalars], dtype=np.uint64))
        _check(lib().helrm_mul_scalar(self.h, _ptr(a), sc.ctypes.data_as(_u64p), _ptr(out), len(ia), pa, batch,
                                      _stream(stream)))

    def helrm_from_signed(self, d_in, d_out, prime_index: Sequence[int], batch: int, stream=None):
        ia, pa = _i32(prime_index)
        _check(lib().helrm_from_signed(self.h, _ptr(d_in), _ptr(d_out), len(ia), pa, batch, _stream(stream)))

    def helrm_keyswitch_hoisted(self, ct, level: int, steps: Sequence[int], out, out_basis: int, batch: int,
                                stream=None):
        sa, ps = _i32(steps)
        _check(lib().helrm_keyswitch_hoisted(self.h, _ptr(ct), level, ps, len(sa), _ptr(out), out_basis, batch,
                                             _stream(stream)))

    def helrm_rescale(self, d_in, level: int, d_out, batch: int, stream=None):
        _check(lib().helrm_rescale(self.h, _ptr(d_in), level, _ptr(d_out), batch, _stream(stream)))

    def helrm_plan_create(self, level: int, m: int, n1: int, n2: int, radix: int,
                          diag: Sequence[int], coeffs: np.ndarray, sign: int = 1, fold_span: int = 0) -> "Plan":
        da, pd = _i32(diag)
        co = np.ascontiguousarray(coeffs, dtype=np.int64)
        assert co.shape == (len(da), self.N)
        desc = helrm_plan_desc(level, m, n1, n2, radix, len(da), pd, co.ctypes.data_as(_i64p), sign, fold_span)
        h = ctypes.c_void_p()
        _check(lib().helrm_plan_create(self.h, ctypes.byref(desc), ctypes.byref(h)))
        return Plan(self, h, level, m, n1, n2, radix)

    def helrm_ptxt_ct_matvec_diag(self, plan: "Plan", ct, out, batch: int, stream=None):
        _check(lib().helrm_ptxt_ct_matvec_diag(self.h, plan.h, _ptr(ct), _ptr(out), batch, _stream(stream)))

    def helrm_lookup_packed(self, plan: "Plan", sel, batch: int, out, stream=None):
        _check(lib().helrm_lookup_packed(self.h, plan.h, _ptr(sel), batch, _ptr(out), _stream(stream)))

    def helrm_calibrate_alu(self, kind: int, prime_index: int = 0, stream=None) -> float:
        v = ctypes.c_double()
        _check(lib().helrm_calibrate_alu(self.h, kind, prime_index, _stream(stream), ctypes.byref(v)))
        return v.value

    def helrm_lookup_packed_noalloc(self, plan: "Plan", sel, batch: int, out, stream=None):
        _check(lib().helrm_lookup_packed_noalloc(self.h, plan.h, _ptr(sel), batch, _ptr(out), _stream(stream)))

    def helrm_lookup_multi(self, plans: Sequence["Plan"], sel, batch: int, out, stream=None):
        arr = (_vp * len(plans))(*[p.h for p in plans])
        _check(lib().helrm_lookup_multi(self.h, arr, len(plans), _ptr(sel), batch, _ptr(out), _stream(stream)))

    def helrm_footprint(self, plan: "Plan", batch: int) -> int:
        v = ctypes.c_size_t()
        _check(lib().helrm_footprint(self.h, plan.h, batch, ctypes.byref(v)))
        return int(v.value)

    def helrm_reserve(self, plan: "Plan", batch: int, stream=None):
        _check(lib().helrm_reserve(self.h, plan.h, batch, _stream(stream)))

    def helrm_release_stream(self, stream=None):
        _check(lib().helrm_release_stream(self.h, _stream(stream)))

    def helrm_footprint_multi(self, plans: Sequence["Plan"], batch: int) -> int:
        arr = (_vp * len(plans))(*[p.h for p in plans])
        v = ctypes.c_size_t()
        _check(lib().helrm_footprint_multi(self.h, arr, len(plans), batch, ctypes.byref(v)))
        return int(v.value)

    def helrm_reserve_multi(self, plans: Sequence["Plan"], batch: int, stream=None):
        arr = (_vp * len(plans))(*[p.h for p in plans])
        _check(lib().helrm_reserve_multi(self.h, arr, len(plans), batch, _stream(stream)))

    def helrm_batch_graph_create(self, plans: Sequence["Plan"], sel, batch: int, out) -> "Graph":
        """sel and out stay bound to the graph: keep the tensors alive and
        write the next selectors into sel before each replay."""
        arr = (_vp * len(plans))(*[p.h for p in plans])
        h = ctypes.c_void_p()
        _check(lib().helrm_batch_graph_create(self.h, arr, len(plans), _ptr(sel), batch, _ptr(out),
                                              ctypes.byref(h)))
        return Graph(self, h, list(plans), sel, out)

    def helrm_lookup_batch(self, plans: Sequence["Plan"], sel, out, stream=None):
        """Element b of sel goes through plans[b]."""
        arr = (_vp * len(plans))(*[p.h for p in plans])
        _check(lib().helrm_lookup_batch(self.h, arr, _ptr(sel), len(plans), _ptr(out), _stream(stream)))

    def helrm_footprint_batch(self, plans: Sequence["Plan"]) -> int:
        arr = (_vp * len(plans))(*[p.h for p in plans])
        v = ctypes.c_size_t()
        _check(lib().helrm_footprint_batch(self.h, arr, len(plans), ctypes.byref(v)))
        return v.value

    def helrm_reserve_batch(self, plans: Sequence["Plan"], stream=None):
        arr = (_vp * len(plans))(*[p.h for p in plans])
        _check(lib().helrm_reserve_batch(self.h, arr, len(plans), _stream(stream)))

    def helrm_batch_graph_create_mixed(self, plans: Sequence["Plan"], sel, out) -> "Graph":
        """Element b goes through plans[b]; sel and out stay bound to the graph."""
        arr = (_vp * len(plans))(*[p.h for p in plans])
        h = ctypes.c_void_p()
        _check(lib().helrm_batch_graph_create_mixed(self.h, arr, _ptr(sel), len(plans), _ptr(out), ctypes.byref(h)))
        return Graph(self, h, list(plans), sel, out)

    def helrm_mul_relin(self, a, b, level: int, out, batch: int, stream=None):
        _check(lib().helrm_mul_relin(self.h, _ptr(a), _ptr(b), level, _ptr(out), batch, _stream(stream)))

    def helrm_add_plain(self, ct, pt, level: int, out, batch: int, stream=None):
        _check(lib().helrm_add_plain(self.h, _ptr(ct), _ptr(pt), level, _ptr(out), batch, _stream(stream)))

    def helrm_mod_drop(self, d_in, level_in: int, d_out, level_out: int, batch: int, stream=None):
        _check(lib().helrm_mod_drop(self.h, _ptr(d_in), level_in, _ptr(d_out), level_out, batch, _stream(stream)))

    def helrm_set_tuning(self, knob: str, value: int):
        _check(lib().helrm_set_tuning(self.h, knob.encode(), int(value)))

    def helrm_timing_enable(self, enable: bool):
        _check(lib().helrm_timing_enable(self.h, 1 if enable else 0))

    def helrm_timing_read(self, kernel: str):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        by, ops = ctypes.c_double(), ctypes.c_double()
        _check(lib().helrm_timing_read(self.h, kernel.encode(), ctypes.byref(ms), ctypes.byref(n),
                                       ctypes.byref(by), ctypes.byref(ops)))
        return {"ms": ms.value, "launches": int(n.value), "bytes": by.value, "ops": ops.value}


class Plan:
    def __init__(self, ctx: Context, h, level, m, n1, n2, radix):
        self.ctx, self.h = ctx, h
        self.level, self.m, self.n1, self.n2, self.radix = level, m, n1, n2, radix

    def helrm_plan_fold_keys(self) -> int:
        """Fold the loaded keys into the plan (batched lookups); returns the bytes kept."""
        v = ctypes.c_size_t()
        _check(lib().helrm_plan_fold_keys(self.ctx.h, self.h, ctypes.byref(v)))
        return v.value

    def rotation_steps(self):
        n = ctypes.c_int()
        buf = np.zeros(4096, dtype=np.int32)
        _check(lib().helrm_plan_rotation_steps(self.h, buf.ctypes.data_as(_i32p), len(buf), ctypes.byref(n)))
        return [int(x) for x in buf[: n.value]]

    def close(self):
        if getattr(self, "h", None):
            _check(lib().helrm_plan_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """An helrm_graph handle; holds references to the plans and the bound
    selector / output tensors so they outlive it."""

    def __init__(self, ctx: Context, h, plans, sel, out):
        self.ctx, self.h, self.plans, self.sel, self.out = ctx, h, plans, sel, out

    def helrm_batch_graph_replay(self, stream=None):
        _check(lib().helrm_batch_graph_replay(self.h, _stream(stream)))

    def replay(self, stream=None):
        self.helrm_batch_graph_replay(stream)

    def close(self):
        if getattr(self, "h", None):
            _check(lib().helrm_batch_graph_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_u64(arr: np.ndarray, device="cuda") -> torch.Tensor:
    """Host uint64 array -> device tensor (int64 storage of the same bits)."""
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).to(device)


def host_u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().contiguous().numpy().view(np.uint64)
