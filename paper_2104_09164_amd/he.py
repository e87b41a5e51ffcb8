"""Python binding of the C ABI in include/he.h (argument marshalling only).

Every step of the hot path runs in the HIP kernels of libhe.so; this module
only allocates device memory through torch (the caller owns all device
memory), passes pointers, sizes and the current torch stream, and raises
HeError on a negative return code.  If libhe.so is missing it raises: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhe.so")

HE_MAX_BATCH = 64


class HeError(RuntimeError):
    def __init__(self, code: int, where: str):
        detail = lib().he_last_error().decode() if code == -7 else ""
        super().__init__(f"{where}: {lib().he_strerror(code).decode()} ({code})" + (f" [{detail}]" if detail else ""))
        self.code = code


class _Ct(C.Structure):
    _fields_ = [("dev", C.c_void_p), ("level", C.c_uint32), ("scale", C.c_double)]


class _TraceEntry(C.Structure):
    _fields_ = [("kernel", C.c_char_p), ("launches", C.c_uint64), ("ms", C.c_double), ("bytes", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("log_n", C.c_uint32), ("n_q", C.c_uint32), ("q", C.POINTER(C.c_uint64)),
                ("n_p", C.c_uint32), ("p", C.POINTER(C.c_uint64)), ("alpha", C.c_uint32)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_2104_09164_amd/build.py")
        # torch ships its own HIP runtime with the same soname; it must be
        # loaded first so that libhe.so binds to it.  Otherwise the process
        # would hold two HIP/HSA runtimes and the device memory and streams
        # torch hands over would belong to the other one.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, u32, u64, i32, sz, dbl = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_size_t, C.c_double
        ctp = C.POINTER(_Ct)
        sig = {
            "he_strerror": (C.c_char_p, [C.c_int]),
            "he_last_error": (C.c_char_p, []),
            "he_gen_primes": (C.c_int, [u32, u32, u32, C.POINTER(u64), u32, C.POINTER(u64)]),
            "he_ctx_create": (C.c_int, [C.POINTER(_Params), vp, C.POINTER(vp)]),
            "he_ctx_destroy": (C.c_int, [vp]),
            "he_ctx_set_stream": (C.c_int, [vp, vp]),
            "he_ct_bytes": (sz, [vp, u32]),
            "he_key_bytes": (sz, [vp, u32]),
            "he_workspace_bytes": (sz, [vp, u32, u32, u32]),
            "he_dense_bytes": (sz, [vp, u32, u32, C.c_int]),
            "he_dense_bytes_ex": (sz, [vp, u32, u32, C.c_int, u32]),
            "he_ctx_bind": (C.c_int, [vp, vp, sz, u32, u32, u32]),
            "he_load_keys": (C.c_int, [vp, vp, u32, C.POINTER(i32), C.POINTER(vp), vp, sz]),
            "he_dense_load": (C.c_int, [vp, u32, u32, u32, u32, vp, vp, dbl, dbl, vp, sz, C.POINTER(vp)]),
            "he_dense_load_ex": (C.c_int, [vp, u32, u32, u32, u32, vp, vp, dbl, dbl, u32, vp, sz, C.POINTER(vp)]),
            "he_dense_free": (C.c_int, [vp]),
            "he_linear_bytes": (sz, [vp, u32, u32, u32, u32, u32]),
            "he_linear_load": (C.c_int, [vp, u32, u32, u32, u32, u32, C.POINTER(i32), C.POINTER(i32), vp, dbl, vp, sz,
                                         C.POINTER(vp)]),
            "he_linear_free": (C.c_int, [vp]),
            "he_linear_scratch_bytes": (sz, [vp, u32, u32, u32]),
            "he_eval_linear": (C.c_int, [vp, ctp, vp, vp, sz, ctp]),
            "he_eval_linear_batch": (C.c_int, [vp, u32, ctp, vp, vp, sz, ctp]),
            "he_ct_import": (C.c_int, [vp, vp, u32, dbl, ctp]),
            "he_ct_export": (C.c_int, [vp, ctp, vp]),
            "he_ct_from_coeff_dev": (C.c_int, [vp, vp, u32, dbl, ctp]),
            "he_ct_to_coeff_dev": (C.c_int, [vp, ctp, vp]),
            "he_eval_dense": (C.c_int, [vp, ctp, vp, ctp]),
            "he_square": (C.c_int, [vp, ctp, ctp]),
            "he_rotate": (C.c_int, [vp, ctp, i32, ctp]),
            "he_rotate_hoisted": (C.c_int, [vp, ctp, u32, C.POINTER(i32), ctp]),
            "he_rescale": (C.c_int, [vp, ctp, ctp]),
            "he_add": (C.c_int, [vp, ctp, ctp, ctp]),
            "he_eval_dense_batch": (C.c_int, [vp, u32, ctp, vp, ctp]),
            "he_square_batch": (C.c_int, [vp, u32, ctp, ctp]),
            "he_rescale_batch": (C.c_int, [vp, u32, ctp, ctp]),
            "he_rescale_batch_noalloc": (C.c_int, [vp, u32, ctp, ctp]),
            "he_rotate_hoisted_batch": (C.c_int, [vp, u32, ctp, u32, C.POINTER(i32), ctp]),
            "he_ntt": (C.c_int, [vp, u32, C.POINTER(vp), u32, u32, C.c_int]),
            "he_sync": (C.c_int, [vp]),
            "he_ctx_set_knob": (C.c_int, [vp, C.c_char_p, C.c_int64]),
            "he_ctx_get_knob": (C.c_int, [vp, C.c_char_p, C.POINTER(C.c_int64)]),
            "he_trace_read": (C.c_int, [vp, C.POINTER(_TraceEntry), u32, C.POINTER(u32)]),
            "he_client_create": (C.c_int, [vp, u32, vp, vp, C.POINTER(vp)]),
            "he_client_destroy": (C.c_int, [vp]),
            "he_encode": (C.c_int, [vp, u32, vp, dbl, u32, vp]),
            "he_encrypt": (C.c_int, [vp, u32, vp, vp, u32, dbl, ctp]),
            "he_decrypt": (C.c_int, [vp, u32, ctp, vp]),
            "he_decode": (C.c_int, [vp, u32, vp, u32, dbl, vp]),
            "he_graph_begin": (C.c_int, [vp]),
            "he_graph_end": (C.c_int, [vp, C.POINTER(vp)]),
            "he_graph_launch": (C.c_int, [vp, vp]),
            "he_graph_free": (C.c_int, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


EXPORTED = ("he_strerror", "he_last_error", "he_gen_primes", "he_ctx_create", "he_ctx_destroy", "he_ctx_set_stream", "he_ct_bytes",
            "he_key_bytes", "he_workspace_bytes", "he_dense_bytes", "he_ctx_bind", "he_load_keys", "he_dense_load",
            "he_dense_free", "he_ct_import", "he_ct_export", "he_ct_from_coeff_dev", "he_ct_to_coeff_dev",
            "he_eval_dense", "he_square", "he_rotate", "he_rotate_hoisted", "he_rescale", "he_add",
            "he_eval_dense_batch", "he_square_batch", "he_rescale_batch", "he_rotate_hoisted_batch", "he_ntt",
            "he_sync", "he_ctx_set_knob", "he_ctx_get_knob", "he_trace_read", "he_dense_bytes_ex",
            "he_dense_load_ex", "he_linear_bytes", "he_linear_load", "he_linear_free", "he_linear_scratch_bytes",
            "he_eval_linear", "he_eval_linear_batch", "he_client_create", "he_client_destroy", "he_encode",
            "he_encrypt", "he_decrypt", "he_decode", "he_rescale_batch_noalloc", "he_graph_begin",
            "he_graph_end", "he_graph_launch", "he_graph_free")

HE_DENSE_QP = 1
HE_DENSE_RS_SHIFT = 8


def _check(rc: int, where: str) -> None:
    if rc != 0:
        raise HeError(rc, where)


def gen_primes(log_n: int, bits: int, count: int, taken=()) -> list[int]:
    t = (C.c_uint64 * max(1, len(taken)))(*taken)
    out = (C.c_uint64 * count)()
    _check(lib().he_gen_primes(log_n, bits, count, t, len(taken), out), "he_gen_primes")
    return list(out)


def prime_chain(log_n: int, q_bits, p_bits) -> tuple[list[int], list[int]]:
    taken: list[int] = []
    for b in list(q_bits) + list(p_bits):
        taken += gen_primes(log_n, b, 1, taken)
    return taken[: len(q_bits)], taken[len(q_bits):]


def _torch():
    import torch
    return torch


@dataclass
class Ct:
    """A ciphertext resident in device memory (NTT form, [2][level+1][N])."""
    buf: object          # torch.int64 tensor owning the memory
    level: int
    scale: float

    def _c(self) -> _Ct:
        return _Ct(self.buf.data_ptr(), self.level, self.scale)


class Dense:
    def __init__(self, ctx: "Context", handle, buf, level, m, n, n1, pt_scale, bias_scale, qp=False, rs_bits=0):
        self.ctx, self.h, self.buf = ctx, handle, buf
        self.level, self.m, self.n, self.n1 = level, m, n, n1
        self.pt_scale, self.bias_scale, self.qp, self.rs_bits = pt_scale, bias_scale, qp, rs_bits

    def __del__(self):
        try:
            lib().he_dense_free(self.h)
        except Exception:
            pass


class Linear:
    def __init__(self, ctx: "Context", handle, buf, level, n_out, n_giant, n_in, n_baby, baby, giant, pt_scale):
        self.ctx, self.h, self.buf = ctx, handle, buf
        self.level, self.n_out, self.n_giant, self.n_in, self.n_baby = level, n_out, n_giant, n_in, n_baby
        self.baby, self.giant, self.pt_scale = list(baby), list(giant), pt_scale
        self.scratch = None

    def __del__(self):
        try:
            lib().he_linear_free(self.h)
        except Exception:
            pass


class Client:
    """Device-side encode / encrypt / decrypt / decode for the key holders
    (he_client_*).  Slot tensors: complex128 [n][N/2]; plaintext tensors:
    int64 storage of uint64 residues [n][level+1][N]; noise: int32 [n][3][N]."""

    def __init__(self, ctx: "Context", max_batch: int, pk: np.ndarray | None = None, sk: np.ndarray | None = None):
        self.ctx, self.max_batch = ctx, max_batch
        pkh = np.ascontiguousarray(pk, dtype=np.uint64) if pk is not None else None
        skh = np.ascontiguousarray(sk, dtype=np.int64) if sk is not None else None
        if pkh is not None and pkh.shape != (2, len(ctx.q), ctx.N):
            raise ValueError(f"pk shape {pkh.shape}, expected {(2, len(ctx.q), ctx.N)}")
        if skh is not None and skh.shape != (ctx.N,):
            raise ValueError(f"sk shape {skh.shape}, expected {(ctx.N,)}")
        h = C.c_void_p()
        _check(lib().he_client_create(ctx.h, max_batch, C.c_void_p(pkh.ctypes.data) if pkh is not None else None,
                                      C.c_void_p(skh.ctypes.data) if skh is not None else None, C.byref(h)),
               "he_client_create")
        self.h = h

    def __del__(self):
        try:
            lib().he_client_destroy(self.h)
        except Exception:
            pass

    def encode(self, slots, scale: float, level: int):
        torch = _torch()
        z = slots.to(device=self.ctx.device, dtype=torch.complex128).contiguous()
        n = z.shape[0]
        if z.shape != (n, self.ctx.N // 2):
            raise ValueError(f"slots shape {tuple(z.shape)}, expected (n, {self.ctx.N // 2})")
        pt = torch.empty((n, level + 1, self.ctx.N), dtype=torch.int64, device=self.ctx.device)
        _check(lib().he_encode(self.h, n, C.c_void_p(z.data_ptr()), scale, level, C.c_void_p(pt.data_ptr())),
               "he_encode")
        return pt

    def encrypt(self, pt, noise, level: int, scale: float, outs=None):
        torch = _torch()
        n = pt.shape[0]
        if pt.shape != (n, level + 1, self.ctx.N) or noise.shape != (n, 3, self.ctx.N) or noise.dtype != torch.int32:
            raise ValueError("plaintexts [n][level+1][N] and int32 noise [n][3][N] expected")
        outs = outs or [self.ctx.new_ct(level) for _ in range(n)]
        arr = (_Ct * max(1, n))(*[o._c() for o in outs])
        _check(lib().he_encrypt(self.h, n, C.c_void_p(pt.data_ptr()), C.c_void_p(noise.data_ptr()), level, scale,
                                arr), "he_encrypt")
        for o in outs:
            o.level, o.scale = level, scale
        return outs

    def decrypt(self, cts):
        torch = _torch()
        n = len(cts)
        level = cts[0].level if n else 0
        pt = torch.empty((n, level + 1, self.ctx.N), dtype=torch.int64, device=self.ctx.device)
        arr = (_Ct * max(1, n))(*[c._c() for c in cts])
        _check(lib().he_decrypt(self.h, n, arr, C.c_void_p(pt.data_ptr())), "he_decrypt")
        return pt

    def decode(self, pt, level: int, scale: float):
        torch = _torch()
        n = pt.shape[0]
        if pt.shape != (n, level + 1, self.ctx.N):
            raise ValueError("plaintexts [n][level+1][N] expected")
        z = torch.empty((n, self.ctx.N // 2), dtype=torch.complex128, device=self.ctx.device)
        _check(lib().he_decode(self.h, n, C.c_void_p(pt.data_ptr()), level, scale, C.c_void_p(z.data_ptr())),
               "he_decode")
        return z


class Graph:
    """A captured sequence of library calls (he_graph_*); replay() launches it
    on its context's current stream."""

    def __init__(self, ctx, handle):
        self.ctx, self.h = ctx, handle

    def replay(self) -> None:
        _check(lib().he_graph_launch(self.ctx.h, self.h), "he_graph_launch")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            lib().he_graph_free(self.h)
            self.h = None


class Context:
    def __init__(self, log_n: int, q, p, alpha: int, device: str = "cuda:0"):
        torch = _torch()
        self.device = torch.device(device)
        self.log_n, self.N = log_n, 1 << log_n
        self.q, self.p, self.alpha = [int(v) for v in q], [int(v) for v in p], alpha
        qa = (C.c_uint64 * len(self.q))(*self.q)
        pa = (C.c_uint64 * max(1, len(self.p)))(*self.p)
        prm = _Params(log_n, len(self.q), qa, len(self.p), pa, alpha)
        self._keep = (qa, pa)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _check(lib().he_ctx_create(C.byref(prm), C.c_void_p(stream), C.byref(h)), "he_ctx_create")
        self.h = h
        self.ws = None
        self.keys = None

    def __del__(self):
        try:
            lib().he_ctx_destroy(self.h)
        except Exception:
            pass

    @property
    def L(self) -> int:
        return len(self.q) - 1

    def use_current_stream(self):
        torch = _torch()
        _check(lib().he_ctx_set_stream(self.h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)),
               "he_ctx_set_stream")

    # ------------------------------------------------------------ graphs
    def capture(self, fn) -> "Graph":
        """Record the library calls fn() makes on this context's stream into a
        HIP graph (he_graph_begin / he_graph_end) instead of running them;
        the capture is ended even when fn raises."""
        _check(lib().he_graph_begin(self.h), "he_graph_begin")
        try:
            fn()
        finally:
            g = C.c_void_p()
            rc = lib().he_graph_end(self.h, C.byref(g))
        _check(rc, "he_graph_end")
        return Graph(self, g)

    # ------------------------------------------------------------ memory
    def _alloc(self, nbytes: int):
        torch = _torch()
        return torch.empty((nbytes + 7) // 8, dtype=torch.int64, device=self.device)

    def ct_bytes(self, level: int) -> int:
        return int(lib().he_ct_bytes(self.h, level))

    def new_ct(self, level: int, scale: float = 1.0) -> Ct:
        return Ct(self._alloc(self.ct_bytes(level)), level, scale)

    def workspace_bytes(self, max_batch: int = 1, max_n1: int = 1, max_n2: int = 1) -> int:
        return int(lib().he_workspace_bytes(self.h, max_batch, max_n1, max_n2))

    def bind(self, max_batch: int = 1, max_n1: int = 1, max_n2: int = 1) -> None:
        nbytes = self.workspace_bytes(max_batch, max_n1, max_n2)
        ws = self._alloc(nbytes)
        _check(lib().he_ctx_bind(self.h, C.c_void_p(ws.data_ptr()), nbytes, max_batch, max_n1, max_n2),
               "he_ctx_bind")
        self.ws = ws

    def load_keys(self, relin: np.ndarray | None, rot: dict) -> None:
        steps = sorted(rot)
        nbytes = int(lib().he_key_bytes(self.h, len(steps)))
        kbuf = self._alloc(nbytes)
        arrs = [np.ascontiguousarray(rot[s], dtype=np.uint64) for s in steps]
        ptrs = (C.c_void_p * max(1, len(arrs)))(*[a.ctypes.data for a in arrs])
        st = (C.c_int32 * max(1, len(steps)))(*steps)
        rl = np.ascontiguousarray(relin, dtype=np.uint64) if relin is not None else None
        _check(lib().he_load_keys(self.h, C.c_void_p(rl.ctypes.data) if rl is not None else None, len(steps), st,
                                  ptrs, C.c_void_p(kbuf.data_ptr()), nbytes), "he_load_keys")
        self.keys = kbuf
        self.key_steps = steps

    def dense_load(self, level: int, m: int, n: int, n1: int, pts: np.ndarray, bias: np.ndarray | None,
                   pt_scale: float, bias_scale: float, qp: bool = False, rs_bits: int = 0) -> Dense:
        """qp: diagonals over q_0..q_level, p_0..p_{K-1} (lazy-ModDown form, HE_DENSE_QP);
        rs_bits: hoisted rotate-and-sum groups (HE_DENSE_RS), 0 = sequential."""
        pts = np.ascontiguousarray(pts, dtype=np.uint64)
        b = np.ascontiguousarray(bias, dtype=np.uint64) if bias is not None else None
        flags = (HE_DENSE_QP if qp else 0) | (int(rs_bits) << HE_DENSE_RS_SHIFT)
        if pts.shape != (m, level + 1 + (len(self.p) if qp else 0), self.N):
            raise ValueError(f"diagonals of shape {pts.shape} for m={m}, level={level}, qp={qp}")
        nbytes = int(lib().he_dense_bytes_ex(self.h, level, m, b is not None, flags))
        buf = self._alloc(nbytes)
        h = C.c_void_p()
        _check(lib().he_dense_load_ex(self.h, level, m, n, n1, C.c_void_p(pts.ctypes.data),
                                      C.c_void_p(b.ctypes.data) if b is not None else None, pt_scale, bias_scale,
                                      flags, C.c_void_p(buf.data_ptr()), nbytes, C.byref(h)), "he_dense_load_ex")
        return Dense(self, h, buf, level, m, n, n1, pt_scale, bias_scale, qp, rs_bits)

    def linear_load(self, level: int, baby, giant, pts: np.ndarray, pt_scale: float) -> Linear:
        """pts: uint64 [n_giant][n_out][n_in][n_baby][level+1][N] (coefficient form)."""
        pts = np.ascontiguousarray(pts, dtype=np.uint64)
        n_giant, n_out, n_in, n_baby = pts.shape[:4]
        if pts.shape[4:] != (level + 1, self.N) or len(baby) != n_baby or len(giant) != n_giant:
            raise ValueError(f"plaintexts of shape {pts.shape} for baby {baby}, giant {giant}, level {level}")
        nbytes = int(lib().he_linear_bytes(self.h, level, n_out, n_giant, n_in, n_baby))
        buf = self._alloc(nbytes)
        b = (C.c_int32 * n_baby)(*baby)
        g = (C.c_int32 * n_giant)(*giant)
        h = C.c_void_p()
        _check(lib().he_linear_load(self.h, level, n_out, n_giant, n_in, n_baby, b, g, C.c_void_p(pts.ctypes.data),
                                    pt_scale, C.c_void_p(buf.data_ptr()), nbytes, C.byref(h)), "he_linear_load")
        return Linear(self, h, buf, level, n_out, n_giant, n_in, n_baby, baby, giant, pt_scale)

    def eval_linear(self, cts, lt: Linear, outs=None):
        """One request: cts = its n_in inputs; returns its n_out outputs."""
        return self.eval_linear_batch(cts, lt, outs)

    def eval_linear_batch(self, cts, lt: Linear, outs=None):
        """R requests: cts = R x n_in inputs (request-major); returns R x n_out outputs."""
        if len(cts) % lt.n_in:
            raise ValueError(f"{len(cts)} inputs for a transform of {lt.n_in}")
        R = len(cts) // lt.n_in
        outs = outs or [self.new_ct(lt.level) for _ in range(R * lt.n_out)]
        nb = R * int(lib().he_linear_scratch_bytes(self.h, lt.level, lt.n_in, lt.n_baby))
        if lt.scratch is None or lt.scratch.numel() * lt.scratch.element_size() < nb:
            lt.scratch = self._alloc(nb)
        ia, oa = self._arr(cts), self._arr(outs)
        _check(lib().he_eval_linear_batch(self.h, R, ia, lt.h, C.c_void_p(lt.scratch.data_ptr()),
                                          lt.scratch.numel() * lt.scratch.element_size(), oa), "he_eval_linear_batch")
        self._sync_meta(outs, oa)
        return outs

    # ------------------------------------------------------ import/export
    def import_ct(self, coeff: np.ndarray, level: int, scale: float) -> Ct:
        coeff = np.ascontiguousarray(coeff, dtype=np.uint64)
        assert coeff.size == 2 * (level + 1) * self.N
        ct = self.new_ct(level, scale)
        c = ct._c()
        _check(lib().he_ct_import(self.h, C.c_void_p(coeff.ctypes.data), level, scale, C.byref(c)), "he_ct_import")
        return ct

    def export_ct(self, ct: Ct) -> np.ndarray:
        out = np.empty((2, ct.level + 1, self.N), dtype=np.uint64)
        c = ct._c()
        _check(lib().he_ct_export(self.h, C.byref(c), C.c_void_p(out.ctypes.data)), "he_ct_export")
        return out

    # -------------------------------------------------------- evaluation
    @staticmethod
    def _arr(cts):
        return (_Ct * len(cts))(*[c._c() for c in cts])

    @staticmethod
    def _sync_meta(cts, arr):
        for c, a in zip(cts, arr):
            c.level, c.scale = int(a.level), float(a.scale)

    def eval_dense(self, ct: Ct, d: Dense, out: Ct | None = None) -> Ct:
        return self.eval_dense_batch([ct], d, [out] if out is not None else None)[0]

    def eval_dense_batch(self, cts, d: Dense, outs=None):
        outs = outs or [self.new_ct(d.level) for _ in cts]
        ia, oa = self._arr(cts), self._arr(outs)
        _check(lib().he_eval_dense_batch(self.h, len(cts), ia, d.h, oa), "he_eval_dense_batch")
        self._sync_meta(outs, oa)
        return outs

    def square(self, ct: Ct, out: Ct | None = None) -> Ct:
        return self.square_batch([ct], [out] if out is not None else None)[0]

    def square_batch(self, cts, outs=None):
        outs = outs or [self.new_ct(c.level) for c in cts]
        ia, oa = self._arr(cts), self._arr(outs)
        _check(lib().he_square_batch(self.h, len(cts), ia, oa), "he_square_batch")
        self._sync_meta(outs, oa)
        return outs

    def rescale(self, ct: Ct, out: Ct | None = None) -> Ct:
        return self.rescale_batch([ct], [out] if out is not None else None)[0]

    def rescale_batch(self, cts, outs=None):
        outs = outs or [self.new_ct(c.level - 1) for c in cts]
        ia, oa = self._arr(cts), self._arr(outs)
        _check(lib().he_rescale_batch(self.h, len(cts), ia, oa), "he_rescale_batch")
        self._sync_meta(outs, oa)
        return outs

    def rescale_batch_noalloc(self, cts, outs):
        """he_rescale_batch_noalloc: the same results with the library's static
        per-GPU scratch (no workspace, no allocation; outs must be given)."""
        ia, oa = self._arr(cts), self._arr(outs)
        _check(lib().he_rescale_batch_noalloc(self.h, len(cts), ia, oa), "he_rescale_batch_noalloc")
        self._sync_meta(outs, oa)
        return outs

    def rotate(self, ct: Ct, step: int, out: Ct | None = None) -> Ct:
        out = out or self.new_ct(ct.level)
        a, o = ct._c(), out._c()
        _check(lib().he_rotate(self.h, C.byref(a), int(step), C.byref(o)), "he_rotate")
        out.level, out.scale = int(o.level), float(o.scale)
        return out

    def rotate_hoisted(self, ct: Ct, steps) -> list:
        return self.rotate_hoisted_batch([ct], steps)

    def rotate_hoisted_batch(self, cts, steps, outs=None):
        outs = outs or [self.new_ct(c.level) for c in cts for _ in steps]
        st = (C.c_int32 * len(steps))(*steps)
        ia, oa = self._arr(cts), self._arr(outs)
        _check(lib().he_rotate_hoisted_batch(self.h, len(cts), ia, len(steps), st, oa), "he_rotate_hoisted_batch")
        self._sync_meta(outs, oa)
        return outs

    def add(self, a: Ct, b: Ct, out: Ct | None = None) -> Ct:
        out = out or self.new_ct(a.level)
        x, y, o = a._c(), b._c(), out._c()
        _check(lib().he_add(self.h, C.byref(x), C.byref(y), C.byref(o)), "he_add")
        out.level, out.scale = int(o.level), float(o.scale)
        return out

    def ntt(self, bufs, first_prime: int, limbs: int, inverse: bool) -> None:
        ptrs = (C.c_void_p * len(bufs))(*[b.data_ptr() for b in bufs])
        _check(lib().he_ntt(self.h, len(bufs), ptrs, first_prime, limbs, int(inverse)), "he_ntt")

    def set_knob(self, key: str, value: int) -> None:
        _check(lib().he_ctx_set_knob(self.h, key.encode(), int(value)), f"he_ctx_set_knob({key})")

    def get_knob(self, key: str) -> int:
        v = C.c_int64()
        _check(lib().he_ctx_get_knob(self.h, key.encode(), C.byref(v)), f"he_ctx_get_knob({key})")
        return int(v.value)

    def trace_read(self) -> dict:
        """{kernel class: (launches, ms, algorithmic bytes)} since the last read."""
        cap = 64
        arr = (_TraceEntry * cap)()
        n = C.c_uint32()
        _check(lib().he_trace_read(self.h, arr, cap, C.byref(n)), "he_trace_read")
        return {arr[i].kernel.decode(): (int(arr[i].launches), float(arr[i].ms), float(arr[i].bytes))
                for i in range(min(n.value, cap))}

    def client(self, max_batch: int, pk: np.ndarray | None = None, sk: np.ndarray | None = None) -> Client:
        return Client(self, max_batch, pk, sk)

    def sync(self) -> None:
        _check(lib().he_sync(self.h), "he_sync")
