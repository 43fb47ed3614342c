"""ctypes binding of libgbs_lhaf.so (the C ABI declared in include/gbs_lhaf.h).

Argument marshalling only: every step of the loop-hafnian path runs in the HIP
library.  Host entry points take numpy arrays; the device entry point takes
torch tensors (device memory and the caller's HIP stream).  Loading fails
loudly when the library has not been built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# GBS_LIB_PATH loads another build of the same library instead (e.g. the
# host-sanitized build that tests/sanitize/run_host_asan.sh makes).
LIB_PATH = os.environ.get("GBS_LIB_PATH") or os.path.join(HERE, "libgbs_lhaf.so")

GBS_FP64 = 0
GBS_FP32_COMP = 1
GBS_DD = 2
GBS_CHARPOLY_LABUDDE = 0
GBS_CHARPOLY_EIGEN = 1
MAX_DIM = 64  # GBS_MAX_DIM
MAX_BATCH_DIM = 56  # GBS_MAX_BATCH_DIM

STATUS = {
    0: "GBS_OK", -1: "GBS_E_ARG", -2: "GBS_E_NOT_SYMMETRIC", -3: "GBS_E_NONFINITE", -4: "GBS_E_TOO_LARGE",
    -5: "GBS_E_NOT_PURE", -6: "GBS_E_NOT_PD", -7: "GBS_E_DEVICE", -8: "GBS_E_NOMEM", -9: "GBS_E_UNSUPPORTED",
}


class GbsError(RuntimeError):
    def __init__(self, code, detail):
        super().__init__(f"{STATUS.get(code, code)}: {detail}")
        self.code = code


class gbs_z(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class gbs_diag(ctypes.Structure):
    _fields_ = [("abs_sum", ctypes.c_double), ("kappa", ctypes.c_double), ("subset_terms", ctypes.c_uint64),
                ("kernel_ms", ctypes.c_double), ("n_pairs", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("lhaf_lo", gbs_z)]


class gbs_tune_report(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("layout", ctypes.c_int32 * 33), ("ns_per_subset", (ctypes.c_double * 4) * 33)]


LAYOUTS = {0: "4x4", 1: "8x4", 2: "8x8", 3: "8x4/1"}


class gbs_batch_info(ctypes.Structure):
    _fields_ = [("items", ctypes.c_int32), ("tiles", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("kernel_nodes", ctypes.c_int32), ("subset_terms", ctypes.c_int64), ("tile_subsets", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("yardstick_flops", ctypes.c_double), ("tune_ms", ctypes.c_double)]


class gbs_sample_info(ctypes.Structure):
    _fields_ = [("loop_hafnians", ctypes.c_int64), ("subset_terms", ctypes.c_int64), ("max_dim", ctypes.c_int32),
                ("groups", ctypes.c_int32), ("setup_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


class gbs_profile(ctypes.Structure):
    _fields_ = [("charpoly_ms", ctypes.c_double), ("series_ms", ctypes.c_double), ("reduce_ms", ctypes.c_double),
                ("charpoly_launches", ctypes.c_int64), ("series_launches", ctypes.c_int64),
                ("reduce_launches", ctypes.c_int64), ("charpoly_flops", ctypes.c_double),
                ("subset_terms", ctypes.c_double), ("dominant_kernel", ctypes.c_char * 96),
                ("dominant_ms", ctypes.c_double), ("dominant_flops", ctypes.c_double),
                ("dominant_launches", ctypes.c_int64)]


_L = None
ZP = ctypes.POINTER(gbs_z)
I32P = ctypes.POINTER(ctypes.c_int32)
U64P = ctypes.POINTER(ctypes.c_uint64)
DP = ctypes.POINTER(ctypes.c_double)


def lib():
    """The loaded library (raises if it has not been built)."""
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_2010_15595_amd.build")
        # torch ships its own libamdhip64.so.7; the dynamic loader keeps the first
        # library loaded under that soname.  Loading torch first makes the whole
        # process share torch's HIP runtime, so device pointers and streams from
        # torch are valid in this library (loading ours first breaks torch's init).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int
        L.gbs_init.argtypes = [ctypes.c_int]
        L.gbs_init.restype = st
        L.gbs_finalize.argtypes = []
        L.gbs_finalize.restype = None
        L.gbs_status_string.argtypes = [st]
        L.gbs_status_string.restype = ctypes.c_char_p
        L.gbs_last_error.argtypes = []
        L.gbs_last_error.restype = ctypes.c_char_p
        L.gbs_max_dim.argtypes = []
        L.gbs_max_dim.restype = ctypes.c_int32
        L.gbs_expand.argtypes = [ZP, ctypes.c_int32, ctypes.c_int64, ZP, I32P, ZP, ctypes.c_int64, I32P]
        L.gbs_expand.restype = st
        L.gbs_pure_state.argtypes = [ZP, ZP, ctypes.c_int32, ZP, ZP, DP]
        L.gbs_pure_state.restype = st
        L.gbs_lhaf.argtypes = [ZP, ctypes.c_int32, ctypes.c_int64, ZP, I32P, ctypes.c_int, ZP,
                               ctypes.POINTER(gbs_diag)]
        L.gbs_lhaf.restype = st
        L.gbs_haf.argtypes = [ZP, ctypes.c_int32, ctypes.c_int64, ctypes.c_int, ZP, ctypes.POINTER(gbs_diag)]
        L.gbs_haf.restype = st
        L.gbs_probability.argtypes = [ZP, ZP, I32P, ctypes.c_int32, ctypes.c_int, DP, ZP, ctypes.POINTER(gbs_diag)]
        L.gbs_probability.restype = st
        L.gbs_probability_mixed.argtypes = [ZP, ZP, I32P, ctypes.c_int32, ctypes.c_int, DP, ZP,
                                            ctypes.POINTER(gbs_diag)]
        L.gbs_probability_mixed.restype = st
        L.gbs_sample_pure.argtypes = [ZP, ZP, ctypes.c_int32, ctypes.c_int32, DP, DP, ctypes.c_int32, ctypes.c_int,
                                      I32P, DP, ctypes.POINTER(gbs_sample_info)]
        L.gbs_sample_pure.restype = st
        L.gbs_lhaf_method.argtypes = [ZP, ctypes.c_int32, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ZP,
                                      ctypes.POINTER(gbs_diag)]
        L.gbs_lhaf_method.restype = st
        L.gbs_lhaf_terms.argtypes = [ZP, ctypes.c_int32, ctypes.c_int64, U64P, ctypes.c_int64, ctypes.c_int, ZP]
        L.gbs_lhaf_terms.restype = st
        L.gbs_lhaf_device.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]
        L.gbs_lhaf_device.restype = st
        L.gbs_lhaf_device_noalloc.argtypes = L.gbs_lhaf_device.argtypes
        L.gbs_lhaf_device_noalloc.restype = st
        L.gbs_lhaf_device_shard.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        L.gbs_lhaf_device_shard.restype = st
        L.gbs_combine_partials.argtypes = [DP, ctypes.c_int32, ZP, DP]
        L.gbs_combine_partials.restype = st
        L.gbs_selftest.argtypes = [I32P]
        L.gbs_selftest.restype = st
        L.gbs_profile_enable.argtypes = [ctypes.c_int]
        L.gbs_profile_enable.restype = st
        L.gbs_profile_read.argtypes = [ctypes.POINTER(gbs_profile)]
        L.gbs_profile_read.restype = st
        L.gbs_set_layout.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.gbs_set_layout.restype = st
        L.gbs_autotune.argtypes = [ctypes.c_int32, ctypes.POINTER(gbs_tune_report)]
        L.gbs_autotune.restype = st
        L.gbs_batch_plan_create.argtypes = [I32P, ctypes.c_int32, ctypes.c_int, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_void_p)]
        L.gbs_batch_plan_create.restype = st
        L.gbs_batch_plan_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(gbs_batch_info)]
        L.gbs_batch_plan_info.restype = st
        L.gbs_batch_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.gbs_batch_run.restype = st
        L.gbs_batch_plan_destroy.argtypes = [ctypes.c_void_p]
        L.gbs_batch_plan_destroy.restype = None
        L.gbs_yardstick_flops.argtypes = [ctypes.c_int32]
        L.gbs_yardstick_flops.restype = ctypes.c_double
        _L = L
    return _L


def _check(code):
    if code != 0:
        raise GbsError(code, lib().gbs_last_error().decode())


def _zarr(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _zp(a):
    return a.ctypes.data_as(ZP) if a is not None and a.size else None


def _diag_dict(d):
    out = {f: getattr(d, f) for f, _ in gbs_diag._fields_}
    out["lhaf_lo"] = complex(d.lhaf_lo.re, d.lhaf_lo.im)
    return out


def init(device=0):
    _check(lib().gbs_init(int(device)))


def finalize():
    lib().gbs_finalize()


def max_dim():
    return lib().gbs_max_dim()


def expand(B, gamma=None, mult=None):
    B = _zarr(B)
    M = B.shape[0]
    g = _zarr(gamma) if gamma is not None else None
    mu = np.ascontiguousarray(mult, dtype=np.int32) if mult is not None else None
    N = int(mu.sum()) if mu is not None else M
    out = np.zeros((max(N, 1), max(N, 1)), dtype=np.complex128)
    nout = ctypes.c_int32(0)
    _check(lib().gbs_expand(_zp(B), M, M, _zp(g), mu.ctypes.data_as(I32P) if mu is not None else None,
                            out.ctypes.data_as(ZP), out.size, ctypes.byref(nout)))
    return out[: nout.value, : nout.value].copy()


def pure_state(Q, alpha):
    Q = _zarr(Q)
    al = _zarr(alpha)
    M = Q.shape[0] // 2
    B = np.zeros((M, M), dtype=np.complex128)
    g = np.zeros(M, dtype=np.complex128)
    pv = ctypes.c_double(0)
    _check(lib().gbs_pure_state(_zp(Q), _zp(al), M, B.ctypes.data_as(ZP), g.ctypes.data_as(ZP), ctypes.byref(pv)))
    return B, g, pv.value


def lhaf(A, gamma=None, mult=None, prec=GBS_FP64, with_diag=False):
    """lhaf(filldiag(A_S, gamma_S)) on the GPU (host arrays in, complex out)."""
    A = _zarr(A)
    M = A.shape[0]
    g = _zarr(gamma) if gamma is not None else None
    mu = np.ascontiguousarray(mult, dtype=np.int32) if mult is not None else None
    out = gbs_z()
    d = gbs_diag()
    _check(lib().gbs_lhaf(_zp(A), M, M, _zp(g), mu.ctypes.data_as(I32P) if mu is not None else None, prec,
                          ctypes.byref(out), ctypes.byref(d)))
    val = complex(out.re, out.im)
    return (val, _diag_dict(d)) if with_diag else val


def lhaf_method(A, method=GBS_CHARPOLY_LABUDDE, prec=GBS_FP64, with_diag=False):
    """lhaf on the LDS-resident reference kernels with La Budde (method 0) or
    eigenvalue (method 1) characteristic polynomials."""
    A = _zarr(A)
    out = gbs_z()
    d = gbs_diag()
    _check(lib().gbs_lhaf_method(_zp(A), A.shape[0], A.shape[0], prec, method, ctypes.byref(out), ctypes.byref(d)))
    val = complex(out.re, out.im)
    return (val, _diag_dict(d)) if with_diag else val


def haf(A, prec=GBS_FP64, with_diag=False):
    A = _zarr(A)
    out = gbs_z()
    d = gbs_diag()
    _check(lib().gbs_haf(_zp(A), A.shape[0], A.shape[0], prec, ctypes.byref(out), ctypes.byref(d)))
    val = complex(out.re, out.im)
    return (val, _diag_dict(d)) if with_diag else val


def probability(Q, alpha, pattern, prec=GBS_FP64, with_lhaf=False):
    Q = _zarr(Q)
    al = _zarr(alpha)
    pat = np.ascontiguousarray(pattern, dtype=np.int32)
    M = pat.shape[0]
    p = ctypes.c_double(0)
    lh = gbs_z()
    _check(lib().gbs_probability(_zp(Q), _zp(al), pat.ctypes.data_as(I32P), M, prec, ctypes.byref(p),
                                 ctypes.byref(lh), None))
    return (p.value, complex(lh.re, lh.im)) if with_lhaf else p.value


def probability_mixed(Q, alpha, pattern, prec=GBS_FP64, with_lhaf=False, with_diag=False):
    """Eq. (11): p(vac) lhaf(filldiag(A_S, gamma_S)) / prod s_i! for a general
    Gaussian state (alpha None = no displacement)."""
    Q = _zarr(Q)
    al = _zarr(alpha) if alpha is not None else None
    pat = np.ascontiguousarray(pattern, dtype=np.int32)
    M = pat.shape[0]
    p = ctypes.c_double(0)
    lh = gbs_z()
    d = gbs_diag()
    _check(lib().gbs_probability_mixed(_zp(Q), _zp(al), pat.ctypes.data_as(I32P), M, prec, ctypes.byref(p),
                                       ctypes.byref(lh), ctypes.byref(d)))
    out = [p.value]
    if with_lhaf:
        out.append(complex(lh.re, lh.im))
    if with_diag:
        out.append(_diag_dict(d))
    return out[0] if len(out) == 1 else tuple(out)


def sample_pure(Q, alpha, cutoff, normals, uniforms, prec=GBS_FP64, with_probs=False, with_info=False):
    """Samples of a pure state by the conditional chain of Sec. III.

    normals: (nsamples, 2 (M - 1)) standard normals of the heterodyne outcomes
    of modes 2..M; uniforms: (nsamples, M) in [0, 1) for the photon-number
    draws.  Returns the (nsamples, M) int32 patterns, plus the (nsamples, M,
    cutoff + 1) normalised conditional probabilities and/or an info dict."""
    Q = _zarr(Q)
    al = _zarr(alpha)
    M = Q.shape[0] // 2
    u = np.ascontiguousarray(uniforms, dtype=np.float64).reshape(-1, M)
    ns = u.shape[0]
    z = np.ascontiguousarray(normals, dtype=np.float64).reshape(ns, 2 * (M - 1))
    out = np.zeros((ns, M), dtype=np.int32)
    probs = np.zeros((ns, M, cutoff + 1)) if with_probs else None
    info = gbs_sample_info()
    _check(lib().gbs_sample_pure(_zp(Q), _zp(al), M, cutoff, z.ctypes.data_as(DP) if z.size else None,
                                 u.ctypes.data_as(DP), ns, prec, out.ctypes.data_as(I32P),
                                 probs.ctypes.data_as(DP) if with_probs else None, ctypes.byref(info)))
    res = [out]
    if with_probs:
        res.append(probs)
    if with_info:
        res.append({f: getattr(info, f) for f, _ in gbs_sample_info._fields_})
    return res[0] if len(res) == 1 else tuple(res)


def lhaf_terms(A, masks, prec=GBS_FP64):
    """Signed subset terms t_S for the given pair-subset masks."""
    A = _zarr(A)
    mk = np.ascontiguousarray(masks, dtype=np.uint64)
    out = np.zeros(mk.shape[0], dtype=np.complex128)
    _check(lib().gbs_lhaf_terms(_zp(A), A.shape[0], A.shape[0], mk.ctypes.data_as(U64P), mk.shape[0], prec,
                                out.ctypes.data_as(ZP)))
    return out


def lhaf_device(A, out, abs_sum=None, stream=None, prec=GBS_FP64):
    """Stream-ordered lhaf of a device-resident N x N torch.complex128 matrix.
    ``out`` (torch.complex128, >= 1 element) and ``abs_sum`` (torch.float64)
    receive the result on the device; nothing is synchronised."""
    import torch

    if A.dtype != torch.complex128 or not A.is_cuda or not A.is_contiguous():
        raise ValueError("A must be a contiguous complex128 device tensor")
    if out.dtype != torch.complex128 or not out.is_cuda:
        raise ValueError("out must be a complex128 device tensor")
    if abs_sum is not None and (abs_sum.dtype != torch.float64 or not abs_sum.is_cuda):
        raise ValueError("abs_sum must be a float64 device tensor")
    N = A.shape[0]
    if stream is None:
        stream = torch.cuda.current_stream(A.device)
    _check(lib().gbs_lhaf_device(ctypes.c_void_p(A.data_ptr()), N, prec, ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(abs_sum.data_ptr()) if abs_sum is not None else None,
                                 ctypes.c_void_p(stream.cuda_stream)))


def lhaf_device_noalloc(A, out, abs_sum=None, stream=None, prec=GBS_FP64):
    """lhaf_device through the entry point that allocates nothing (its scratch
    is a fixed per-device array; init() must come first).  Calls on one device
    must not overlap in time."""
    import torch

    if A.dtype != torch.complex128 or not A.is_cuda or not A.is_contiguous():
        raise ValueError("A must be a contiguous complex128 device tensor")
    if out.dtype != torch.complex128 or not out.is_cuda:
        raise ValueError("out must be a complex128 device tensor")
    if abs_sum is not None and (abs_sum.dtype != torch.float64 or not abs_sum.is_cuda):
        raise ValueError("abs_sum must be a float64 device tensor")
    N = A.shape[0]
    if stream is None:
        stream = torch.cuda.current_stream(A.device)
    _check(lib().gbs_lhaf_device_noalloc(ctypes.c_void_p(A.data_ptr()), N, prec, ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(abs_sum.data_ptr()) if abs_sum is not None else None,
                                         ctypes.c_void_p(stream.cuda_stream)))


def lhaf_device_shard(A, record, shard, nshards, stream=None, prec=GBS_FP64):
    """Shard ``shard`` of ``nshards`` of the subset sum of a device-resident
    N x N torch.complex128 matrix: its compensated partial record (five
    float64 values: sum re, compensation re, sum im, compensation im,
    sum |t_S|) is written to the device tensor ``record``; stream-ordered."""
    import torch

    if A.dtype != torch.complex128 or not A.is_cuda or not A.is_contiguous():
        raise ValueError("A must be a contiguous complex128 device tensor")
    if record.dtype != torch.float64 or not record.is_cuda or not record.is_contiguous() or record.numel() < 5:
        raise ValueError("record must be a contiguous float64 device tensor of >= 5 elements")
    N = A.shape[0]
    if stream is None:
        stream = torch.cuda.current_stream(A.device)
    _check(lib().gbs_lhaf_device_shard(ctypes.c_void_p(A.data_ptr()), N, prec, int(shard), int(nshards),
                                       ctypes.c_void_p(record.data_ptr()), ctypes.c_void_p(stream.cuda_stream)))


def combine_partials(records):
    """Fold shard records (array of shape (G, 5), in shard order) into
    (loop hafnian, sum |t_S|)."""
    r = np.ascontiguousarray(np.asarray(records, dtype=np.float64).reshape(-1, 5))
    out = gbs_z()
    ab = ctypes.c_double()
    _check(lib().gbs_combine_partials(r.ctypes.data_as(DP), r.shape[0], ctypes.byref(out), ctypes.byref(ab)))
    return complex(out.re, out.im), ab.value


def selftest():
    f = ctypes.c_int32(-1)
    _check(lib().gbs_selftest(ctypes.byref(f)))
    return f.value


def profile_enable(on=True):
    _check(lib().gbs_profile_enable(1 if on else 0))


def profile_read():
    p = gbs_profile()
    _check(lib().gbs_profile_read(ctypes.byref(p)))
    out = {f: getattr(p, f) for f, _ in gbs_profile._fields_}
    out["dominant_kernel"] = p.dominant_kernel.decode()
    return out


def yardstick_flops(N):
    return lib().gbs_yardstick_flops(int(N))


def set_layout(n, s, layout):
    """Force the per-subset kernel lane grid (0 = 4x4, 1 = 8x4, 2 = 8x8, -1 =
    default) for size-s subsets of n-pair loop hafnians (0 = all)."""
    _check(lib().gbs_set_layout(int(n), int(s), int(layout)))


def autotune(n):
    """Run the autotuner for n pairs; returns {s: (layout, {layout: ns/subset})}."""
    r = gbs_tune_report()
    _check(lib().gbs_autotune(int(n), ctypes.byref(r)))
    out = {}
    for s in range(1, n + 1):
        times = {LAYOUTS[k]: r.ns_per_subset[s][k] for k in range(4) if r.ns_per_subset[s][k] > 0}
        out[s] = (LAYOUTS[r.layout[s]], times)
    return out


def pack(mats):
    """Packed batch input: the matrices' row-major blocks concatenated."""
    flat = [np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).ravel() for a in mats]
    return np.concatenate(flat) if flat else np.zeros(0, dtype=np.complex128)


class BatchPlan:
    """A captured schedule for a batch of loop hafnians of the given
    dimensions (gbs_batch_plan_create); run() replays it on a stream."""

    def __init__(self, dims, prec=GBS_FP64, autotune=False):
        d = np.ascontiguousarray(dims, dtype=np.int32)
        self.count = int(d.shape[0])
        h = ctypes.c_void_p()
        _check(lib().gbs_batch_plan_create(d.ctypes.data_as(I32P), self.count, prec, 1 if autotune else 0,
                                           ctypes.byref(h)))
        self._h = h

    def info(self):
        i = gbs_batch_info()
        _check(lib().gbs_batch_plan_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in gbs_batch_info._fields_}

    def run(self, mats_dev, out, abs_sum=None, stream=None):
        """mats_dev: packed complex128 device tensor; out: complex128 device
        tensor of length count; abs_sum: float64 device tensor or None."""
        import torch

        if mats_dev.dtype != torch.complex128 or not mats_dev.is_cuda or not mats_dev.is_contiguous():
            raise ValueError("mats_dev must be a contiguous complex128 device tensor")
        if out.dtype != torch.complex128 or not out.is_cuda or out.numel() < self.count:
            raise ValueError("out must be a complex128 device tensor with one entry per item")
        if abs_sum is not None and (abs_sum.dtype != torch.float64 or not abs_sum.is_cuda):
            raise ValueError("abs_sum must be a float64 device tensor")
        if stream is None:
            stream = torch.cuda.current_stream(out.device)
        _check(lib().gbs_batch_run(self._h, ctypes.c_void_p(mats_dev.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(abs_sum.data_ptr()) if abs_sum is not None else None,
                                   ctypes.c_void_p(stream.cuda_stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().gbs_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
