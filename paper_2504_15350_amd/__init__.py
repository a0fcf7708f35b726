"""Python binding of librpod.so (randomized POD on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/rpod.h. PyTorch supplies device
memory and streams. There is no fallback path: if the library is not built,
every entry point raises.

Layout convention: a column-major m x n matrix is a row-major torch tensor
of shape (n, m). So the snapshot matrix S is passed as St with St[j] =
snapshot j, the modes come back as Phi_t (r, m) with Phi_t[k] = mode k, and
the coefficients as A_t (n, r) with A_t[j, k] = coefficient k of snapshot j.
"""

import ctypes
import os

import numpy as np
import torch

__all__ = ["RpodError", "Plan", "BatchPlan", "Tuning", "autotune", "WarmModel", "WarmPlan", "AdaptivePlan", "rpod", "generate_omega", "sketch_bits", "lib", "LIB_PATH",
           "STATUS", "FLAG_SHIFTED", "FLAG_BREAKDOWN", "FLAG_NONFINITE", "FLAG_JACOBI_SLOW", "FLAG_RANK_CUT"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpod.so")

STATUS = {0: "RPOD_OK", 1: "RPOD_EINVAL", 2: "RPOD_EINVAL_DATA", 3: "RPOD_ENOMEM", 4: "RPOD_EHIP",
          5: "RPOD_EUNSUPPORTED", 6: "RPOD_EBREAKDOWN"}
FLAG_SHIFTED, FLAG_BREAKDOWN, FLAG_NONFINITE, FLAG_JACOBI_SLOW, FLAG_RANK_CUT = 0x1, 0x2, 0x4, 0x8, 0x20

_DTYPES = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2, torch.float16: 3}


class RpodError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("r", ctypes.c_int32), ("p", ctypes.c_int32),
                ("q", ctypes.c_int32), ("flags", ctypes.c_uint32), ("block_cols", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    """Launch-shape knobs of a plan (rpod_tuning); 0 = library default."""
    _fields_ = [("stq_workgroups", ctypes.c_int32), ("gram_workgroups", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 6)]

    def __repr__(self):
        return f"Tuning(stq_workgroups={self.stq_workgroups}, gram_workgroups={self.gram_workgroups})"


class _WarmDesc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("r", ctypes.c_int32), ("max_train", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class _WarmLayout(ctypes.Structure):
    _fields_ = [(k, ctypes.c_size_t) for k in ("params", "grads", "adam_m", "adam_v", "bank", "gram", "gram8",
                                                "total")]


WARM_PARAMS = 69128
WARM_BANK = 8
FLAG_RESIDUAL = 0x10

_lib = None


def lib():
    """Load librpod.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2504_15350_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        sig = {
            "rpod_workspace_size": [ctypes.POINTER(_Desc), ctypes.POINTER(ctypes.c_size_t)],
            "rpod_plan_create": [ctypes.POINTER(vp), ctypes.POINTER(_Desc), vp, ctypes.c_size_t, vp],
            "rpod_plan_destroy": [vp],
            "rpod_compute": [vp, vp, u64, vp, vp, vp],
            "rpod_status_query": [vp, ctypes.POINTER(i32)],
            "rpod_energy": [vp, i32, ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)],
            "rpod_reconstruct_workspace_size": [i64, i32, ctypes.POINTER(ctypes.c_size_t)],
            "rpod_reconstruct": [i32, i64, i32, i64, vp, vp, vp, vp, vp, i64, vp, ctypes.c_size_t, vp,
                                 ctypes.POINTER(ctypes.c_double)],
            "rpod_reconstruct_noalloc": [i32, i64, i32, i64, vp, vp, vp, vp, vp, i64, vp,
                                         ctypes.POINTER(ctypes.c_double)],
            "rpod_generate_omega": [u64, i64, i32, i32, vp, i64, vp],
            "rpod_sketch_bits": [u64, i64, i32, vp, vp],
            "rpod_plan_set_timing": [vp, i32],
            "rpod_plan_get_timing": [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
            "rpod_workspace_size_batched": [ctypes.POINTER(_Desc), i32, ctypes.POINTER(ctypes.c_size_t)],
            "rpod_plan_create_batched": [ctypes.POINTER(vp), ctypes.POINTER(_Desc), i32, vp, ctypes.c_size_t, vp],
            "rpod_compute_batched": [vp, ctypes.POINTER(vp), ctypes.POINTER(u64), ctypes.POINTER(vp),
                                     ctypes.POINTER(vp), ctypes.POINTER(vp)],
            "rpod_status_query_batched": [vp, ctypes.POINTER(i32)],
            "rpod_workspace_size_tuned": [ctypes.POINTER(_Desc), i32, ctypes.POINTER(Tuning),
                                          ctypes.POINTER(ctypes.c_size_t)],
            "rpod_plan_create_tuned": [ctypes.POINTER(vp), ctypes.POINTER(_Desc), i32, ctypes.POINTER(Tuning), vp,
                                       ctypes.c_size_t, vp],
            "rpod_autotune_workspace_size": [ctypes.POINTER(_Desc), i32, ctypes.POINTER(ctypes.c_size_t)],
            "rpod_autotune": [ctypes.POINTER(_Desc), i32, ctypes.POINTER(vp), vp, ctypes.c_size_t, vp, i32,
                              ctypes.c_char_p, ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_double)],
            "rpod_warm_layout_of": [ctypes.POINTER(_WarmDesc), ctypes.POINTER(_WarmLayout)],
            "rpod_warm_create": [ctypes.POINTER(vp), ctypes.POINTER(_WarmDesc), vp, ctypes.c_size_t, vp],
            "rpod_warm_destroy": [vp],
            "rpod_warm_set_bank": [vp, ctypes.POINTER(vp)],
            "rpod_warm_targets": [vp, vp, vp],
            "rpod_warm_loss_grad": [vp, vp, vp, i32, vp],
            "rpod_warm_train": [vp, vp, vp, i32, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float, vp],
            "rpod_warm_predict": [vp, vp, i32, vp],
            "rpod_workspace_size_warm": [ctypes.POINTER(_Desc), vp, i32, ctypes.POINTER(ctypes.c_size_t)],
            "rpod_plan_create_warm": [ctypes.POINTER(vp), ctypes.POINTER(_Desc), vp, i32, ctypes.c_double, vp,
                                      ctypes.c_size_t, vp],
            "rpod_compute_warm": [vp, vp, ctypes.POINTER(ctypes.c_float), u64, vp, vp, vp, ctypes.POINTER(i32),
                                  ctypes.POINTER(ctypes.c_double)],
            "rpod_warm_residuals": [vp, ctypes.POINTER(ctypes.c_double)],
            "rpod_workspace_size_adaptive": [ctypes.POINTER(_Desc), ctypes.c_double, ctypes.POINTER(ctypes.c_size_t)],
            "rpod_plan_create_adaptive": [ctypes.POINTER(vp), ctypes.POINTER(_Desc), ctypes.c_double, vp,
                                          ctypes.c_size_t, vp],
            "rpod_compute_adaptive": [vp, vp, u64, vp, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                      ctypes.POINTER(ctypes.c_double)],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.rpod_last_error.argtypes = []
        L.rpod_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise RpodError(status, lib().rpod_last_error().decode())


def _stream_ptr(stream, device):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream), s


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def make_desc(m, n, r, p, q, dtype, ld=None, flags=0, block_cols=0):
    if dtype not in _DTYPES:
        raise TypeError(f"unsupported dtype {dtype}")
    return _Desc(int(m), int(n), int(m if ld is None else ld), _DTYPES[dtype], int(r), int(p), int(q), int(flags),
                 int(block_cols))


DESC_ENERGY = 0x1  # rpod_desc.flags: compute ||S||_F^2 for rpod_energy


def workspace_size(m, n, r, p, q, dtype, ld=None, block_cols=0, flags=0):
    d = make_desc(m, n, r, p, q, dtype, ld, flags=flags, block_cols=block_cols)
    out = ctypes.c_size_t(0)
    _check(lib().rpod_workspace_size(ctypes.byref(d), ctypes.byref(out)))
    return out.value


def workspace_size_batched(descs, tuning=None):
    arr = (_Desc * len(descs))(*descs)
    out = ctypes.c_size_t(0)
    if tuning is None:
        _check(lib().rpod_workspace_size_batched(arr, len(descs), ctypes.byref(out)))
    else:
        _check(lib().rpod_workspace_size_tuned(arr, len(descs), ctypes.byref(tuning), ctypes.byref(out)))
    return out.value


def _shape_descs(shapes, q, dtype):
    out = []
    for sh in shapes:
        m, n, r, p = (int(x) for x in sh[:4])
        ld = int(sh[4]) if len(sh) > 4 else m
        bc = int(sh[5]) if len(sh) > 5 else 0  # block_cols: fluctuations about block time averages
        out.append(((m, n, r, p, ld), make_desc(m, n, r, p, q, dtype, ld, block_cols=bc)))
    return out


def autotune(shapes, q, Sts, dtype=None, repeats=3, cache=None, device=None, stream=None):
    """rpod_autotune over a batch given as shapes (m, n, r, p[, ld]) and the
    device tensors Sts; returns (Tuning, ms per call). cache: a text file
    path (default: environment variable RPOD_TUNE_CACHE, if set)."""
    dtype = Sts[0].dtype if dtype is None else dtype
    dev = _norm_device(Sts[0].device if device is None else device)
    sd = _shape_descs(shapes, q, dtype)
    for St, ((m, n, _r, _p, ld), _d) in zip(Sts, sd):
        _check_St(St, dtype, dev, m, n, ld)
    arr = (_Desc * len(sd))(*[d for _, d in sd])
    nbytes = ctypes.c_size_t(0)
    _check(lib().rpod_autotune_workspace_size(arr, len(sd), ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    sptr, _s = _stream_ptr(stream, dev)
    S_arr = (ctypes.c_void_p * len(sd))(*[St.data_ptr() for St in Sts])
    cache = os.environ.get("RPOD_TUNE_CACHE") if cache is None else cache
    best = Tuning()
    ms = ctypes.c_double(0)
    _check(lib().rpod_autotune(arr, len(sd), S_arr, _dev_ptr(ws), nbytes.value, sptr, int(repeats),
                               None if cache is None else str(cache).encode(), ctypes.byref(best), ctypes.byref(ms)))
    del ws
    return best, ms.value


class _PlanBase:
    def set_timing(self, enable=True):
        """Record HIP events around every pass over S of later compute calls."""
        _check(lib().rpod_plan_set_timing(self._h, 1 if enable else 0))

    def timing(self, pass_kind):
        """(launches, total_ms, bytes_per_launch, flops_per_launch) of pass 0 (S X), 1 (S^T Q) or 2
        (the 16-bit refinement S^T Q with Q as hi + lo)."""
        n = ctypes.c_int64(0)
        t, b, f = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        _check(lib().rpod_plan_get_timing(self._h, int(pass_kind), ctypes.byref(n), ctypes.byref(t),
                                          ctypes.byref(b), ctypes.byref(f)))
        return n.value, t.value, b.value, f.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().rpod_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_St(St, dtype, device, m, n, ld):
    if St.dtype != dtype or St.device != device:
        raise TypeError("St must be a tensor of the plan's dtype on the plan's device")
    if St.dim() != 2 or St.shape[0] != n or St.shape[1] < m:
        raise ValueError(f"St must have shape ({n}, >= {m})")
    if St.stride(1) != 1 or St.stride(0) != ld:
        raise ValueError("St must be row-major with row stride equal to the plan's ld")


def reconstruct(Phi_t, alpha_t, mean=None, ref_t=None, want_fields=True, stream=None):
    """rpod_reconstruct: fields mean + Phi alpha and the relative L2 error of the time averages.

    Phi_t (r, m), alpha_t (T, r), mean (m,) or None, ref_t (T, ld_ref) or None, all on
    one device in float32 or float64 (the column-major layouts of the C ABI).
    Returns (fields_t (T, m) or None, eps or None).
    """
    dt = Phi_t.dtype
    if dt not in (torch.float32, torch.float64):
        raise TypeError("Phi must be float32 or float64")
    r, m = Phi_t.shape
    T = alpha_t.shape[0]
    for t in (alpha_t, mean, ref_t):
        if t is not None and (t.dtype != dt or t.device != Phi_t.device or not t.is_contiguous()):
            raise ValueError("alpha, mean and ref must be contiguous tensors of Phi's dtype and device")
    if not Phi_t.is_contiguous() or alpha_t.shape[1] != r:
        raise ValueError("Phi_t must be contiguous (r, m) and alpha_t (T, r)")
    dev = Phi_t.device
    nb = ctypes.c_size_t(0)
    _check(lib().rpod_reconstruct_workspace_size(m, r, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    out = torch.empty((T, m), dtype=dt, device=dev) if want_fields else None
    eps = ctypes.c_double(0.0)
    ld_ref = ref_t.shape[1] if ref_t is not None else m
    sptr, _s = _stream_ptr(stream, dev)
    vp = ctypes.c_void_p
    _check(lib().rpod_reconstruct(_DTYPES[dt], m, r, T, _dev_ptr(Phi_t),
                                  _dev_ptr(mean) if mean is not None else vp(None), _dev_ptr(alpha_t),
                                  _dev_ptr(out) if out is not None else vp(None),
                                  _dev_ptr(ref_t) if ref_t is not None else vp(None), ld_ref, _dev_ptr(ws), nb.value,
                                  sptr, ctypes.byref(eps)))
    if ref_t is None:
        torch.cuda.synchronize(dev)
    return out, (eps.value if ref_t is not None else None)


def _norm_device(device):
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


class Plan(_PlanBase):
    """A plan for one matrix shape: rpod_plan_create / rpod_compute / rpod_status_query."""

    def __init__(self, m, n, r, p, q, dtype=torch.float32, ld=None, device="cuda", stream=None, block_cols=0,
                 energy=False):
        self.device = _norm_device(device)
        self.m, self.n, self.r, self.p, self.q = int(m), int(n), int(r), int(p), int(q)
        self.ld = self.m if ld is None else int(ld)
        self.dtype = dtype
        self.block_cols = int(block_cols)  # > 0: decompose the fluctuations about block time averages
        self.out_dtype = torch.float64 if dtype == torch.float64 else torch.float32
        flags = DESC_ENERGY if energy else 0
        self._desc = make_desc(m, n, r, p, q, dtype, ld, flags=flags, block_cols=block_cols)
        nbytes = workspace_size(m, n, r, p, q, dtype, ld, block_cols=block_cols, flags=flags)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        sptr, self.stream = _stream_ptr(stream, self.device)
        h = ctypes.c_void_p()
        _check(lib().rpod_plan_create(ctypes.byref(h), ctypes.byref(self._desc), _dev_ptr(self.workspace),
                                      nbytes, sptr))
        self._h = h

    def compute(self, St, seed, out=None, check=True):
        """rPOD of the column-major S given as St (n, ld) -> (Phi_t (r, m), sigma (r,), A_t (n, r)).

        With check=True the stream is synchronised and the device status
        word is turned into an exception; check=False only enqueues.
        """
        _check_St(St, self.dtype, self.device, self.m, self.n, self.ld)
        if out is None:
            Phi = torch.empty((self.r, self.m), dtype=self.out_dtype, device=self.device)
            sigma = torch.empty((self.r,), dtype=torch.float64, device=self.device)
            A = torch.empty((self.n, self.r), dtype=self.out_dtype, device=self.device)
        else:
            Phi, sigma, A = out
        _check(lib().rpod_compute(self._h, _dev_ptr(St), ctypes.c_uint64(int(seed) & (2 ** 64 - 1)),
                                  _dev_ptr(Phi), _dev_ptr(sigma), _dev_ptr(A)))
        if check:
            self.status()
        return Phi, sigma, A

    def energy(self, delta):
        """rpod_energy after a compute call (plans made with energy=True):
        (e_k = sum_{i<=k} sigma_i^2 / ||S||_F^2 for k = 1..r+p as a numpy array,
        the smallest k with e_k >= delta or -1)."""
        import numpy as np
        e = (ctypes.c_double * (self.r + self.p))()
        rk = ctypes.c_int32(0)
        _check(lib().rpod_energy(self._h, 0, ctypes.c_double(float(delta)), e, ctypes.byref(rk)))
        return np.array(e[:], dtype=np.float64), rk.value

    def status(self):
        """Synchronise and return the device flags; raise on an error status."""
        fl = ctypes.c_int32(0)
        st = lib().rpod_status_query(self._h, ctypes.byref(fl))
        self.last_flags = fl.value
        _check(st)
        return fl.value



class BatchPlan(_PlanBase):
    """A plan for a batch of matrices: rpod_plan_create_batched / rpod_compute_batched.

    shapes: list of (m, n, r, p), (m, n, r, p, ld) or (m, n, r, p, ld, block_cols);
    all share dtype and q.
    """

    def __init__(self, shapes, q, dtype=torch.float32, device="cuda", stream=None, tuning=None):
        self.device = _norm_device(device)
        self.dtype = dtype
        self.q = int(q)
        self.out_dtype = torch.float64 if dtype == torch.float64 else torch.float32
        sd = _shape_descs(shapes, q, dtype)
        self.shapes = [sh for sh, _ in sd]
        descs = [d for _, d in sd]
        self.count = len(descs)
        self.tuning = tuning
        self._descs = (_Desc * self.count)(*descs)
        nbytes = workspace_size_batched(descs, tuning)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        sptr, self.stream = _stream_ptr(stream, self.device)
        h = ctypes.c_void_p()
        if tuning is None:
            _check(lib().rpod_plan_create_batched(ctypes.byref(h), self._descs, self.count,
                                                  _dev_ptr(self.workspace), nbytes, sptr))
        else:
            _check(lib().rpod_plan_create_tuned(ctypes.byref(h), self._descs, self.count, ctypes.byref(tuning),
                                                _dev_ptr(self.workspace), nbytes, sptr))
        self._h = h

    def alloc_outputs(self):
        outs = []
        for (m, n, r, _p, _ld) in self.shapes:
            outs.append((torch.empty((r, m), dtype=self.out_dtype, device=self.device),
                         torch.empty((r,), dtype=torch.float64, device=self.device),
                         torch.empty((n, r), dtype=self.out_dtype, device=self.device)))
        return outs

    def compute(self, Sts, seeds, outs=None, check=True):
        """rPOD of every matrix; Sts[i] is (n_i, ld_i). Returns a list of (Phi_t, sigma, A_t)."""
        if len(Sts) != self.count or len(seeds) != self.count:
            raise ValueError(f"expected {self.count} matrices and seeds")
        for St, (m, n, _r, _p, ld) in zip(Sts, self.shapes):
            _check_St(St, self.dtype, self.device, m, n, ld)
        if outs is None:
            outs = self.alloc_outputs()
        vp = ctypes.c_void_p
        S_arr = (vp * self.count)(*[St.data_ptr() for St in Sts])
        seed_arr = (ctypes.c_uint64 * self.count)(*[int(s) & (2 ** 64 - 1) for s in seeds])
        P_arr = (vp * self.count)(*[o[0].data_ptr() for o in outs])
        s_arr = (vp * self.count)(*[o[1].data_ptr() for o in outs])
        A_arr = (vp * self.count)(*[o[2].data_ptr() for o in outs])
        _check(lib().rpod_compute_batched(self._h, S_arr, seed_arr, P_arr, s_arr, A_arr))
        if check:
            self.status()
        return outs

    def status(self):
        """Synchronise; per-matrix device flags (list); raise on an error status."""
        fl = (ctypes.c_int32 * self.count)()
        st = lib().rpod_status_query_batched(self._h, fl)
        self.last_flags = list(fl)
        _check(st)
        return list(fl)


class WarmModel:
    """The learned warm start's network and basis bank (rpod_warm_*).

    Bases, parameter vectors and targets are device tensors; a basis of m
    rows and r columns is passed as an (r, m) tensor (column-major m x r).
    """

    def __init__(self, m, r, max_train=128, seed=0, device="cuda", stream=None):
        self.device = _norm_device(device)
        self.m, self.r, self.max_train = int(m), int(r), int(max_train)
        self._desc = _WarmDesc(self.m, self.r, self.max_train, int(seed) & (2 ** 64 - 1))
        self.layout = _WarmLayout()
        _check(lib().rpod_warm_layout_of(ctypes.byref(self._desc), ctypes.byref(self.layout)))
        self.workspace = torch.empty(self.layout.total, dtype=torch.uint8, device=self.device)
        sptr, self.stream = _stream_ptr(stream, self.device)
        h = ctypes.c_void_p()
        _check(lib().rpod_warm_create(ctypes.byref(h), ctypes.byref(self._desc), _dev_ptr(self.workspace),
                                      self.layout.total, sptr))
        self._h = h

    def _view(self, off, count, dtype):
        nbytes = count * torch.empty((), dtype=dtype).element_size()
        return self.workspace[off:off + nbytes].view(dtype)

    def params(self):
        return self._view(self.layout.params, WARM_PARAMS, torch.float32)

    def grads(self):
        return self._view(self.layout.grads, WARM_PARAMS, torch.float32)

    def gram(self):
        k = WARM_BANK * self.r
        return self._view(self.layout.gram, k * k, torch.float64).view(k, k)

    def gram8(self):
        return self._view(self.layout.gram8, WARM_BANK * WARM_BANK, torch.float64).view(WARM_BANK, WARM_BANK)

    def _basis_ok(self, B):
        if B.dtype != torch.float32 or B.device != self.device or tuple(B.shape) != (self.r, self.m) \
                or not B.is_contiguous():
            raise ValueError(f"a basis must be a contiguous float32 ({self.r}, {self.m}) tensor on {self.device}")

    def set_bank(self, bases):
        if len(bases) != WARM_BANK:
            raise ValueError(f"the bank holds {WARM_BANK} bases")
        for B in bases:
            self._basis_ok(B)
        arr = (ctypes.c_void_p * WARM_BANK)(*[B.data_ptr() for B in bases])
        _check(lib().rpod_warm_set_bank(self._h, arr))

    def targets(self, basis):
        self._basis_ok(basis)
        b = torch.empty(WARM_BANK, dtype=torch.float64, device=self.device)
        _check(lib().rpod_warm_targets(self._h, _dev_ptr(basis), _dev_ptr(b)))
        return b

    def _pairs_ok(self, mu, b=None):
        if mu.dtype != torch.float32 or mu.dim() != 2 or mu.shape[1] != 4 or not mu.is_contiguous() \
                or mu.device != self.device:
            raise ValueError("mu must be a contiguous float32 (N, 4) device tensor")
        if b is not None and (b.dtype != torch.float64 or tuple(b.shape) != (mu.shape[0], WARM_BANK)
                              or not b.is_contiguous() or b.device != self.device):
            raise ValueError("b must be a contiguous float64 (N, 8) device tensor")

    def loss_grad(self, mu, b):
        self._pairs_ok(mu, b)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(lib().rpod_warm_loss_grad(self._h, _dev_ptr(mu), _dev_ptr(b), mu.shape[0], _dev_ptr(loss)))
        return loss

    def train(self, mu, b, epochs, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-5):
        self._pairs_ok(mu, b)
        losses = torch.empty(max(1, int(epochs)), dtype=torch.float32, device=self.device)
        _check(lib().rpod_warm_train(self._h, _dev_ptr(mu), _dev_ptr(b), mu.shape[0], int(epochs), lr, beta1,
                                     beta2, eps, weight_decay, _dev_ptr(losses)))
        return losses[:int(epochs)]

    def predict(self, mu):
        self._pairs_ok(mu)
        c = torch.empty((mu.shape[0], WARM_BANK), dtype=torch.float32, device=self.device)
        _check(lib().rpod_warm_predict(self._h, _dev_ptr(mu), mu.shape[0], _dev_ptr(c)))
        return c

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().rpod_warm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AdaptivePlan(_PlanBase):
    """Adaptive-rank plan (rpod_plan_create_adaptive / rpod_compute_adaptive):
    the sketch grows by `block` columns, up to l_max, until the captured
    energy ||Q^T S||_F^2 / ||S||_F^2 reaches delta."""

    def __init__(self, m, n, l_max, block, q, delta, dtype=torch.float32, ld=None, device="cuda", stream=None):
        self.device = _norm_device(device)
        self.m, self.n, self.l_max, self.block, self.q = int(m), int(n), int(l_max), int(block), int(q)
        self.delta = float(delta)
        self.ld = self.m if ld is None else int(ld)
        self.dtype = dtype
        self.out_dtype = torch.float64 if dtype == torch.float64 else torch.float32
        self._desc = make_desc(m, n, l_max, block, q, dtype, ld)
        nbytes = ctypes.c_size_t(0)
        _check(lib().rpod_workspace_size_adaptive(ctypes.byref(self._desc), self.delta, ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        sptr, self.stream = _stream_ptr(stream, self.device)
        h = ctypes.c_void_p()
        _check(lib().rpod_plan_create_adaptive(ctypes.byref(h), ctypes.byref(self._desc), self.delta,
                                               _dev_ptr(self.workspace), nbytes.value, sptr))
        self._h = h

    def compute(self, St, seed, out=None, check=True, info=True):
        """-> (Phi_t (l, m), sigma (l,), A_t (n, l), l, rank, residual); l is the sketch
        width used, rank the energy rank (-1 if l_max fell short), residual
        ||S - Q B||_F^2 / ||S||_F^2. With info=False the call only enqueues and
        returns the full buffers (l_max modes, of which the first l are valid)
        with l, rank, residual None."""
        _check_St(St, self.dtype, self.device, self.m, self.n, self.ld)
        if out is None:
            out = (torch.empty((self.l_max, self.m), dtype=self.out_dtype, device=self.device),
                   torch.empty((self.l_max,), dtype=torch.float64, device=self.device),
                   torch.empty((self.n * self.l_max,), dtype=self.out_dtype, device=self.device))
        Phi, sigma, A = out
        lu, rk, res = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0)
        _check(lib().rpod_compute_adaptive(self._h, _dev_ptr(St), ctypes.c_uint64(int(seed) & (2 ** 64 - 1)),
                                           _dev_ptr(Phi), _dev_ptr(sigma), _dev_ptr(A),
                                           ctypes.byref(lu) if info else None, ctypes.byref(rk) if info else None,
                                           ctypes.byref(res) if info else None))
        if check:
            self.status()
        if not info:
            return Phi, sigma, A, None, None, None
        l = lu.value
        return Phi[:l], sigma[:l], A.view(-1)[:self.n * l].view(self.n, l), l, rk.value, res.value

    def status(self):
        fl = ctypes.c_int32(0)
        st = lib().rpod_status_query(self._h, ctypes.byref(fl))
        self.last_flags = fl.value
        _check(st)
        return fl.value


class WarmPlan(_PlanBase):
    """A warm-started plan for one matrix shape (rpod_plan_create_warm / rpod_compute_warm)."""

    def __init__(self, model, n, p, q, q_fallback=2, tol=1e-3, dtype=torch.float32, ld=None, device="cuda",
                 stream=None):
        self.model = model  # must outlive the plan
        self.device = _norm_device(device)
        self.m, self.n, self.r, self.p, self.q = model.m, int(n), model.r, int(p), int(q)
        self.ld = self.m if ld is None else int(ld)
        self.dtype = dtype
        self.out_dtype = torch.float32
        self._desc = make_desc(self.m, self.n, self.r, self.p, self.q, dtype, self.ld)
        nbytes = ctypes.c_size_t(0)
        _check(lib().rpod_workspace_size_warm(ctypes.byref(self._desc), model._h, int(q_fallback),
                                              ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        sptr, self.stream = _stream_ptr(stream, self.device)
        h = ctypes.c_void_p()
        _check(lib().rpod_plan_create_warm(ctypes.byref(h), ctypes.byref(self._desc), model._h, int(q_fallback),
                                           float(tol), _dev_ptr(self.workspace), nbytes.value, sptr))
        self._h = h

    def compute(self, St, mu, seed, out=None, check=True, decision=True):
        """-> (Phi_t (r, m), sigma (r,), A_t (n, r), fell_back, rho). With
        decision=False the call only enqueues and fell_back, rho are None."""
        _check_St(St, self.dtype, self.device, self.m, self.n, self.ld)
        if out is None:
            out = (torch.empty((self.r, self.m), dtype=torch.float32, device=self.device),
                   torch.empty((self.r,), dtype=torch.float64, device=self.device),
                   torch.empty((self.n, self.r), dtype=torch.float32, device=self.device))
        Phi, sigma, A = out
        mu_arr = (ctypes.c_float * 4)(*[float(x) for x in mu])
        fb = ctypes.c_int32(0)
        rho = ctypes.c_double(0)
        _check(lib().rpod_compute_warm(self._h, _dev_ptr(St), mu_arr, ctypes.c_uint64(int(seed) & (2 ** 64 - 1)),
                                       _dev_ptr(Phi), _dev_ptr(sigma), _dev_ptr(A),
                                       ctypes.byref(fb) if decision else None,
                                       ctypes.byref(rho) if decision else None))
        if check:
            self.status()
        if not decision:
            return Phi, sigma, A, None, None
        return Phi, sigma, A, bool(fb.value), rho.value

    def residuals(self):
        """rho_k of the last call's warm result (numpy, r values)."""
        buf = (ctypes.c_double * self.r)()
        _check(lib().rpod_warm_residuals(self._h, buf))
        return np.array(buf[:], dtype=np.float64)

    def status(self):
        fl = ctypes.c_int32(0)
        st = lib().rpod_status_query(self._h, ctypes.byref(fl))
        self.last_flags = fl.value
        _check(st)
        return fl.value


def rpod(St, r, p, q, seed, stream=None):
    """One-shot rPOD of St (n, m), a column-major m x n snapshot matrix."""
    n, m = St.shape
    plan = Plan(m, n, r, p, q, dtype=St.dtype, ld=St.stride(0), device=St.device, stream=stream)
    out = plan.compute(St, seed)
    plan.close()
    return out


def generate_omega(seed, n, l, dtype=torch.float64, device="cuda", stream=None):
    """The n x l Gaussian sketch as an (l, n) tensor (column-major n x l)."""
    out = torch.empty((l, n), dtype=dtype, device=device)
    sptr, s = _stream_ptr(stream, torch.device(device))
    _check(lib().rpod_generate_omega(ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), n, l, _DTYPES[dtype],
                                     _dev_ptr(out), n, sptr))
    s.synchronize()
    return out


def sketch_bits(seed, n, l, device="cuda", stream=None):
    """Raw Philox words as an int32 tensor of shape (n, ceil(l/2), 4) (bit pattern of uint32)."""
    out = torch.empty((n, (l + 1) // 2, 4), dtype=torch.int32, device=device)
    sptr, s = _stream_ptr(stream, torch.device(device))
    _check(lib().rpod_sketch_bits(ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), n, l, _dev_ptr(out), sptr))
    s.synchronize()
    return out
