"""Python binding of libccham (ctypes): argument marshalling only.

Every step of the Hamiltonian build and the Davidson solve runs in the HIP
kernels of libccham.so (built by `build.py` for gfx950). There is no CPU
fallback: importing this package without the built library raises.

The functions mirror include/ccham.h; `Context` wraps one cch_ctx.
Arrays may be NumPy arrays (host) or torch CUDA tensors (device); device
tensors are passed with CCH_MEM_DEVICE.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccham.so")

CCH_OK = 0
CCH_E_INVALID_ARG = -1
CCH_E_STATE = -2
CCH_E_INPUT = -3
CCH_E_LIMIT = -4
CCH_E_OOM = -5
CCH_E_HIP = -6
CCH_E_NOT_CONVERGED = -7
CCH_MEM_HOST = 0
CCH_MEM_DEVICE = 1
CCH_DAV_RESIDUALS = 2
CCH_DAV_SPARSE_L2 = 4
CCH_RESTART_AUTO, CCH_RESTART_THICK, CCH_RESTART_PREV = 0, 1, 2
CCH_LOWER = 8
CCH_PLAN_SPARSE_L2 = 1
CCH_PREC_FP64 = 0
CCH_PREC_FP32 = 1
CCH_PREC_SPLIT_BF16 = 2
CCH_PRECOND_JACOBI = 0
CCH_PRECOND_MLP = 1
CCH_EIG_AUTO = 0
CCH_EIG_JACOBI = 1
CCH_PAIRS_TARGET = 0
CCH_PAIRS_L2 = 1
CCH_PAIRS_L2_TARGET = 2

EXPORTS = [
    "cch_version", "cch_probe_fp64", "cch_create", "cch_destroy", "cch_last_error", "cch_sync", "cch_set_orbitals",
    "cch_set_integrals", "cch_add_target_symmetry", "cch_add_target_symmetry_spin", "cch_add_target_symmetry_csf", "cch_set_l2", "cch_set_l2_csf", "cch_set_target_energies", "cch_plan", "cch_build",
    "cch_get_dim", "cch_get_matrix", "cch_matrix_device", "cch_get_diagonal", "cch_get_elements", "cch_get_block", "cch_block_shape", "cch_get_labels",
    "cch_davidson", "cch_build_time", "cch_work_counts", "cch_batch_create", "cch_batch_build",
    "cch_batch_time", "cch_batch_info", "cch_batch_destroy", "cch_batch_last_error",
    "cch_mlp_num_params", "cch_mlp_create", "cch_mlp_destroy", "cch_mlp_last_error", "cch_mlp_set_weights",
    "cch_mlp_get_weights", "cch_mlp_forward", "cch_mlp_grad", "cch_mlp_train_step", "cch_mlp_features",
    "cch_davidson_set_mlp", "cch_subspace_eig", "cch_plan_info", "cch_subspace_eig_noalloc",
    "cch_work_detail", "cch_target_hamiltonian", "cch_eig_all", "cch_set_integrals_packed", "cch_apply",
]
CCH_BATCH_AUTOTUNE = 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run paper_1709_03005_amd/build.py (hipcc, gfx950)")
# torch ships its own HIP runtime (soname libamdhip64.so.7, loaded by the
# unversioned name). Loading torch first lets this library bind to that same
# runtime; loading it first would put two HIP/HSA runtimes in one process,
# after which the second one to initialise finds no device.
import torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)


class PlanOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("split_slices", C.c_int32), ("autotune", C.c_int32),
                ("flags", C.c_int32), ("max_device_bytes", C.c_int64)]


class DavOpts(C.Structure):
    _fields_ = [("k", C.c_int32), ("max_iter", C.c_int32), ("max_subspace", C.c_int32),
                ("precond", C.c_int32), ("tol", C.c_double), ("block", C.c_int32), ("restart", C.c_int32)]


class EigInfo(C.Structure):
    _fields_ = [("tridiag_ms", C.c_double), ("eigenvalues_ms", C.c_double), ("vectors_ms", C.c_double),
                ("clusters", C.c_int32), ("clustered", C.c_int32), ("tridiag_bytes", C.c_double),
                ("backtransform_flops", C.c_double)]


class DavInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("matvecs", C.c_int32), ("converged", C.c_int32),
                ("fallbacks", C.c_int32), ("max_residual", C.c_double), ("seconds", C.c_double),
                ("matvec_ms", C.c_double), ("matvec_launches", C.c_int32), ("rr_fallbacks", C.c_int32),
                ("rr_ms", C.c_double), ("rr_flops", C.c_double), ("rr_calls", C.c_int32), ("dropped", C.c_int32),
                ("restarts", C.c_int32), ("prev_kept", C.c_int32)]


P = C.c_void_p
i32, i64 = C.c_int32, C.c_int64
_SIG = {
    "cch_version": (C.c_char_p, []),
    "cch_probe_fp64": (i32, [i32, P, P]),
    "cch_create": (i32, [C.POINTER(P), i32, P]),
    "cch_destroy": (i32, [P]),
    "cch_last_error": (C.c_char_p, [P]),
    "cch_sync": (i32, [P]),
    "cch_set_orbitals": (i32, [P, i32, P, i32, P, i32]),
    "cch_set_integrals": (i32, [P, P, P, P, P, P, C.c_double, i32]),
    "cch_set_integrals_packed": (i32, [P, P, P, P, P, P, C.c_double, i32]),
    "cch_add_target_symmetry": (i32, [P, i32, i32, i32, P, i32, P, i32, C.POINTER(i32)]),
    "cch_add_target_symmetry_spin": (i32, [P, i32, i32, i32, P, P, i32, P, i32, C.POINTER(i32)]),
    "cch_add_target_symmetry_csf": (i32, [P, i32, i32, P, i32, P, P, i32, P, i32, P]),
    "cch_set_l2": (i32, [P, i32, i32, P, i32]),
    "cch_set_l2_csf": (i32, [P, i32, P, i32, P, P, i32]),
    "cch_set_target_energies": (i32, [P, P, i64, i32]),
    "cch_plan": (i32, [P, C.POINTER(PlanOpts)]),
    "cch_build": (i32, [P]),
    "cch_get_dim": (i32, [P, C.POINTER(i64), C.POINTER(i64)]),
    "cch_get_matrix": (i32, [P, P, i64, i32]),
    "cch_matrix_device": (i32, [P, C.POINTER(P), C.POINTER(i64)]),
    "cch_get_diagonal": (i32, [P, P, i32]),
    "cch_apply": (i32, [P, P, i64, i32, P, i64, i32]),
    "cch_get_block": (i32, [P, i32, i32, i32, P, i64, i32]),
    "cch_get_elements": (i32, [P, i64, P, P, P, i32]),
    "cch_block_shape": (i32, [P, i32, i32, i32, C.POINTER(i64), C.POINTER(i64)]),
    "cch_get_labels": (i32, [P, i32, i32, i32, P, P, P, P, P, i64, C.POINTER(i64)]),
    "cch_davidson": (i32, [P, C.POINTER(DavOpts), P, P, C.POINTER(DavInfo), i32]),
    "cch_build_time": (i32, [P, C.POINTER(C.c_float), P]),
    "cch_work_counts": (i32, [P, P]),
    "cch_work_detail": (i32, [P, P, i32]),
    "cch_target_hamiltonian": (i32, [P, i32, i32, P, i64, i32]),
    "cch_eig_all": (i32, [P, P, i64, i32, P, P, i64, i32, C.POINTER(EigInfo)]),
    "cch_batch_create": (i32, [C.POINTER(P), P, i32, i32]),
    "cch_batch_build": (i32, [P]),
    "cch_batch_time": (i32, [P, C.POINTER(C.c_float)]),
    "cch_batch_info": (i32, [P, P]),
    "cch_batch_destroy": (i32, [P]),
    "cch_batch_last_error": (C.c_char_p, [P]),
    "cch_mlp_num_params": (i32, []),
    "cch_mlp_create": (i32, [C.POINTER(P), i32, P, C.c_uint64]),
    "cch_mlp_destroy": (i32, [P]),
    "cch_mlp_last_error": (C.c_char_p, [P]),
    "cch_mlp_set_weights": (i32, [P, P, i64, i32]),
    "cch_mlp_get_weights": (i32, [P, P, i64, i32]),
    "cch_mlp_forward": (i32, [P, P, i64, P, i32]),
    "cch_mlp_grad": (i32, [P, P, P, P, P, i64, C.POINTER(C.c_double), P, i32]),
    "cch_mlp_train_step": (i32, [P, P, P, P, P, i64, C.c_float, C.POINTER(C.c_double), i32]),
    "cch_mlp_features": (i32, [P, C.c_double, P, i32]),
    "cch_davidson_set_mlp": (i32, [P, P]),
    "cch_subspace_eig": (i32, [P, P, i32, i32, P, P, i32, i32, C.POINTER(i32), i32]),
    "cch_subspace_eig_noalloc": (i32, [P, P, i32, i32, P, P, i32, i32, C.POINTER(i32), i32]),
    "cch_plan_info": (i32, [P, C.POINTER(i64), C.POINTER(i32)]),
}
for _n, (_r, _a) in _SIG.items():
    _f = getattr(lib, _n)
    _f.restype = _r
    _f.argtypes = _a


class CchError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ccham error {code}: {msg}")
        self.code = code


def probe_fp64(device=0, stream=None):
    """cch_probe_fp64: measured FP64 rates (TFLOP/s) of the 16x16x4 MFMA, the
    four-block 4x4x4 MFMA and the vector FMA on `device`."""
    r = np.zeros(3)
    rc = lib.cch_probe_fp64(device, stream, r.ctypes.data_as(C.c_void_p))
    if rc != CCH_OK:
        raise CchError(rc, "cch_probe_fp64 failed")
    return {"mfma_16x16x4": float(r[0]), "mfma_4x4x4": float(r[1]), "fma": float(r[2])}


def version() -> str:
    return lib.cch_version().decode()


def _arr(a, dtype):
    """(pointer, flags, keepalive) for a NumPy array or a torch tensor."""
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        if a.is_cuda:
            t = a.contiguous()
            return C.c_void_p(t.data_ptr()), CCH_MEM_DEVICE, t
        a = a.numpy()
    x = np.ascontiguousarray(a, dtype=dtype)
    return x.ctypes.data_as(C.c_void_p), CCH_MEM_HOST, x


class Context:
    """One cch_ctx on `device`, ordering its work on `stream` (a HIP stream
    handle as an int, e.g. torch.cuda.current_stream().cuda_stream)."""

    def __init__(self, device: int = 0, stream: int | None = None):
        h = C.c_void_p()
        rc = lib.cch_create(C.byref(h), device, C.c_void_p(stream or 0))
        if rc != CCH_OK:
            raise CchError(rc, lib.cch_last_error(None).decode())
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            lib.cch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _ck(self, rc, ok=(CCH_OK,)):
        if rc not in ok:
            raise CchError(rc, lib.cch_last_error(self.h).decode())
        return rc

    def last_error(self) -> str:
        return lib.cch_last_error(self.h).decode()

    def sync(self):
        self._ck(lib.cch_sync(self.h))

    def set_orbitals(self, n_o, tgt_irrep, n_irrep, n_c_per_irrep, total_irrep=0):
        p1, _, k1 = _arr(tgt_irrep, np.uint8)
        p2, _, k2 = _arr(n_c_per_irrep, np.int32)
        self._ck(lib.cch_set_orbitals(self.h, int(n_o), p1, int(n_irrep), p2, int(total_irrep)))

    def set_integrals(self, h, tttt, tttc, ttcc, tctc, e_core=0.0):
        ps = [_arr(x, np.float64) for x in (h, tttt, tttc, ttcc, tctc)]
        flags = ps[0][1]
        self._ck(lib.cch_set_integrals(self.h, *[p[0] for p in ps], float(e_core), flags))

    def set_integrals_packed(self, h, tttt, tttc, ttcc, tctc, e_core=0.0):
        """cch_set_integrals_packed: (tt|cc) and (tc|tc) in the symmetry-packed layout."""
        ps = [_arr(x, np.float64) for x in (h, tttt, tttc, ttcc, tctc)]
        flags = ps[0][1]
        self._ck(lib.cch_set_integrals_packed(self.h, *[p[0] for p in ps], float(e_core), flags))

    def add_target_symmetry(self, irrep, dets, ci, cont_spin=None) -> int:
        """cch_add_target_symmetry, or cch_add_target_symmetry_spin when
        cont_spin (0 alpha / 1 beta per determinant) is given."""
        pd, fd, kd = _arr(dets, np.uint64)
        pc, fc, kc = _arr(ci, np.float64)
        n_det, n_words = kd.shape
        if kc.ndim != 2 or kc.shape[0] != n_det:
            # the library reads n_det rows of ci: refuse a shorter array here
            raise CchError(CCH_E_INVALID_ARG, f"ci has shape {tuple(kc.shape)}, expected ({n_det}, n_states)")
        sid = i32()
        if cont_spin is None:
            self._ck(lib.cch_add_target_symmetry(self.h, int(irrep), int(n_det), int(n_words), pd,
                                                 int(kc.shape[1]), pc, fd, C.byref(sid)))
        else:
            sp = np.ascontiguousarray(cont_spin, dtype=np.int8)
            if sp.shape != (n_det,):
                raise CchError(CCH_E_INVALID_ARG, f"cont_spin has shape {sp.shape}, expected ({n_det},)")
            if fd != CCH_MEM_HOST:
                raise CchError(CCH_E_INVALID_ARG, "continuum spins are passed with host determinants")
            self._ck(lib.cch_add_target_symmetry_spin(self.h, int(irrep), int(n_det), int(n_words), pd,
                                                      sp.ctypes.data_as(C.c_void_p), int(kc.shape[1]), pc, fd,
                                                      C.byref(sid)))
        self._ndet = getattr(self, "_ndet", []) + [int(n_det)]
        return sid.value

    def add_target_symmetry_csf(self, irrep, csf_start, dets, coef, ci) -> int:
        """cch_add_target_symmetry_csf: CSF m = sum of coef[t] |dets[t]> over
        t in [csf_start[m], csf_start[m + 1]); ci[n_csf][n_states]."""
        def host(a, dt):   # a set-up call: every list is read from host memory
            if hasattr(a, "detach"):
                a = a.detach().cpu().numpy()
            return np.ascontiguousarray(a, dtype=dt)
        st = host(csf_start, np.int32)
        kd, kk, kc = host(dets, np.uint64), host(coef, np.float64), host(ci, np.float64)
        if kd.ndim != 2:
            raise CchError(CCH_E_INVALID_ARG, "dets must be [n_terms][n_words]")
        pd, pk, pc = (x.ctypes.data_as(C.c_void_p) for x in (kd, kk, kc))
        fd = CCH_MEM_HOST
        n_csf = st.size - 1
        n_terms, n_words = kd.shape
        if n_csf <= 0 or st[-1] != n_terms or kk.shape[0] != n_terms or kc.ndim != 2 or kc.shape[0] != n_csf:
            raise CchError(CCH_E_INVALID_ARG, "inconsistent CSF arrays")
        sid = i32()
        self._ck(lib.cch_add_target_symmetry_csf(self.h, int(irrep), int(n_csf), st.ctypes.data_as(C.c_void_p),
                                                 int(n_words), pd, pk, int(kc.shape[1]), pc, fd, C.byref(sid)))
        # the library keeps the distinct determinants of the terms
        self._ndet = getattr(self, "_ndet", []) + [int(np.unique(kd, axis=0).shape[0])]
        return sid.value

    def set_l2(self, dets):
        pd, fd, kd = _arr(dets, np.uint64)
        n = kd.shape[0]
        w = kd.shape[1] if kd.ndim == 2 else 0
        self._ck(lib.cch_set_l2(self.h, int(n), int(w), pd, fd))

    def set_l2_csf(self, csf_start, dets, coef):
        """cch_set_l2_csf: L2 function l = sum over terms t in
        [csf_start[l], csf_start[l+1]) of coef[t] |dets[t]>."""
        st = np.ascontiguousarray(csf_start, dtype=np.int32)
        d = np.ascontiguousarray(dets, dtype=np.uint64)
        cf = np.ascontiguousarray(coef, dtype=np.float64)
        if d.ndim != 2 or d.shape[0] != cf.size or st.size < 2:
            raise CchError(CCH_E_INVALID_ARG, "CSF terms and coefficients differ in count")
        self._ck(lib.cch_set_l2_csf(self.h, int(st.size - 1), st.ctypes.data_as(C.c_void_p), int(d.shape[1]),
                                    d.ctypes.data_as(C.c_void_p), cf.ctypes.data_as(C.c_void_p), CCH_MEM_HOST))

    def set_target_energies(self, energies):
        """Target energies on the diagonal (one array per target symmetry, or
        one flat array over all states); None switches the option off."""
        if energies is None:
            self._ck(lib.cch_set_target_energies(self.h, None, 0, 0))
            return
        if isinstance(energies, (list, tuple)):
            energies = np.concatenate([np.ravel(np.asarray(e, dtype=np.float64)) for e in energies]) \
                if len(energies) else np.zeros(0)
        pe, fe, ke = _arr(energies, np.float64)
        n = int(ke.numel()) if hasattr(ke, "numel") else int(ke.size)
        if n == 0:
            raise CchError(CCH_E_INVALID_ARG, "empty energy list (pass None to switch the option off)")
        self._ck(lib.cch_set_target_energies(self.h, pe, n, fe))

    def plan(self, precision=CCH_PREC_FP64, split_slices=0, autotune=0, max_device_bytes=0, sparse_l2=False):
        """cch_plan; sparse_l2=True: classes 2 and 8 built and stored as CSR."""
        o = PlanOpts(precision, split_slices, autotune, CCH_PLAN_SPARSE_L2 if sparse_l2 else 0, max_device_bytes)
        self._ck(lib.cch_plan(self.h, C.byref(o)))

    def build(self):
        self._ck(lib.cch_build(self.h))

    def dim(self):
        D, Dc = i64(), i64()
        self._ck(lib.cch_get_dim(self.h, C.byref(D), C.byref(Dc)))
        return D.value, Dc.value

    def get_matrix(self, out=None, lower=False):
        """The matrix (D x D); with lower=True only the lower triangle is
        guaranteed (the rest of a new array is zero)."""
        D, _ = self.dim()
        if out is None:
            out = np.zeros((D, D)) if lower else np.empty((D, D))
        p, f, k = _arr(out, np.float64)
        self._ck(lib.cch_get_matrix(self.h, p, D, f | (CCH_LOWER if lower else 0)))
        return out

    def matrix_device(self):
        p, ld = C.c_void_p(), i64()
        self._ck(lib.cch_matrix_device(self.h, C.byref(p), C.byref(ld)))
        return p.value, ld.value

    def get_diagonal(self):
        D, _ = self.dim()
        out = np.empty(D)
        self._ck(lib.cch_get_diagonal(self.h, out.ctypes.data_as(C.c_void_p), CCH_MEM_HOST))
        return out

    def apply(self, V):
        """cch_apply: H V for the rows of V (b x D, host), as a b x D array."""
        D, _ = self.dim()
        V = np.ascontiguousarray(np.atleast_2d(V), dtype=np.float64)
        if V.shape[1] != D:
            raise CchError(CCH_E_INVALID_ARG, f"vectors of length {V.shape[1]}, D = {D}")
        W = np.zeros_like(V)
        self._ck(lib.cch_apply(self.h, V.ctypes.data_as(C.c_void_p), D, V.shape[0], W.ctypes.data_as(C.c_void_p),
                               D, CCH_MEM_HOST))
        return W

    def get_elements(self, rows, cols):
        """cch_get_elements: H[rows[i]][cols[i]] without copying the matrix."""
        r = np.ascontiguousarray(rows, dtype=np.int64)
        c = np.ascontiguousarray(cols, dtype=np.int64)
        if r.shape != c.shape:
            raise CchError(CCH_E_INVALID_ARG, "rows and cols differ in shape")
        out = np.zeros(r.size)
        self._ck(lib.cch_get_elements(self.h, int(r.size), r.ctypes.data_as(C.c_void_p),
                                      c.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p), CCH_MEM_HOST))
        return out.reshape(r.shape)

    def get_block(self, cls, sym_a=0, sym_b=0):
        """cch_get_block: one class block (elements outside the class are 0)."""
        r, c = i64(), i64()
        self._ck(lib.cch_block_shape(self.h, cls, sym_a, sym_b, C.byref(r), C.byref(c)))
        out = np.zeros((r.value, c.value))
        if out.size:
            self._ck(lib.cch_get_block(self.h, cls, sym_a, sym_b, out.ctypes.data_as(C.c_void_p), max(c.value, 1),
                                       CCH_MEM_HOST))
        return out

    def get_labels(self, which, sym_a=0, sym_b=0):
        n = i64()
        self._ck(lib.cch_get_labels(self.h, which, sym_a, sym_b, None, None, None, None, None, 0,
                                    C.byref(n)))
        cap = n.value
        x = np.zeros(cap, np.int32); y = np.zeros(cap, np.int32)
        d = np.zeros(cap, np.int8); lab = np.zeros(cap, np.uint64); ph = np.zeros(cap, np.int8)
        ptr = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
        self._ck(lib.cch_get_labels(self.h, which, sym_a, sym_b, ptr(x), ptr(y), ptr(d), ptr(lab),
                                    ptr(ph), cap, C.byref(n)))
        return dict(x=x, y=y, deg=d, label=lab, phase=ph)

    def davidson(self, k, tol=1e-8, max_iter=200, max_subspace=0, precond=CCH_PRECOND_JACOBI,
                 want_vectors=True, residuals=False, block=0, sparse_l2=False, restart=CCH_RESTART_AUTO):
        """(eigenvalues, vectors or None, info, status); with residuals=True the
        vectors array has 2k rows, residuals H x - theta x after the vectors."""
        D, _ = self.dim()
        ev = np.zeros(k)
        vec = np.zeros((2 * k if residuals else k, D)) if (want_vectors or residuals) else None
        info = DavInfo()
        o = DavOpts(k, max_iter, max_subspace, precond, tol, block, restart)
        rc = lib.cch_davidson(self.h, C.byref(o), ev.ctypes.data_as(C.c_void_p),
                              vec.ctypes.data_as(C.c_void_p) if vec is not None else None,
                              C.byref(info), CCH_MEM_HOST | (CCH_DAV_RESIDUALS if residuals else 0)
                              | (CCH_DAV_SPARSE_L2 if sparse_l2 else 0))
        self._ck(rc, ok=(CCH_OK, CCH_E_NOT_CONVERGED))
        return ev, vec, info, rc

    def work_counts(self):
        out = np.zeros(8)
        self._ck(lib.cch_work_counts(self.h, out.ctypes.data_as(C.c_void_p)))
        keys = ["lower_elements", "gemm_flops", "target_pairs", "l2_target_pairs", "relayout_bytes",
                "class4_outputs", "l2_lower_elements", "sym_pairs"]
        return dict(zip(keys, out.tolist()))

    def eig_all(self, A=None, vectors=True, device=False):
        """cch_eig_all: (eigenvalues ascending, eigenvectors as rows or None,
        EigInfo) of a host matrix A, or of the built matrix when A is None.
        With device=True the results are float64 torch tensors on the
        context's GPU (A, if given, is then such a tensor too)."""
        if device:
            import torch
            dev = torch.device("cuda", self.device)
            if A is None:
                n, _ = self.dim()
                pa, lda = None, 0
            else:
                A = A.to(device=dev, dtype=torch.float64).contiguous()
                n = A.shape[0]
                pa, lda = C.c_void_p(A.data_ptr()), A.shape[1]
            w = torch.zeros(n, dtype=torch.float64, device=dev)
            V = torch.zeros((n, n), dtype=torch.float64, device=dev) if vectors else None
            torch.cuda.synchronize(dev)
            info = EigInfo()
            self._ck(lib.cch_eig_all(self.h, pa, lda, n if A is not None else 0, C.c_void_p(w.data_ptr()),
                                     C.c_void_p(V.data_ptr()) if vectors else None, n, CCH_MEM_DEVICE,
                                     C.byref(info)))
            return w, V, info
        if A is None:
            n, _ = self.dim()
            pa, lda = None, 0
        else:
            A = np.ascontiguousarray(A, dtype=np.float64)
            n = A.shape[0]
            pa, lda = A.ctypes.data_as(C.c_void_p), A.shape[1]
        w = np.zeros(n)
        V = np.zeros((n, n)) if vectors else None
        info = EigInfo()
        self._ck(lib.cch_eig_all(self.h, pa, lda, n if A is not None else 0, w.ctypes.data_as(C.c_void_p),
                                 V.ctypes.data_as(C.c_void_p) if vectors else None, n, CCH_MEM_HOST,
                                 C.byref(info)))
        return w, V, info

    def target_hamiltonian(self, sym_a, sym_b):
        """cch_target_hamiltonian: <D_ax|H|D_by> over target determinants."""
        ma = self._ndet[sym_a]
        mb = self._ndet[sym_b]
        out = np.zeros((ma, mb))
        self._ck(lib.cch_target_hamiltonian(self.h, sym_a, sym_b, out.ctypes.data_as(C.c_void_p), max(mb, 1),
                                            CCH_MEM_HOST))
        return out

    def work_detail(self):
        """cch_work_detail: the work counts plus the per-kernel algorithmic work
        of the last build."""
        out = np.zeros(16)
        self._ck(lib.cch_work_detail(self.h, out.ctypes.data_as(C.c_void_p), 16))
        keys = ["lower_elements", "gemm_flops", "target_pairs", "l2_target_pairs", "relayout_bytes",
                "class4_outputs", "l2_lower_elements", "sym_pairs", "density_pairs", "density_flops",
                "class4_flops", "l2_pairs", "mirror_bytes"]
        return dict(zip(keys, out.tolist()))

    def plan_info(self):
        """(device bytes held, expansion passes)."""
        b = C.c_int64()
        n = C.c_int32()
        self._ck(lib.cch_plan_info(self.h, C.byref(b), C.byref(n)))
        return b.value, n.value

    def subspace_eig(self, G, method=CCH_EIG_AUTO):
        """(theta ascending, Y with eigenvectors in columns, fell_back) for a
        small symmetric host matrix G (m <= 96), solved on the device."""
        G = np.ascontiguousarray(G, dtype=np.float64)
        m = G.shape[0]
        theta = np.zeros(m)
        Y = np.zeros((m, m))
        fb = C.c_int32()
        self._ck(lib.cch_subspace_eig(self.h, G.ctypes.data_as(C.c_void_p), G.shape[1], m,
                                      theta.ctypes.data_as(C.c_void_p), Y.ctypes.data_as(C.c_void_p), m, method,
                                      C.byref(fb), CCH_MEM_HOST))
        return theta, Y, bool(fb.value)

    def subspace_eig_noalloc(self, G, method=CCH_EIG_AUTO):
        """cch_subspace_eig_noalloc: as subspace_eig, with no device allocation."""
        G = np.ascontiguousarray(G, dtype=np.float64)
        m = G.shape[0]
        theta = np.zeros(m)
        Y = np.zeros((m, m))
        fb = C.c_int32()
        self._ck(lib.cch_subspace_eig_noalloc(self.h, G.ctypes.data_as(C.c_void_p), G.shape[1], m,
                                              theta.ctypes.data_as(C.c_void_p), Y.ctypes.data_as(C.c_void_p), m,
                                              method, C.byref(fb), CCH_MEM_HOST))
        return theta, Y, bool(fb.value)

    def mlp_features(self, theta):
        D, _ = self.dim()
        X = np.zeros((D, 4), np.float32)
        self._ck(lib.cch_mlp_features(self.h, float(theta), X.ctypes.data_as(C.c_void_p), CCH_MEM_HOST))
        return X

    def set_mlp(self, mlp):
        self._ck(lib.cch_davidson_set_mlp(self.h, mlp.h if mlp is not None else None))
        self._mlp = mlp

    def build_time(self):
        t = C.c_float()
        ph = (C.c_float * 8)()
        self._ck(lib.cch_build_time(self.h, C.byref(t), C.cast(ph, C.c_void_p)))
        return t.value, list(ph)


class Mlp:
    """cch_mlp: the learned Davidson preconditioner's network."""

    def __init__(self, device=0, stream=None, seed=0):
        h = C.c_void_p()
        rc = lib.cch_mlp_create(C.byref(h), device, C.c_void_p(stream or 0), seed)
        if rc != CCH_OK:
            raise CchError(rc, lib.cch_mlp_last_error(None).decode())
        self.h = h
        self.n_params = lib.cch_mlp_num_params()

    def _ck(self, rc):
        if rc != CCH_OK:
            raise CchError(rc, lib.cch_mlp_last_error(self.h).decode())

    def weights(self):
        w = np.zeros(self.n_params, np.float32)
        self._ck(lib.cch_mlp_get_weights(self.h, w.ctypes.data_as(C.c_void_p), self.n_params, CCH_MEM_HOST))
        return w

    def set_weights(self, w):
        p, f, k = _arr(w, np.float32)
        self._ck(lib.cch_mlp_set_weights(self.h, p, int(k.size if hasattr(k, "size") else k.numel()), f))

    def forward(self, X):
        p, f, k = _arr(X, np.float32)
        n = k.shape[0]
        if f == CCH_MEM_DEVICE:
            import torch
            g = torch.empty(n, dtype=torch.float32, device=k.device)
            self._ck(lib.cch_mlp_forward(self.h, p, n, C.c_void_p(g.data_ptr()), f))
            return g
        g = np.zeros(n, np.float32)
        self._ck(lib.cch_mlp_forward(self.h, p, n, g.ctypes.data_as(C.c_void_p), f))
        return g

    def grad(self, X, tj, e, w):
        args = [_arr(a, np.float32) for a in (X, tj, e, w)]
        f = args[0][1]
        n = args[0][2].shape[0]
        loss = C.c_double()
        g = np.zeros(self.n_params, np.float32)
        if f == CCH_MEM_DEVICE:
            import torch
            gd = torch.empty(self.n_params, dtype=torch.float32, device=args[0][2].device)
            self._ck(lib.cch_mlp_grad(self.h, *[a[0] for a in args], n, C.byref(loss),
                                      C.c_void_p(gd.data_ptr()), f))
            return loss.value, gd.cpu().numpy()
        self._ck(lib.cch_mlp_grad(self.h, *[a[0] for a in args], n, C.byref(loss),
                                  g.ctypes.data_as(C.c_void_p), f))
        return loss.value, g

    def train_step(self, X, tj, e, w, lr=1e-3):
        args = [_arr(a, np.float32) for a in (X, tj, e, w)]
        loss = C.c_double()
        self._ck(lib.cch_mlp_train_step(self.h, *[a[0] for a in args], args[0][2].shape[0], float(lr),
                                        C.byref(loss), args[0][1]))
        return loss.value

    def close(self):
        if getattr(self, "h", None):
            lib.cch_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """cch_batch over planned contexts (kept alive by this object)."""

    def __init__(self, contexts, autotune=True):
        self.contexts = list(contexts)
        arr = (C.c_void_p * len(self.contexts))(*[c.h.value for c in self.contexts])
        h = C.c_void_p()
        rc = lib.cch_batch_create(C.byref(h), C.cast(arr, C.c_void_p), len(self.contexts),
                                  CCH_BATCH_AUTOTUNE if autotune else 0)
        if rc != CCH_OK:
            raise CchError(rc, lib.cch_batch_last_error(None).decode())
        self.h = h

    def build(self):
        rc = lib.cch_batch_build(self.h)
        if rc != CCH_OK:
            raise CchError(rc, lib.cch_batch_last_error(self.h).decode())

    def time_ms(self) -> float:
        t = C.c_float()
        lib.cch_batch_time(self.h, C.byref(t))
        return t.value

    def info(self) -> dict:
        o = np.zeros(8, np.int32)
        lib.cch_batch_info(self.h, o.ctypes.data_as(C.c_void_p))
        keys = ["tile_rows", "grid_expand", "grid_class4", "grid_l2", "autotuned", "from_cache",
                "graph_nodes", "instances"]
        return dict(zip(keys, [int(x) for x in o]))

    def close(self):
        if getattr(self, "h", None):
            lib.cch_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_instance(inst, device=0, stream=None, plan=True, target_energies=None, **plan_kw) -> Context:
    """Context loaded with an instance object carrying the fields the
    interface takes (n_o, tgt_irrep, n_irrep, n_c, total_irrep, h, tttt,
    tttc, ttcc, tctc, e_core, syms[i].irrep/.dets/.ci, l2_dets, and for L2
    functions given as CSFs l2_csf_start and l2_coef); with
    target_energies (one array per symmetry) the option of target energies on
    the diagonal is set before the plan."""
    ctx = Context(device, stream)
    ctx.set_orbitals(inst.n_o, inst.tgt_irrep, inst.n_irrep, inst.n_c, inst.total_irrep)
    if getattr(inst, "packed", False):
        ctx.set_integrals_packed(inst.h, inst.tttt, inst.tttc, inst.ttcc, inst.tctc, inst.e_core)
    else:
        ctx.set_integrals(inst.h, inst.tttt, inst.tttc, inst.ttcc, inst.tctc, inst.e_core)
    for s in inst.syms:
        ctx.add_target_symmetry(s.irrep, s.dets, s.ci, getattr(s, "cont_spin", None))
    if getattr(inst, "l2_csf_start", None) is not None:
        ctx.set_l2_csf(inst.l2_csf_start, inst.l2_dets, inst.l2_coef)
    elif inst.l2_dets is not None and len(inst.l2_dets):
        ctx.set_l2(inst.l2_dets)
    if target_energies is not None:
        ctx.set_target_energies(target_energies)
    if plan:
        ctx.plan(**plan_kw)
    return ctx
