"""ctypes binding of libksh.so: argument marshalling only.

Every computation happens in the HIP library; this module converts torch
device tensors and numpy host arrays into the pointers and structs declared
in include/ksh.h.  Importing works without a GPU; ``load()`` raises if the
shared library has not been built.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libksh.so")

KS_FP64, KS_MIXED_FP32, KS_MIXED_BF16X3 = 0, 1, 2
KS_PRECOND_NONE, KS_PRECOND_TPA, KS_PRECOND_CNN, KS_PRECOND_CNN_TPA = 0, 1, 2, 3
KS_CNN_NPARAM = 9106
KS_OP_APPLY_H, KS_OP_PRECOND, KS_OP_LOBPCG, KS_OP_JD, KS_OP_PRECOND_CNN, KS_OP_ANGLE, KS_OP_SCF = 1, 2, 3, 4, 5, 6, 7
# status words of a LOBPCG step
KS_STATUS_WORDS = 8
KS_ST_FLAGS, KS_ST_DEAD_W, KS_ST_DEAD_P, KS_ST_DEAD_BASIS, KS_ST_DEAD_X, KS_ST_INFO = range(6)
KS_FLAG_DEFLATED, KS_FLAG_SOLVE_FAILED, KS_FLAG_NONFINITE = 1, 2, 4
KS_E_HIP, KS_E_WORKSPACE, KS_E_NUMERIC, KS_E_UNSUPPORTED = -1000, -2001, -2002, -2003

EXPORTS = (
    "ks_plan_create",
    "ks_plan_create_k",
    "ks_plan_destroy",
    "ks_workspace_size",
    "ks_apply_h",
    "ks_precond_apply",
    "ks_subspace_sin",
    "ks_gram_workspace_size",
    "ks_gram_general",
    "ks_rotate_block",
    "ks_density",
    "ks_hartree",
    "ks_lda_xc",
    "ks_scf_potential",
    "ks_mix_density",
    "hegv_reduce_solve",
    "hegv_workspace_size",
    "hegv_reduce_solve_noalloc",
    "hegv_reduce_variant",
    "sygv_reduce_variant",
    "sygv_reduce_workspace_size",
    "lobpcg_init",
    "lobpcg_step",
    "ks_jd_correction",
    "cnn_workspace_size",
    "cnn_forward",
    "cnn_backward",
    "cnn_loss",
    "cnn_adam_step",
    "cnn_make_input",
    "cnn_add_skip",
    "cnn_infer",
    "cnn_conv16_bf16",
    "ks_kernel_timer",
    "ks_kernel_timer_read",
    "ks_last_error",
)

# kernel families of ks_kernel_timer
(KF_GRAM, KF_ROTATE, KF_PASS_A, KF_PASS_B, KF_PASS_C, KF_NL_PROJECT, KF_HEGV, KF_ZGEMM, KF_GRAM_BASIS,
 KF_NL_SCATTER) = range(10)


class KsGrid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("L", C.c_double * 3)]


class KsProjset(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32),
        ("n_proj", C.c_int32),
        ("n_supp", C.c_int64),
        ("atom_supp_ptr", C.POINTER(C.c_int32)),
        ("supp_idx", C.POINTER(C.c_int32)),
        ("atom_proj_ptr", C.POINTER(C.c_int32)),
        ("beta_ptr", C.POINTER(C.c_int64)),
        ("beta", C.POINTER(C.c_double)),
        ("D", C.POINTER(C.c_double)),
    ]


class KsLobpcgState(C.Structure):
    _fields_ = [
        ("nb", C.c_int32),
        ("has_p", C.c_int32),
        ("ld", C.c_int64),
        ("X", C.c_void_p),
        ("AX", C.c_void_p),
        ("W", C.c_void_p),
        ("AW", C.c_void_p),
        ("P", C.c_void_p),
        ("AP", C.c_void_p),
        ("Xn", C.c_void_p),
        ("Pn", C.c_void_p),
        ("T1", C.c_void_p),
        ("theta", C.c_void_p),
        ("res", C.c_void_p),
        ("status", C.c_void_p),
        ("host_summary", C.c_void_p),
        ("iter", C.c_int32),
        ("p_gram_ok", C.c_int32),
        ("p_gram", C.c_void_p),
    ]


class KsLobpcgOpts(C.Structure):
    _fields_ = [("precond", C.c_int32), ("pad_", C.c_int32), ("lock_tol", C.c_double), ("cnn_params", C.c_void_p)]


class KsError(RuntimeError):
    pass


_lib = None
# Plans alive in this process; destroyed by an exit hook while the HIP
# runtime is still up (a plan's tables must not be freed from a finaliser
# that runs during interpreter or runtime teardown).
_live_plans = weakref.WeakSet()
_exiting = False


def _destroy_live_plans():
    global _exiting
    for plan in list(_live_plans):
        plan.destroy()
    _exiting = True


atexit.register(_destroy_live_plans)


def load() -> C.CDLL:
    """Load libksh.so and declare its signatures; raises when not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise KsError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    lib.ks_plan_create.argtypes = [C.POINTER(vp), C.POINTER(KsGrid), C.POINTER(KsProjset), i32, i32, vp]
    lib.ks_plan_create_k.argtypes = [C.POINTER(vp), C.POINTER(KsGrid), C.POINTER(C.c_double), C.POINTER(KsProjset),
                                     C.POINTER(C.c_double), i32, i32, vp]
    lib.ks_plan_destroy.argtypes = [vp]
    lib.ks_workspace_size.argtypes = [vp, i32, i32, C.POINTER(sz)]
    lib.ks_apply_h.argtypes = [vp, vp, vp, i64, vp, i64, i32, vp, sz, vp]
    lib.ks_precond_apply.argtypes = [vp, C.POINTER(KsLobpcgOpts), vp, vp, vp, vp, i64, i32, vp, vp, vp, sz, vp]
    lib.ks_subspace_sin.argtypes = [vp, vp, vp, i64, i32, vp, vp, sz, vp]
    lib.ks_gram_workspace_size.argtypes = [i64, i32, C.POINTER(sz)]
    lib.ks_density.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    lib.ks_hartree.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.ks_lda_xc.argtypes = [vp, vp, vp, vp, vp]
    lib.ks_scf_potential.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    lib.ks_mix_density.argtypes = [vp, C.c_double, vp, vp, vp, vp, vp, sz, vp]
    lib.ks_gram_general.argtypes = [i32, i64, i32, vp, vp, i64, vp, i32, vp, sz, vp]
    lib.ks_rotate_block.argtypes = [i32, i64, i32, vp, i64, vp, i32, i32, vp, i64, vp]
    lib.hegv_reduce_solve.argtypes = [i32, i32, vp, i32, vp, i32, vp, vp, i32, vp, sz, vp, vp]
    lib.hegv_workspace_size.argtypes = [i32, i32, C.POINTER(sz)]
    lib.hegv_reduce_solve_noalloc.argtypes = [i32, i32, vp, i32, vp, i32, vp, vp, i32, vp, vp]
    lib.hegv_reduce_variant.argtypes = [i32, i32, vp, i32, vp, i32, vp, i32, vp, sz, vp, vp]
    lib.sygv_reduce_variant.argtypes = [i32, i32, vp, i32, vp, i32, vp, i32, vp, sz, vp, vp]
    lib.sygv_reduce_workspace_size.argtypes = [i32, C.POINTER(sz)]
    lib.lobpcg_init.argtypes = [vp, vp, C.POINTER(KsLobpcgState), vp, sz, vp]
    lib.lobpcg_step.argtypes = [vp, vp, C.POINTER(KsLobpcgState), C.POINTER(KsLobpcgOpts), vp, sz, vp]
    f32 = C.c_float
    lib.ks_jd_correction.argtypes = [vp, vp, vp, vp, vp, i64, i32, i32, C.c_double, vp, vp, vp, sz, vp]
    lib.cnn_workspace_size.argtypes = [vp, i32, C.POINTER(sz), C.POINTER(sz)]
    lib.cnn_forward.argtypes = [vp, vp, i32, vp, vp, vp, vp]
    lib.cnn_backward.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, sz, vp]
    lib.cnn_loss.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp]
    lib.cnn_adam_step.argtypes = [vp, vp, vp, vp, i32, i32, f32, vp]
    lib.cnn_make_input.argtypes = [vp, vp, i64, vp, vp, vp, i32, vp, vp]
    lib.cnn_add_skip.argtypes = [vp, i32, vp, vp, vp]
    lib.cnn_infer.argtypes = [vp, vp, i32, vp, vp, vp, vp]
    lib.cnn_conv16_bf16.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp]
    lib.ks_kernel_timer.argtypes = [i32, i32]
    lib.ks_kernel_timer_read.argtypes = [i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.ks_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name != "ks_last_error":
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def check(rc: int, what: str) -> None:
    if rc != 0:
        msg = load().ks_last_error().decode()
        raise KsError(f"{what} failed with {rc}: {msg}")


def _ptr(t) -> int:
    return int(t.data_ptr())


def _stream(stream=None) -> int:
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _work(nbytes: int, device):
    import torch

    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


@dataclass
class ProjectorArrays:
    """Host copies of the projector set (numpy), kept alive for the call."""

    atom_supp_ptr: np.ndarray
    supp_idx: np.ndarray
    atom_proj_ptr: np.ndarray
    beta_ptr: np.ndarray
    beta: np.ndarray
    D: np.ndarray
    # (n_supp, 3) displacements of the support points from their atoms
    # (plans with a Bloch vector only)
    supp_disp: np.ndarray = None

    @classmethod
    def from_cell(cls, cell):
        disp = getattr(cell, "supp_disp", None)
        return cls(
            np.ascontiguousarray(cell.atom_supp_ptr, np.int32),
            np.ascontiguousarray(cell.supp_idx, np.int32),
            np.ascontiguousarray(cell.atom_proj_ptr, np.int32),
            np.ascontiguousarray(cell.beta_ptr, np.int64),
            np.ascontiguousarray(cell.beta, np.float64),
            np.ascontiguousarray(cell.D, np.float64),
            None if disp is None else np.ascontiguousarray(disp, np.float64),
        )

    def struct(self) -> KsProjset:
        ps = KsProjset()
        ps.n_atoms = len(self.atom_supp_ptr) - 1
        ps.n_proj = len(self.D)
        ps.n_supp = len(self.supp_idx)
        ps.atom_supp_ptr = self.atom_supp_ptr.ctypes.data_as(C.POINTER(C.c_int32))
        ps.supp_idx = self.supp_idx.ctypes.data_as(C.POINTER(C.c_int32))
        ps.atom_proj_ptr = self.atom_proj_ptr.ctypes.data_as(C.POINTER(C.c_int32))
        ps.beta_ptr = self.beta_ptr.ctypes.data_as(C.POINTER(C.c_int64))
        ps.beta = self.beta.ctypes.data_as(C.POINTER(C.c_double))
        ps.D = self.D.ctypes.data_as(C.POINTER(C.c_double))
        return ps


class Plan:
    """Owns a ks_plan*.  With ``k`` (3 floats, 1/bohr) the plan acts on the
    periodic part of Bloch orbitals at that vector (ks_plan_create_k; the
    projector set then needs its support displacements)."""

    def __init__(self, n, L, proj: ProjectorArrays | None, nb_max: int, precision: int = KS_FP64, stream=None,
                 k=None):
        lib = load()
        g = KsGrid()
        for a in range(3):
            g.n[a] = int(n[a] if hasattr(n, "__len__") else n)
            g.L[a] = float(L[a] if hasattr(L, "__len__") else L)
        self.n = tuple(int(g.n[a]) for a in range(3))
        self.Ng = self.n[0] * self.n[1] * self.n[2]
        self.nb_max = int(nb_max)
        self.precision = int(precision)
        self._proj = proj
        ps = proj.struct() if proj is not None and len(proj.D) > 0 else None
        h = C.c_void_p()
        self.k = None if k is None else np.ascontiguousarray(k, np.float64).reshape(3)
        if self.k is None:
            rc = lib.ks_plan_create(C.byref(h), C.byref(g), C.byref(ps) if ps is not None else None, self.nb_max,
                                    self.precision, C.c_void_p(_stream(stream)))
            check(rc, "ks_plan_create")
        else:
            disp = None if proj is None or proj.supp_disp is None else proj.supp_disp
            dp = None if disp is None else disp.ctypes.data_as(C.POINTER(C.c_double))
            rc = lib.ks_plan_create_k(C.byref(h), C.byref(g), self.k.ctypes.data_as(C.POINTER(C.c_double)),
                                      C.byref(ps) if ps is not None else None, dp, self.nb_max, self.precision,
                                      C.c_void_p(_stream(stream)))
            check(rc, "ks_plan_create_k")
        self.handle = h
        _live_plans.add(self)

    @property
    def complex_dtype(self):
        import torch

        return torch.complex128 if self.precision == KS_FP64 else torch.complex64

    @property
    def real_dtype(self):
        import torch

        return torch.float64 if self.precision == KS_FP64 else torch.float32

    def workspace_size(self, op: int, nb: int) -> int:
        n = C.c_size_t()
        check(load().ks_workspace_size(self.handle, op, nb, C.byref(n)), "ks_workspace_size")
        return int(n.value)

    def destroy(self):
        """Free the plan's device tables now (idempotent)."""
        if getattr(self, "handle", None):
            load().ks_plan_destroy(self.handle)
            self.handle = None
        _live_plans.discard(self)

    def __del__(self):  # pragma: no cover
        # after the exit hook has run, a finaliser frees nothing: the exit
        # hook destroyed every live plan already
        if _exiting:
            return
        try:
            self.destroy()
        except Exception:
            pass


def ks_apply_h(plan: Plan, v, psi, hpsi, nb: int | None = None, work=None, stream=None):
    """hpsi = H psi for torch blocks of shape (nb, >=Ng) on the device."""
    nb = psi.shape[0] if nb is None else nb
    need = plan.workspace_size(KS_OP_APPLY_H, nb)
    if work is None:
        work = _work(need, psi.device)
    rc = load().ks_apply_h(plan.handle, _ptr(v), _ptr(psi), psi.stride(0), _ptr(hpsi), hpsi.stride(0), nb,
                           _ptr(work), work.numel(), C.c_void_p(_stream(stream)))
    check(rc, "ks_apply_h")
    return hpsi


def _opts(precond: int, lock_tol: float, cnn_params=None) -> KsLobpcgOpts:
    o = KsLobpcgOpts()
    o.precond = int(precond)
    o.lock_tol = float(lock_tol)
    if cnn_params is not None:
        if cnn_params.numel() != KS_CNN_NPARAM:
            raise KsError("cnn_params must hold KS_CNN_NPARAM values")
        o.cnn_params = _ptr(cnn_params)
    return o


def ks_precond_apply(plan: Plan, kind: int, X, AX, theta, W, res, lock_tol: float = 0.0, v=None, cnn_params=None,
                     work=None, stream=None):
    """W = K(AX - X diag(theta)) and res = its column norms; the learned
    kinds need v (the local potential) and cnn_params."""
    nb = X.shape[0]
    learned = kind in (KS_PRECOND_CNN, KS_PRECOND_CNN_TPA)
    need = plan.workspace_size(KS_OP_PRECOND_CNN if learned else KS_OP_PRECOND, nb)
    if work is None:
        work = _work(need, X.device)
    o = _opts(kind, lock_tol, cnn_params)
    rc = load().ks_precond_apply(plan.handle, C.byref(o), None if v is None else _ptr(v), _ptr(X), _ptr(AX),
                                 _ptr(theta), X.stride(0), nb, _ptr(W), _ptr(res), _ptr(work), work.numel(),
                                 C.c_void_p(_stream(stream)))
    check(rc, "ks_precond_apply")
    return W


def ks_subspace_sin(plan: Plan, A, B, k: int, out=None, work=None, stream=None):
    """Device double: sine of the largest principal angle between the spans
    of the first k rows (columns of the blocks) of A and B."""
    import torch

    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=A.device)
    if work is None:
        work = _work(plan.workspace_size(KS_OP_ANGLE, k), A.device)
    rc = load().ks_subspace_sin(plan.handle, _ptr(A), _ptr(B), A.stride(0), int(k), _ptr(out), _ptr(work),
                                work.numel(), C.c_void_p(_stream(stream)))
    check(rc, "ks_subspace_sin")
    return out


def _scf_work(plan: Plan, device):
    return _work(plan.workspace_size(KS_OP_SCF, 1), device)


def ks_density(plan: Plan, X, nocc: int, n, occ=None, stream=None):
    """n (Ng float64) = electrons per grid point of the first nocc rows of X."""
    check(load().ks_density(plan.handle, _ptr(X), X.stride(0), int(nocc), None if occ is None else _ptr(occ), _ptr(n),
                            C.c_void_p(_stream(stream))), "ks_density")
    return n


def ks_hartree(plan: Plan, n, v_h, work=None, stream=None):
    work = _scf_work(plan, n.device) if work is None else work
    check(load().ks_hartree(plan.handle, _ptr(n), _ptr(v_h), _ptr(work), work.numel(), C.c_void_p(_stream(stream))),
          "ks_hartree")
    return v_h


def ks_lda_xc(plan: Plan, n, v_xc, e_xc=None, stream=None):
    check(load().ks_lda_xc(plan.handle, _ptr(n), _ptr(v_xc), None if e_xc is None else _ptr(e_xc),
                           C.c_void_p(_stream(stream))), "ks_lda_xc")
    return v_xc


def ks_scf_potential(plan: Plan, n, v_ion, v_eff, terms, work=None, stream=None):
    """v_eff = v_ion + V_H[n] + v_xc[n] (plan precision); terms (4 float64)."""
    work = _scf_work(plan, n.device) if work is None else work
    check(load().ks_scf_potential(plan.handle, _ptr(n), _ptr(v_ion), _ptr(v_eff), _ptr(terms), _ptr(work),
                                  work.numel(), C.c_void_p(_stream(stream))), "ks_scf_potential")
    return v_eff


def ks_mix_density(plan: Plan, alpha: float, n_in, n_out, n_next, resid, work=None, stream=None):
    work = _scf_work(plan, n_in.device) if work is None else work
    check(load().ks_mix_density(plan.handle, float(alpha), _ptr(n_in), _ptr(n_out), _ptr(n_next), _ptr(resid),
                                _ptr(work), work.numel(), C.c_void_p(_stream(stream))), "ks_mix_density")
    return n_next


def ks_gram_general(precision: int, A, B, G, work=None, stream=None):
    """G (m x m complex128, column-major: a tensor whose transpose is
    contiguous) = A^H B for blocks A, B of shape (m, K) (rows are columns)."""
    m, K = A.shape
    if work is None:
        n = C.c_size_t()
        check(load().ks_gram_workspace_size(K, m, C.byref(n)), "ks_gram_workspace_size")
        work = _work(n.value, A.device)
    check(load().ks_gram_general(precision, K, m, _ptr(A), _ptr(B), A.stride(0), _ptr(G), G.stride(1), _ptr(work),
                                 work.numel(), C.c_void_p(_stream(stream))), "ks_gram_general")
    return G


def ks_rotate_block(precision: int, V, Cm, Y, stream=None):
    """Y (ncol, K) = (V^T C)^T for V of shape (m, K) and C (m x ncol,
    column-major, the block precision)."""
    m, K = V.shape
    ncol = Y.shape[0]
    check(load().ks_rotate_block(precision, K, m, _ptr(V), V.stride(0), _ptr(Cm), Cm.stride(1), ncol, _ptr(Y),
                                 Y.stride(0), C.c_void_p(_stream(stream))), "ks_rotate_block")
    return Y


def kernel_timer(enable: bool, family: int) -> None:
    check(load().ks_kernel_timer(1 if enable else 0, family), "ks_kernel_timer")


def kernel_timer_read(family: int):
    """(total milliseconds, launches) recorded since the timer was enabled."""
    ms = C.c_double()
    n = C.c_int64()
    check(load().ks_kernel_timer_read(family, C.byref(ms), C.byref(n)), "ks_kernel_timer_read")
    return float(ms.value), int(n.value)


def hegv_workspace_size(n: int, nev: int) -> int:
    b = C.c_size_t()
    check(load().hegv_workspace_size(n, nev, C.byref(b)), "hegv_workspace_size")
    return int(b.value)


def hegv_reduce_solve(H, S, nev: int, w, Cmat, info, work=None, stream=None):
    """H, S: (n, n) complex128 column-major device matrices, i.e. torch
    tensors whose transpose is contiguous (pass A.T.contiguous().T)."""
    n = H.shape[0]
    if work is None:
        work = _work(hegv_workspace_size(n, nev), H.device)
    rc = load().hegv_reduce_solve(n, nev, _ptr(H), H.stride(1), _ptr(S), S.stride(1), _ptr(w), _ptr(Cmat),
                                  Cmat.stride(1), _ptr(work), work.numel(), _ptr(info), C.c_void_p(_stream(stream)))
    check(rc, "hegv_reduce_solve")


KS_REDUCE_INVERSE, KS_REDUCE_TWO_TRSM, KS_REDUCE_TWO_SIDED = 0, 1, 2


def hegv_reduce_variant(variant: int, H, S, K, info, work=None, stream=None):
    """S <- chol(S) (lower) and K = L^-1 H L^-H by the chosen method;
    column-major n x n complex128 device matrices (transposes contiguous)."""
    n = H.shape[0]
    if work is None:
        work = _work(hegv_workspace_size(n, 1), H.device)
    check(load().hegv_reduce_variant(variant, n, _ptr(H), H.stride(1), _ptr(S), S.stride(1), _ptr(K), K.stride(1),
                                     _ptr(work), work.numel(), _ptr(info), C.c_void_p(_stream(stream))),
          "hegv_reduce_variant")
    return K


def sygv_reduce_workspace_size(n: int) -> int:
    out = C.c_size_t()
    check(load().sygv_reduce_workspace_size(n, C.byref(out)), "sygv_reduce_workspace_size")
    return out.value


def sygv_reduce_variant(variant: int, H, S, K, info, work=None, stream=None):
    """The real-symmetric reduction: S <- chol(S) (lower) and K = L^-1 H L^-T;
    column-major n x n float64 device matrices (transposes contiguous)."""
    n = H.shape[0]
    if work is None:
        work = _work(sygv_reduce_workspace_size(n), H.device)
    check(load().sygv_reduce_variant(variant, n, _ptr(H), H.stride(1), _ptr(S), S.stride(1), _ptr(K), K.stride(1),
                                     _ptr(work), work.numel(), _ptr(info), C.c_void_p(_stream(stream))),
          "sygv_reduce_variant")
    return K


class Lobpcg:
    """Device buffers of one LOBPCG run and the calls that advance it.

    With ``summary=True`` (the default) every init/step ends with the one
    device-to-host copy of (theta, res, status) into pinned host memory,
    readable afterwards as ``theta_host``, ``res_host`` and ``status_host``;
    with ``summary=False`` the calls never wait for the device."""

    BLOCKS = ("X", "AX", "W", "AW", "P", "AP", "Xn", "Pn", "T1")

    def __init__(self, plan: Plan, v, X0, stream=None, summary: bool = True):
        import torch

        self.plan = plan
        self.v = v
        nb = X0.shape[0]
        self.nb = nb
        dev = X0.device
        self.buf = {}
        for name in self.BLOCKS:
            self.buf[name] = torch.empty((nb, plan.Ng), dtype=plan.complex_dtype, device=dev)
        self.buf["X"].copy_(X0)
        self.theta = torch.zeros(nb, dtype=torch.float64, device=dev)
        self.res = torch.zeros(nb, dtype=torch.float64, device=dev)
        self.status = torch.zeros(KS_STATUS_WORDS, dtype=torch.int32, device=dev)
        # the next step's P Gram, carried from step to step
        self.p_gram = torch.zeros((nb, nb), dtype=torch.complex128, device=dev)
        self.work = _work(plan.workspace_size(KS_OP_LOBPCG, nb), dev)
        self._by_ptr = {_ptr(t): t for t in self.buf.values()}
        st = KsLobpcgState()
        st.nb = nb
        st.ld = plan.Ng
        for name in self.BLOCKS:
            setattr(st, name, _ptr(self.buf[name]))
        st.theta = _ptr(self.theta)
        st.res = _ptr(self.res)
        st.status = _ptr(self.status)
        st.p_gram = _ptr(self.p_gram)
        self.summary = None
        if summary:
            self.summary = torch.zeros(16 * nb + 4 * KS_STATUS_WORDS, dtype=torch.uint8, pin_memory=True)
            st.host_summary = self.summary.data_ptr()
        self.st = st
        self.stream = stream

    def block(self, name: str):
        return self._by_ptr[int(getattr(self.st, name))]

    def init(self):
        rc = load().lobpcg_init(self.plan.handle, _ptr(self.v), C.byref(self.st), _ptr(self.work), self.work.numel(),
                                C.c_void_p(_stream(self.stream)))
        check(rc, "lobpcg_init")

    def step(self, precond: int = KS_PRECOND_TPA, lock_tol: float = 0.0, cnn_params=None):
        """One iteration; ``cnn_params`` (FP32 device tensor of KS_CNN_NPARAM
        values) is required for KS_PRECOND_CNN and KS_PRECOND_CNN_TPA."""
        o = _opts(precond, lock_tol, cnn_params)
        rc = load().lobpcg_step(self.plan.handle, _ptr(self.v), C.byref(self.st), C.byref(o), _ptr(self.work),
                                self.work.numel(), C.c_void_p(_stream(self.stream)))
        check(rc, "lobpcg_step")

    def _summary_np(self):
        if self.summary is None:
            raise KsError("this run has no host summary buffer")
        return self.summary.numpy()

    @property
    def theta_host(self):
        """Ritz values from the last call's summary copy (numpy, no device access)."""
        return self._summary_np()[: 8 * self.nb].view(np.float64).copy()

    @property
    def res_host(self):
        """Residual norms of the block the last step started from (numpy)."""
        return self._summary_np()[8 * self.nb: 16 * self.nb].view(np.float64).copy()

    @property
    def status_host(self):
        return self._summary_np()[16 * self.nb:].view(np.int32).copy()

    @property
    def X(self):
        return self.block("X")

    @property
    def AX(self):
        return self.block("AX")

    @property
    def P(self):
        return self.block("P") if self.st.has_p else None

    @property
    def AP(self):
        return self.block("AP") if self.st.has_p else None


def ks_jd_correction(plan: Plan, v, X, theta, R, T, iters, maxit: int = 500, rtol: float = 1e-6, work=None,
                     stream=None):
    """T = CG solution of P (H - theta_i) P t_i = P r_i for every column."""
    nb = X.shape[0]
    if work is None:
        work = _work(plan.workspace_size(KS_OP_JD, nb), X.device)
    rc = load().ks_jd_correction(plan.handle, _ptr(v), _ptr(X), _ptr(theta), _ptr(R), X.stride(0), nb, int(maxit),
                                 float(rtol), _ptr(T), _ptr(iters), _ptr(work), work.numel(),
                                 C.c_void_p(_stream(stream)))
    check(rc, "ks_jd_correction")
    return T


class Cnn:
    """Parameters, Adam state and buffers of the learned preconditioner."""

    def __init__(self, plan: Plan, params, nbatch: int):
        import torch

        self.plan = plan
        self.nbatch = nbatch
        dev = params.device
        self.params = params.contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.t = 0
        a = C.c_size_t()
        wb = C.c_size_t()
        check(load().cnn_workspace_size(plan.handle, nbatch, C.byref(a), C.byref(wb)), "cnn_workspace_size")
        self.acts = torch.empty(int(a.value), dtype=torch.float32, device=dev)
        self.work = _work(int(wb.value), dev)
        self.y = torch.empty((nbatch, 2, plan.Ng), dtype=torch.float32, device=dev)
        self.gy = torch.empty_like(self.y)
        self.loss = torch.zeros(nbatch, dtype=torch.float64, device=dev)
        self.sums = torch.zeros(3 * nbatch, dtype=torch.float64, device=dev)

    def forward(self, x, nb=None, skip=False, stream=None):
        """y = net(x), plus the first two input channels when ``skip``."""
        nb = x.shape[0] if nb is None else nb
        check(load().cnn_forward(self.plan.handle, _ptr(self.params), nb, _ptr(x), _ptr(self.y), _ptr(self.acts),
                                 C.c_void_p(_stream(stream))), "cnn_forward")
        if skip:
            cnn_add_skip(self.plan, x, self.y, nb, stream)
        return self.y[:nb]

    def infer(self, x, nb=None, stream=None):
        """y = net(x) as lobpcg_step applies it (the same bfloat16
        matrix-core layers as ``forward``, no activations kept); uses the
        activation buffer as scratch and returns the same buffer as
        ``forward``."""
        nb = x.shape[0] if nb is None else nb
        check(load().cnn_infer(self.plan.handle, _ptr(self.params), nb, _ptr(x), _ptr(self.y), _ptr(self.acts),
                               C.c_void_p(_stream(stream))), "cnn_infer")
        return self.y[:nb]

    def loss_grad(self, t, nb=None, stream=None):
        nb = t.shape[0] if nb is None else nb
        check(load().cnn_loss(nb, self.plan.Ng, _ptr(self.y), _ptr(t), _ptr(self.gy), _ptr(self.loss), _ptr(self.sums),
                              C.c_void_p(_stream(stream))), "cnn_loss")
        return self.loss[:nb]

    def backward(self, x, gy=None, nb=None, stream=None):
        nb = x.shape[0] if nb is None else nb
        g = self.gy if gy is None else gy
        check(load().cnn_backward(self.plan.handle, _ptr(self.params), nb, _ptr(x), _ptr(self.acts), _ptr(g),
                                  _ptr(self.grads), _ptr(self.work), self.work.numel(), C.c_void_p(_stream(stream))),
              "cnn_backward")
        return self.grads

    def adam(self, lr: float = 1e-3, stream=None):
        self.t += 1
        check(load().cnn_adam_step(_ptr(self.params), _ptr(self.grads), _ptr(self.m), _ptr(self.v),
                                   self.params.numel(), self.t, float(lr), C.c_void_p(_stream(stream))),
              "cnn_adam_step")


def cnn_make_input(plan: Plan, R, rnorm, v, theta, x, stream=None):
    """x = network input of the columns of R; rnorm None: each column is
    scaled by its own norm (computed by the library)."""
    nb = R.shape[0]
    check(load().cnn_make_input(plan.handle, _ptr(R), R.stride(0), None if rnorm is None else _ptr(rnorm), _ptr(v),
                                _ptr(theta), nb, _ptr(x), C.c_void_p(_stream(stream))), "cnn_make_input")
    return x


def cnn_conv16_bf16(plan: Plan, x, w, b, y, silu=True, nbatch=None, stream=None):
    """y = conv(x; w, b) (16 -> 16 channels, periodic 3x3x3) with bfloat16
    products, then SiLU when ``silu``; x, y: (nbatch, 16, Ng) float32."""
    nb = x.shape[0] if nbatch is None else nbatch
    check(load().cnn_conv16_bf16(plan.handle, nb, _ptr(x), _ptr(w), _ptr(b), 1 if silu else 0, _ptr(y),
                                 C.c_void_p(_stream(stream))), "cnn_conv16_bf16")


def cnn_add_skip(plan: Plan, x, y, nbatch=None, stream=None):
    """y[:, 0:2] += x[:, 0:2] (skip connection of the residual network)."""
    nb = x.shape[0] if nbatch is None else nbatch
    check(load().cnn_add_skip(plan.handle, nb, _ptr(x), _ptr(y), C.c_void_p(_stream(stream))), "cnn_add_skip")
    return y
