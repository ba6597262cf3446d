"""MI355X (gfx950) DF-SS-FNO-EA-ADC(3): thin Python binding of the C ABI in include/adc3ea.h.

Every step of the method runs in the HIP library libadc3ea.so; this module only
marshals arguments.  Device buffers are torch tensors (float64, contiguous, on the
current HIP device); work runs on torch's current stream.  The library must be
built (``python -m paper_2511_05897_amd.build``); importing the binding without it
raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadc3ea.so")

ADC3_OK, ADC3_WNOCONV = 0, 1
ADC3_EINVAL, ADC3_ENOMEM, ADC3_EHIP, ADC3_ENUMERIC, ADC3_EUNSUP = -1, -2, -3, -4, -5

# every symbol declared in include/adc3ea.h
EXPORTS = ["adc3_default_opts", "adc3_last_error", "adc3_ea_solve_workspace_bytes", "adc3_ea_solve",
           "adc3_ea_setup_workspace_bytes", "adc3_ea_setup", "adc3_ctx_destroy", "adc3_ea_dim",
           "adc3_ea_sigma", "adc3_ea_diagonal", "adc3_ea_davidson", "adc3_ea_dense_matrix",
           "adc3_ea_intermediate", "adc3_profile_enable", "adc3_profile_query", "adc3_mlp_nparams",
           "adc3_ea_set_preconditioner", "adc3_mlp_collect", "adc3_mlp_workspace_bytes", "adc3_mlp_loss_grad",
           "adc3_mlp_forward", "adc3_mlp_train", "adc3_ea_precondition", "adc3_ea_solve_batched_workspace_bytes",
           "adc3_ea_solve_batched", "adc3_ea_set_sigma_graphs", "adc3_profile_query_bound",
           "adc3_ea_setup_workspace_bytes_ex", "adc3_ea_setup_ex", "adc3_set_chunk_elems",
           "adc3_ladder_workspace_bytes", "adc3_ladder_apply", "adc3_eigh_workspace_bytes", "adc3_eigh",
           "adc3_eigh_batched_workspace_bytes", "adc3_eigh_batched", "adc3_ladder_apply_static",
           "adc3_ea_davidson_guess", "adc3_ea_setup_sm", "adc3_debug_inject_nan", "adc3_ea_spectral_amplitudes",
           "adc3_debug_ladder_offset_limit"]

# size of the static device scratch of adc3_ladder_apply_static (ADC3_STATIC_SCRATCH_BYTES)
STATIC_SCRATCH_BYTES = 256 << 20


class adc3_opts(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int), ("max_iter", ctypes.c_int), ("max_subspace", ctypes.c_int),
                ("fno_correction", ctypes.c_int), ("precision", ctypes.c_int), ("precond", ctypes.c_int),
                ("mlp_weights", ctypes.c_void_p), ("sigma_graphs", ctypes.c_int), ("ladder", ctypes.c_int),
                ("sm_x", ctypes.c_double), ("fno_mode", ctypes.c_int), ("fno_keep_frac", ctypes.c_double),
                ("init_guess", ctypes.c_void_p), ("n_guess", ctypes.c_int), ("vectors_out", ctypes.c_void_p),
                ("dyson_out", ctypes.c_void_p), ("lockstep", ctypes.c_int)]


class adc3_instance(ctypes.Structure):
    _fields_ = [("eps_occ", ctypes.c_void_p), ("eps_vir", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("nocc", ctypes.c_int), ("nvir", ctypes.c_int), ("naux", ctypes.c_int), ("nroots", ctypes.c_int),
                ("fno_thresh", ctypes.c_double), ("naf_thresh", ctypes.c_double), ("conv", ctypes.c_double)]


class adc3_root_report(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("omega_uncorr", ctypes.c_double),
                ("omega_adc2_can", ctypes.c_double), ("omega_adc2_fno", ctypes.c_double),
                ("resnorm", ctypes.c_double), ("nvir_kept", ctypes.c_int), ("naux_kept", ctypes.c_int),
                ("iters", ctypes.c_int), ("sigma_builds", ctypes.c_int), ("omega_lowp", ctypes.c_double),
                ("iters_lowp", ctypes.c_int), ("err_bound", ctypes.c_double), ("pole_strength", ctypes.c_double),
                ("sigma_builds_final", ctypes.c_int)]


class ADCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("adc3 status %d: %s" % (status, msg))
        self.status = status


_lib = None


def load():
    """Load libadc3ea.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError("libadc3ea.so not built: run python -m paper_2511_05897_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, S, LL = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_longlong
    lib.adc3_default_opts.argtypes = [ctypes.POINTER(adc3_opts)]
    lib.adc3_default_opts.restype = None
    lib.adc3_last_error.restype = ctypes.c_char_p
    lib.adc3_ea_solve_workspace_bytes.argtypes = [I, I, I, I, ctypes.POINTER(adc3_opts)]
    lib.adc3_ea_solve_workspace_bytes.restype = S
    lib.adc3_ea_solve.argtypes = [P, P, P, I, I, I, I, D, D, D, ctypes.POINTER(adc3_opts),
                                  ctypes.POINTER(D), ctypes.POINTER(adc3_root_report), P, S, P]
    lib.adc3_ea_solve.restype = I
    lib.adc3_ea_setup_workspace_bytes.argtypes = [I, I, I, I, I, I]
    lib.adc3_ea_setup_workspace_bytes.restype = S
    lib.adc3_ea_setup.argtypes = [P, P, P, I, I, I, I, I, P, S, P, ctypes.POINTER(P)]
    lib.adc3_ea_setup.restype = I
    lib.adc3_ea_setup_workspace_bytes_ex.argtypes = [I, I, I, I, I, I, I]
    lib.adc3_ea_setup_workspace_bytes_ex.restype = S
    lib.adc3_ea_setup_ex.argtypes = [P, P, P, I, I, I, I, I, I, P, S, P, ctypes.POINTER(P)]
    lib.adc3_ea_setup_ex.restype = I
    lib.adc3_set_chunk_elems.argtypes = [LL]
    lib.adc3_set_chunk_elems.restype = LL
    lib.adc3_ladder_workspace_bytes.argtypes = [I, I, I, I]
    lib.adc3_ladder_workspace_bytes.restype = S
    lib.adc3_ladder_apply.argtypes = [P, P, P, I, I, I, I, P, S, P]
    lib.adc3_eigh_workspace_bytes.argtypes = [I]
    lib.adc3_eigh_workspace_bytes.restype = S
    lib.adc3_eigh.argtypes = [P, P, P, I, P, S, P]
    lib.adc3_eigh.restype = I
    lib.adc3_eigh_batched_workspace_bytes.argtypes = [I, I]
    lib.adc3_eigh_batched_workspace_bytes.restype = S
    lib.adc3_eigh_batched.argtypes = [P, P, P, I, I, P, S, P]
    lib.adc3_eigh_batched.restype = I
    lib.adc3_ladder_apply.restype = I
    lib.adc3_ladder_apply_static.argtypes = [P, P, P, I, I, I, I, P]
    lib.adc3_ladder_apply_static.restype = I
    lib.adc3_ctx_destroy.argtypes = [P]
    lib.adc3_ctx_destroy.restype = None
    lib.adc3_ea_dim.argtypes = [P]
    lib.adc3_ea_dim.restype = LL
    lib.adc3_ea_sigma.argtypes = [P, P, P, I, I, P]
    lib.adc3_ea_sigma.restype = I
    lib.adc3_ea_diagonal.argtypes = [P, P, P]
    lib.adc3_ea_diagonal.restype = I
    lib.adc3_ea_davidson.argtypes = [P, I, D, I, I, I, ctypes.POINTER(D), P, ctypes.POINTER(D),
                                     ctypes.POINTER(I), P]
    lib.adc3_ea_davidson.restype = I
    lib.adc3_ea_davidson_guess.argtypes = [P, I, D, I, I, I, P, I, ctypes.POINTER(D), P, ctypes.POINTER(D),
                                           ctypes.POINTER(I), P]
    lib.adc3_ea_davidson_guess.restype = I
    lib.adc3_ea_setup_sm.argtypes = [P, P, P, I, I, I, D, I, I, P, S, P, ctypes.POINTER(P)]
    lib.adc3_ea_setup_sm.restype = I
    lib.adc3_ea_spectral_amplitudes.argtypes = [P, P, I, P, P]
    lib.adc3_ea_spectral_amplitudes.restype = I
    lib.adc3_debug_inject_nan.argtypes = [I]
    lib.adc3_debug_inject_nan.restype = None
    lib.adc3_debug_ladder_offset_limit.argtypes = [ctypes.c_longlong]
    lib.adc3_debug_ladder_offset_limit.restype = None
    lib.adc3_ea_dense_matrix.argtypes = [P, P, I, P]
    lib.adc3_ea_dense_matrix.restype = I
    lib.adc3_ea_intermediate.argtypes = [P, I, P, ctypes.POINTER(LL), P]
    lib.adc3_ea_intermediate.restype = I
    lib.adc3_profile_enable.argtypes = [I]
    lib.adc3_profile_enable.restype = None
    lib.adc3_profile_query.argtypes = [I, ctypes.POINTER(D), ctypes.POINTER(LL), ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.adc3_profile_query.restype = I
    lib.adc3_profile_query_bound.argtypes = [I, ctypes.POINTER(D)]
    lib.adc3_profile_query_bound.restype = I
    U64 = ctypes.c_ulonglong
    lib.adc3_mlp_nparams.argtypes = []
    lib.adc3_mlp_nparams.restype = I
    lib.adc3_ea_set_preconditioner.argtypes = [P, P]
    lib.adc3_ea_set_preconditioner.restype = I
    lib.adc3_mlp_collect.argtypes = [P, I, D, I, I, I, U64, P, P, P, ctypes.POINTER(I), P]
    lib.adc3_mlp_collect.restype = I
    lib.adc3_mlp_workspace_bytes.argtypes = [I, I]
    lib.adc3_mlp_workspace_bytes.restype = S
    lib.adc3_mlp_loss_grad.argtypes = [P, P, P, P, I, I, P, ctypes.POINTER(D), P, S, P]
    lib.adc3_mlp_loss_grad.restype = I
    lib.adc3_mlp_forward.argtypes = [P, P, LL, P, P, S, P]
    lib.adc3_mlp_forward.restype = I
    lib.adc3_mlp_train.argtypes = [P, P, P, P, I, I, I, I, D, U64, P, P, S, P]
    lib.adc3_mlp_train.restype = I
    lib.adc3_ea_precondition.argtypes = [P, D, P, P, ctypes.POINTER(I), P]
    lib.adc3_ea_precondition.restype = I
    lib.adc3_ea_solve_batched_workspace_bytes.argtypes = [ctypes.POINTER(adc3_instance), I,
                                                          ctypes.POINTER(adc3_opts), I]
    lib.adc3_ea_solve_batched_workspace_bytes.restype = S
    lib.adc3_ea_solve_batched.argtypes = [ctypes.POINTER(adc3_instance), I, ctypes.POINTER(adc3_opts), I,
                                          ctypes.POINTER(D), ctypes.POINTER(adc3_root_report), ctypes.POINTER(I),
                                          P, S, P]
    lib.adc3_ea_solve_batched.restype = I
    lib.adc3_ea_set_sigma_graphs.argtypes = [P, I]
    lib.adc3_ea_set_sigma_graphs.restype = I
    _lib = lib
    return lib


def _check(status, allow_noconv=False):
    if status == ADC3_OK or (allow_noconv and status == ADC3_WNOCONV):
        return status
    raise ADCError(status, load().adc3_last_error().decode())


def _ptr(t):
    import torch
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _ptrf(t):
    import torch
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(nbytes):
    import torch
    if nbytes == 0:
        raise ADCError(ADC3_EINVAL, "workspace size query failed (invalid arguments)")
    return torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")


def adc3_default_opts():
    o = adc3_opts()
    load().adc3_default_opts(ctypes.byref(o))
    return o


def adc3_ea_solve_workspace_bytes(nocc, nvir, naux, nroots, opts=None):
    o = opts if opts is not None else adc3_default_opts()
    return load().adc3_ea_solve_workspace_bytes(nocc, nvir, naux, nroots, ctypes.byref(o))


def adc3_ea_solve(eps_occ, eps_vir, B, nroots, fno_thresh, naf_thresh, conv, opts=None, workspace=None):
    """Full SS-FNO/NAF EA-ADC solve on device tensors.  Returns (roots[nroots], reports, status)."""
    lib = load()
    o = opts if opts is not None else adc3_default_opts()
    nocc, nvir, naux = int(eps_occ.numel()), int(eps_vir.numel()), int(B.shape[0])
    if workspace is None:
        workspace = _workspace(adc3_ea_solve_workspace_bytes(nocc, nvir, naux, nroots, o))
    roots = (ctypes.c_double * nroots)()
    reps = (adc3_root_report * nroots)()
    st = lib.adc3_ea_solve(_ptr(eps_occ), _ptr(eps_vir), _ptr(B), nocc, nvir, naux, nroots,
                           float(fno_thresh), float(naf_thresh), float(conv), ctypes.byref(o), roots, reps,
                           ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream())
    _check(st, allow_noconv=True)
    reports = [{f: getattr(r, f) for f, _ in adc3_root_report._fields_} for r in reps]
    return np.array(roots[:]), reports, st


def _instances(instances):
    arr = (adc3_instance * len(instances))()
    for i, d in enumerate(instances):
        eo, ev, B = d["eps_occ"], d["eps_vir"], d["B"]
        arr[i] = adc3_instance(_ptr(eo).value, _ptr(ev).value, _ptr(B).value, int(eo.numel()), int(ev.numel()),
                               int(B.shape[0]), int(d["nroots"]), float(d.get("fno_thresh", 0.0)),
                               float(d.get("naf_thresh", 0.0)), float(d["conv"]))
    return arr


def adc3_ea_solve_batched_workspace_bytes(instances, opts=None, nstreams=0):
    o = opts if opts is not None else adc3_default_opts()
    arr = _instances(instances)
    return load().adc3_ea_solve_batched_workspace_bytes(arr, len(instances), ctypes.byref(o), nstreams)


def adc3_ea_solve_batched(instances, opts=None, nstreams=0, workspace=None):
    """Solve a ragged list of instances (dicts: eps_occ, eps_vir, B device tensors, nroots, conv,
    fno_thresh, naf_thresh).  Returns (list of root arrays, list of report lists, statuses, status)."""
    lib = load()
    o = opts if opts is not None else adc3_default_opts()
    arr = _instances(instances)
    n = len(instances)
    if workspace is None:
        workspace = _workspace(lib.adc3_ea_solve_batched_workspace_bytes(arr, n, ctypes.byref(o), nstreams))
    tot = sum(int(d["nroots"]) for d in instances)
    roots = (ctypes.c_double * tot)()
    reps = (adc3_root_report * tot)()
    sts = (ctypes.c_int * n)()
    st = lib.adc3_ea_solve_batched(arr, n, ctypes.byref(o), nstreams, roots, reps, sts,
                                   ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream())
    _check(st, allow_noconv=True)
    out_r, out_p, k = [], [], 0
    for d in instances:
        m = int(d["nroots"])
        out_r.append(np.array(roots[k:k + m]))
        out_p.append([{f: getattr(r, f) for f, _ in adc3_root_report._fields_} for r in reps[k:k + m]])
        k += m
    return out_r, out_p, list(sts), st


def adc3_ea_setup_workspace_bytes(nocc, nvir, naux, level, nroots=0, precision=0, ladder=0):
    return load().adc3_ea_setup_workspace_bytes_ex(nocc, nvir, naux, level, nroots, precision, ladder)


def adc3_set_chunk_elems(n):
    """Set (n > 0) or query (n <= 0) the element budget of one chunk of the large setup tensors."""
    return load().adc3_set_chunk_elems(int(n))


def adc3_ladder_workspace_bytes(nvir, naux, nrows, precision=0):
    return load().adc3_ladder_workspace_bytes(nvir, naux, nrows, precision)


def adc3_ladder_apply(Bvv, Z, precision=0, out=None, workspace=None, workspace_bytes=None):
    """C[m] = sum_Q B^Q Z[m] B^Q (the ladder term from the DF factor), Bvv [X][v][v], Z [M][v][v] FP64 device.
    workspace_bytes (default: one chunk of all auxiliary functions) sets the chunking."""
    import torch
    X, v = int(Bvv.shape[0]), int(Bvv.shape[1])
    M = int(Z.shape[0])
    if out is None:
        out = torch.empty_like(Z)
    if workspace is None:
        if workspace_bytes is None:
            eb = 8 if precision == 0 else 4 if precision == 1 else 2
            workspace_bytes = adc3_ladder_workspace_bytes(v, X, M, precision) + (max(X, 1) - 1) * M * v * v * eb + 512
        workspace = _workspace(workspace_bytes)
    _check(load().adc3_ladder_apply(_ptr(Bvv), _ptr(Z), _ptr(out), v, X, M, precision,
                                    ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream()))
    return out


def adc3_ladder_apply_static(Bvv, Z, precision=0, out=None):
    """The same ladder as adc3_ladder_apply with the library's static device scratch (no allocation by
    the library; calls on one GPU must not overlap)."""
    import torch
    X, v = int(Bvv.shape[0]), int(Bvv.shape[1])
    M = int(Z.shape[0])
    if out is None:
        out = torch.empty_like(Z)
    _check(load().adc3_ladder_apply_static(_ptr(Bvv), _ptr(Z), _ptr(out), v, X, M, precision, _stream()))
    return out


def adc3_eigh_workspace_bytes(n):
    return load().adc3_eigh_workspace_bytes(n)


def adc3_eigh(A):
    """Eigenvalues (ascending) and eigenvectors (columns) of the symmetric part of A [n][n] (FP64 device)."""
    import torch
    n = int(A.shape[0])
    w = torch.empty(n, dtype=torch.float64, device=A.device)
    V = torch.empty((n, n), dtype=torch.float64, device=A.device)
    ws = _workspace(adc3_eigh_workspace_bytes(n))
    _check(load().adc3_eigh(_ptr(A), _ptr(w), _ptr(V), n, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return w, V


def adc3_eigh_batched(A):
    """Eigenvalues (ascending) and eigenvectors of each symmetric part of A [nb][n][n] (FP64 device)."""
    import torch
    nb, n = int(A.shape[0]), int(A.shape[1])
    w = torch.empty((nb, n), dtype=torch.float64, device=A.device)
    V = torch.empty((nb, n, n), dtype=torch.float64, device=A.device)
    ws = _workspace(load().adc3_eigh_batched_workspace_bytes(n, nb))
    _check(load().adc3_eigh_batched(_ptr(A), _ptr(w), _ptr(V), n, nb, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    _stream()))
    return w, V


class Context:
    """Secular-matrix context (adc3_ea_setup ... adc3_ctx_destroy)."""

    def __init__(self, eps_occ, eps_vir, B, level, nroots=8, precision=0, ladder=0, sm_x=None):
        """level 2 or 3; sm_x (level 3 only): the scaled-matrix ADC M_ADC(2) + sm_x (M_ADC(3) - M_ADC(2))."""
        lib = load()
        self.nocc, self.nvir, self.naux = int(eps_occ.numel()), int(eps_vir.numel()), int(B.shape[0])
        self.level = level
        self.precision = precision
        self.workspace = _workspace(adc3_ea_setup_workspace_bytes(self.nocc, self.nvir, self.naux, level, nroots,
                                                                  precision, ladder))
        h = ctypes.c_void_p()
        ws = (ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(), _stream(), ctypes.byref(h))
        if sm_x is None:
            _check(lib.adc3_ea_setup_ex(_ptr(eps_occ), _ptr(eps_vir), _ptr(B), self.nocc, self.nvir, self.naux,
                                        level, precision, ladder, *ws))
        else:
            if level != 3:
                raise ValueError("sm_x needs level 3")
            _check(lib.adc3_ea_setup_sm(_ptr(eps_occ), _ptr(eps_vir), _ptr(B), self.nocc, self.nvir, self.naux,
                                        float(sm_x), precision, ladder, *ws))
        self.handle = h
        self.N = lib.adc3_ea_dim(h)

    def close(self):
        if self.handle:
            load().adc3_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sigma(self, r, out=None, precision=0):
        import torch
        r = r.contiguous()
        nvec = 1 if r.dim() == 1 else r.shape[0]
        if out is None:
            out = torch.empty_like(r)
        _check(load().adc3_ea_sigma(self.handle, _ptr(r), _ptr(out), nvec, precision, _stream()))
        return out

    def diagonal(self):
        import torch
        d = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(load().adc3_ea_diagonal(self.handle, _ptr(d), _stream()))
        return d

    def davidson(self, nroots, conv, max_iter=500, max_subspace=0, want_vectors=False, precision=0, guess=None):
        """(omega, vectors or None, resnorm, iterations, status); guess: device [n][N] start vectors."""
        import torch
        w = (ctypes.c_double * nroots)()
        rn = (ctypes.c_double * nroots)()
        it = ctypes.c_int()
        vec = torch.empty((nroots, self.N), dtype=torch.float64, device="cuda") if want_vectors else None
        g = guess.contiguous() if guess is not None else None
        ng = 0 if g is None else (1 if g.dim() == 1 else int(g.shape[0]))
        st = load().adc3_ea_davidson_guess(self.handle, nroots, conv, max_iter, max_subspace, precision,
                                           _ptr(g) if g is not None else None, ng, w,
                                           _ptr(vec) if vec is not None else None, rn, ctypes.byref(it), _stream())
        _check(st, allow_noconv=True)
        return np.array(w[:]), vec, np.array(rn[:]), it.value, st

    def set_sigma_graphs(self, on=True):
        """Replay sigma passes from captured HIP graphs (on a non-null stream)."""
        _check(load().adc3_ea_set_sigma_graphs(self.handle, 1 if on else 0))

    def set_preconditioner(self, weights):
        """Learned preconditioner for davidson() (float32 device weights; None: Jacobi)."""
        self._mlp_weights = weights
        _check(load().adc3_ea_set_preconditioner(self.handle, _ptrf(weights)))

    def precondition(self, theta, r):
        """(t, fallback): one preconditioning step on residual r (learned if set, else Jacobi)."""
        import torch
        t = torch.empty_like(r)
        fb = ctypes.c_int()
        _check(load().adc3_ea_precondition(self.handle, float(theta), _ptr(r.contiguous()), _ptr(t),
                                           ctypes.byref(fb), _stream()))
        return t, bool(fb.value)

    def mlp_collect(self, nroots, conv, group_size, max_groups, seed, max_iter=500):
        """Training groups from a Jacobi Davidson solve: (feat[G,S,6], a0[G,S], target[G,S], status)."""
        import torch
        F = torch.zeros((max_groups, group_size, 6), dtype=torch.float64, device="cuda")
        A = torch.zeros((max_groups, group_size), dtype=torch.float64, device="cuda")
        T = torch.zeros((max_groups, group_size), dtype=torch.float64, device="cuda")
        ng = ctypes.c_int()
        st = load().adc3_mlp_collect(self.handle, nroots, conv, max_iter, group_size, max_groups, seed, _ptr(F),
                                     _ptr(A), _ptr(T), ctypes.byref(ng), _stream())
        _check(st, allow_noconv=True)
        g = ng.value
        return F[:g], A[:g], T[:g], st

    def spectral_amplitudes(self, vecs):
        """x[nvec, nocc + nvir] = Y^T f (eqs 7-8) of device vectors vecs[nvec, N] in this basis."""
        import torch
        vecs = vecs.contiguous()
        n = 1 if vecs.dim() == 1 else int(vecs.shape[0])
        x = torch.empty((n, self.nocc + self.nvir), dtype=torch.float64, device="cuda")
        _check(load().adc3_ea_spectral_amplitudes(self.handle, _ptr(vecs), n, _ptr(x), _stream()))
        return x

    def dense(self):
        import torch
        M = torch.empty((self.N, self.N), dtype=torch.float64, device="cuda")
        _check(load().adc3_ea_dense_matrix(self.handle, _ptr(M), self.N, _stream()))
        return M

    def intermediate(self, which):
        import torch
        n = ctypes.c_longlong()
        _check(load().adc3_ea_intermediate(self.handle, which, None, ctypes.byref(n), _stream()))
        out = torch.empty(n.value, dtype=torch.float64, device="cuda")
        _check(load().adc3_ea_intermediate(self.handle, which, _ptr(out), None, _stream()))
        return out


adc3_ea_setup = Context


def adc3_debug_inject_nan(iteration):
    """Arm the error-path hook: the next Davidson iteration >= iteration writes NaN into one sigma vector."""
    load().adc3_debug_inject_nan(int(iteration))


def adc3_debug_ladder_offset_limit(nbytes):
    """Test hook: byte limit of one k-major ladder chunk's operand span (0 restores 2^31 - 1)."""
    load().adc3_debug_ladder_offset_limit(int(nbytes))


def adc3_mlp_nparams():
    return load().adc3_mlp_nparams()


def adc3_mlp_workspace_bytes(batch_groups, group_size):
    return load().adc3_mlp_workspace_bytes(batch_groups, group_size)


def adc3_mlp_loss_grad(weights, feat, a0, target, want_grad=True):
    """(loss, grad[nparams] float64 device tensor or None) for groups feat[G,S,6], a0/target[G,S]."""
    import torch
    G, S = int(a0.shape[0]), int(a0.shape[1])
    ws = _workspace(adc3_mlp_workspace_bytes(G, S))
    grad = torch.empty(adc3_mlp_nparams(), dtype=torch.float64, device="cuda") if want_grad else None
    loss = ctypes.c_double()
    _check(load().adc3_mlp_loss_grad(_ptrf(weights), _ptr(feat.contiguous()), _ptr(a0.contiguous()),
                                     _ptr(target.contiguous()), G, S, _ptr(grad), ctypes.byref(loss),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return loss.value, grad


def adc3_mlp_forward(weights, feat):
    """u[n] = MLP(feat[n,6]) as in training (FP32 matrix cores)."""
    import torch
    n = int(feat.shape[0])
    ws = _workspace(adc3_mlp_workspace_bytes(1, n))
    u = torch.empty(n, dtype=torch.float64, device="cuda")
    _check(load().adc3_mlp_forward(_ptrf(weights), _ptr(feat.contiguous()), n, _ptr(u),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return u


def adc3_mlp_train(weights, feat, a0, target, epochs, batch_groups, lr, seed):
    """Adam training in place on float32 device weights; returns the mean loss of every epoch."""
    G, S = int(a0.shape[0]), int(a0.shape[1])
    b = min(batch_groups, G)
    ws = _workspace(adc3_mlp_workspace_bytes(b, S))
    losses = (ctypes.c_double * epochs)()
    _check(load().adc3_mlp_train(_ptrf(weights), _ptr(feat.contiguous()), _ptr(a0.contiguous()),
                                 _ptr(target.contiguous()), G, S, epochs, b, float(lr), seed, losses,
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return np.array(losses[:])


PROF_LADDER, PROF_SIGMA, PROF_SETUP, PROF_DAVIDSON, PROF_EIG, PROF_LADDER_LP = range(6)


def adc3_profile_enable(on=True):
    load().adc3_profile_enable(1 if on else 0)


def adc3_profile_query(kernel):
    """(total_ms, launches, flops, bytes) recorded for a timing id since the last enable."""
    ms, n, f, b = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
    _check(load().adc3_profile_query(kernel, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(f), ctypes.byref(b)))
    return ms.value, n.value, f.value, b.value


def adc3_profile_query_bound(kernel):
    """Summed roofline time (ms) of the timed launches of a ladder id."""
    b = ctypes.c_double()
    _check(load().adc3_profile_query_bound(kernel, ctypes.byref(b)))
    return b.value
