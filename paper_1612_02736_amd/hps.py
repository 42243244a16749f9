"""ctypes binding of libhps.so (argument marshalling only).

Every step of the build and solve runs in the library's HIP kernels; this
module converts arguments (torch device tensors -> pointers, host arrays ->
numpy) and raises on error codes.  There is no fallback: a missing library
or a CPU tensor is an error.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhps.so")

HPS_PREC_FP64, HPS_PREC_MIXED, HPS_PREC_FP32 = 0, 1, 2
HPS_SOLVE_NOALLOC_MAX_BYTES = 256 << 20      # size of the fixed work array (hps.h)
HPS_BC_DIRICHLET, HPS_BC_NEUMANN, HPS_BC_PERIODIC = 0, 1, 2
_BC_CODES = {"D": HPS_BC_DIRICHLET, "N": HPS_BC_NEUMANN, "P": HPS_BC_PERIODIC}
_ERRS = {-1: "HPS_EINVAL", -2: "HPS_ETREE", -3: "HPS_ESINGULAR",
         -4: "HPS_ENONFINITE", -5: "HPS_ENOCONV", -6: "HPS_EHIP", -7: "HPS_ENOMEM"}

EXPORTS = ["hps_tree_uniform", "hps_tree_refine_point", "hps_tree_set_bc", "hps_tree_info",
           "hps_tree_counts", "hps_leaf_cheb_nodes", "hps_leaf_boxes",
           "hps_bdry_gauss_nodes", "hps_gauss_nodes", "hps_tree_free",
           "hps_build", "hps_refactor", "hps_build_workspace_size", "hps_solve",
           "hps_solve_noalloc",
           "hps_solve_adjoint", "hps_coeff_grad_c", "hps_apply_operator",
           "hps_handle_free", "hps_last_error"]


class HPSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRS.get(code, code)}: {msg}")
        self.code = code


class TreeInfo(ctypes.Structure):
    _fields_ = [("n_problems", ctypes.c_int), ("n_leaves", ctypes.c_int),
                ("n_boxes", ctypes.c_int), ("n_levels", ctypes.c_int),
                ("max_depth", ctypes.c_int)]


class BuildOpts(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("keep_fp32", ctypes.c_int), ("economic", ctypes.c_int),
                ("translation_invariant", ctypes.c_int), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("ir_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("u_gauss", ctypes.c_void_p), ("iters_out", ctypes.c_void_p),
                ("resid_out", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libhps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_1612_02736_amd.build_lib")
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.hps_tree_uniform.argtypes = [dp, dp, dp, dp, ip, ip, ip, ctypes.POINTER(vp)]
    L.hps_tree_refine_point.argtypes = [vp, ip, dp, dp, ip, dp]
    L.hps_tree_set_bc.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int)]
    L.hps_tree_info.argtypes = [vp, ctypes.POINTER(TreeInfo)]
    L.hps_tree_counts.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64)]
    L.hps_leaf_cheb_nodes.argtypes = [vp, ip, vp]
    L.hps_leaf_boxes.argtypes = [vp, vp]
    L.hps_bdry_gauss_nodes.argtypes = [vp, ip, vp]
    L.hps_gauss_nodes.argtypes = [vp, ip, vp]
    L.hps_tree_free.argtypes = [vp]
    L.hps_tree_free.restype = None
    L.hps_build.argtypes = [vp, vp, ip, ctypes.POINTER(BuildOpts), ctypes.POINTER(vp)]
    L.hps_refactor.argtypes = [vp, vp, vp]
    L.hps_build_workspace_size.argtypes = [vp, ip, ctypes.POINTER(BuildOpts)]
    L.hps_build_workspace_size.restype = ctypes.c_size_t
    L.hps_solve.argtypes = [vp, vp, vp, ip, vp, ctypes.POINTER(SolveOpts)]
    L.hps_solve_noalloc.argtypes = [vp, vp, vp, ip, vp, ctypes.POINTER(SolveOpts)]
    L.hps_solve_adjoint.argtypes = [vp, vp, ip, vp, vp, ctypes.POINTER(SolveOpts)]
    L.hps_coeff_grad_c.argtypes = [vp, vp, vp, ip, vp, vp]
    L.hps_apply_operator.argtypes = [vp, vp, ip, dp, vp, vp]
    L.hps_handle_free.argtypes = [vp]
    L.hps_handle_free.restype = None
    L.hps_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise HPSError(rc, lib().hps_last_error().decode())


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _dev_ptr(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Tree:
    """A forest of rectangles split into leaf boxes (host object)."""

    def __init__(self, x0=0.0, x1=1.0, y0=0.0, y1=1.0, nx=1, ny=1, n_problems=1):
        h = ctypes.c_void_p()
        _check(lib().hps_tree_uniform(x0, x1, y0, y1, nx, ny, n_problems, ctypes.byref(h)))
        self._h = h

    def refine_point(self, problem, px, py, n_ref, t=np.sqrt(2.0)):
        _check(lib().hps_tree_refine_point(self._h, problem, px, py, n_ref, t))
        return self

    def set_bc(self, bc, problem=-1):
        """Side conditions of sides S, E, N, W: a string such as "NPNP" (D
        Dirichlet, N Neumann, P periodic) or four HPS_BC_* codes;
        problem=-1: every problem."""
        codes = [_BC_CODES[c] if isinstance(c, str) else int(c) for c in bc]
        if len(codes) != 4:
            raise ValueError("bc needs four sides")
        arr = (ctypes.c_int * 4)(*codes)
        _check(lib().hps_tree_set_bc(self._h, problem, arr))
        return self

    def info(self):
        i = TreeInfo()
        _check(lib().hps_tree_info(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in TreeInfo._fields_}

    @property
    def n_leaves(self):
        return self.info()["n_leaves"]

    def counts(self, q):
        ng, nb = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().hps_tree_counts(self._h, q, ctypes.byref(ng), ctypes.byref(nb)))
        return ng.value, nb.value

    def leaf_cheb_nodes(self, p):
        out = np.empty((self.n_leaves, p * p, 2))
        _check(lib().hps_leaf_cheb_nodes(self._h, p, _np_ptr(out)))
        return out

    def leaf_boxes(self):
        out = np.empty((self.n_leaves, 4))
        _check(lib().hps_leaf_boxes(self._h, _np_ptr(out)))
        return out

    def bdry_gauss_nodes(self, q):
        _, nb = self.counts(q)
        out = np.empty((nb, 2))
        _check(lib().hps_bdry_gauss_nodes(self._h, q, _np_ptr(out)))
        return out

    def gauss_nodes(self, q):
        ng, _ = self.counts(q)
        out = np.empty((ng, 2))
        _check(lib().hps_gauss_nodes(self._h, q, _np_ptr(out)))
        return out

    def workspace_bytes(self, p, q=0, economic=False, translation_invariant=False):
        """Device bytes of the operators a build stores (economic: without
        the leaf F, the storage-efficient version of Sec. 5.4;
        translation_invariant: one copy per distinct box)."""
        o = BuildOpts(q=q, economic=int(economic),
                      translation_invariant=int(translation_invariant))
        return lib().hps_build_workspace_size(self._h, p, ctypes.byref(o))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hps_tree_free(self._h)
            self._h = None


class Solver:
    """Handle of a built solution operator (Algorithm 1)."""

    def __init__(self, tree, coeffs, p, q=0, keep_fp32=False, economic=False,
                 translation_invariant=False, stream=None, workspace=None):
        """workspace: None (the library allocates the operator memory), True
        (a torch uint8 tensor of tree.workspace_bytes(...) bytes, owned by this
        Solver) or a contiguous CUDA tensor of at least that many bytes, which
        the Solver keeps alive."""
        import torch
        self.tree, self.p = tree, p
        self.q = q if q > 0 else p - 1
        self.n_leaves = tree.n_leaves
        self.n_gauss, self.n_bdry = tree.counts(self.q)
        if tuple(coeffs.shape) != (self.n_leaves, 6, p * p):
            raise ValueError(f"coeffs must be [{self.n_leaves}, 6, {p * p}]")
        self.workspace = None
        wp, wb = None, 0
        if workspace is not None and workspace is not False:
            if workspace is True:
                need = tree.workspace_bytes(p, self.q, economic, translation_invariant)
                workspace = torch.empty(need, dtype=torch.uint8, device=coeffs.device)
            if not (isinstance(workspace, torch.Tensor) and workspace.is_cuda
                    and workspace.is_contiguous()):
                raise TypeError("workspace must be a contiguous CUDA tensor")
            self.workspace = workspace
            wp, wb = ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
        o = BuildOpts(q=self.q, stream=_stream(stream), keep_fp32=int(keep_fp32),
                      economic=int(economic),
                      translation_invariant=int(translation_invariant),
                      workspace=wp, workspace_bytes=wb)
        h = ctypes.c_void_p()
        _check(lib().hps_build(tree._h, _dev_ptr(coeffs, "coeffs"), p, ctypes.byref(o),
                               ctypes.byref(h)))
        self._h = h
        self.device = coeffs.device
        self._torch = torch
        # counts refactorizations, so holders of earlier operators can tell
        self.version = 0

    def refactor(self, coeffs, stream=None):
        """Algorithm 1 again for new coefficients, reusing the device memory."""
        if tuple(coeffs.shape) != (self.n_leaves, 6, self.p * self.p):
            raise ValueError("coeffs has the wrong shape")
        self.version += 1
        _check(lib().hps_refactor(self._h, _dev_ptr(coeffs, "coeffs"), _stream(stream)))

    def solve(self, f, g, precision=HPS_PREC_FP64, ir_tol=1e-10, max_iter=0,
              u_gauss=False, stream=None, stats=None):
        """f: [nrhs, n_bdry], g: [nrhs, n_leaves, (p-2)^2] -> u [nrhs, n_leaves, p^2]."""
        torch = self._torch
        nrhs = f.shape[0]
        if tuple(f.shape) != (nrhs, self.n_bdry):
            raise ValueError("f has the wrong shape")
        if tuple(g.shape) != (nrhs, self.n_leaves, (self.p - 2) ** 2):
            raise ValueError("g has the wrong shape")
        u = torch.empty((nrhs, self.n_leaves, self.p * self.p), dtype=torch.float64,
                        device=self.device)
        ug = None
        if u_gauss:
            ug = torch.empty((nrhs, self.n_gauss), dtype=torch.float64, device=self.device)
        iters = ctypes.c_int(0)
        res = ctypes.c_double(0.0)
        o = SolveOpts(precision=precision, ir_tol=ir_tol, max_iter=max_iter,
                      stream=_stream(stream),
                      u_gauss=ctypes.c_void_p(ug.data_ptr()) if ug is not None else None,
                      iters_out=ctypes.cast(ctypes.pointer(iters), ctypes.c_void_p),
                      resid_out=ctypes.cast(ctypes.pointer(res), ctypes.c_void_p))
        _check(lib().hps_solve(self._h, _dev_ptr(f, "f"), _dev_ptr(g, "g"), nrhs,
                               _dev_ptr(u, "u"), ctypes.byref(o)))
        if stats is not None:
            stats["iters"] = iters.value
            stats["resid"] = res.value
        return (u, ug) if u_gauss else u

    def solve_noalloc(self, f, g, u, precision=HPS_PREC_FP64, stream=None):
        """hps_solve_noalloc: Algorithm 2 into the caller's u [nrhs, n_leaves, p^2],
        with the library's fixed work array (no device allocation)."""
        nrhs = f.shape[0]
        if tuple(f.shape) != (nrhs, self.n_bdry):
            raise ValueError("f has the wrong shape")
        if tuple(g.shape) != (nrhs, self.n_leaves, (self.p - 2) ** 2):
            raise ValueError("g has the wrong shape")
        if tuple(u.shape) != (nrhs, self.n_leaves, self.p * self.p):
            raise ValueError("u has the wrong shape")
        o = SolveOpts(precision=precision, stream=_stream(stream))
        _check(lib().hps_solve_noalloc(self._h, _dev_ptr(f, "f"), _dev_ptr(g, "g"), nrhs,
                                       _dev_ptr(u, "u"), ctypes.byref(o)))
        return u

    def solve_adjoint(self, ubar, stream=None):
        """ubar: [nrhs, n_leaves, p^2] -> (fbar [nrhs, n_bdry], gbar [nrhs, n_leaves, mi])."""
        torch = self._torch
        nrhs = ubar.shape[0]
        fb = torch.empty((nrhs, self.n_bdry), dtype=torch.float64, device=self.device)
        gb = torch.empty((nrhs, self.n_leaves, (self.p - 2) ** 2), dtype=torch.float64,
                         device=self.device)
        o = SolveOpts(precision=HPS_PREC_FP64, stream=_stream(stream))
        _check(lib().hps_solve_adjoint(self._h, _dev_ptr(ubar, "ubar"), nrhs,
                                       _dev_ptr(fb, "fbar"), _dev_ptr(gb, "gbar"),
                                       ctypes.byref(o)))
        return fb, gb

    def apply_operator(self, u, sigma, stream=None):
        """sigma u - A u at the interior nodes: u [nrhs, n_leaves, p^2] ->
        [nrhs, n_leaves, (p-2)^2] (the right side of an implicit step)."""
        torch = self._torch
        nrhs = u.shape[0]
        if tuple(u.shape) != (nrhs, self.n_leaves, self.p * self.p):
            raise ValueError("u has the wrong shape")
        out = torch.empty((nrhs, self.n_leaves, (self.p - 2) ** 2), dtype=torch.float64,
                          device=self.device)
        _check(lib().hps_apply_operator(self._h, _dev_ptr(u, "u"), nrhs, float(sigma),
                                        _dev_ptr(out, "out"), _stream(stream)))
        return out

    def coeff_grad_c(self, u, gbar, stream=None):
        torch = self._torch
        nrhs = u.shape[0]
        cb = torch.empty_like(u)
        _check(lib().hps_coeff_grad_c(self._h, _dev_ptr(u, "u"), _dev_ptr(gbar, "gbar"),
                                      nrhs, _dev_ptr(cb, "cbar"), _stream(stream)))
        return cb

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hps_handle_free(self._h)
            self._h = None


# -- test hooks (include/hps_debug.h) ----------------------------------------
def _debug_lib():
    L = lib()
    if not hasattr(L, "_dbg"):
        vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.hps_debug_gemm.argtypes = [ip, ip, ip, dp, vp, ip, vp, ip, vp, ip, vp]
        L.hps_debug_invert.argtypes = [ip, ip, vp, vp, vp]
        L.hps_debug_gemm_variant.argtypes = [ip, ip, ip, ip, dp, vp, ip, vp, ip, vp, ip, vp]
        L.hps_debug_gemm_choices.argtypes = [vp, vp, ip, ctypes.POINTER(ctypes.c_int)]
        L.hps_debug_solve_work_bytes.argtypes = [vp, ip]
        L.hps_debug_solve_work_bytes.restype = ctypes.c_size_t
        L.hps_debug_boxes.argtypes = [vp, ctypes.POINTER(ctypes.c_int), vp]
        L.hps_debug_box_nodes.argtypes = [vp, ip, ip, vp]
        L.hps_debug_box_op.argtypes = [vp, ip, ip, vp, ctypes.POINTER(ctypes.c_int64)]
        L._dbg = True
    return L


def debug_gemm(A, B, alpha=1.0, variant=0):
    """C = alpha A B on the library's MFMA GEMM (column-major device copies),
    tile variant `variant`."""
    import torch
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    Ad = A.t().contiguous()          # column-major storage of A
    Bd = B.t().contiguous()
    C = torch.empty((N, M), dtype=torch.float64, device=A.device)
    _check(_debug_lib().hps_debug_gemm_variant(variant, M, N, K, alpha, _dev_ptr(Ad, "A"), M,
                                               _dev_ptr(Bd, "B"), K, _dev_ptr(C, "C"), M,
                                               _stream(None)))
    return C.t()


def debug_gemm_choices(solver):
    """Tile variant the tuner chose for each GEMM step of the build program."""
    L = _debug_lib()
    n = ctypes.c_int()
    _check(L.hps_debug_gemm_choices(solver._h, None, 0, ctypes.byref(n)))
    out = np.zeros(n.value, dtype=np.int32)
    _check(L.hps_debug_gemm_choices(solver._h, _np_ptr(out), n.value, ctypes.byref(n)))
    return [int(v) for v in out]


def debug_invert(A):
    """Batch of n x n inverses by the build's Gauss-Jordan kernels."""
    import torch
    b, n, _ = A.shape
    Ad = A.transpose(1, 2).contiguous()
    X = torch.empty_like(Ad)
    _check(_debug_lib().hps_debug_invert(n, b, _dev_ptr(Ad, "A"), _dev_ptr(X, "X"), _stream(None)))
    return X.transpose(1, 2)


def debug_solve_work_bytes(solver, nrhs):
    """Bytes of solve work memory nrhs right-hand sides take on this handle."""
    return int(_debug_lib().hps_debug_solve_work_bytes(solver._h, nrhs))


def debug_boxes(solver):
    L = _debug_lib()
    n = ctypes.c_int()
    _check(L.hps_debug_boxes(solver._h, ctypes.byref(n), None))
    out = np.empty((n.value, 8), dtype=np.int32)
    _check(L.hps_debug_boxes(solver._h, ctypes.byref(n), _np_ptr(out)))
    return out


def debug_box_nodes(solver, box, which):
    info = debug_boxes(solver)[box]
    cnt = {0: info[5], 1: info[6], 2: info[7]}[which]
    out = np.empty(cnt, dtype=np.int64)
    _check(_debug_lib().hps_debug_box_nodes(solver._h, box, which, _np_ptr(out)))
    return out


def debug_box_op(solver, box, which, shape):
    L = _debug_lib()
    cnt = ctypes.c_int64()
    _check(L.hps_debug_box_op(solver._h, box, which, None, ctypes.byref(cnt)))
    out = np.empty(cnt.value)
    _check(L.hps_debug_box_op(solver._h, box, which, _np_ptr(out), ctypes.byref(cnt)))
    return out.reshape(shape, order="F")


PROFILE_KINDS = {0: "gemm", 1: "gj_leaf", 2: "gj_interface", 3: "interface_diff",
                 4: "gj_panel", 5: "gj_colperm", 6: "apply", 9: "leaf_b"}


def debug_profile(solver, enable=True):
    L = _debug_lib()
    if not hasattr(L, "_prof"):
        L.hps_debug_profile.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.hps_debug_profile_read.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int)]
        L._prof = True
    _check(L.hps_debug_profile(solver._h, int(enable)))


def debug_profile_read(solver, max_n=100000, with_work=False):
    """[(kind, variant, ms)] of every launch step since the last read, or
    [(kind, variant, ms, work)] with the launch's algorithmic work (flops, or
    operator elements per right-hand side for applies)."""
    L = _debug_lib()
    kinds = np.zeros(max_n, dtype=np.int32)
    ms = np.zeros(max_n)
    work = np.zeros(max_n)
    n = ctypes.c_int()
    _check(L.hps_debug_profile_read(solver._h, _np_ptr(kinds), _np_ptr(ms), _np_ptr(work), max_n,
                                    ctypes.byref(n)))
    k = min(n.value, max_n)
    out = []
    for i in range(k):
        t = (PROFILE_KINDS.get(int(kinds[i]) // 16, "?"), int(kinds[i]) % 16, float(ms[i]))
        out.append(t + (float(work[i]),) if with_work else t)
    return out
