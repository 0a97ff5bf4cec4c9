"""Python binding of libnmodes (ctypes): argument marshalling only.

Every computation runs in the HIP library (include/nmodes.h).  torch is
imported first so that the library binds to the HIP runtime torch loaded;
device arrays are torch tensors on the current device and the library runs
on torch's current stream.  If the library is not built the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:
    import torch
except ImportError:  # pragma: no cover - the GPU path needs torch
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmodes.so")

NM_OK, NM_PARTIAL = 0, 1
MAT_AG, MAT_M, MAT_R, MAT_KP, MAT_EG = range(5)
OP_AG, OP_M, OP_R, OP_KP, OP_EG, OP_EGT, OP_KPINV, OP_A, OP_MINV, OP_B = range(10)

EXPORTED = ["nm_assemble", "nm_pencil_info_get", "nm_pencil_export_csr", "nm_pencil_nodes", "nm_pencil_apply",
            "nm_filter_coeffs", "nm_filter_degree", "nm_filter_apply", "nm_spectrum_bounds", "nm_filtered_eig",
            "nm_filtered_eig_slices", "nm_project_rotation", "nm_pencil_autotune", "nm_server_create",
            "nm_server_submit", "nm_server_wait", "nm_server_result_free", "nm_server_destroy",
            "nm_result_copy_vectors", "nm_rot_copy_vectors", "nm_result_free", "nm_rot_result_free",
            "nm_pencil_free", "nm_last_error", "nm_version", "nm_set_allocator", "nm_max_block_columns", "nm_pencil_apply_noalloc",
            "nm_spectrum_dos", "nm_dos_count", "nm_dos_slices", "nm_spectrum_dos_weighted", "nm_dos_count_weighted",
            "nm_dos_slices_weighted", "nm_spectrum_bound_rigorous", "nm_refine_rotation",
            "nm_selfgrav_build", "nm_selfgrav_info", "nm_selfgrav_apply", "nm_selfgrav_field",
            "nm_pencil_attach_selfgrav", "nm_selfgrav_free", "nm_gemm_tn", "nm_gemm_nn"]


class NMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("nmodes status %d: %s" % (status, msg))
        self.status = status


class _Mesh(C.Structure):
    _fields_ = [("n_vert", C.c_int64), ("n_tet", C.c_int64), ("xyz", C.c_void_p), ("tet", C.c_void_p),
                ("region", C.c_void_p), ("disp_order", C.c_int32), ("pres_order", C.c_int32)]


class _Material(C.Structure):
    _fields_ = [("rho", C.c_void_p), ("lam", C.c_void_p), ("mu", C.c_void_p), ("gprime", C.c_void_p),
                ("grad_gprime", C.c_void_p), ("gprime_np", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("n_geom", C.c_int64), ("n_node", C.c_int64), ("n_solid", C.c_int64), ("n_disp", C.c_int64),
                ("n_pres", C.c_int64), ("nnzb", C.c_int64), ("nnz_kp", C.c_int64), ("nnzb_eg", C.c_int64),
                ("n_fs_faces", C.c_int64), ("minv_lo", C.c_double), ("minv_hi", C.c_double),
                ("kp_lo", C.c_double), ("kp_hi", C.c_double)]


class _ApplyOpts(C.Structure):
    _fields_ = [("kM", C.c_int32), ("kP", C.c_int32), ("minv_tol", C.c_double), ("kp_tol", C.c_double),
                ("precision", C.c_int32), ("mass_passes", C.c_int32)]


class _EigOpts(C.Structure):
    _fields_ = [("degree", C.c_int32), ("block", C.c_int32), ("precision", C.c_int32), ("max_basis", C.c_int32),
                ("null_filter", C.c_int32), ("verbose", C.c_int32), ("minv_tol", C.c_double),
                ("kp_tol", C.c_double), ("lmin", C.c_double), ("lmax", C.c_double), ("guard", C.c_double),
                ("seed", C.c_uint64), ("stream", C.c_void_p), ("refine", C.c_int32), ("mass_passes", C.c_int32)]


class _EigResult(C.Structure):
    _fields_ = [("count", C.c_int32), ("n", C.c_int64), ("lam", C.POINTER(C.c_double)),
                ("resid", C.POINTER(C.c_double)), ("X", C.c_void_p), ("degree", C.c_int32), ("kM", C.c_int32),
                ("kP", C.c_int32), ("block", C.c_int32), ("basis", C.c_int32), ("bapps", C.c_int64),
                ("lmin", C.c_double), ("lmax", C.c_double), ("seconds", C.c_double), ("bytes", C.c_double),
                ("filter_seconds", C.c_double), ("hot_launches", C.c_int64), ("hot_samples", C.c_int64),
                ("hot_ms", C.c_double), ("hot_bytes", C.c_double), ("refine_passes", C.c_int32),
                ("refine_degree", C.c_int32), ("refine_seconds", C.c_double), ("refine_bapps", C.c_int64),
                ("mass_passes", C.c_int32), ("mass_pass_steps", C.c_int32), ("hot_kernel", C.c_int32)]


class _RotResult(C.Structure):
    _fields_ = [("count", C.c_int32), ("n", C.c_int64), ("omega", C.POINTER(C.c_double)), ("U", C.c_void_p),
                ("seconds", C.c_double), ("resid", C.POINTER(C.c_double)), ("iters", C.c_int32),
                ("basis", C.c_int32), ("degree", C.c_int32)]


class _Request(C.Structure):
    _fields_ = [("mesh", _Mesh), ("material", _Material), ("omega", C.c_double * 3), ("nslices", C.c_int32),
                ("a", C.c_void_p), ("b", C.c_void_p), ("nev", C.c_void_p), ("tol", C.c_double),
                ("opts", _EigOpts), ("rotate", C.c_int32)]


class _ServerResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("error", C.c_char * 256), ("nslices", C.c_int32),
                ("slices", C.POINTER(C.POINTER(_EigResult))), ("rotation", C.POINTER(_RotResult)),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_end", C.c_double),
                ("est_bytes", C.c_double)]


_lib = None

# device allocator callbacks of nm_set_allocator
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
# every installed pair stays alive: memory it allocated is freed through it later
_allocator_refs = []


def library_path() -> str:
    return LIB_PATH


def load_library(path: str | None = None):
    """Load libnmodes.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError("libnmodes.so is not built: run paper_1906_11082_amd.build.build()")
    lib = C.CDLL(path)
    P = C.c_void_p
    sig = {
        "nm_assemble": ([C.POINTER(_Mesh), C.POINTER(_Material), P, P, C.POINTER(P)], C.c_int32),
        "nm_pencil_info_get": ([P, C.POINTER(_Info)], C.c_int32),
        "nm_pencil_export_csr": ([P, C.c_int32] + [C.POINTER(C.c_int64)] * 3 + [P, P, P], C.c_int32),
        "nm_pencil_nodes": ([P, P, P], C.c_int32),
        "nm_pencil_apply": ([P, C.c_int32, C.c_int32, P, P, C.POINTER(_ApplyOpts), P], C.c_int32),
        "nm_filter_coeffs": ([C.c_double] * 4 + [C.c_int32, P], C.c_int32),
        "nm_filter_degree": ([C.c_double] * 5 + [C.c_int32, C.POINTER(C.c_int32)], C.c_int32),
        "nm_filter_apply": ([P, P, C.c_int32] + [C.c_double] * 4 + [C.c_int32, P, P, C.POINTER(_ApplyOpts), P],
                            C.c_int32),
        "nm_spectrum_bounds": ([P, C.c_int32, C.c_uint64, P, C.POINTER(C.c_double), C.POINTER(C.c_double)],
                               C.c_int32),
        "nm_filtered_eig": ([P, C.c_double, C.c_double, C.c_int32, C.c_double, C.POINTER(_EigOpts),
                             C.POINTER(C.POINTER(_EigResult))], C.c_int32),
        "nm_pencil_autotune": ([P, C.c_int32, P, C.POINTER(C.c_int32), C.POINTER(C.c_double)], C.c_int32),
        "nm_server_create": ([C.c_double, C.c_int32, C.POINTER(C.c_void_p)], C.c_int32),
        "nm_server_submit": ([P, C.POINTER(_Request), C.POINTER(C.c_int64)], C.c_int32),
        "nm_server_wait": ([P, C.c_int64, C.POINTER(C.POINTER(_ServerResult))], C.c_int32),
        "nm_server_result_free": ([C.POINTER(_ServerResult)], None),
        "nm_server_destroy": ([P], C.c_int32),
        "nm_filtered_eig_slices": ([P, C.c_int32, P, P, P, C.c_double, C.POINTER(_EigOpts),
                                    C.POINTER(C.POINTER(_EigResult))], C.c_int32),
        "nm_project_rotation": ([P, C.POINTER(_EigResult), C.c_double, C.c_double, P,
                                 C.POINTER(C.POINTER(_RotResult))], C.c_int32),
        "nm_result_copy_vectors": ([C.POINTER(_EigResult), P, C.c_int32], C.c_int32),
        "nm_rot_copy_vectors": ([C.POINTER(_RotResult), P, C.c_int32], C.c_int32),
        "nm_result_free": ([C.POINTER(_EigResult)], None),
        "nm_rot_result_free": ([C.POINTER(_RotResult)], None),
        "nm_pencil_free": ([P], None),
        "nm_last_error": ([], C.c_char_p),
        "nm_version": ([], C.c_char_p),
        "nm_set_allocator": ([_ALLOC_FN, _FREE_FN, P], C.c_int32),
        "nm_max_block_columns": ([C.c_int64, C.POINTER(C.c_int64)], C.c_int32),
        "nm_pencil_apply_noalloc": ([P, C.c_int32, C.c_int32, P, P, C.POINTER(_ApplyOpts), P], C.c_int32),
        "nm_selfgrav_build": ([P, C.POINTER(_Mesh), C.POINTER(_Material), C.c_double, P, C.POINTER(P)], C.c_int32),
        "nm_selfgrav_info": ([P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64), P], C.c_int32),
        "nm_selfgrav_apply": ([P, C.c_int32, P, P, P], C.c_int32),
        "nm_selfgrav_field": ([P, C.c_int64, P, P, P], C.c_int32),
        "nm_pencil_attach_selfgrav": ([P, P], C.c_int32),
        "nm_selfgrav_free": ([P], None),
        "nm_refine_rotation": ([P, C.POINTER(_EigResult), C.POINTER(_RotResult), C.c_double, C.c_double, C.c_int32,
                                C.c_int32, C.c_double, P, C.POINTER(C.POINTER(_RotResult))], C.c_int32),
        "nm_spectrum_dos": ([P, C.c_double, C.c_double, C.c_int32, C.c_int32, P, C.POINTER(_ApplyOpts), P, P],
                            C.c_int32),
        "nm_dos_count": ([P, C.c_int32] + [C.c_double] * 4 + [C.POINTER(C.c_double)], C.c_int32),
        "nm_dos_slices": ([P, C.c_int32] + [C.c_double] * 4 + [C.c_int32, P], C.c_int32),
        "nm_spectrum_dos_weighted": ([P, C.c_double, C.c_double, C.c_int32, C.c_int32, P, C.POINTER(_ApplyOpts), P,
                                      P], C.c_int32),
        "nm_dos_count_weighted": ([P, C.c_int32] + [C.c_double] * 4 + [C.POINTER(C.c_double)], C.c_int32),
        "nm_dos_slices_weighted": ([P, C.c_int32] + [C.c_double] * 4 + [C.c_int32, P], C.c_int32),
        "nm_spectrum_bound_rigorous": ([P, P, C.POINTER(C.c_double)], C.c_int32),
        "nm_gemm_tn": ([C.c_int64, C.c_int32, C.c_int32, P, C.c_int32, P, C.c_int32, P, P], C.c_int32),
        "nm_gemm_nn": ([C.c_int64, C.c_int32, C.c_int32, C.c_double, P, C.c_int32, P, C.c_int32, C.c_double, P,
                        C.c_int32, P], C.c_int32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(st, partial_ok=False):
    if st == NM_OK or (partial_ok and st == NM_PARTIAL):
        return st
    raise NMError(st, _lib.nm_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else C.c_void_p(a.data_ptr())


def _rows(a, name):
    if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64 and a.dim() == 2
            and (a.shape[1] <= 1 or a.stride(1) == 1)):
        raise ValueError("%s: a 2-D float64 CUDA tensor with contiguous rows" % name)
    return max(a.stride(0), a.shape[1]) if a.shape[0] <= 1 else a.stride(0)


def gemm_tn(A, B, K=None, q=None):
    """C = A[:, :K]^T B[:, :q] (K x q) through nm_gemm_tn, the solver's block
    product on the FP64 matrix cores.  A, B: float64 CUDA tensors [n][*] with
    contiguous rows (leading dimensions from their row strides)."""
    lib = load_library()
    lda, ldb = _rows(A, "A"), _rows(B, "B")
    if A.shape[0] != B.shape[0]:
        raise ValueError("A and B need the same number of rows")
    K = A.shape[1] if K is None else K
    q = B.shape[1] if q is None else q
    Ct = torch.empty((q, K), dtype=torch.float64, device=A.device)  # column-major K x q
    _check(lib.nm_gemm_tn(A.shape[0], K, q, _ptr(A), lda, _ptr(B), ldb, _ptr(Ct), _stream()))
    return Ct.t()


def gemm_nn(A, Cm, D=None, alpha=1.0, beta=0.0):
    """D = alpha A[:, :K] Cm + beta D through nm_gemm_nn (Cm: K x q, any
    layout; D: [n][q'] float64 CUDA tensor with contiguous rows, q' >= q,
    created when None).  Returns D."""
    lib = load_library()
    lda = _rows(A, "A")
    K, q = Cm.shape
    Cc = Cm.detach().to(device=A.device, dtype=torch.float64).t().contiguous()  # column-major K x q
    if D is None:
        D = torch.empty((A.shape[0], q), dtype=torch.float64, device=A.device)
    ldd = _rows(D, "D")
    if D.shape[0] != A.shape[0] or D.shape[1] < q:
        raise ValueError("D must be [n][>= q]")
    _check(lib.nm_gemm_nn(A.shape[0], K, q, float(alpha), _ptr(A), lda, _ptr(Cc), K, float(beta), _ptr(D), ldd,
                           _stream()))
    return D


def set_allocator(alloc=None, free=None):
    """Device buffers of the library through alloc(nbytes) -> device pointer
    (int, 256-byte aligned, 0 on failure) and free(pointer), called after a
    device synchronisation; both None restores hipMalloc / hipFree
    (nm_set_allocator).  Call it while no library call is in flight."""
    lib = load_library()
    if alloc is None and free is None:
        _check(lib.nm_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
        return
    if alloc is None or free is None:
        raise ValueError("set both allocator functions or neither")
    a = _ALLOC_FN(lambda nbytes, stream, ctx: alloc(int(nbytes)) or None)
    f = _FREE_FN(lambda ptr, stream, ctx: free(int(ptr)))
    _allocator_refs.append((a, f))
    _check(lib.nm_set_allocator(a, f, None))


def use_torch_allocator():
    """Device buffers of the library from torch's caching allocator, on the
    device current now."""
    dev = torch.cuda.current_device()
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, device=dev), torch.cuda.caching_allocator_delete)


def max_block_columns(n_disp):
    """Widest vector block (columns) the kernels accept for n_disp displacement rows."""
    lib = load_library()
    out = C.c_int64()
    _check(lib.nm_max_block_columns(int(n_disp), C.byref(out)))
    return out.value


def dos_count(tau, lmin, lmax, a, b, weighted=False):
    """Estimated eigenvalue count in [a, b] from density-of-states traces
    (nm_dos_count; weighted: traces of T_k B, nm_dos_count_weighted)."""
    lib = load_library()
    tau = np.ascontiguousarray(tau, np.float64)
    out = C.c_double()
    fn = lib.nm_dos_count_weighted if weighted else lib.nm_dos_count
    _check(fn(_ptr(tau), len(tau) - 1, lmin, lmax, a, b, C.byref(out)))
    return out.value


def dos_slices(tau, lmin, lmax, a, b, nslices, weighted=False):
    """Ends of nslices equal-count windows of [a, b] (nm_dos_slices, or
    nm_dos_slices_weighted for weighted traces)."""
    lib = load_library()
    tau = np.ascontiguousarray(tau, np.float64)
    edges = np.zeros(nslices + 1)
    fn = lib.nm_dos_slices_weighted if weighted else lib.nm_dos_slices
    _check(fn(_ptr(tau), len(tau) - 1, lmin, lmax, a, b, int(nslices), _ptr(edges)))
    return edges


def filter_coeffs(a, b, lmin, lmax, m):
    lib = load_library()
    mu = np.zeros(m + 1)
    _check(lib.nm_filter_coeffs(a, b, lmin, lmax, m, _ptr(mu)))
    return mu


def filter_degree(a, b, lmin, lmax, guard=1.0, mode=1):
    """mode 0: no damping below a; 1: damping below a; 2: null factor."""
    lib = load_library()
    m = C.c_int32()
    _check(lib.nm_filter_degree(a, b, lmin, lmax, guard, int(mode), C.byref(m)))
    return m.value


class EigResult:
    """Eigenpairs: lam (numpy, ascending), resid (numpy), X (torch, device,
    [n, count]) and solve statistics."""

    def __init__(self, ptr, keep_vectors=True):
        r = ptr.contents
        self.count = r.count
        self.lam = np.array([r.lam[i] for i in range(r.count)])
        self.resid = np.array([r.resid[i] for i in range(r.count)])
        self.stats = dict(degree=r.degree, kM=r.kM, kP=r.kP, block=r.block, basis=r.basis, bapps=r.bapps,
                          lmin=r.lmin, lmax=r.lmax, seconds=r.seconds, bytes=r.bytes,
                          filter_seconds=r.filter_seconds, hot_launches=r.hot_launches,
                          hot_samples=r.hot_samples, hot_ms=r.hot_ms, hot_bytes=r.hot_bytes,
                          refine_passes=r.refine_passes, refine_degree=r.refine_degree,
                          refine_seconds=r.refine_seconds, refine_bapps=r.refine_bapps,
                          mass_passes=r.mass_passes, mass_pass_steps=r.mass_pass_steps,
                          hot_kernel=("per-row", "row-group", "tile")[r.hot_kernel])
        self._ptr = ptr
        self.n = r.n
        self.X = None
        if keep_vectors and r.count:
            self.X = torch.empty((r.n, r.count), dtype=torch.float64, device="cuda")
            _check(_lib.nm_result_copy_vectors(ptr, _ptr(self.X), 1))

    def __del__(self):
        if getattr(self, "_ptr", None) is not None and _lib is not None:
            _lib.nm_result_free(self._ptr)
            self._ptr = None


class RotResult:
    """Rotating modes: omega (numpy, ascending), U (torch complex, device,
    [n, count]), resid (QEP residuals) and statistics.  An owned result keeps
    the library's copy (needed to refine it) until the object is released."""

    def __init__(self, ptr, owned=True):
        r = ptr.contents
        self.count = r.count
        self.omega = np.array([r.omega[i] for i in range(r.count)])
        self.resid = np.array([r.resid[i] for i in range(r.count)]) if r.resid else None
        self.seconds = r.seconds
        self.iters, self.basis, self.degree = r.iters, r.basis, r.degree
        self.U = None
        if r.count:
            buf = torch.empty((r.n, r.count, 2), dtype=torch.float64, device="cuda")
            _check(_lib.nm_rot_copy_vectors(ptr, _ptr(buf), 1))
            self.U = torch.view_as_complex(buf)
        self._ptr = ptr if owned else None

    def __del__(self):
        if getattr(self, "_ptr", None) is not None and _lib is not None:
            _lib.nm_rot_result_free(self._ptr)
            self._ptr = None


def _planet_structs(planet: dict, omega=None):
    """nm_mesh / nm_material views of a planet dict (arrays kept alive in `keep`)."""
    xyz = np.ascontiguousarray(planet["xyz"], np.float64)
    tet = np.ascontiguousarray(planet["tet"], np.int32)
    reg = np.ascontiguousarray(planet["region"], np.int8)
    order, porder = int(planet["disp_order"]), int(planet["pres_order"])
    rho = np.ascontiguousarray(planet["rho"], np.float64)
    lam = np.ascontiguousarray(planet["lam"], np.float64)
    mu = np.ascontiguousarray(planet["mu"], np.float64)
    gp, dgp = planet.get("gprime"), planet.get("grad_gprime")
    mesh = _Mesh(len(xyz), len(tet), _ptr(xyz), _ptr(tet), _ptr(reg), order, porder)
    keep = [xyz, tet, reg, rho, lam, mu]
    if gp is not None:
        gp = np.ascontiguousarray(gp, np.float64)
        dgp = np.ascontiguousarray(dgp, np.float64)
        keep += [gp, dgp]
        mat = _Material(_ptr(rho), _ptr(lam), _ptr(mu), _ptr(gp), _ptr(dgp), gp.shape[1])
    else:
        mat = _Material(_ptr(rho), _ptr(lam), _ptr(mu), None, None, 0)
    om = np.ascontiguousarray(planet.get("omega", (0, 0, 0)) if omega is None else omega, np.float64)
    keep.append(om)
    return mesh, mat, om, keep


class Pencil:
    """Device-resident pencil of one planet (A_G, M, R, K_p, E_G)."""

    def __init__(self, planet: dict, omega=None):
        lib = load_library()
        mesh, mat, om, keep = _planet_structs(planet, omega)
        h = C.c_void_p()
        _check(lib.nm_assemble(C.byref(mesh), C.byref(mat), _ptr(om), _stream(), C.byref(h)))
        self._h = h
        info = _Info()
        _check(lib.nm_pencil_info_get(h, C.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _Info._fields_}
        self.n = self.info["n_disp"]
        self.n_p = self.info["n_pres"]
        self.N = self.info["n_node"]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.nm_pencil_free(self._h)
            self._h = None

    def export_csr(self, which):
        nr, nc, nnz = C.c_int64(), C.c_int64(), C.c_int64()
        _check(_lib.nm_pencil_export_csr(self._h, which, C.byref(nr), C.byref(nc), C.byref(nnz), None, None, None))
        ptr = np.zeros(nr.value + 1, np.int64)
        col = np.zeros(max(nnz.value, 1), np.int32)
        val = np.zeros(max(nnz.value, 1), np.float64)
        _check(_lib.nm_pencil_export_csr(self._h, which, C.byref(nr), C.byref(nc), C.byref(nnz), _ptr(ptr),
                                         _ptr(col), _ptr(val)))
        return ptr, col[:nnz.value], val[:nnz.value], (nr.value, nc.value)

    def nodes(self):
        ng = np.zeros(self.N, np.int64)
        pg = np.zeros(max(self.n_p, 1), np.int64)
        _check(_lib.nm_pencil_nodes(self._h, _ptr(ng), _ptr(pg)))
        return ng, pg[:self.n_p]

    @staticmethod
    def _opts(kM=0, kP=0, minv_tol=0.0, kp_tol=0.0, precision=0, mass_passes=0):
        return _ApplyOpts(kM, kP, minv_tol, kp_tol, precision, mass_passes)

    def apply(self, op, X, out_rows=None, **kw):
        """Y = op(X) for a device tensor X [rows, ncols] (float64, or float32
        with precision=1)."""
        X = X.contiguous()
        rows = out_rows if out_rows is not None else (self.n_p if op in (OP_EGT, OP_KP, OP_KPINV) else self.n)
        Y = torch.empty((rows, X.shape[1]), dtype=X.dtype, device=X.device)
        o = self._opts(**kw)
        _check(_lib.nm_pencil_apply(self._h, op, X.shape[1], _ptr(X), _ptr(Y), C.byref(o), _stream()))
        torch.cuda.synchronize()
        return Y

    def apply_noalloc(self, op, X, Y, **kw):
        """Y = op(X) through nm_pencil_apply_noalloc into the caller's Y (no
        device allocation, no synchronisation: Y is ready when torch's current
        stream reaches this point)."""
        o = self._opts(**kw)
        _check(_lib.nm_pencil_apply_noalloc(self._h, op, X.shape[1], _ptr(X), _ptr(Y), C.byref(o), _stream()))
        return Y

    def filter_apply(self, mu, c, e, X, null_shift=0.0, null_scale=0.0, **kw):
        mu = np.ascontiguousarray(mu, np.float64)
        X = X.contiguous()
        Y = torch.empty_like(X)
        o = self._opts(**kw)
        _check(_lib.nm_filter_apply(self._h, _ptr(mu), len(mu) - 1, c, e, null_shift, null_scale, X.shape[1],
                                    _ptr(X), _ptr(Y), C.byref(o), _stream()))
        return Y

    def spectrum_dos(self, lmin, lmax, m, Z, weighted=False, **kw):
        """Density-of-states traces tau[0..m] from the columns of the device
        block Z [n, nvec] (float64, canonical order; nm_spectrum_dos, or
        nm_spectrum_dos_weighted: traces of T_k B, blind to the null space)."""
        Z = Z.contiguous()
        tau = np.zeros(m + 1)
        o = self._opts(**kw)
        fn = _lib.nm_spectrum_dos_weighted if weighted else _lib.nm_spectrum_dos
        _check(fn(self._h, lmin, lmax, int(m), Z.shape[1], _ptr(Z), C.byref(o), _stream(), _ptr(tau)))
        return tau

    def dos_slice_edges(self, a, b, nslices, lmin, lmax, m=1000, nvec=32, seed=0, weighted=False):
        """Ends of nslices windows of [a, b] with equal estimated eigenvalue
        counts, from density-of-states traces of degree m on nvec Gaussian
        columns drawn with torch (seeded); returns (edges, tau)."""
        g = torch.Generator(device="cuda").manual_seed(int(seed))
        Z = torch.randn(self.n, nvec, generator=g, dtype=torch.float64, device="cuda")
        tau = self.spectrum_dos(lmin, lmax, m, Z, weighted=weighted)
        return dos_slices(tau, lmin, lmax, a, b, nslices, weighted=weighted), tau

    def spectrum_bound_rigorous(self):
        """An upper bound of the pencil's spectrum that provably holds (nm_spectrum_bound_rigorous)."""
        hi = C.c_double()
        _check(_lib.nm_spectrum_bound_rigorous(self._h, _stream(), C.byref(hi)))
        return hi.value

    def spectrum_bounds(self, steps=60, seed=1):
        lo, hi = C.c_double(), C.c_double()
        _check(_lib.nm_spectrum_bounds(self._h, steps, seed, _stream(), C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    def filtered_eig(self, a, b, nev, tol, degree=0, block=0, precision=0, max_basis=0, null_filter=-1,
                     verbose=0, minv_tol=0.0, kp_tol=0.0, lmin=0.0, lmax=0.0, guard=0.0, seed=1,
                     allow_partial=False, refine=0, mass_passes=0):
        o = _EigOpts(degree, block, precision, max_basis, null_filter, verbose, minv_tol, kp_tol, lmin, lmax,
                     guard, seed, _stream(), refine, mass_passes)
        r = C.POINTER(_EigResult)()
        st = _lib.nm_filtered_eig(self._h, a, b, nev, tol, C.byref(o), C.byref(r))
        if st == NM_PARTIAL and allow_partial and r:
            res = EigResult(r)
            res.partial = True
            return res
        _check(st)
        res = EigResult(r)
        res.partial = False
        return res

    def autotune(self, precision=0):
        """Pick the fastest block width and mass-solve kernel; returns (block, microseconds per column-step)."""
        blk, us = C.c_int32(), C.c_double()
        _check(_lib.nm_pencil_autotune(self._h, int(precision), _stream(), C.byref(blk), C.byref(us)))
        return blk.value, us.value

    def filtered_eig_slices(self, windows, nev, tol, degree=0, block=0, precision=0, max_basis=0, null_filter=-1,
                            verbose=0, minv_tol=0.0, kp_tol=0.0, lmin=0.0, lmax=0.0, guard=0.0, seed=1,
                            allow_partial=False, refine=0, mass_passes=0):
        """One solve per window (a, b), their filter applications batched; returns a list of EigResult."""
        S = len(windows)
        a = np.ascontiguousarray([w[0] for w in windows], np.float64)
        b = np.ascontiguousarray([w[1] for w in windows], np.float64)
        nv = np.ascontiguousarray(nev if np.ndim(nev) else [nev] * S, np.int32)
        o = _EigOpts(degree, block, precision, max_basis, null_filter, verbose, minv_tol, kp_tol, lmin, lmax,
                     guard, seed, _stream(), refine, mass_passes)
        outs = (C.POINTER(_EigResult) * S)()
        st = _lib.nm_filtered_eig_slices(self._h, S, _ptr(a), _ptr(b), _ptr(nv), tol, C.byref(o), outs)
        if not (st == NM_PARTIAL and allow_partial):
            _check(st)
        res = []
        for i in range(S):
            r = EigResult(outs[i])
            r.partial = st == NM_PARTIAL
            res.append(r)
        return res

    def project_rotation(self, basis: EigResult, a, b):
        r = C.POINTER(_RotResult)()
        _check(_lib.nm_project_rotation(self._h, basis._ptr, a, b, _stream(), C.byref(r)))
        return RotResult(r)

    def refine_rotation(self, basis: EigResult, rot: "RotResult", a, b, iters=3, degree=0, tol=1e-8):
        """Refine projected rotating modes toward the exact QEP (nm_refine_rotation)."""
        r = C.POINTER(_RotResult)()
        _check(_lib.nm_refine_rotation(self._h, basis._ptr, rot._ptr, a, b, int(iters), int(degree), tol, _stream(),
                                       C.byref(r)))
        return RotResult(r)


class SelfGravity:
    """Self-gravitation of a pencil's planet as an N-body problem
    (nm_selfgrav_build): apply(X) = -C^T S C X, field(points) = the reference
    field from the element masses; attach() makes the pencil's operator
    include it."""

    def __init__(self, pencil: "Pencil", planet: dict, G=1.0 / np.pi):
        lib = load_library()
        mesh, mat, om, keep = _planet_structs(planet)
        h = C.c_void_p()
        _check(lib.nm_selfgrav_build(pencil._h, C.byref(mesh), C.byref(mat), float(G), _stream(), C.byref(h)))
        self._h = h
        self._pencil = pencil  # the pencil must outlive this object
        nb, nt, nf = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib.nm_selfgrav_info(h, C.byref(nb), C.byref(nt), C.byref(nf), None))
        self.n_body, self.n_tet, self.n_face = nb.value, nt.value, nf.value

    def inv_R(self):
        out = np.zeros(self.n_body)
        _check(_lib.nm_selfgrav_info(self._h, None, None, None, _ptr(out)))
        return out

    def apply(self, X):
        X = X.contiguous()
        Y = torch.empty_like(X)
        _check(_lib.nm_selfgrav_apply(self._h, X.shape[1], _ptr(X), _ptr(Y), _stream()))
        return Y

    def field(self, pts):
        pts = pts.contiguous()
        g = torch.empty_like(pts)
        _check(_lib.nm_selfgrav_field(self._h, pts.shape[0], _ptr(pts), _ptr(g), _stream()))
        return g

    def attach(self, on=True):
        _check(_lib.nm_pencil_attach_selfgrav(self._pencil._h, self._h if on else None))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.nm_selfgrav_free(self._h)
            self._h = None


class Server:
    """Continuous batching of eigensolves on this GPU (see nm_server_create)."""

    def __init__(self, hbm_budget_gb=200.0, max_active=4):
        lib = load_library()
        h = C.c_void_p()
        _check(lib.nm_server_create(float(hbm_budget_gb) * 1e9, int(max_active), C.byref(h)))
        self._h = h

    def submit(self, planet: dict, windows, nev, tol, rotate=False, degree=0, block=0, precision=0, max_basis=0,
               null_filter=-1, minv_tol=0.0, kp_tol=0.0, guard=0.0, seed=1, refine=0, verbose=0, mass_passes=0):
        mesh, mat, om, keep = _planet_structs(planet)
        S = len(windows)
        a = np.ascontiguousarray([w[0] for w in windows], np.float64)
        b = np.ascontiguousarray([w[1] for w in windows], np.float64)
        nv = np.ascontiguousarray(nev if np.ndim(nev) else [nev] * S, np.int32)
        o = _EigOpts(degree, block, precision, max_basis, null_filter, verbose, minv_tol, kp_tol, 0.0, 0.0, guard,
                     seed, None, refine, mass_passes)
        req = _Request(mesh, mat, (C.c_double * 3)(*om), S, _ptr(a).value, _ptr(b).value, _ptr(nv).value, tol, o,
                       1 if rotate else 0)
        t = C.c_int64()
        _check(_lib.nm_server_submit(self._h, C.byref(req), C.byref(t)))
        return t.value

    def wait(self, ticket):
        """Block until the request is done: dict(status, error, slices [EigResult], rotation, t_submit,
        t_start, t_end, est_bytes)."""
        r = C.POINTER(_ServerResult)()
        _check(_lib.nm_server_wait(self._h, int(ticket), C.byref(r)))
        c = r.contents
        out = dict(status=c.status, error=c.error.decode(), t_submit=c.t_submit, t_start=c.t_start,
                   t_end=c.t_end, est_bytes=c.est_bytes, slices=[], rotation=None)
        for i in range(c.nslices):
            if c.slices[i]:
                e = EigResult(c.slices[i])
                e.partial = c.status == NM_PARTIAL
                e._ptr = None  # owned by the server result, freed below
                out["slices"].append(e)
        if c.rotation:
            out["rotation"] = RotResult(c.rotation, owned=False)
        _lib.nm_server_result_free(r)
        return out

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _check(_lib.nm_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
