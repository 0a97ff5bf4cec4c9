/*
 * nmodes -- seismic normal modes of layered, rotating planets on AMD MI355X.
 *
 * C ABI of the GPU library.  It computes the eigenpairs of the mixed
 * continuous-Galerkin elastic-gravitational pencil of
 *   Shi, Li, Xi, Saad, de Hoop, "A non-perturbative approach to computing
 *   seismic normal modes in rotating planets" (arXiv 1906.11082),
 * in the Cowling approximation (Sec. 6.2, eq. "cowling"):
 *
 *     (A_G - E_G A_p^{-1} E_G^T) u = omega^2 M u,           (Omega = 0)
 *     omega^2 M u - 2 i omega R u - A u = 0                  (Sec. 7, eq. "simplequad")
 *
 * with the matrices of the table of implicit matrix definitions (Sec. 4.2)
 * built by the element formulas of Appendix A, on unstructured tetrahedral
 * meshes with solid and fluid regions.
 *
 * Conventions used by every entry point
 * -------------------------------------
 * - Status: 0 success, NM_PARTIAL (1) a solve returned fewer converged pairs
 *   than requested, negative values are errors (NM_E*).  nm_last_error()
 *   returns a message for the last failing call on the calling thread.
 * - Host arrays passed in are borrowed for the duration of the call only.
 * - Threads: different pencils may be used from different host threads at
 *   once; calls on one pencil must not overlap (they share its rocBLAS
 *   handle), except inside nm_filtered_eig_slices, which runs its windows
 *   on threads of its own, each with its own stream and rocBLAS handle.
 * - Device arrays are plain device pointers (hipMalloc'd or from any
 *   allocator in the same process), row-major [rows][ncols] with the ncols
 *   columns of a row contiguous.  A displacement block therefore is
 *   [N][3][ncols]: node-major, components x,y,z, then columns.
 * - "stream" is a hipStream_t (NULL = the default stream).  Calls that
 *   return host data synchronise that stream before returning.
 * - Displacement DOF numbering (the numbering is part of the result and is
 *   bit-exact reproducible): geometric nodes are the vertices in input order,
 *   then (degree 2) one node per edge, edges ordered by (min vertex, max
 *   vertex).  A node carries a solid copy if it belongs to a solid
 *   tetrahedron and a fluid copy if it belongs to a fluid one; the elements
 *   are non-conforming across fluid-solid boundaries (Sec. 4.1).  All solid
 *   copies come first, by geometric id, then all fluid copies.  DOF =
 *   3*node + component.  Pressure DOFs: geometric nodes of the pressure
 *   degree that belong to a fluid tetrahedron, by geometric id.
 * - Element-local node order (for per-element-node inputs): vertices 0..3
 *   of tet[k], then edge midpoints of edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3).
 */
#ifndef NMODES_H
#define NMODES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nm_status;
enum {
  NM_OK = 0,
  NM_PARTIAL = 1,     /* solve finished with fewer converged pairs than asked */
  NM_EINVAL = -1,     /* invalid argument (sizes, window, options) */
  NM_EBADMESH = -2,   /* index out of range or tetrahedron with J <= 0 */
  NM_ENOMEM = -3,     /* device or host allocation failed */
  NM_EDEVICE = -4,    /* HIP / rocBLAS / rocSOLVER call failed */
  NM_ENOCONV = -5     /* filter blow-up or Lanczos breakdown not recovered */
};

/* Matrices held by a pencil (nm_pencil_export_csr, nm_pencil_apply). */
enum {
  NM_MAT_AG = 0,   /* A_G: solid stiffness with gravity (n x n); the fluid block
                      A_f is zero (buoyancy N^2 = 0, no fluid-fluid interface) */
  NM_MAT_M = 1,    /* M = M_s (x) I_3, mass (n x n) */
  NM_MAT_R = 2,    /* R = M_s (x) [Omega]_x, Coriolis int rho v.(Omega x u) (n x n) */
  NM_MAT_KP = 3,   /* K_p = -A_p = int kappa^{-1} v^p p, SPD (n_p x n_p) */
  NM_MAT_EG = 4    /* E_G = [E_FS; A_dg] (n x n_p) */
};

/* Operators of nm_pencil_apply (Y = op(X)). */
enum {
  NM_OP_AG = 0,     /* Y = A_G X                               X:[n][c]   Y:[n][c]   */
  NM_OP_M = 1,      /* Y = M X                                 [n][c] -> [n][c]       */
  NM_OP_R = 2,      /* Y = R X                                 [n][c] -> [n][c]       */
  NM_OP_KP = 3,     /* Y = K_p X                               [n_p][c] -> [n_p][c]   */
  NM_OP_EG = 4,     /* Y = E_G X                               [n_p][c] -> [n][c]     */
  NM_OP_EGT = 5,    /* Y = E_G^T X                             [n][c] -> [n_p][c]     */
  NM_OP_KPINV = 6,  /* Y = S_p(X), fixed-k Chebyshev-Jacobi solve with K_p          */
  NM_OP_A = 7,      /* Y = (A_G + E_G S_p E_G^T) X, the Cowling operator            */
  NM_OP_MINV = 8,   /* Y = S_M(X), fixed-k Chebyshev-Jacobi solve with M            */
  NM_OP_B = 9       /* Y = S_M(A X)                                                 */
};

typedef struct nm_pencil nm_pencil;

typedef struct {
  int64_t n_vert;          /* V */
  int64_t n_tet;           /* T */
  const double* xyz;       /* host [V][3] */
  const int32_t* tet;      /* host [T][4], vertex ids, positive orientation */
  const int8_t* region;    /* host [T], 0 solid, 1 fluid */
  int32_t disp_order;      /* 1 or 2 */
  int32_t pres_order;      /* 1 or 2, <= disp_order */
} nm_mesh;

typedef struct {
  const double* rho;          /* host [T] density */
  const double* lam;          /* host [T] Lame lambda (fluid: kappa) */
  const double* mu;           /* host [T] shear modulus (0 in fluid) */
  const double* gprime;       /* host [T][Np][3] g' at element nodes, or NULL (no gravity) */
  const double* grad_gprime;  /* host [T][Np][3][3], [i][j] = d_i g'_j, or NULL */
  int32_t gprime_np;          /* Np of the two arrays above (4 or 10) */
} nm_material;

typedef struct {
  int64_t n_geom;     /* geometric nodes (vertices + edges) */
  int64_t n_node;     /* displacement nodes N (solid copies + fluid copies) */
  int64_t n_solid;    /* solid copies */
  int64_t n_disp;     /* n = 3 N */
  int64_t n_pres;     /* pressure DOFs n_p */
  int64_t nnzb;       /* blocks of the node graph (= nnz of M_s) */
  int64_t nnz_kp;     /* nnz of K_p */
  int64_t nnzb_eg;    /* (node, pressure) pairs of E_G */
  int64_t n_fs_faces; /* fluid-solid faces */
  double minv_lo, minv_hi;  /* element bounds of spec(D^{-1} M) */
  double kp_lo, kp_hi;      /* element bounds of spec(D^{-1} K_p) */
} nm_pencil_info;

typedef struct {
  int32_t kM;          /* Chebyshev-Jacobi steps of the M solve (0 = from minv_tol) */
  int32_t kP;          /* steps of the K_p solve (0 = from kp_tol) */
  double minv_tol;     /* bound 2 r^k of the M solve (0 = 1e-12) */
  double kp_tol;       /* bound of the K_p solve (0 = 1e-13) */
  int32_t precision;   /* 0 FP64, 1 FP32 values, vectors and accumulation */
  int32_t mass_passes; /* M solve of NM_OP_MINV / NM_OP_B and nm_filter_apply, precision 0:
                          0 one FP64 Chebyshev-Jacobi pass; P = 2..8: P passes in FP32 with
                          FP64 residual corrections (see nm_filtered_eig), each of kM steps
                          if kM > 0, else of the steps that bring (2 r^k)^P to minv_tol */
} nm_apply_opts;

typedef struct {
  int32_t degree;      /* filter degree, 0 = chosen from the spectrum bounds */
  int32_t block;       /* block width b, 0 = auto */
  int32_t precision;   /* 0 FP64 filter; 1 FP32 filter + FP64 Lanczos/RR/residual */
  int32_t max_basis;   /* cap of the Krylov basis size, 0 = auto */
  int32_t null_filter; /* lower side of the filter: -1 auto (no damping below a when the
                          pencil has fluid, else damping), 0 damping below a, 1 factor
                          lambda/b, 2 no damping below a, 3 spectrum slice: damping on both
                          sides beyond a - guard (b - a) and b + guard (b - a) */
  int32_t verbose;     /* 0 quiet, 1 per-block log on stderr */
  double minv_tol;     /* M-solve bound inside the filter (0: 0.3 tol clamped to [1e-12, 1e-7] in FP64, 1e-7 in FP32) */
  double kp_tol;       /* K_p-solve bound (0 = 1e-13 FP64, 1e-7 FP32) */
  double lmin, lmax;   /* spectrum bounds of M^{-1}A; lmax <= lmin: estimate */
  double guard;        /* transition width beyond b as a fraction of b (0 = 1.0) */
  uint64_t seed;       /* start block seed */
  void* stream;        /* hipStream_t */
  int32_t refine;      /* at most this many FP64 refinement passes of the window pairs
                          (0 = 3, -1 = none; see nm_filtered_eig) */
  int32_t mass_passes; /* M solve inside an FP64 filter: 0 one FP64 pass; P = 2..8 passes in
                          FP32 with FP64 residual corrections (see nm_filtered_eig) */
} nm_eig_opts;

typedef struct {
  int32_t count;        /* pairs returned, lambda ascending */
  int64_t n;            /* rows of X */
  double* lambda;       /* host [count] omega^2 */
  double* resid;        /* host [count] ||A x - l M x|| / (|l| ||M x||) */
  double* X;            /* device [n][count], M-orthonormal, largest entry of each column > 0 */
  int32_t degree;       /* filter degree used */
  int32_t kM, kP;       /* inner solve steps used */
  int32_t block;        /* block width used */
  int32_t basis;        /* final Krylov basis size */
  int64_t bapps;        /* column applications of B = M^{-1} A */
  double lmin, lmax;    /* spectrum bounds used */
  double seconds;       /* wall time of the solve */
  double bytes;         /* algorithmic HBM bytes of all filter applications */
  double filter_seconds;/* time inside filter applications */
  /* hot kernel (a middle Chebyshev-Jacobi step of the M solve inside the
     filter): launches, sampled launches timed with HIP events on the solve's
     stream, their mean duration, and its algorithmic bytes per launch */
  int64_t hot_launches, hot_samples;
  double hot_ms, hot_bytes;
  /* FP64 refinement: passes run, degree of the last low-pass polynomial,
     their wall time and column B-applications */
  int32_t refine_passes, refine_degree;
  double refine_seconds;
  int64_t refine_bapps;
  /* M solve inside the filter: FP32 passes (0: one FP64 pass of kM steps) and steps per pass */
  int32_t mass_passes, mass_pass_steps;
  /* kernel of the middle mass-solve steps: 0 per-row, 1 row groups, 2 LDS tiles */
  int32_t hot_kernel;
} nm_eig_result;

typedef struct {
  int32_t count;        /* rotating modes with omega > 0, omega^2 in [a, b] */
  int64_t n;
  double* omega;        /* host [count] ascending */
  double* U;            /* device [n][count][2] complex (re, im) modes, normalised by
                           u^H M u - (i/omega) u^H R u = 1, largest entry real > 0 */
  double seconds;
  double* resid;        /* host [count] QEP residuals ||w^2 M u - 2 i w R u - A u|| / (w^2 ||M u||) */
  int32_t iters;        /* refinement passes run (nm_refine_rotation; 0 for a projection) */
  int32_t basis;        /* size of the projection space */
  int32_t degree;       /* degree of the correction series (refinement) */
} nm_rot_result;

/* Build the pencil: numbering, CSR patterns and all matrix values on the
 * device (Sec. 4.2 table, Appendix A).  omega: rotation vector (may be
 * NULL = 0).  Fails with NM_EBADMESH naming the first tetrahedron with
 * J <= 0 or an index out of range. */
nm_status nm_assemble(const nm_mesh* mesh, const nm_material* mat, const double omega[3],
                      void* stream, nm_pencil** out);

nm_status nm_pencil_info_get(const nm_pencil* p, nm_pencil_info* info);

/* Two-call CSR export of one matrix (NM_MAT_*) into caller host buffers:
 * with row_ptr == NULL only *nrows, *ncols, *nnz are filled; then call again
 * with row_ptr [nrows+1], col [nnz], val [nnz] (val may be NULL).
 * Columns of a row strictly increase; the vector matrices are exported with
 * full 3x3 blocks (zeros stored). */
nm_status nm_pencil_export_csr(const nm_pencil* p, int32_t which, int64_t* nrows, int64_t* ncols,
                               int64_t* nnz, int64_t* row_ptr, int32_t* col, double* val);

/* Geometric node of each displacement node (host [N]) and of each pressure
 * DOF (host [n_p]); either may be NULL. */
nm_status nm_pencil_nodes(const nm_pencil* p, int64_t* node_geom, int64_t* pres_geom);

/* Y = op(X) on the device (NM_OP_*), X and Y device arrays as above, X != Y.
 * opts may be NULL (FP64, default tolerances).  With precision 1 the
 * arrays are float. */
nm_status nm_pencil_apply(const nm_pencil* p, int32_t op, int32_t ncols, const void* X, void* Y,
                          const nm_apply_opts* opts, void* stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * operators as nm_pencil_apply with every buffer beyond X and Y (the vectors
 * in the internal node order, the iterates of the inner Chebyshev-Jacobi
 * solves) in a static device array of NM_NOALLOC_SCRATCH_BYTES per device,
 * held from library load to process end.  Calls no hipMalloc / hipFree and no
 * allocating routine, and does not synchronise: Y is complete when the stream
 * reaches the end of the call.  All calls on one device share the array:
 * calls that overlap in time on one device (other streams or host threads)
 * race; calls ordered on one stream do not.  NM_EINVAL: an operator whose
 * buffers exceed NM_NOALLOC_SCRATCH_BYTES (the message gives the bytes
 * needed), opts->mass_passes != 0, precision 1 before the pencil's FP32
 * matrices exist (any allocating FP32 operator or solve creates them), or a
 * current device other than the pencil's. */
#define NM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
nm_status nm_pencil_apply_noalloc(const nm_pencil* p, int32_t op, int32_t ncols, const void* X, void* Y,
                                  const nm_apply_opts* opts, void* stream);

/* Autotuning of the mass-solve step (the hot loop of every filter step) on
 * this pencil, in FP64 (precision 0) or FP32 (1): times middle
 * Chebyshev-Jacobi steps for block widths 8, 16, 32 and 64 with the per-row
 * kernel, the row-group kernel at groups of 4 and of 8 rows (the block size
 * of the grouped format: rows times the union of their columns), each as one
 * workgroup per share or as a persistent launch, and the LDS-tile kernel at
 * tiles of 32 and 64 rows, then keeps the fastest per
 * column: nm_filtered_eig with block 0 uses that width (at most nev / 4,
 * rounded down to a multiple of 8, at least 8) and every later mass solve
 * that kernel and block size (the row groups and tiles are rebuilt for it).
 * Allocates 3 x 64 columns of work vectors for the duration of the call; do
 * not call it while another call uses the pencil.  block / us_per_column
 * (may be NULL): the winner and its time per column and step in
 * microseconds. */
nm_status nm_pencil_autotune(nm_pencil* p, int32_t precision, void* stream, int32_t* block, double* us_per_column);

/* Jackson-damped Chebyshev coefficients mu[0..m] of the indicator of [a, b]
 * after mapping [lmin, lmax] onto [-1, 1] (the polynomial filter). */
nm_status nm_filter_coeffs(double a, double b, double lmin, double lmax, int32_t m, double* mu);

/* Filter degree chosen by the library: the smallest degree whose filter
 * stays below 1 % of its window-edge level beyond b (1 + guard) (guard <= 0:
 * 1.0).  mode 0: no requirement below a (the spectrum below the window is
 * an exactly degenerate null space); mode 1: the same bound below
 * a - guard (a - lmin); mode 2: the filter carries the factor lambda / b;
 * mode 3 (spectrum slices): the bound beyond b + guard (b - a) and below
 * a - guard (b - a). */
nm_status nm_filter_degree(double a, double b, double lmin, double lmax, double guard, int32_t mode,
                           int32_t* m);

/* Y = p(B) X (null_scale == 0) or Y = ((B - null_shift)/null_scale) p(B) X,
 * p(t) = sum_k mu_k T_k((t - c)/e), B = S_M A: one polynomial-filter
 * application (Sec. 6.1, polynomial filtering), device arrays [n][ncols]. */
nm_status nm_filter_apply(const nm_pencil* p, const double* mu, int32_t m, double c, double e,
                          double null_shift, double null_scale, int32_t ncols, const void* X,
                          void* Y, const nm_apply_opts* opts, void* stream);

/* Bounds [lmin, lmax] enclosing the spectrum of M^{-1} A (the
 * interval the Chebyshev filter is defined on), from `steps` Lanczos steps
 * in the M-inner product with the random start vector of `seed`. */
nm_status nm_spectrum_bounds(const nm_pencil* p, int32_t steps, uint64_t seed, void* stream, double* lmin,
                             double* lmax);
/* An upper bound that provably holds for every eigenvalue of the Cowling
 * pencil without the self-gravitation term: with D = diag(M), Gershgorin row
 * sums of D^{-1/2} A_G D^{-1/2}, plus those of D^{-1/2} E_G D_p^{-1} E_G^T
 * D^{-1/2} over the reference element's lower Jacobi bound of K_p, over the
 * element's lower Jacobi bound of M.  Looser than the Lanczos estimate
 * (about 6x on the small test planets); the filtered solve uses it for its
 * last blow-up restart.  Synchronises the stream. */
nm_status nm_spectrum_bound_rigorous(const nm_pencil* p, void* stream, double* lmax);

/* Density of states of B = M^{-1} A by the kernel polynomial method (the
 * spectrum slicing of Sec. 6.1 follows EVSL, which places slices by such an
 * estimate): tau[k] = (1/nvec) sum_v z_v^T T_k((B - c)/e) z_v, k = 0..m,
 * c -+ e = [lmin, lmax], by the filter's three-term recurrence on the nvec
 * columns of Z (device, [n][nvec], canonical order, caller-drawn; with
 * E[z z^T] = I each tau[k] estimates tr T_k).  FP64 operators (opts as for
 * nm_pencil_apply; precision must be 0).  tau: host [m + 1]. */
nm_status nm_spectrum_dos(const nm_pencil* p, double lmin, double lmax, int32_t m, int32_t nvec, const double* Z,
                          const nm_apply_opts* opts, void* stream, double* tau);
/* Estimated number of eigenvalues in [a, b] from traces tau[0..m]: the
 * Jackson-damped Chebyshev series of the indicator (nm_filter_coeffs) dotted
 * with tau.  Host only. */
nm_status nm_dos_count(const double* tau, int32_t m, double lmin, double lmax, double a, double b, double* count);
/* Ends edges[0..nslices] (edges[0] = a, edges[nslices] = b) of nslices
 * windows of [a, b] with equal estimated counts (bisection on the
 * cumulative count).  Host only. */
nm_status nm_dos_slices(const double* tau, int32_t m, double lmin, double lmax, double a, double b, int32_t nslices,
                        double* edges);

/* Null-free density of states for pencils with a large null space (the
 * fluid's, exactly degenerate at 0): the same traces with the recurrence
 * started from B z, tau[k] = (1/nvec) sum_v z_v^T T_k((B - c)/e) B z_v,
 * estimating tr(T_k(.) B) = sum_i T_k(t_i) lambda_i, in which every
 * eigenvalue 0 weighs nothing.  Counts then use the Jackson-damped series of
 * 1/lambda on [a, b] (a > 0), so the kernel's finite resolution cannot leak
 * the null cluster into a low window (at the benchmark planet's spectrum
 * width the unweighted kernel smears it over several units of lambda even
 * at degree 3000).  Arguments as nm_spectrum_dos, nm_dos_count and
 * nm_dos_slices; NM_EINVAL when a <= 0. */
nm_status nm_spectrum_dos_weighted(const nm_pencil* p, double lmin, double lmax, int32_t m, int32_t nvec,
                                   const double* Z, const nm_apply_opts* opts, void* stream, double* tau);
nm_status nm_dos_count_weighted(const double* tau, int32_t m, double lmin, double lmax, double a, double b,
                                double* count);
nm_status nm_dos_slices_weighted(const double* tau, int32_t m, double lmin, double lmax, double a, double b,
                                 int32_t nslices, double* edges);

/* Eigenpairs of the Cowling pencil with a <= omega^2 <= b: the min(nev,
 * count) smallest, by polynomial-filtered block Lanczos in the M-inner
 * product with Rayleigh-Ritz on (A, M) (Sec. 6.1).  tol bounds the
 * residual of every returned pair.  Rounding inside the filter (FP64:
 * about eps64 times the degree; precision 1, the filter in FP32 values,
 * vectors and accumulation: eps32) leaves the window residuals at a floor
 * near eps * lambda_max / lambda.  The Lanczos therefore stops when they are
 * below tol or no longer improve, and the window pairs are refined in FP64:
 * each pass applies q(B) ((B / b) q(B) after an FP32 filter), q a Chebyshev
 * low-pass polynomial (1 at b, small beyond a cut-off chosen from the floor),
 * to the window Ritz vectors and to those just above and below the window,
 * and runs Rayleigh-Ritz on (A, M) over the refined vectors.
 * opts->mass_passes P >= 2 (precision 0): every M solve inside the filter
 * runs as P Chebyshev-Jacobi passes in FP32, the first on A W, each later one
 * on the FP64 residual of the sum so far, with the sum kept in FP64
 * (iterative refinement of the solve; the paper fixes only that M^{-1} is
 * applied through products with M, Sec. 6.1).  Its error operator (I - S M)^P
 * has the bound of one FP64 pass of P k steps, and the rounding a pass leaves
 * is relative to the correction it computes; the refinement above runs in
 * FP64 throughout.  NM_PARTIAL:
 * the pairs returned are those found, some with residual above tol, or the
 * basis cap was reached first. */
nm_status nm_filtered_eig(const nm_pencil* p, double a, double b, int32_t nev, double tol,
                          const nm_eig_opts* opts, nm_eig_result** out);

/* Several windows [a[i], b[i]] of one pencil (spectrum slicing, Sec. 6.1),
 * nev[i] pairs each, solved together: one block Lanczos per window, each in
 * its own host thread and HIP stream, with their filter applications batched
 * into one block of concatenated columns (one Chebyshev series per column,
 * zero-padded to the largest degree), so the matrices are streamed once per
 * step for all windows.  A window's result is the one nm_filtered_eig gives
 * for it with the same bounds and seed.  All windows use one filter interval
 * (opts->lmin/lmax, or estimated once) and opts otherwise as
 * nm_filtered_eig; the null factor (null_filter 1) is not allowed.  out:
 * caller array of nslices (1..64) result pointers, each freed with
 * nm_result_free; NM_PARTIAL if any window is partial (all results set); on
 * an error no result is returned. */
nm_status nm_filtered_eig_slices(const nm_pencil* p, int32_t nslices, const double* a, const double* b,
                                 const int32_t* nev, double tol, const nm_eig_opts* opts, nm_eig_result** out);

/* ---- Request server (continuous batching of solves on one GPU) ----
 * Requests (a planet, its windows and options) are admitted in arrival order
 * while the sum of their estimated device memory stays within the budget and
 * at most max_active run at once; each admitted request runs on its own host
 * thread and HIP stream (assembly, then nm_filtered_eig_slices over its
 * windows, then optionally nm_project_rotation over their union), so requests
 * that arrive while others run overlap with them on the device.  A request's
 * results are those it gives alone.  The memory estimate is made from the
 * mesh sizes before assembly (node count from vertices, tets and order;
 * matrices, assembly staging, Krylov bases and work blocks per window). */
typedef struct nm_server nm_server;

typedef struct {
  nm_mesh mesh;          /* borrowed during nm_server_submit only (copied) */
  nm_material material;  /* borrowed during nm_server_submit only (copied) */
  double omega[3];       /* rotation vector */
  int32_t nslices;       /* windows, 1..64 */
  const double* a;       /* host [nslices] lower ends (copied) */
  const double* b;       /* host [nslices] upper ends (copied) */
  const int32_t* nev;    /* host [nslices] (copied) */
  double tol;            /* residual bound */
  nm_eig_opts opts;      /* as for nm_filtered_eig; opts.stream is ignored */
  int32_t rotate;        /* 1: also project the Coriolis term over the union of the windows */
} nm_request;

typedef struct {
  int32_t status;            /* nm_status of the request (NM_PARTIAL: some pairs above tol) */
  char error[256];           /* message when status < 0 */
  int32_t nslices;
  nm_eig_result** slices;    /* [nslices] results (NULL entries on error) */
  nm_rot_result* rotation;   /* NULL unless requested and found */
  double t_submit, t_start, t_end;  /* seconds since nm_server_create */
  double est_bytes;          /* the admission estimate */
} nm_server_result;

/* max_active >= 1; the server admits the first queued request whenever
 * nothing runs, whatever its estimate. */
nm_status nm_server_create(double hbm_budget_bytes, int32_t max_active, nm_server** out);
/* Queue a request; *ticket identifies it for nm_server_wait. */
nm_status nm_server_submit(nm_server* s, const nm_request* req, int64_t* ticket);
/* Block until the request has finished; *out is freed with nm_server_result_free.
 * Each ticket can be waited for once: a later (or concurrent) wait on the
 * same ticket returns NM_EINVAL. */
nm_status nm_server_wait(nm_server* s, int64_t ticket, nm_server_result** out);
void nm_server_result_free(nm_server_result* r);
/* Run every queued request to completion, then free the server (results not
 * waited for are discarded). */
nm_status nm_server_destroy(nm_server* s);

/* Rotating modes by projection on the non-rotating eigenvectors of basis
 * (Sec. 7, eqs. "linearpb", "sublinear0"): keeps omega > 0 with omega^2 in
 * [a, b].  Uses the pencil's Omega.  The paper's setting (Sec. 3, eq.
 * "freq") has the window far above |Omega| + (|Omega|^2 + max N^2)^(1/2),
 * which with N^2 = 0 is 2 |Omega|, the top of the rotating fluid's
 * continuous spectrum; the projection does not test this (the paper gives
 * no threshold), so windows near 2 |Omega| are the caller's to avoid. */
nm_status nm_project_rotation(const nm_pencil* p, const nm_eig_result* basis, double a, double b,
                              void* stream, nm_rot_result** out);

/* Refinement of the rotating modes of a projection toward the exact QEP
 * (Sec. 7, eq. "simplequad"; the paper notes after eq. "sublinear0" that
 * solving it exactly improves on the projection): up to `iters` passes of
 * Rayleigh-Ritz for the QEP over span(X_e) enlarged by two directions per
 * mode, g(B) M^{-1} Re r and g(B) M^{-1} Im r, r = w^2 M u - 2 i w R u - A u
 * its residual and g the Jackson-damped Chebyshev series (degree `degree`,
 * 0 = chosen from the spectrum bound) of the regularised resolvent
 * (l - w^2) / ((l - w^2)^2 + (w^2 / 4)^2) on the basis's spectrum bounds;
 * the enlarged span is projected by eq. "sublinear0" on the eigenvectors of
 * V^T A V (all of them: rigid motions and the fluid null space, absent
 * from the window basis, enter through the corrections; directions of
 * clearly negative V^T A V are left out).  A pass is kept only if every mode
 * it returns has a residual below the previous pass's largest (Rayleigh-Ritz
 * for the QEP can return spurious window values on the enlarged span, seen
 * on fluid planets); the refinement stops at the first pass that is not, or
 * when every residual is <= tol.
 * basis: the Omega = 0 window pairs the projection used; rot: its result.
 * out->resid holds the final residuals; out->iters the passes kept. */
nm_status nm_refine_rotation(const nm_pencil* p, const nm_eig_result* basis, const nm_rot_result* rot, double a,
                             double b, int32_t iters, int32_t degree, double tol, void* stream, nm_rot_result** out);

/* ---- Self-gravitation as an N-body problem (Sec. 5) ----
 * Bodies: the tetrahedra (barycentres) and the faces where the density jumps
 * (outer surface, fluid-solid faces; centroids).  A displacement gives them
 * charges q = C u (eqs. "ph1body2", "ph1surface2": int_K div(rho u) per
 * tetrahedron, int_E (nu . u)[rho] per face, each side of a fluid-solid face
 * with its own displacement and density); the incremental potential is
 * S q, S_ij = G / |r_i - r_j| and S_ii = G / R_i with 1/R_i the mean of
 * 1/|r_i - x| over body i (eqs. "k2local", "l2local"); the operator gains
 * -C^T S C (eq. "eigfull").  The sums S q are direct, tiled on the device:
 * FP32 pair terms, FP64 accumulation over source tiles. */
typedef struct nm_selfgrav nm_selfgrav;
/* Bodies, C (device) and the self-terms for the pencil's planet: mesh and
 * mat must be the arrays the pencil was assembled from (checked: sizes and
 * order).  G: the gravitational constant in the planet's units (1/pi for
 * radius, mean density and sqrt(pi G rho) as units).  The result refers to
 * the pencil, which must outlive it. */
nm_status nm_selfgrav_build(nm_pencil* p, const nm_mesh* mesh, const nm_material* mat, double G, void* stream,
                            nm_selfgrav** out);
/* Counts and (inv_R host [nbody], may be NULL) the self-terms 1/R_i. */
nm_status nm_selfgrav_info(const nm_selfgrav* sg, int64_t* nbody, int64_t* ntet, int64_t* nface, double* inv_R);
/* Y = -C^T S C X, device [n][ncols] canonical order.  Calls on one self-gravitation object must not
 * overlap (they share its work buffers). */
nm_status nm_selfgrav_apply(const nm_selfgrav* sg, int32_t ncols, const double* X, double* Y, void* stream);
/* Reference field of Sec. 5.1 at npts points (device [npts][3]): g(x) = -G sum_k m_k (x - r_k) / |x - r_k|^3
 * over the element masses m_k = rho_k |K_k| at the barycentres (device out [npts][3]). */
nm_status nm_selfgrav_field(const nm_selfgrav* sg, int64_t npts, const double* pts, double* g, void* stream);
/* The pencil's operator A becomes A_G + E_G K_p^{-1} E_G^T - C^T S C (eq. "eigfull") for every later
 * operator application and solve (FP64 filters only; NM_EINVAL with precision 1); sg NULL detaches. */
nm_status nm_pencil_attach_selfgrav(nm_pencil* p, const nm_selfgrav* sg);
void nm_selfgrav_free(nm_selfgrav* sg);

/* Copy the eigenvectors of a result into dst (device if dst_is_device,
 * else host), row-major [n][count] (rotation: [n][count][2]). */
nm_status nm_result_copy_vectors(const nm_eig_result* r, void* dst, int32_t dst_is_device);
nm_status nm_rot_copy_vectors(const nm_rot_result* r, void* dst, int32_t dst_is_device);

void nm_result_free(nm_eig_result* r);
void nm_rot_result_free(nm_rot_result* r);
void nm_pencil_free(nm_pencil* p);

/* Device memory of the library's own buffers (pencil matrices, Krylov bases,
 * work vectors) through the caller's allocator, e.g. a framework's caching
 * allocator, instead of hipMalloc / hipFree; alloc == free_ == NULL restores
 * those (NM_EINVAL if only one is NULL).  alloc(bytes, stream, ctx) returns
 * device memory of the current device aligned to 256 bytes, or NULL (the
 * call that needed it then fails with NM_ENOMEM); stream is NULL: the memory
 * may be used on any stream.  free_(ptr, stream, ctx) is called after a
 * device synchronisation, when no kernel uses the memory any more, with the
 * functions and ctx that allocated it (a later change does not affect memory
 * already allocated).  Result vectors (nm_eig_result.X, nm_rot_result.U)
 * stay hipMalloc'd and are freed by nm_result_free / nm_rot_result_free.
 * Call it while no other call of the library is in flight. */
nm_status nm_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                           void (*free_)(void* ptr, void* stream, void* ctx), void* ctx);

/* Widest vector block the kernels accept for n_disp displacement rows: one
 * launch indexes a block [N][3][ncols] with 32-bit offsets, so n_disp * ncols
 * must stay below 2^32.  nm_pencil_apply, nm_filter_apply, nm_filtered_eig
 * (block width) and nm_filtered_eig_slices (the sum of the windows' block
 * widths, which share one block) return NM_EINVAL for wider blocks before
 * allocating or launching anything.  Host-only; NM_EINVAL if n_disp <= 0. */
nm_status nm_max_block_columns(int64_t n_disp, int64_t* max_cols);

/* Dense block products of the filtered Lanczos (Sec. 6.2: the Gram-Schmidt
 * projections of a new block against the basis, the Gram matrices of its
 * Cholesky orthonormalisation and the Rayleigh-Ritz matrices V^T A V), on the
 * FP64 matrix cores — the kernels the solver uses, for callers that build or
 * orthogonalise their own blocks.  All matrices are FP64 device memory owned
 * by the caller; work is enqueued on `stream` (NULL: the default stream).
 *
 * nm_gemm_tn: C = A^T B, K x q, column-major with leading dimension K; A is
 * row-major [n][lda] (its first K columns are used, lda >= K), B row-major
 * [n][ldb] (first q columns, ldb >= q).  The rows are summed in fixed chunks
 * whose partial products are added in chunk order (the result does not
 * depend on scheduling); the partials (n-dependent, at most about
 * 4096 / ceil(K/64) / ceil(q/64) chunks of K x q) are allocated for the call,
 * which synchronises the stream before it returns.  n = 0 gives C = 0.
 *
 * nm_gemm_nn: D = alpha A C + beta D; A row-major [n][lda] (first K columns),
 * C column-major K x q with leading dimension ldc >= K, D row-major [n][ldd]
 * (first q columns, ldd >= q; not read when beta is 0); A and D must not be
 * the same array.  Asynchronous, allocates nothing.
 *
 * NM_EINVAL on negative sizes, leading dimensions below the used widths,
 * null matrices of a non-empty product, or A == D. */
nm_status nm_gemm_tn(int64_t n, int32_t K, int32_t q, const double* A, int32_t lda, const double* B, int32_t ldb,
                     double* C, void* stream);
nm_status nm_gemm_nn(int64_t n, int32_t K, int32_t q, double alpha, const double* A, int32_t lda, const double* C,
                     int32_t ldc, double beta, double* D, int32_t ldd, void* stream);

/* Message of the last failing call on this thread ("" if none). */
const char* nm_last_error(void);

/* Library version string. */
const char* nm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NMODES_H */
