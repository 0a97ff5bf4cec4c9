// Internal declarations of the nmodes GPU library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <condition_variable>
#include <exception>
#include <mutex>
#include <vector>

#include "../../include/nmodes.h"

namespace nm {

struct Error : std::runtime_error {
  nm_status code;
  Error(nm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_error(const std::string& m);

// body of a C entry point: status codes, no exception crosses the ABI
#define NM_TRY(...)                                    \
  try {                                                \
    nm::set_error("");                                 \
    __VA_ARGS__;                                       \
    return NM_OK;                                      \
  } catch (const nm::Error& e) {                       \
    nm::set_error(e.what());                           \
    return e.code;                                     \
  } catch (const std::bad_alloc&) {                    \
    nm::set_error("host allocation failed");           \
    return NM_ENOMEM;                                  \
  } catch (const std::exception& e) {                  \
    nm::set_error(e.what());                           \
    return NM_EDEVICE;                                 \
  }


#define NM_HIP(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      throw ::nm::Error(NM_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));    \
  } while (0)
#define NM_BLAS(x)                                                                      \
  do {                                                                                  \
    rocblas_status s_ = (x);                                                            \
    if (s_ != rocblas_status_success)                                                   \
      throw ::nm::Error(NM_EDEVICE, std::string(#x) + ": rocblas status " +             \
                                        std::to_string((int)s_));                       \
  } while (0)
#define NM_REQUIRE(cond, code, msg)                                                     \
  do {                                                                                  \
    if (!(cond)) throw ::nm::Error(code, msg);                                          \
  } while (0)

// Device allocator of the library's buffers (nm_set_allocator): the caller's
// functions, or hipMalloc / hipFree when none are set.
struct AllocHooks {
  void* (*alloc)(size_t, void*, void*) = nullptr;
  void (*free_)(void*, void*, void*) = nullptr;
  void* ctx = nullptr;
};
void set_alloc_hooks(const AllocHooks& h);
// allocates `bytes` with the current hooks and records them in *used (throws NM_ENOMEM)
void* dev_alloc(size_t bytes, AllocHooks* used);
// frees with the hooks that allocated p (caller's free after a device synchronisation)
void dev_free(void* p, const AllocHooks& used) noexcept;

// Owning device buffer.
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  AllocHooks h;  // the allocator that produced p
  DBuf() = default;
  explicit DBuf(size_t count) { alloc(count); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), h(o.h) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; h = o.h; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count) p = (T*)dev_alloc(count * sizeof(T), &h);
    n = count;
  }
  void release() {
    if (p) dev_free(p, h);
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// Reference-element tables (Appendix A): nodal Lagrange bases on the
// reference tetrahedron I = {r_i >= -1, r1+r2+r3 <= -1} and triangle.
struct RefTables {
  int nd, npp, nfd, nfp;          // nodes: disp/pres on tet, disp/pres on face
  double MM[10][10];              // mass  int_I l_a l_b
  double KR[3][3][10][10];        // (D_j^T M D_l)_{ab}
  double DR[3][10][10];           // (D_j^T M)_{ac}
  double Mp[10][10];              // pressure mass
  double Mfp[10][10];             // mixed mass int l^f_a l^p_c
  double QP[3][10][10];           // (M_fp D^p_l)_{ac} = int l^f_a d_l l^p_c
  double M2[6][6];                // face mass (disp)
  double M2sp[6][6];              // face mixed mass (disp x pres)
  double m_lo, m_hi, p_lo, p_hi;  // element bounds of spec(D^{-1} M), spec(D^{-1} K_p)
};
void build_ref_tables(int disp_order, int pres_order, RefTables& t);

// Small dense symmetric eigensolver (cyclic Jacobi), host, column-major a[n*n].
void jacobi_eig(int n, std::vector<double>& a, std::vector<double>& w, std::vector<double>* v);

}  // namespace nm

// The pencil: device-resident matrices and numbering.
struct nm_pencil {
  int device = 0;
  int disp_order = 1, pres_order = 1, nd = 4, npp = 4;
  int64_t V = 0, T = 0, n_geom = 0, N = 0, n_solid = 0, n_pres = 0;
  int64_t nnzb = 0, nnz_kp = 0, nnzb_eg = 0, n_fs = 0;
  double omega[3] = {0, 0, 0};
  bool gravity = false;
  nm::RefTables ref;
  // node graph (shared by A_G, M_s, R)
  nm::DBuf<int32_t> row_ptr, col;
  nm::DBuf<double> ag, ms, mdinv;  // ag [nnzb][9], ms [nnzb], mdinv [N] = 1/diag(M_s)
  // pressure graph
  nm::DBuf<int32_t> kp_ptr, kp_col;
  nm::DBuf<double> kp, kpdinv;
  // E_G by displacement node rows and its transpose by pressure rows, 3-vectors
  nm::DBuf<int32_t> eg_ptr, eg_col, egt_ptr, egt_col;
  nm::DBuf<double> eg_val, egt_val;
  // FP32 shadows (built on first use)
  nm::DBuf<float> ag32, ms32, mdinv32, kp32, kpdinv32, eg_val32, egt_val32;
  // numbering (device): canonical node -> geometric node; canonical <-> internal
  // (Hilbert-curve) order of the displacement nodes: internal = perm[canonical],
  // canonical = iperm[internal]
  nm::DBuf<int32_t> node_geom, pres_geom, perm, iperm;
  // row groups of the node graph (grouped mass solve): grp_rows 0 -> per-row kernel
  int grp_rows = 0;
  nm::DBuf<int32_t> grp_ptr, grp_col;
  nm::DBuf<double> grp_coef;
  nm::DBuf<float> grp_coef32;  // FP32 shadow (built with the other FP32 shadows)
  int grouped = 1;  // 0: per-row kernels only; 1: grouped from 32 columns; 2: grouped at any width
  int persist = 0;  // 1: each row-group step as one persistent launch (k_cj_group_persist)
  // LDS tiles of the node graph (tiled mass solve): tile_rows consecutive internal rows, the
  // sorted union of their columns, and each nonzero's position in its tile's union;
  // tile_umax / tile_emax: largest union and largest entry count of a tile (0: no tiles)
  int tile_rows = 0, tile_umax = 0, tile_emax = 0;
  int tiled = 0;  // 0: off (default); 1: tiles where they fit
  nm::DBuf<int32_t> tile_ptr, tile_col;
  nm::DBuf<uint16_t> tile_lcol;
  int tuned_block = 0;  // block width chosen by the autotuner (0: none)
  int tuned_tile = 0;   // tile rows chosen by the autotuner (0: none or no tiles)
  rocblas_handle blas = nullptr;
  // self-gravitation attached by nm_pencil_attach_selfgrav: A includes -C^T S C (FP64 operators)
  const nm_selfgrav* selfgrav = nullptr;
  std::mutex fp32_mx;  // the window threads of one pencil create the FP32 shadows once
  void ensure_fp32(hipStream_t st);
};

namespace nm {
// pattern + assembly (nm_assemble.hip)
void assemble(nm_pencil* P, const nm_mesh* mesh, const nm_material* mat, hipStream_t st);
// row groups and LDS tiles (nm_groups.hip)
// rows 0: from the environment (NM_ROW_GROUPS, NM_GROUP_ROWS; default 4), else groups of `rows` (4 or 8)
void build_row_groups(nm_pencil* P, hipStream_t st, int rows = 0);
// tiles of `rows` rows (0: NM_TILE_ROWS or 32, and NM_TILES=0 switches them off)
void build_tiles(nm_pencil* P, hipStream_t st, int rows = 0);

// operators (nm_ops.hip)
// Sampled HIP-event timing of the hot kernel (a middle Chebyshev-Jacobi
// step of the M solve): one launch in `every` is bracketed by events on
// its own stream; harvest() adds the elapsed times once the stream passed.
struct KernelProf {
  int every = 32;
  int64_t launches = 0, samples = 0;
  double ms = 0.0;
  std::vector<hipEvent_t> pool;  // pairs (start, stop)
  int used = 0;
  void before(hipStream_t st, bool& sampled);
  void after(hipStream_t st);
  void harvest();
  ~KernelProf();
};

struct ApplyCfg {
  int kM = 0, kP = 0;
  int precision = 0;
  // mass solve of an FP64 filter as mixP >= 2 FP32 Chebyshev-Jacobi passes of
  // mixK steps with FP64 residual corrections between them (0: one FP64 pass of kM)
  int mixP = 0, mixK = 0;
  KernelProf* prof = nullptr;
};
int cheb_steps(double lo, double hi, double tol);
// kernel of the middle mass-solve steps on b columns (FP32 or FP64 steps): 0 per-row, 1 row groups,
// 2 LDS tiles
int mass_kernel_kind(const nm_pencil* P, int b, bool fp32);
// sets cfg.mixP / mixK for `passes` (0 or 2..8; FP64 filters only) from the overall
// bound mtol, or kM_pass steps per pass when > 0; creates the FP32 shadows it reads
void set_mass_passes(nm_pencil* P, ApplyCfg& cfg, int passes, double mtol, int kM_pass, hipStream_t st);
// fastest block width and mass-solve kernel for this pencil (sets tuned_block and grouped)
void autotune(nm_pencil* P, int precision, hipStream_t st, int* best_b, double* best_us_per_col);
// dense block products on the FP64 matrix cores (nm_gemm.hip):
// C (col-major K x q) = A^T B with A [n][lda], B [n][ldb] row-major; ws: row-chunk partials
void gemm_tn(int64_t n, int K, int q, const double* A, int lda, const double* B, int ldb, double* C, DBuf<double>& ws,
             hipStream_t st);
// D ([n][ldd] row-major) = alpha A C + beta D with A [n][lda] row-major, C col-major K x q (ld ldc)
void gemm_nn(int64_t n, int K, int q, double alpha, const double* A, int lda, const double* C, int ldc, double beta,
             double* D, int ldd, hipStream_t st);
// work buffers of apply_op_ws for op on b columns: nvec vectors of `vec` elements,
// then npres vectors of `pres` elements (elements of the operator's precision)
struct OpWorkElems {
  size_t vec = 0, pres = 0;
  int nvec = 0, npres = 0;
  size_t elems() const { return vec * nvec + pres * npres; }
};
OpWorkElems op_work_elems(const nm_pencil* P, int op, int b);
// Y = op(X) in the internal node order with the work buffers in `work` (op_work_elems; no
// allocation, no synchronisation; FP32 operators need the FP32 matrices to exist; no mixed solve)
void apply_op_ws(const nm_pencil* P, int op, int ncols, const void* X, void* Y, const ApplyCfg& cfg, void* work,
                 hipStream_t st);
// operators on vectors in the internal node order
void apply_op(const nm_pencil* P, int op, int ncols, const void* X, void* Y, const ApplyCfg& cfg,
              hipStream_t st);
// the same on vectors in the canonical node order (C ABI)
void api_apply(const nm_pencil* P, int op, int ncols, const void* X, void* Y, const ApplyCfg& cfg,
               hipStream_t st);
// dst[r] = src[map[r]] for rows of w elements (8 or 4 bytes each)
void permute_rows(int64_t rows, int w, const void* src, void* dst, const int32_t* map, int elem_bytes,
                  hipStream_t st);

// work buffers of one B application: f, ya, yb [N][3b]; pt, pa, pb [n_p][b]
template <class T>
struct BWork {
  T *f = nullptr, *ya = nullptr, *yb = nullptr, *pt = nullptr, *pa = nullptr, *pb = nullptr;
};

// workspace for filter applications on a block of ncols columns
template <class T>
struct FilterWork {
  int b = 0;
  DBuf<T> x0, w0, w1, f, ya, yb, pt, ps, pa, pb;
  DBuf<T> mucols;  // per-column series coefficients of filter_apply_cols
  DBuf<float> s0, s1, s2, s3;  // FP32 right-hand side, iterates and first result of the mixed mass solve
  void ensure(const nm_pencil* P, int ncols);
  void ensure_mixed(const nm_pencil* P, int ncols);
  BWork<T> bwork() const { return BWork<T>{f.p, ya.p, yb.p, pt.p, pa.p, pb.p}; }
};
template <class T>
void filter_apply(const nm_pencil* P, const double* mu, int m, double c, double e, double l0,
                  double s0, int ncols, const T* X, T* Y, const ApplyCfg& cfg, FilterWork<T>& w,
                  hipStream_t st);
// one Chebyshev series per column: mu_cols host [m+1][ncols] (row k: the k-th coefficient of every column)
template <class T>
void filter_apply_cols(const nm_pencil* P, const double* mu_cols, int m, double c, double e, int ncols, const T* X,
                       T* Y, const ApplyCfg& cfg, FilterWork<T>& w, hipStream_t st);
template <class T>
void b_apply(const nm_pencil* P, int ncols, const T* X, T* Y, const ApplyCfg& cfg, FilterWork<T>& w,
             hipStream_t st);

// density of states: tau_k = (1/s) sum_v z_v . T_k((B - c)/e) z_v, k = 0..m (host tau[m+1]),
// Z device [n][s] in the internal node order
void dos_traces(const nm_pencil* P, double lmin, double lmax, int m, int s, const double* Z, const ApplyCfg& cfg,
                hipStream_t st, double* tau, bool weighted = false);
// column dot products out[v] = sum_r X[r*ldx+v] Y[r*ldy+v] (deterministic)
void col_dots(int64_t rows, int ncols, const double* X, int ldx, const double* Y, int ldy,
              double* out_dev, hipStream_t st);
void convert_f64_f32(int64_t n, const double* a, float* b, hipStream_t st);
void convert_f32_f64(int64_t n, const float* a, double* b, hipStream_t st);

// filter design (nm_eig.hip)
void jackson_chebyshev(double a, double b, double lmin, double lmax, int m, double* mu);
int choose_degree(double a, double b, double lmin, double lmax, double guard, int mode);
double cheb_eval(const double* mu, int m, double t);

void spectrum_bounds(const nm_pencil* P, int steps, uint64_t seed, hipStream_t st, double* lmin, double* lmax);
// rigorous upper bound of the Cowling pencil's spectrum (Gershgorin on D^{-1/2} A D^{-1/2}, element bounds)
double lmax_rigorous(const nm_pencil* P, hipStream_t st);
// Filter applications of several concurrent solves on one pencil, batched
// into one block (columns concatenated, one Chebyshev series per column):
// every solve thread submits its block and waits; the submission that
// completes the batch (all active solves waiting) runs it on the batch
// stream.  All solves share the filter interval [c - e, c + e] and the
// inner-solve configuration.
class FilterBatcher {
 public:
  FilterBatcher(const nm_pencil* P, int precision, const ApplyCfg& cfg, double c, double e, int active,
                hipStream_t st);
  // X, Y: device FP64 [n][bs], X complete when called; returns the degree applied (the batch's largest;
  // the series of lower-degree solves is zero-padded, which leaves their result unchanged)
  int filter(const double* X, double* Y, const double* mu, int m, int bs);
  // a solve stops submitting (finished or failed)
  void leave();
  KernelProf prof;

 private:
  struct Req {
    const double* X;
    double* Y;
    const double* mu;
    int m, bs, deg;
    bool done;
    std::exception_ptr err;
  };
  void run_locked();
  const nm_pencil* P_;
  int prec_;
  ApplyCfg cfg_;
  double c_, e_;
  int active_;
  hipStream_t st_;
  std::mutex mx_;
  std::condition_variable cv_;
  std::vector<Req*> pend_;
  FilterWork<double> fw_;
  FilterWork<float> fw32_;
  DBuf<double> xb_, yb_;
  DBuf<float> x32_, y32_;
};

// One solve's place in a FilterBatcher: left once, when the solve stops filtering (the end
// of its Lanczos loop, or an error), so the others' batches do not wait for its refinement.
struct BatchSeat {
  FilterBatcher* fb = nullptr;
  bool left = false;
  void leave() {
    if (fb && !left) fb->leave();
    left = true;
  }
};

// block width of a solve (options, autotuner, default)
int solve_block_width(const nm_pencil* P, const nm_eig_opts& o, int nev);
// seat: batch the filter applications with other solves (null factor not allowed);
// blas: rocBLAS handle to use (null: the pencil's)
void filtered_eig(const nm_pencil* P, double a, double b, int nev, double tol, const nm_eig_opts& o,
                  nm_eig_result** out, BatchSeat* seat = nullptr, rocblas_handle blas = nullptr);
// one solve per window [a[i], b[i]] (nev[i] pairs), each in its own host thread and stream,
// their filter applications batched; out[i] receives each result (NM_PARTIAL if any is partial)
void filtered_eig_slices(const nm_pencil* P, int S, const double* a, const double* b, const int* nev, double tol,
                         const nm_eig_opts& o, nm_eig_result** out);
// F -= C^T S C X (internal node order, FP64 [N][3 nc]; nm_selfgrav.hip)
void selfgrav_add(const nm_selfgrav* sg, int nc, const double* X, double* F, hipStream_t st);
void refine_rotation(const nm_pencil* P, const nm_eig_result* basis, const nm_rot_result* rot, double a, double b,
                     int iters, int degree, double tol, hipStream_t st, nm_rot_result** out);
void project_rotation(const nm_pencil* P, const nm_eig_result* basis, double a, double b,
                      hipStream_t st, nm_rot_result** out);

// Vector-block kernels index a block [N][3][ncols] with 32-bit lane ids and
// element offsets (row * 3 ncols + entry): a block of one launch must hold
// fewer than 2^32 elements.  Widest block for n = 3N displacement rows:
constexpr int64_t BLOCK_ELEMS_MAX = (int64_t)UINT32_MAX;
inline int64_t max_block_columns(int64_t n_disp) { return n_disp > 0 ? (BLOCK_ELEMS_MAX - 1) / n_disp : 0; }
// throws NM_EINVAL unless n_disp x ncols fits (checked before any allocation or launch)
inline void check_block(int64_t n_disp, int64_t ncols) {
  NM_REQUIRE(ncols >= 1 && ncols <= max_block_columns(n_disp), NM_EINVAL,
             "vector block of " + std::to_string(ncols) + " columns x " + std::to_string(n_disp) +
                 " rows exceeds the 2^32 elements a launch indexes (at most " +
                 std::to_string(max_block_columns(n_disp)) + " columns)");
}

// launch geometry: grid padded to a multiple of 8 workgroups so that the
// XCD-aware remap in the kernels is a bijection
inline unsigned grid_for(int64_t threads, int block = 256) {
  int64_t g = (threads + block - 1) / block;
  g = (g + 7) / 8 * 8;
  if (g < 8) g = 8;
  return (unsigned)g;
}
}  // namespace nm

// Workgroups are dispatched round-robin over the 8 XCDs (blockIdx % 8).
// Remap so that each XCD works on one contiguous eighth of the index range:
// neighbouring rows share vector gathers through that XCD's L2.
__device__ __forceinline__ int64_t nm_xcd_block() {
  const unsigned per = gridDim.x >> 3;
  return (int64_t)(blockIdx.x & 7u) * per + (blockIdx.x >> 3);
}
