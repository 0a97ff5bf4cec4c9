// nm_pencil_apply_noalloc: the operators of nm_pencil_apply for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops).  Every buffer beyond the caller's X and Y -- the vectors permuted to
// the internal node order and the iterates of the inner Chebyshev-Jacobi
// solves -- lives in one file-scope device array, `scratch`, of
// NM_SCRATCH_BYTES.  Each device holds its own copy of the array (from module
// load to process end); host code reaches it only through the device address
// that hipGetSymbolAddress returns for it, looked up once per device on the
// first call there.  Calls on one device share the array: calls that overlap
// in time on that device (other streams or threads) race on it; calls on one
// stream are ordered.  Nothing in the array needs to start at zero: every
// operator writes its work vectors before reading them.
#include <mutex>

#include "nm_internal.h"

namespace {

constexpr size_t NM_SCRATCH_BYTES = NM_NOALLOC_SCRATCH_BYTES;  // 256 MiB per device

static __device__ __align__(256) unsigned char scratch[NM_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mx;
void* g_scratch_ptr[MAX_DEVICES] = {};

// device address of this device's scratch array (looked up once per device, with that device current)
void* scratch_for(int dev) {
  NM_REQUIRE(dev >= 0 && dev < MAX_DEVICES, NM_EINVAL, "device id out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mx);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    NM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    NM_REQUIRE(p != nullptr, NM_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" {

nm_status nm_pencil_apply_noalloc(const nm_pencil* p, int32_t op, int32_t ncols, const void* X, void* Y,
                                  const nm_apply_opts* o, void* stream) {
  NM_TRY({
    NM_REQUIRE(p && X && Y && X != Y, NM_EINVAL, "invalid pointers");
    NM_REQUIRE(op >= NM_OP_AG && op <= NM_OP_B, NM_EINVAL, "unknown operator");
    nm::check_block(3 * p->N, ncols);
    NM_REQUIRE(!o || o->mass_passes == 0, NM_EINVAL,
               "mass_passes is not available without allocation (its FP32 work vectors)");
    int dev = -1;
    NM_HIP(hipGetDevice(&dev));
    NM_REQUIRE(dev == p->device, NM_EINVAL, "the pencil's device is not the current device");
    nm::ApplyCfg cfg;
    const double mt = (o && o->minv_tol > 0) ? o->minv_tol : 1e-12;
    const double pt = (o && o->kp_tol > 0) ? o->kp_tol : 1e-13;
    cfg.kM = (o && o->kM > 0) ? o->kM : nm::cheb_steps(p->ref.m_lo, p->ref.m_hi, mt);
    cfg.kP = (o && o->kP > 0) ? o->kP : nm::cheb_steps(p->ref.p_lo, p->ref.p_hi, pt);
    cfg.precision = o ? o->precision : 0;
    NM_REQUIRE(cfg.precision == 0 || cfg.precision == 1, NM_EINVAL, "precision must be 0 or 1");
    NM_REQUIRE(cfg.kM >= 2 && cfg.kP >= 1, NM_EINVAL, "kM must be >= 2 and kP >= 1");
    NM_REQUIRE(cfg.precision == 0 || p->ms32.p, NM_EINVAL,
               "precision 1 needs the pencil's FP32 matrices: run one FP32 operator or solve with allocation first");
    // scratch layout: [X permuted][Y internal][operator work], each 256-byte aligned
    const size_t eb = cfg.precision == 1 ? 4 : 8;
    const bool in_disp = !(op == NM_OP_KP || op == NM_OP_EG || op == NM_OP_KPINV);
    const bool out_disp = !(op == NM_OP_KP || op == NM_OP_EGT || op == NM_OP_KPINV);
    const size_t blk = (size_t)p->N * 3 * ncols * eb;
    const size_t xb = in_disp ? round256(blk) : 0, yb = out_disp ? round256(blk) : 0;
    const size_t wb = round256(nm::op_work_elems(p, op, ncols).elems() * eb);
    const size_t need = xb + yb + wb;
    NM_REQUIRE(need <= NM_SCRATCH_BYTES, NM_EINVAL,
               "operator " + std::to_string(op) + " on " + std::to_string(ncols) + " columns needs " +
                   std::to_string(need) + " bytes of scratch; the no-allocation entry point holds " +
                   std::to_string(NM_SCRATCH_BYTES) + " (use nm_pencil_apply)");
    hipStream_t st = (hipStream_t)stream;
    unsigned char* base = (unsigned char*)scratch_for(dev);
    const void* xin = X;
    void* yout = Y;
    const int w = 3 * ncols;
    if (in_disp) {
      nm::permute_rows(p->N, w, X, base, p->iperm.p, (int)eb, st);
      xin = base;
    }
    if (out_disp) yout = base + xb;
    nm::apply_op_ws(p, op, ncols, xin, yout, cfg, base + xb + yb, st);
    if (out_disp) nm::permute_rows(p->N, w, yout, Y, p->perm.p, (int)eb, st);
    NM_HIP(hipGetLastError());
  })
}

}  // extern "C"
