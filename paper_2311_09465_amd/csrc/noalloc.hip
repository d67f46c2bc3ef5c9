// Reduced-basis projection for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the reductions of tsgls_rb_project with their block partial
// sums and the projected mean held in one fixed device array per GPU instead
// of buffers allocated per call.  Public ABI in include/tsgls.h.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/tsgls.h"
#include "internal.h"

using namespace tsgls;

namespace {

// Block partials of the multi-dot (multidot_blocks() gives at most 1024
// blocks, each writing one value per basis vector, r <= 1024) followed by the
// projected mean (r values): 1024 * 1024 + 1024 doubles, 8.0 MiB per GPU,
// held until the process ends.
constexpr int kMaxBasis = 1024;
constexpr int64_t kPartialDoubles = (int64_t)1024 * kMaxBasis;
constexpr int64_t kScratchDoubles = kPartialDoubles + kMaxBasis;
static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of each GPU's copy of scratch, looked up on the first call
// made with that GPU current.  The symbol's name is a host-side stand-in and
// is never passed to a kernel; only these addresses are.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

int scratch_address(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return TSGLS_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return TSGLS_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TSGLS_EHIP;
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return TSGLS_OK;
}

}  // namespace

extern "C" int tsgls_rb_project_noalloc(const double* Phi, int r, int64_t D, const double* Y,
                                        int64_t N, const double* mean, double* coef,
                                        void* hip_stream) {
  if (!Phi || !Y || !mean || !coef || r < 1 || D < 1 || N < 0) return TSGLS_EINVAL;
  if (r > kMaxBasis) return TSGLS_ESCRATCH;
  const int nb = multidot_blocks(D);
  if ((int64_t)nb * r > kPartialDoubles) return TSGLS_ESCRATCH;
  double* base = nullptr;
  const int rc = scratch_address(&base);
  if (rc != TSGLS_OK) return rc;
  double* partial = base;                  // [nb][r], fully written by each multi-dot
  double* pm = base + kPartialDoubles;     // [r] Phi mean, written by the first reduction
  hipStream_t st = (hipStream_t)hip_stream;
  if (launch_multidot(Phi, D, r, mean, partial, nb, D, st) != hipSuccess) return TSGLS_EHIP;
  if (launch_reduce_partials(partial, nb, r, pm, st) != hipSuccess) return TSGLS_EHIP;
  for (int64_t i = 0; i < N; ++i) {   // coef_i = Phi (y_i - mean)
    if (launch_multidot(Phi, D, r, Y + i * D, partial, nb, D, st) != hipSuccess) return TSGLS_EHIP;
    if (launch_reduce_partials(partial, nb, r, coef + i * r, st) != hipSuccess) return TSGLS_EHIP;
    if (launch_axpy(-1.0, pm, coef + i * r, r, st) != hipSuccess) return TSGLS_EHIP;
  }
  return TSGLS_OK;
}
