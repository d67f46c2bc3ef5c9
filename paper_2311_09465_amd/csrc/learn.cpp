// Learned warm start: a reduced basis of modal solutions (greedy selection
// with CGS2 orthonormalization on the Krylov kernels) and a tanh MLP that maps
// inflow parameters to reduced-basis coefficients, trained with Adam on the
// MFMA kernels of mlp.hip.  Public ABI in include/tsgls.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "../../include/tsgls.h"
#include "internal.h"

using namespace tsgls;

struct tsgls_mlp {
  int n_in = 0, width = 0, n_hidden = 0, n_out = 0, bf16 = 1;
  hipStream_t st = nullptr;
  std::vector<int> dims;                 // d[0] = n_in, d[1..n_hidden] = width, d[L] = n_out
  std::vector<int64_t> woff, boff;       // offsets of W_l [d[l+1]][d[l]] and b_l in params
  int64_t n_params = 0;
  float* params = nullptr;               // FP32 master weights
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* dloss = nullptr;
  int64_t step = 0;
  int batch_cap = 0;                     // activation buffers sized for this batch
  std::vector<float*> H;                 // [n_hidden] layer outputs [B][width]
  float* O = nullptr;                    // [B][n_out]
  float* dZa = nullptr;                  // ping-pong gradients [B][max d]
  float* dZb = nullptr;
  std::string err;
};

namespace {

int mfail(tsgls_mlp* m, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (m) m->err = buf;
  return code;
}

#define MHIP(m, call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return mfail(m, TSGLS_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define RHIP(call)                                          \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) { rc = TSGLS_EHIP; goto done; }   \
  } while (0)

// splitmix64 (Steele, Lea, Flood 2014) -> uniform in [-1, 1)
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform_pm1(uint64_t& s) { return (double)(splitmix64(s) >> 11) * 0x1.0p-52 - 1.0; }

void free_acts(tsgls_mlp* m) {
  for (float* p : m->H) (void)hipFree(p);
  m->H.clear();
  (void)hipFree(m->O);
  (void)hipFree(m->dZa);
  (void)hipFree(m->dZb);
  m->O = m->dZa = m->dZb = nullptr;
  m->batch_cap = 0;
}

int ensure_acts(tsgls_mlp* m, int B) {
  if (B <= m->batch_cap) return TSGLS_OK;
  free_acts(m);
  const int dmax = *std::max_element(m->dims.begin(), m->dims.end());
  m->H.assign(m->n_hidden, nullptr);
  for (int l = 0; l < m->n_hidden; ++l) MHIP(m, hipMalloc(&m->H[l], sizeof(float) * (size_t)B * m->width));
  MHIP(m, hipMalloc(&m->O, sizeof(float) * (size_t)B * m->n_out));
  MHIP(m, hipMalloc(&m->dZa, sizeof(float) * (size_t)B * dmax));
  MHIP(m, hipMalloc(&m->dZb, sizeof(float) * (size_t)B * dmax));
  m->batch_cap = B;
  return TSGLS_OK;
}

// y = MLP(x) for B rows; layer outputs kept in m->H, result in m->O.
int forward(tsgls_mlp* m, const float* x, int B) {
  const int L = m->n_hidden + 1;
  const float* in = x;
  for (int l = 0; l < L; ++l) {
    const int din = m->dims[l], dout = m->dims[l + 1];
    float* out = l < L - 1 ? m->H[l] : m->O;
    const float* W = m->params + m->woff[l];
    const float* b = m->params + m->boff[l];
    // out[b][j] = act(sum_k in[b][k] W[j][k] + b[j])
    MHIP(m, launch_mlp_gemm(m->bf16, l < L - 1 ? 1 : 0, B, dout, din, in, din, 1, W, 1, din, b,
                            nullptr, out, dout, m->st));
    in = out;
  }
  return TSGLS_OK;
}

}  // namespace

extern "C" {

int tsgls_mlp_create(int n_in, int width, int n_hidden, int n_out, int precision, uint64_t seed,
                     void* hip_stream, tsgls_mlp** out) {
  if (!out) return TSGLS_EINVAL;
  *out = nullptr;
  if (n_in < 1 || width < 1 || n_hidden < 1 || n_out < 1 || n_in > 65536 || width > 65536 ||
      n_hidden > 64 || n_out > 65536 || (precision != TSGLS_MLP_BF16 && precision != TSGLS_MLP_F32))
    return TSGLS_EINVAL;
  tsgls_mlp* m = new (std::nothrow) tsgls_mlp();
  if (!m) return TSGLS_ENOMEM;
  *out = m;
  m->n_in = n_in;
  m->width = width;
  m->n_hidden = n_hidden;
  m->n_out = n_out;
  m->bf16 = precision == TSGLS_MLP_BF16;
  m->st = (hipStream_t)hip_stream;
  m->dims.push_back(n_in);
  for (int l = 0; l < n_hidden; ++l) m->dims.push_back(width);
  m->dims.push_back(n_out);
  int64_t off = 0;
  for (int l = 0; l <= n_hidden; ++l) {
    m->woff.push_back(off);
    off += (int64_t)m->dims[l + 1] * m->dims[l];
    m->boff.push_back(off);
    off += m->dims[l + 1];
  }
  m->n_params = off;
  std::vector<float> h((size_t)off, 0.f);
  uint64_t s = seed;
  for (int l = 0; l <= n_hidden; ++l) {   // W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), b = 0
    const double sc = 1.0 / std::sqrt((double)m->dims[l]);
    const int64_t nw = (int64_t)m->dims[l + 1] * m->dims[l];
    for (int64_t i = 0; i < nw; ++i) h[(size_t)(m->woff[l] + i)] = (float)(sc * uniform_pm1(s));
  }
  const size_t bytes = sizeof(float) * (size_t)off;
  MHIP(m, hipMalloc(&m->params, bytes));
  MHIP(m, hipMalloc(&m->grads, bytes));
  MHIP(m, hipMalloc(&m->adam_m, bytes));
  MHIP(m, hipMalloc(&m->adam_v, bytes));
  MHIP(m, hipMalloc(&m->dloss, sizeof(float)));
  MHIP(m, hipMemcpyAsync(m->params, h.data(), bytes, hipMemcpyHostToDevice, m->st));
  std::fill(h.begin(), h.end(), 0.f);
  MHIP(m, hipMemcpyAsync(m->grads, h.data(), bytes, hipMemcpyHostToDevice, m->st));
  MHIP(m, hipMemcpyAsync(m->adam_m, h.data(), bytes, hipMemcpyHostToDevice, m->st));
  MHIP(m, hipMemcpyAsync(m->adam_v, h.data(), bytes, hipMemcpyHostToDevice, m->st));
  MHIP(m, hipStreamSynchronize(m->st));
  return TSGLS_OK;
}

int tsgls_mlp_num_params(const tsgls_mlp* m, int64_t* count) {
  if (!m || !count) return TSGLS_EINVAL;
  *count = m->n_params;
  return TSGLS_OK;
}

int tsgls_mlp_get_params(tsgls_mlp* m, float* host_out, float* grad_out) {
  if (!m || (!host_out && !grad_out)) return TSGLS_EINVAL;
  const size_t bytes = sizeof(float) * (size_t)m->n_params;
  if (host_out) MHIP(m, hipMemcpyAsync(host_out, m->params, bytes, hipMemcpyDeviceToHost, m->st));
  if (grad_out) MHIP(m, hipMemcpyAsync(grad_out, m->grads, bytes, hipMemcpyDeviceToHost, m->st));
  MHIP(m, hipStreamSynchronize(m->st));
  return TSGLS_OK;
}

int tsgls_mlp_set_params(tsgls_mlp* m, const float* host_in) {
  if (!m || !host_in) return TSGLS_EINVAL;
  const size_t bytes = sizeof(float) * (size_t)m->n_params;
  MHIP(m, hipMemcpyAsync(m->params, host_in, bytes, hipMemcpyHostToDevice, m->st));
  MHIP(m, hipStreamSynchronize(m->st));
  m->step = 0;
  return TSGLS_OK;
}

int tsgls_mlp_forward(tsgls_mlp* m, const float* x, int B, float* y) {
  if (!m) return TSGLS_EINVAL;
  if (!x || !y || B < 1) return mfail(m, TSGLS_EINVAL, "bad forward arguments");
  int rc = ensure_acts(m, B);
  if (rc != TSGLS_OK) return rc;
  rc = forward(m, x, B);
  if (rc != TSGLS_OK) return rc;
  MHIP(m, hipMemcpyAsync(y, m->O, sizeof(float) * (size_t)B * m->n_out, hipMemcpyDeviceToDevice, m->st));
  return TSGLS_OK;
}

int tsgls_mlp_gradient(tsgls_mlp* m, const float* x, const float* t, int B, float* loss) {
  if (!m) return TSGLS_EINVAL;
  if (!x || !t || B < 1) return mfail(m, TSGLS_EINVAL, "bad gradient arguments");
  int rc = ensure_acts(m, B);
  if (rc != TSGLS_OK) return rc;
  rc = forward(m, x, B);
  if (rc != TSGLS_OK) return rc;
  const int L = m->n_hidden + 1;
  float* dZ = m->dZa;
  float* dZn = m->dZb;
  MHIP(m, launch_mse(m->O, t, dZ, m->dloss, (int64_t)B * m->n_out, m->st));
  for (int l = L - 1; l >= 0; --l) {
    const int din = m->dims[l], dout = m->dims[l + 1];
    const float* in = l == 0 ? x : m->H[l - 1];
    // dW[j][k] = sum_b dZ[b][j] in[b][k]
    MHIP(m, launch_mlp_gemm(m->bf16, 0, dout, din, B, dZ, 1, dout, in, din, 1, nullptr, nullptr,
                            m->grads + m->woff[l], din, m->st));
    MHIP(m, launch_colsum(dZ, B, dout, m->grads + m->boff[l], m->st));
    if (l > 0) {
      // dZ_prev[b][k] = (sum_j dZ[b][j] W[j][k]) (1 - H_prev[b][k]^2)
      MHIP(m, launch_mlp_gemm(m->bf16, 2, B, din, dout, dZ, dout, 1, m->params + m->woff[l], din, 1,
                              nullptr, m->H[l - 1], dZn, din, m->st));
      std::swap(dZ, dZn);
    }
  }
  if (loss) {
    MHIP(m, hipMemcpyAsync(loss, m->dloss, sizeof(float), hipMemcpyDeviceToHost, m->st));
    MHIP(m, hipStreamSynchronize(m->st));
  }
  return TSGLS_OK;
}

int tsgls_mlp_adam_step(tsgls_mlp* m, float lr, float beta1, float beta2, float eps) {
  if (!m) return TSGLS_EINVAL;
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return mfail(m, TSGLS_EINVAL, "bad Adam parameters");
  ++m->step;
  const float c1 = 1.f - std::pow(beta1, (float)m->step);
  const float c2 = 1.f - std::pow(beta2, (float)m->step);
  MHIP(m, launch_adam(m->params, m->grads, m->adam_m, m->adam_v, m->n_params, lr, beta1, beta2, eps,
                      c1, c2, m->st));
  return TSGLS_OK;
}

const char* tsgls_mlp_last_error(const tsgls_mlp* m) { return m ? m->err.c_str() : "null network"; }

void tsgls_mlp_destroy(tsgls_mlp* m) {
  if (!m) return;
  if (m->st) (void)hipStreamSynchronize(m->st);
  free_acts(m);
  (void)hipFree(m->params);
  (void)hipFree(m->grads);
  (void)hipFree(m->adam_m);
  (void)hipFree(m->adam_v);
  (void)hipFree(m->dloss);
  delete m;
}

// ------------------------------------------------------------ reduced basis
int tsgls_rb_greedy(const double* Y, int64_t N, int64_t D, const double* mean, int r, double* Phi,
                    int32_t* picked, void* hip_stream) {
  if (!Y || !mean || !Phi || !picked || N < 1 || N > 65536 || D < 1 || r < 1 || r > N || r > 1024)
    return TSGLS_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  const int nb = multidot_blocks(D);
  double *Yc = nullptr, *partial = nullptr, *dd = nullptr;
  int rc = TSGLS_OK, built = 0;
  std::vector<double> nrm(N), proj(N, 0.0), c(N), h(r);
  std::vector<char> used(N, 0);
  RHIP(hipMalloc(&Yc, sizeof(double) * (size_t)N * D));
  RHIP(hipMalloc(&partial, sizeof(double) * (size_t)nb * 1024));
  RHIP(hipMalloc(&dd, sizeof(double) * (size_t)std::max<int64_t>(2048, N)));
  // centered snapshots and their squared norms
  RHIP(launch_copy(Y, Yc, N * D, st));
  for (int64_t i = 0; i < N; ++i) RHIP(launch_axpy(-1.0, mean, Yc + i * D, D, st));
  for (int64_t i = 0; i < N; ++i) {
    RHIP(launch_multidot(Yc + i * D, 0, 1, Yc + i * D, partial, nb, D, st));
    RHIP(launch_reduce_partials(partial, nb, 1, dd + i, st));
  }
  RHIP(hipMemcpyAsync(nrm.data(), dd, sizeof(double) * N, hipMemcpyDeviceToHost, st));
  RHIP(hipStreamSynchronize(st));
  {
    const double top = *std::max_element(nrm.begin(), nrm.end());
    for (int s = 0; s < r; ++s) {
      // the snapshot worst represented by the current basis
      int64_t best = -1;
      double bv = -1.0;
      for (int64_t i = 0; i < N; ++i)
        if (!used[i] && nrm[i] - proj[i] > bv) {
          bv = nrm[i] - proj[i];
          best = i;
        }
      if (best < 0 || !(bv > 1e-24 * top)) break;
      used[best] = 1;
      double* phi = Phi + (int64_t)s * D;
      RHIP(launch_copy(Yc + best * D, phi, D, st));
      for (int pass = 0; pass < 2 && s > 0; ++pass) {   // CGS2 against phi_0 .. phi_{s-1}
        RHIP(launch_multidot(Phi, D, s, phi, partial, nb, D, st));
        RHIP(launch_reduce_partials(partial, nb, s, dd, st));
        RHIP(launch_multiaxpy(Phi, D, s, dd, phi, D, st));
      }
      RHIP(launch_multidot(phi, 0, 1, phi, partial, nb, D, st));
      RHIP(launch_reduce_partials(partial, nb, 1, dd, st));
      RHIP(hipMemcpyAsync(h.data(), dd, sizeof(double), hipMemcpyDeviceToHost, st));
      RHIP(hipStreamSynchronize(st));
      if (!(h[0] > 1e-24 * top)) break;
      RHIP(launch_scal_copy(1.0 / std::sqrt(h[0]), phi, phi, D, st));
      // coefficients of every snapshot on the new basis vector (1,024 rows per pass)
      for (int64_t i0 = 0; i0 < N; i0 += 1024) {
        const int J = (int)std::min<int64_t>(1024, N - i0);
        RHIP(launch_multidot(Yc + i0 * D, D, J, phi, partial, nb, D, st));
        RHIP(launch_reduce_partials(partial, nb, J, dd + i0, st));
      }
      RHIP(hipMemcpyAsync(c.data(), dd, sizeof(double) * N, hipMemcpyDeviceToHost, st));
      RHIP(hipStreamSynchronize(st));
      for (int64_t i = 0; i < N; ++i) proj[i] += c[i] * c[i];
      picked[s] = (int32_t)best;
      built = s + 1;
    }
  }
done:
  (void)hipStreamSynchronize(st);
  (void)hipFree(Yc);
  (void)hipFree(partial);
  (void)hipFree(dd);
  return rc == TSGLS_OK ? built : rc;
}

int tsgls_rb_project(const double* Phi, int r, int64_t D, const double* Y, int64_t N,
                     const double* mean, double* coef, void* hip_stream) {
  if (!Phi || !Y || !mean || !coef || r < 1 || r > 1024 || D < 1 || N < 0) return TSGLS_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  const int nb = multidot_blocks(D);
  double *partial = nullptr, *pm = nullptr;
  int rc = TSGLS_OK;
  RHIP(hipMalloc(&partial, sizeof(double) * (size_t)nb * 1024));
  RHIP(hipMalloc(&pm, sizeof(double) * (size_t)r));
  RHIP(launch_multidot(Phi, D, r, mean, partial, nb, D, st));
  RHIP(launch_reduce_partials(partial, nb, r, pm, st));
  for (int64_t i = 0; i < N; ++i) {   // coef_i = Phi (y_i - mean)
    RHIP(launch_multidot(Phi, D, r, Y + i * D, partial, nb, D, st));
    RHIP(launch_reduce_partials(partial, nb, r, coef + i * r, st));
    RHIP(launch_axpy(-1.0, pm, coef + i * r, r, st));
  }
done:
  (void)hipStreamSynchronize(st);
  (void)hipFree(partial);
  (void)hipFree(pm);
  return rc;
}

int tsgls_rb_expand(const double* Phi, int r, int64_t D, const double* coef, const double* mean,
                    double* y, void* hip_stream) {
  if (!Phi || !coef || !mean || !y || r < 1 || r > 1024 || D < 1) return TSGLS_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  if (launch_copy(mean, y, D, st) != hipSuccess) return TSGLS_EHIP;
  if (launch_multiaxpy_add(Phi, D, r, coef, y, D, st) != hipSuccess) return TSGLS_EHIP;
  return TSGLS_OK;
}

}  // extern "C"
