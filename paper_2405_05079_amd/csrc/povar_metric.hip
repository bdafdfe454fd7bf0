// Metric upgrade (autocalibration) of a projective reconstruction with known
// intrinsics: the "Metric Upgrade" section of the supplement (App. D).
//
// Find H = [[A, 0], [c^T, 1]] such that every P_i H is a scaled K_i [R_i | t_i].
// With H~ the three left columns of H and Q_i = K_i^-1 P_i, the constraint is
// alpha_i Q_i H~ H~^T Q_i^T = I, and c with the scales alpha_i minimises
//   f(c) = sum_i || alpha_i Q_i H~(c) H~(c)^T Q_i^T - I ||_F^2
// by variable projection: each alpha_i is linear and eliminated in closed
// form, alpha_i = tr(M_i) / ||M_i||_F^2 with M_i = B_i B_i^T, B_i = Q_i H~;
// Levenberg-Marquardt runs on the reduced residual over c (3 values).
//
// H~ depends on c alone, so A is fixed by a choice of frame: the cameras are
// first moved to the frame where camera 0 is [I | 0] (T = [[M^-1, -M^-1 m],
// [0, 1]] for P_0 = [M | m]), and A = K_0.
//
// Derivatives: B_i = Q_i[:, :3] K_0 + q_i c^T with q_i = Q_i[:, 3], so
// dB_i / dc_k = q_i e_k^T and dM_i / dc_k = q_i b_k^T + b_k q_i^T (b_k the
// k-th column of B_i), the product rule that the theorem on the derivative of
// H~ H~^T in App. D states in Kronecker form; then
// d alpha = (tr dM - 2 alpha <M, dM>) / ||M||^2 and J_k = alpha dM_k + M d alpha.
//
// One thread per camera for the per-camera terms (a 3 x 4 matrix in, ten
// sums out); fixed-order block reductions; one workgroup for the 3 x 3 LM
// step and the accept/reject decision, which stay on the device.  Everything
// is FP64.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include <map>
#include <mutex>

#include "povar.h"
#include "povar_host.h"

// Device scratch of povar_metric_upgrade_noalloc: every buffer of one call
// (control block, camera copies, per-block partials, outputs, traces) is
// carved from this array instead of being allocated.  Each GPU the library
// runs on holds its own copy until the process ends; calls that overlap on
// one GPU share it and race.  In host code `scratch` names a host-side
// stand-in: its device address comes from hipGetSymbolAddress, once per
// device (metric_scratch_init), and only that address is used.
static constexpr size_t kMetricScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kMetricScratchBytes];

namespace povar {

namespace {
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_addr;   // device -> address of `scratch` there

// The scratch address of a device (nullptr until metric_scratch_init ran on it).
char* metric_scratch(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  return it == g_scratch_addr.end() ? nullptr : it->second;
}
}  // namespace

povar_status metric_scratch_init(povar_ctx ctx) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_addr.count(ctx->device)) return POVAR_OK;
  void* ptr = nullptr;   // ctx->device is current (povar_ctx_create)
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    set_error(ctx, "hipGetSymbolAddress of the metric-upgrade scratch failed: %s", hipGetErrorString(e));
    return POVAR_EDEVICE;
  }
  g_scratch_addr[ctx->device] = static_cast<char*>(ptr);
  return POVAR_OK;
}

namespace {

constexpr int kMBlock = 256;
constexpr int kMVals = 10;   // per-block partials: J^T J (6), J^T r (3), cost

struct MetricCtl {
  double T[16];        // reference frame (row-major 4 x 4)
  double K0[9];
  double c[3], c_trial[3];
  double A[6], g[3];   // J^T J (00, 01, 02, 11, 12, 22) and J^T r at c
  double cost, cost_trial, cost0, lambda, ftol;
  double H[16];        // T [[K_0, 0], [c^T, 1]] after the solve
  int32_t need_lin, done, iters, max_iters;
  int32_t status;      // bit 0: camera 0 has a singular 3 x 3 part; bit 1: no step factored
  int32_t have_cost0, debug_no_step;
  int32_t stop;        // 1: small accepted decrease (ftol), 2: damping at its cap, 3: max_iters
  int32_t pad;
};

struct MetricArgs {
  MetricCtl* ctl;
  const double* P;     // n x 12
  const double* K;     // n x 9
  double* Q;           // n x 12
  double* part;        // blocks x kMVals
  double* alpha;       // n
  double* R;           // n x 9
  double* t;           // n x 3
  double* tr_cost;     // max_iters
  int32_t* tr_acc;     // max_iters
  int32_t n, blocks;
};

__device__ __forceinline__ double det3(const double (&m)[9]) {
  return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
         m[2] * (m[3] * m[7] - m[4] * m[6]);
}

// cofactor matrix: inverse transpose times the determinant
__device__ __forceinline__ void cof3(const double (&m)[9], double (&o)[9]) {
  o[0] = m[4] * m[8] - m[5] * m[7];
  o[1] = m[5] * m[6] - m[3] * m[8];
  o[2] = m[3] * m[7] - m[4] * m[6];
  o[3] = m[2] * m[7] - m[1] * m[8];
  o[4] = m[0] * m[8] - m[2] * m[6];
  o[5] = m[1] * m[6] - m[0] * m[7];
  o[6] = m[1] * m[5] - m[2] * m[4];
  o[7] = m[2] * m[3] - m[0] * m[5];
  o[8] = m[0] * m[4] - m[1] * m[3];
}

// K^-1 y for an upper-triangular K (row-major 3 x 3)
__device__ __forceinline__ void ktri_solve(const double* K, double y0, double y1, double y2, double& x0, double& x1,
                                           double& x2) {
  x2 = y2 / K[8];
  x1 = (y1 - K[5] * x2) / K[4];
  x0 = (y0 - K[1] * x1 - K[2] * x2) / K[0];
}

// Sum of kMVals values over the workgroup in a fixed order (LDS tree).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* out) {
  __shared__ double sh[NV][kMBlock];
  const int tid = (int)threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) sh[k][tid] = v[k];
  __syncthreads();
  for (int s = kMBlock / 2; s > 0; s >>= 1) {
    if (tid < s)
#pragma unroll
      for (int k = 0; k < NV; ++k) sh[k][tid] += sh[k][tid + s];
    __syncthreads();
  }
  if (tid < NV) out[tid] = sh[tid][0];
}

// k_metric_frame: T from camera 0, K_0, and the LM state (one thread).
__global__ void k_metric_frame(MetricArgs a, double lambda0) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  MetricCtl& C = *a.ctl;
  double M[9], co[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) M[r * 3 + k] = a.P[r * 4 + k];
  const double det = det3(M);
  double nrm = 0.0;
  for (int k = 0; k < 9; ++k) nrm += M[k] * M[k];
  if (!(fabs(det) > 1e-14 * nrm * sqrt(nrm))) C.status |= 1;
  cof3(M, co);
  const double id = 1.0 / det;
  // M^-1 = co^T / det
  for (int r = 0; r < 3; ++r) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double v = co[k * 3 + r] * id;
      C.T[r * 4 + k] = v;
      s += v * a.P[k * 4 + 3];
    }
    C.T[r * 4 + 3] = -s;
  }
  C.T[12] = C.T[13] = C.T[14] = 0.0;
  C.T[15] = 1.0;
  for (int k = 0; k < 9; ++k) C.K0[k] = a.K[k];
  for (int k = 0; k < 3; ++k) C.c[k] = C.c_trial[k] = 0.0;
  C.lambda = lambda0;
  C.need_lin = 1;
  C.done = 0;
  C.iters = 0;
  C.have_cost0 = 0;
}

// k_metric_normalize: Q_i = K_i^-1 P_i T, one thread per camera.
__global__ void __launch_bounds__(kMBlock) k_metric_normalize(MetricArgs a) {
  const int i = (int)(blockIdx.x * kMBlock + threadIdx.x);
  if (i >= a.n) return;
  const MetricCtl& C = *a.ctl;
  const double* P = a.P + (size_t)i * 12;
  double pt[12];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 4; ++k)
      pt[r * 4 + k] = P[r * 4] * C.T[k] + P[r * 4 + 1] * C.T[4 + k] + P[r * 4 + 2] * C.T[8 + k] + P[r * 4 + 3] * C.T[12 + k];
  const double* K = a.K + (size_t)i * 9;
  double* Q = a.Q + (size_t)i * 12;
  for (int k = 0; k < 4; ++k) {
    double x0, x1, x2;
    ktri_solve(K, pt[k], pt[4 + k], pt[8 + k], x0, x1, x2);
    Q[k] = x0;
    Q[4 + k] = x1;
    Q[8 + k] = x2;
  }
}

// B = Q[:, :3] K_0 + q c^T and M = B B^T for one camera.
struct CamTerms {
  double B[9], q[3], M[6];   // M: 00, 01, 02, 11, 12, 22
  double mm, tr, alpha;
};

__device__ __forceinline__ void cam_terms(const double* Q, const double* K0, const double* c, CamTerms& o) {
  for (int r = 0; r < 3; ++r) {
    o.q[r] = Q[r * 4 + 3];
    for (int k = 0; k < 3; ++k)
      o.B[r * 3 + k] = Q[r * 4] * K0[k] + Q[r * 4 + 1] * K0[3 + k] + Q[r * 4 + 2] * K0[6 + k] + o.q[r] * c[k];
  }
  int u = 0;
  for (int r = 0; r < 3; ++r)
    for (int s = r; s < 3; ++s)
      o.M[u++] = o.B[r * 3] * o.B[s * 3] + o.B[r * 3 + 1] * o.B[s * 3 + 1] + o.B[r * 3 + 2] * o.B[s * 3 + 2];
  o.tr = o.M[0] + o.M[3] + o.M[5];
  o.mm = o.M[0] * o.M[0] + o.M[3] * o.M[3] + o.M[5] * o.M[5] +
         2.0 * (o.M[1] * o.M[1] + o.M[2] * o.M[2] + o.M[4] * o.M[4]);
  o.alpha = o.tr / o.mm;
}

// Frobenius inner product of two symmetric 3 x 3 matrices in the 6-value form
__device__ __forceinline__ double sym_dot(const double (&x)[6], const double (&y)[6]) {
  return x[0] * y[0] + x[3] * y[3] + x[5] * y[5] + 2.0 * (x[1] * y[1] + x[2] * y[2] + x[4] * y[4]);
}

// k_metric_terms: per camera the reduced residual r_i = alpha_i M_i - I and,
// for the linearisation, J_k; per workgroup the sums J^T J, J^T r and the cost.
template <bool Lin>
__global__ void __launch_bounds__(kMBlock) k_metric_terms(MetricArgs a) {
  const MetricCtl& C = *a.ctl;
  if (C.done || (Lin ? !C.need_lin : (C.status & 2) != 0)) return;
  const int i = (int)(blockIdx.x * kMBlock + threadIdx.x);
  double v[kMVals];
  for (int k = 0; k < kMVals; ++k) v[k] = 0.0;
  if (i < a.n) {
    CamTerms m;
    cam_terms(a.Q + (size_t)i * 12, C.K0, Lin ? C.c : C.c_trial, m);
    double r[6];
    for (int k = 0; k < 6; ++k) r[k] = m.alpha * m.M[k];
    r[0] -= 1.0;
    r[3] -= 1.0;
    r[5] -= 1.0;
    v[9] = sym_dot(r, r);
    if (Lin) {
      double J[3][6];
      for (int k = 0; k < 3; ++k) {
        const double b0 = m.B[k], b1 = m.B[3 + k], b2 = m.B[6 + k];
        const double dM[6] = {2.0 * m.q[0] * b0, m.q[0] * b1 + b0 * m.q[1], m.q[0] * b2 + b0 * m.q[2],
                              2.0 * m.q[1] * b1, m.q[1] * b2 + b1 * m.q[2], 2.0 * m.q[2] * b2};
        const double dtr = dM[0] + dM[3] + dM[5];
        const double da = (dtr - 2.0 * m.alpha * sym_dot(m.M, dM)) / m.mm;
        for (int u = 0; u < 6; ++u) J[k][u] = m.alpha * dM[u] + da * m.M[u];
      }
      v[0] = sym_dot(J[0], J[0]);
      v[1] = sym_dot(J[0], J[1]);
      v[2] = sym_dot(J[0], J[2]);
      v[3] = sym_dot(J[1], J[1]);
      v[4] = sym_dot(J[1], J[2]);
      v[5] = sym_dot(J[2], J[2]);
      for (int k = 0; k < 3; ++k) v[6 + k] = sym_dot(J[k], r);
    }
  }
  block_sum<kMVals>(v, a.part + (size_t)blockIdx.x * kMVals);
}

// Workgroup sums of the block partials (value k of each block), fixed order.
__device__ __forceinline__ void reduce_parts(const MetricArgs& a, int nv, double* out) {
  double v[kMVals];
  for (int k = 0; k < kMVals; ++k) v[k] = 0.0;
  for (int b = (int)threadIdx.x; b < a.blocks; b += kMBlock)
    for (int k = 0; k < nv; ++k) v[k] += a.part[(size_t)b * kMVals + (kMVals - nv) + k];
  block_sum<kMVals>(v, out);
}

// k_metric_solve: after a linearisation, the sums into the control block;
// then the damped 3 x 3 step (Cholesky), c_trial = c + delta.
__global__ void __launch_bounds__(kMBlock) k_metric_solve(MetricArgs a) {
  MetricCtl& C = *a.ctl;
  if (C.done) return;
  __shared__ double s[kMVals];
  if (C.need_lin) {
    reduce_parts(a, kMVals, s);
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int k = 0; k < 6; ++k) C.A[k] = s[k];
      for (int k = 0; k < 3; ++k) C.g[k] = s[6 + k];
      C.cost = s[9];
      if (!C.have_cost0) {
        C.cost0 = s[9];
        C.have_cost0 = 1;
      }
      C.need_lin = 0;
    }
  }
  if (threadIdx.x != 0 || C.debug_no_step) return;
  const double dmax = fmax(fmax(C.A[0], C.A[3]), C.A[5]);
  double A[6];
  for (int k = 0; k < 6; ++k) A[k] = C.A[k];
  A[0] += C.lambda * fmax(C.A[0], 1e-12 * dmax);
  A[3] += C.lambda * fmax(C.A[3], 1e-12 * dmax);
  A[5] += C.lambda * fmax(C.A[5], 1e-12 * dmax);
  // Cholesky A = L L^T
  const double l00 = A[0] > 0.0 ? sqrt(A[0]) : NAN;
  const double l10 = A[1] / l00, l20 = A[2] / l00;
  const double d1 = A[3] - l10 * l10;
  const double l11 = d1 > 0.0 ? sqrt(d1) : NAN;
  const double l21 = (A[4] - l20 * l10) / l11;
  const double d2 = A[5] - l20 * l20 - l21 * l21;
  const double l22 = d2 > 0.0 ? sqrt(d2) : NAN;
  const double y0 = -C.g[0] / l00;
  const double y1 = (-C.g[1] - l10 * y0) / l11;
  const double y2 = (-C.g[2] - l20 * y0 - l21 * y1) / l22;
  const double x2 = y2 / l22;
  const double x1 = (y1 - l21 * x2) / l11;
  const double x0 = (y0 - l10 * x1 - l20 * x2) / l00;
  if (isfinite(x0) && isfinite(x1) && isfinite(x2)) {
    C.status &= ~2;
    C.c_trial[0] = C.c[0] + x0;
    C.c_trial[1] = C.c[1] + x1;
    C.c_trial[2] = C.c[2] + x2;
  } else {
    C.status |= 2;
  }
}

// k_metric_decide: the trial cost, accept or reject, the damping schedule and
// the stopping rules.
__global__ void __launch_bounds__(kMBlock) k_metric_decide(MetricArgs a) {
  MetricCtl& C = *a.ctl;
  if (C.done) return;
  __shared__ double s[kMVals];
  const bool failed = (C.status & 2) != 0;
  if (!failed) {
    reduce_parts(a, 1, s);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double ft = failed ? INFINITY : s[0];
  const bool ok = isfinite(ft) && ft < C.cost;
  const int it = C.iters;
  a.tr_cost[it] = ft;
  a.tr_acc[it] = ok ? 1 : 0;
  C.iters = it + 1;
  C.cost_trial = ft;
  if (ok) {
    const bool small = C.cost - ft <= C.ftol * C.cost;
    for (int k = 0; k < 3; ++k) C.c[k] = C.c_trial[k];
    C.cost = ft;
    C.lambda = fmax(C.lambda / 10.0, 1e-12);
    C.need_lin = 1;
    if (small) C.stop = 1;
  } else {
    C.lambda = fmin(C.lambda * 10.0, 1e12);
    if (C.lambda >= 1e12) C.stop = 2;
  }
  if (!C.stop && C.iters >= C.max_iters) C.stop = 3;
  if (C.stop) C.done = 1;
}

// k_metric_finish: alpha_i at the final c, H, and each camera's R_i, t_i with
// P_i H = s_i K_i [R_i | t_i]; R_i the orthogonal polar factor (scaled Newton
// iteration X <- (g X + (g X)^-T) / 2).
__global__ void __launch_bounds__(kMBlock) k_metric_finish(MetricArgs a) {
  const MetricCtl& C = *a.ctl;
  const int i = (int)(blockIdx.x * kMBlock + threadIdx.x);
  double H[16];
  {
    double G[16] = {C.K0[0], C.K0[1], C.K0[2], 0.0, C.K0[3], C.K0[4], C.K0[5], 0.0,
                    C.K0[6], C.K0[7], C.K0[8], 0.0, C.c[0],  C.c[1],  C.c[2],  1.0};
    for (int r = 0; r < 4; ++r)
      for (int k = 0; k < 4; ++k)
        H[r * 4 + k] = C.T[r * 4] * G[k] + C.T[r * 4 + 1] * G[4 + k] + C.T[r * 4 + 2] * G[8 + k] +
                       C.T[r * 4 + 3] * G[12 + k];
  }
  if (i == 0)
    for (int k = 0; k < 16; ++k) a.ctl->H[k] = H[k];
  if (i >= a.n) return;
  CamTerms m;
  cam_terms(a.Q + (size_t)i * 12, C.K0, C.c, m);
  a.alpha[i] = m.alpha;
  if (!a.R) return;
  const double* P = a.P + (size_t)i * 12;
  double B[12];
  for (int k = 0; k < 4; ++k) {
    const double y0 = P[0] * H[k] + P[1] * H[4 + k] + P[2] * H[8 + k] + P[3] * H[12 + k];
    const double y1 = P[4] * H[k] + P[5] * H[4 + k] + P[6] * H[8 + k] + P[7] * H[12 + k];
    const double y2 = P[8] * H[k] + P[9] * H[4 + k] + P[10] * H[8 + k] + P[11] * H[12 + k];
    ktri_solve(a.K + (size_t)i * 9, y0, y1, y2, B[k], B[4 + k], B[8 + k]);
  }
  double X[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) X[r * 3 + k] = B[r * 4 + k];
  double sc = 1.0 / sqrt(m.alpha);
  if (det3(X) < 0.0) sc = -sc;
  for (int k = 0; k < 9; ++k) X[k] /= sc;
  for (int r = 0; r < 3; ++r) a.t[(size_t)i * 3 + r] = B[r * 4 + 3] / sc;
  for (int it = 0; it < 100; ++it) {
    double co[9];
    cof3(X, co);
    const double d = det3(X);
    double nx = 0.0, ni = 0.0;
    for (int k = 0; k < 9; ++k) {
      nx += X[k] * X[k];
      ni += co[k] * co[k];
    }
    ni /= d * d;   // ||X^-1||_F^2 = ||cof(X)||_F^2 / det^2
    const double gm = it < 4 ? sqrt(sqrt(ni / nx)) : 1.0;
    double diff = 0.0;
    for (int k = 0; k < 9; ++k) {
      const double xn = 0.5 * (gm * X[k] + co[k] / (gm * d));
      diff += (xn - X[k]) * (xn - X[k]);
      X[k] = xn;
    }
    if (it >= 4 && diff <= 1e-30) break;
  }
  for (int k = 0; k < 9; ++k) a.R[(size_t)i * 9 + k] = X[k];
}

#define M_TRY(ctx, expr)                                                          \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess) {                                                       \
      set_error((ctx), "%s failed: %s", #expr, hipGetErrorString(_e));            \
      return POVAR_EDEVICE;                                                       \
    }                                                                             \
  } while (0)

size_t align_256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device buffers of one call: allocated per call (owned, freed by the
// destructor), or carved from the device's scratch array (not owned).
struct MetricRun {
  void* mem = nullptr;
  bool owned = false;
  MetricArgs a{};
  ~MetricRun() {
    if (mem && owned) (void)hipFree(mem);
  }
};

// Bytes of device memory a call needs for n cameras and max_iters iterations.
size_t metric_bytes(int32_t n, int32_t max_iters) {
  const int32_t blocks = (n + kMBlock - 1) / kMBlock;
  const int32_t tr = max_iters > 0 ? max_iters : 1;
  return align_256(sizeof(MetricCtl)) + 2 * align_256((size_t)n * 12 * 8) + align_256((size_t)n * 9 * 8) +
         align_256((size_t)blocks * kMVals * 8) + align_256((size_t)n * 8) + align_256((size_t)n * 9 * 8) +
         align_256((size_t)n * 3 * 8) + align_256((size_t)tr * 8) + align_256((size_t)tr * 4);
}

povar_status metric_setup(povar_ctx ctx, int32_t n, const double* cams, const double* K, int32_t max_iters,
                          double ftol, MetricRun& run, char* scratch_base) {
  if (n < 2) {
    set_error(ctx, "the metric upgrade needs at least two cameras (got %d)", n);
    return POVAR_EINVAL;
  }
  if (n > (1 << 26)) {
    set_error(ctx, "n_cams exceeds the supported maximum");
    return POVAR_EINVAL;
  }
  if (!cams || !K) {
    set_error(ctx, "cams and K must not be NULL");
    return POVAR_EINVAL;
  }
  if (max_iters < 0 || max_iters > (1 << 20) || !(ftol >= 0.0 && ftol < 1.0)) {
    set_error(ctx, "max_iters must be in [0, 2^20] and ftol in [0, 1)");
    return POVAR_EINVAL;
  }
  for (int64_t k = 0; k < (int64_t)n * 12; ++k)
    if (!std::isfinite(cams[k])) {
      set_error(ctx, "camera %lld has a non-finite entry", (long long)(k / 12));
      return POVAR_EINVAL;
    }
  for (int32_t i = 0; i < n; ++i) {
    const double* k = K + (size_t)i * 9;
    bool ok = k[3] == 0.0 && k[6] == 0.0 && k[7] == 0.0;
    for (int u = 0; u < 9; ++u) ok = ok && std::isfinite(k[u]);
    ok = ok && k[0] != 0.0 && k[4] != 0.0 && k[8] != 0.0;
    if (!ok) {
      set_error(ctx, "K of camera %d is not a finite upper-triangular matrix with a nonzero diagonal", i);
      return POVAR_EINVAL;
    }
  }
  M_TRY(ctx, hipSetDevice(ctx->device));
  const int32_t blocks = (n + kMBlock - 1) / kMBlock;
  const int32_t tr = max_iters > 0 ? max_iters : 1;
  const size_t b_ctl = align_256(sizeof(MetricCtl)), b_P = align_256((size_t)n * 12 * 8),
               b_K = align_256((size_t)n * 9 * 8), b_part = align_256((size_t)blocks * kMVals * 8),
               b_a = align_256((size_t)n * 8), b_R = align_256((size_t)n * 9 * 8), b_t = align_256((size_t)n * 3 * 8),
               b_tc = align_256((size_t)tr * 8), b_ta = align_256((size_t)tr * 4);
  const size_t total = b_ctl + 2 * b_P + b_K + b_part + b_a + b_R + b_t + b_tc + b_ta;
  if (scratch_base) {
    if (total > kMetricScratchBytes) {
      set_error(ctx, "%d cameras and %d iterations need %zu bytes of device memory; the no-allocation metric "
                "upgrade has %zu bytes of scratch per device", n, max_iters, total, kMetricScratchBytes);
      return POVAR_EINVAL;
    }
    run.mem = scratch_base;
    run.owned = false;
  } else {
    if (hipMalloc(&run.mem, total) != hipSuccess) {
      run.mem = nullptr;
      set_error(ctx, "hipMalloc of %zu bytes for the metric upgrade failed", total);
      return POVAR_ENOMEM;
    }
    run.owned = true;
  }
  char* p = static_cast<char*>(run.mem);
  MetricArgs& a = run.a;
  a.ctl = (MetricCtl*)p;
  p += b_ctl;
  a.P = (const double*)p;
  M_TRY(ctx, hipMemcpyAsync(p, cams, (size_t)n * 12 * 8, hipMemcpyHostToDevice, ctx->stream));
  p += b_P;
  a.K = (const double*)p;
  M_TRY(ctx, hipMemcpyAsync(p, K, (size_t)n * 9 * 8, hipMemcpyHostToDevice, ctx->stream));
  p += b_K;
  a.Q = (double*)p;
  p += b_P;
  a.part = (double*)p;
  p += b_part;
  a.alpha = (double*)p;
  p += b_a;
  a.R = (double*)p;
  p += b_R;
  a.t = (double*)p;
  p += b_t;
  a.tr_cost = (double*)p;
  p += b_tc;
  a.tr_acc = (int32_t*)p;
  a.n = n;
  a.blocks = blocks;
  MetricCtl init{};
  init.max_iters = max_iters;
  init.ftol = ftol;
  M_TRY(ctx, hipMemcpyAsync(a.ctl, &init, sizeof(init), hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(k_metric_frame, dim3(1), dim3(64), 0, ctx->stream, a, 1e-4);
  hipLaunchKernelGGL(k_metric_normalize, dim3(blocks), dim3(kMBlock), 0, ctx->stream, a);
  M_TRY(ctx, hipGetLastError());
  MetricCtl c;
  M_TRY(ctx, hipMemcpyAsync(&c, a.ctl, sizeof(c), hipMemcpyDeviceToHost, ctx->stream));
  M_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (c.status & 1) {
    set_error(ctx, "the left 3x3 block of camera 0 (the reference camera) is singular");
    return POVAR_EINVAL;
  }
  return POVAR_OK;
}

// The LM iterations, the final pass and the copies of the results into the
// caller's host buffers, for a run set up by metric_setup.
povar_status metric_solve(povar_ctx ctx, MetricRun& run, int32_t n_cams, int32_t max_iters, double* H, double* c,
                          double* alpha, double* R, double* t, double* trace_cost, int32_t* trace_accept,
                          povar_metric_report* rep) {
  MetricArgs& a = run.a;
  hipStream_t s = ctx->stream;
  // iterations in groups of 8 between reads of the stop flag; every kernel
  // returns at once after the stop
  for (int32_t done_iters = 0; done_iters < max_iters;) {
    const int32_t k = max_iters - done_iters < 8 ? max_iters - done_iters : 8;
    for (int32_t it = 0; it < k; ++it) {
      hipLaunchKernelGGL(k_metric_terms<true>, dim3(a.blocks), dim3(kMBlock), 0, s, a);
      hipLaunchKernelGGL(k_metric_solve, dim3(1), dim3(kMBlock), 0, s, a);
      hipLaunchKernelGGL(k_metric_terms<false>, dim3(a.blocks), dim3(kMBlock), 0, s, a);
      hipLaunchKernelGGL(k_metric_decide, dim3(1), dim3(kMBlock), 0, s, a);
    }
    M_TRY(ctx, hipGetLastError());
    done_iters += k;
    int32_t done = 0;
    M_TRY(ctx, hipMemcpyAsync(&done, &a.ctl->done, sizeof(done), hipMemcpyDeviceToHost, s));
    M_TRY(ctx, hipStreamSynchronize(s));
    if (done) break;
  }
  if (max_iters == 0) {
    // no iteration: only the cost at c = 0 (control block: no step)
    const int32_t one = 1;
    M_TRY(ctx, hipMemcpyAsync(&a.ctl->debug_no_step, &one, sizeof(one), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_metric_terms<true>, dim3(a.blocks), dim3(kMBlock), 0, s, a);
    hipLaunchKernelGGL(k_metric_solve, dim3(1), dim3(kMBlock), 0, s, a);
  }
  // the cost in the control block is always the one at its c (an accepted
  // step carries its trial cost over)
  hipLaunchKernelGGL(k_metric_finish, dim3(a.blocks), dim3(kMBlock), 0, s, a);
  M_TRY(ctx, hipGetLastError());
  MetricCtl C;
  M_TRY(ctx, hipMemcpyAsync(&C, a.ctl, sizeof(C), hipMemcpyDeviceToHost, s));
  const size_t n = (size_t)n_cams;
  if (alpha) M_TRY(ctx, hipMemcpyAsync(alpha, a.alpha, n * 8, hipMemcpyDeviceToHost, s));
  if (R) M_TRY(ctx, hipMemcpyAsync(R, a.R, n * 9 * 8, hipMemcpyDeviceToHost, s));
  if (t) M_TRY(ctx, hipMemcpyAsync(t, a.t, n * 3 * 8, hipMemcpyDeviceToHost, s));
  M_TRY(ctx, hipStreamSynchronize(s));
  // the first C.iters trace entries (C.iters <= max_iters, the buffers' size)
  if (C.iters > 0 && trace_cost)
    M_TRY(ctx, hipMemcpyAsync(trace_cost, a.tr_cost, (size_t)C.iters * 8, hipMemcpyDeviceToHost, s));
  if (C.iters > 0 && trace_accept)
    M_TRY(ctx, hipMemcpyAsync(trace_accept, a.tr_acc, (size_t)C.iters * 4, hipMemcpyDeviceToHost, s));
  M_TRY(ctx, hipStreamSynchronize(s));
  if (H) std::memcpy(H, C.H, sizeof(C.H));
  if (c) std::memcpy(c, C.c, sizeof(C.c));
  if (rep) {
    rep->cost_initial = C.have_cost0 ? C.cost0 : C.cost;
    rep->cost_final = C.cost;
    rep->lambda = C.lambda;
    rep->iters = C.iters;
    rep->stop = C.stop;
  }
  return POVAR_OK;
}

}  // namespace
}  // namespace povar

using namespace povar;

extern "C" povar_status povar_metric_upgrade(povar_ctx ctx, int32_t n_cams, const double* cams, const double* K,
                                             int32_t max_iters, double ftol, double* H, double* c, double* alpha,
                                             double* R, double* t, double* trace_cost, int32_t* trace_accept,
                                             povar_metric_report* rep) try {
  if (!ctx) return POVAR_EINVAL;
  MetricRun run;
  povar_status st = metric_setup(ctx, n_cams, cams, K, max_iters, ftol, run, nullptr);
  if (st != POVAR_OK) return st;
  return metric_solve(ctx, run, n_cams, max_iters, H, c, alpha, R, t, trace_cost, trace_accept, rep);
} POVAR_HOST_CATCH(ctx)

extern "C" povar_status povar_metric_upgrade_noalloc(povar_ctx ctx, int32_t n_cams, const double* cams,
                                                     const double* K, int32_t max_iters, double ftol, double* H,
                                                     double* c, double* alpha, double* R, double* t,
                                                     double* trace_cost, int32_t* trace_accept,
                                                     povar_metric_report* rep) try {
  if (!ctx) return POVAR_EINVAL;
  char* base = metric_scratch(ctx->device);
  if (!base) {
    set_error(ctx, "no scratch address for device %d (the context was not created through povar_ctx_create)",
              ctx->device);
    return POVAR_ESTATE;
  }
  MetricRun run;
  povar_status st = metric_setup(ctx, n_cams, cams, K, max_iters, ftol, run, base);
  if (st != POVAR_OK) return st;
  return metric_solve(ctx, run, n_cams, max_iters, H, c, alpha, R, t, trace_cost, trace_accept, rep);
} POVAR_HOST_CATCH(ctx)

extern "C" povar_status povar_metric_debug_reduced(povar_ctx ctx, int32_t n_cams, const double* cams,
                                                   const double* K, const double* c, double* alpha, double* JtJ,
                                                   double* Jtr, double* cost) try {
  if (!ctx) return POVAR_EINVAL;
  if (!c || !std::isfinite(c[0]) || !std::isfinite(c[1]) || !std::isfinite(c[2])) {
    set_error(ctx, "c must be three finite values");
    return POVAR_EINVAL;
  }
  MetricRun run;
  povar_status st = metric_setup(ctx, n_cams, cams, K, 1, 0.0, run, nullptr);
  if (st != POVAR_OK) return st;
  MetricArgs& a = run.a;
  hipStream_t s = ctx->stream;
  MetricCtl C;
  M_TRY(ctx, hipMemcpyAsync(&C, a.ctl, sizeof(C), hipMemcpyDeviceToHost, s));
  M_TRY(ctx, hipStreamSynchronize(s));
  for (int k = 0; k < 3; ++k) C.c[k] = c[k];
  C.debug_no_step = 1;
  C.need_lin = 1;
  M_TRY(ctx, hipMemcpyAsync(a.ctl, &C, sizeof(C), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_metric_terms<true>, dim3(a.blocks), dim3(kMBlock), 0, s, a);
  hipLaunchKernelGGL(k_metric_solve, dim3(1), dim3(kMBlock), 0, s, a);
  MetricArgs b = a;
  b.R = nullptr;
  hipLaunchKernelGGL(k_metric_finish, dim3(a.blocks), dim3(kMBlock), 0, s, b);
  M_TRY(ctx, hipGetLastError());
  M_TRY(ctx, hipMemcpyAsync(&C, a.ctl, sizeof(C), hipMemcpyDeviceToHost, s));
  if (alpha) M_TRY(ctx, hipMemcpyAsync(alpha, a.alpha, (size_t)n_cams * 8, hipMemcpyDeviceToHost, s));
  M_TRY(ctx, hipStreamSynchronize(s));
  if (JtJ) {
    const int idx[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
    for (int k = 0; k < 9; ++k) JtJ[k] = C.A[idx[k]];
  }
  if (Jtr)
    for (int k = 0; k < 3; ++k) Jtr[k] = C.g[k];
  if (cost) *cost = C.cost;
  return POVAR_OK;
} POVAR_HOST_CATCH(ctx)
