// HIP kernels of one PoVar outer iteration for gfx950 (CDNA4, wave64).
//
// Notation (Sec. 3.2 and 4 of the paper): camera i is the row-major 3x4
// matrix P_i = [Pbar_i | p4_i]; landmark j is x~_j = (X_j, 1); an observation
// k = (i, j, m).  With a = 1 - eta the pOSE residual (6) is
//   r_k = ( sqrt(a)(u - m1 w), sqrt(a)(v - m2 w), sqrt(eta)(u - m1), sqrt(eta)(v - m2) ),
//   (u, v, w) = P_i x~_j ,
// and its normal-equation blocks (10)-(13) factor through the symmetric 3x3
//   N_k = E_k^T E_k = [[1, 0, -a m1], [0, 1, -a m2], [-a m1, -a m2, a |m|^2]] :
//   J_p^T J_p = N_k (x) x~ x~^T ,   W_k = J_p^T J_l = (N_k Pbar_i) (x) x~_j ,
//   W_k^T x = Pbar_i^T N_k (X_i x~_j) ,   W_k z = vec_row((N_k Pbar_i z) x~_j^T) .
// No Jacobian block is stored: each pass rebuilds what it needs from the
// observation stream (camera or landmark index + measurement) and the
// camera / landmark state.
//
// Passes (all deterministic, no floating-point atomics):
//   k_landmark_solve   closed-form landmarks (8), V_j^+, b_l, z0 = V^+ b_l, cost (9)
//   k_linearize        U_i, b_p, sum_k W_k z0 per camera                  (10)-(13)
//   k_camera_prep      damping, tangent projection, 12x12 inverse, x_0    (14),(17),(20)-(29)
//   k_series_landmark  z_j = V_j^+ sum_k W_k^T x_i                        (17)
//   k_series_camera    x_i = K_i sum_k W_k z_j, acc_i += x_i              (17)
//   k_retract          p_i <- (p_i + acc_i) / |p_i + acc_i|               (Sec. 4.3)
//   k_decide           LM accept / reject and damping update              (Sec. 5.2)
// Landmark-major passes run one lane per landmark over 64-landmark slices
// whose entries are stored lane-interleaved (coalesced); camera-major passes
// run one wave per chunk of <= 256 observations of one camera and combine
// the chunks of a camera in a fixed order in the last-arriving wave.
#include <type_traits>

#include "povar_internal.h"

namespace povar {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ bool map_wave(const Batch& B, int kind, int& p, int& u) {
  int w = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
  w = __builtin_amdgcn_readfirstlane(w);
  if (w >= B.total[kind]) return false;
  const int32_t* off = B.off[kind];
  int lo = 0, hi = B.n_prob;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= w) lo = mid; else hi = mid;
  }
  p = lo;
  u = w - off[lo];
  return true;
}

// Butterfly sum: every lane ends with the same, order-fixed value.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T ld_coherent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Arrival counter for "last wave combines the partials": every wave of a
// group publishes its partial, fences, and bumps the counter; the wave that
// sees count == n-1 owns the combination and resets the counter.
__device__ __forceinline__ bool arrive_last(uint32_t* cnt, uint32_t n) {
  __threadfence();
  uint32_t old = 0;
  if (lane_id() == 0) old = atomicAdd(cnt, 1u);
  old = __shfl(old, 0, kWave);
  if (old != n - 1) return false;
  __threadfence();
  return true;
}

__device__ __forceinline__ void reset_counter(uint32_t* cnt) {
  if (lane_id() == 0) __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T> struct Prec;
template <> struct Prec<float> {
  using T2 = float2;
  __device__ static const float2* cm_m(const DevProblem& D) { return D.cm_m32; }
  __device__ static const float2* e_m(const DevProblem& D) { return D.e_m32; }
  __device__ static float* P(const DevProblem& D, int b) { return D.P32[b]; }
  __device__ static float* X(const DevProblem& D, int b) { return D.X32[b]; }
  __device__ static float* Vp(const DevProblem& D, int b) { return D.Vp32[b]; }
  __device__ static float* z0(const DevProblem& D, int b) { return D.z032[b]; }
  __device__ static float* K(const DevProblem& D) { return D.K32; }
};
template <> struct Prec<double> {
  using T2 = double2;
  __device__ static const double2* cm_m(const DevProblem& D) { return D.cm_m64; }
  __device__ static const double2* e_m(const DevProblem& D) { return D.e_m64; }
  __device__ static double* P(const DevProblem& D, int b) { return D.P64[b]; }
  __device__ static double* X(const DevProblem& D, int b) { return D.X64[b]; }
  __device__ static double* Vp(const DevProblem& D, int b) { return D.Vp64[b]; }
  __device__ static double* z0(const DevProblem& D, int b) { return D.z064[b]; }
  __device__ static double* K(const DevProblem& D) { return D.K64; }
};

template <typename T>
__device__ __forceinline__ void load4(const T* p, T& a, T& b, T& c, T& d) {
  if constexpr (std::is_same<T, float>::value) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    a = v.x; b = v.y; c = v.z; d = v.w;
  } else {
    const double2 v0 = reinterpret_cast<const double2*>(p)[0];
    const double2 v1 = reinterpret_cast<const double2*>(p)[1];
    a = v0.x; b = v0.y; c = v1.x; d = v1.y;
  }
}

template <typename T>
__device__ __forceinline__ void store4(T* p, T a, T b, T c, T d) {
  if constexpr (std::is_same<T, float>::value) {
    *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
  } else {
    reinterpret_cast<double2*>(p)[0] = make_double2(a, b);
    reinterpret_cast<double2*>(p)[1] = make_double2(c, d);
  }
}

template <typename T>
__device__ __forceinline__ void load12(const T* p, T (&v)[12]) {
  load4(p, v[0], v[1], v[2], v[3]);
  load4(p + 4, v[4], v[5], v[6], v[7]);
  load4(p + 8, v[8], v[9], v[10], v[11]);
}

// N q for N = [[1,0,-a m1],[0,1,-a m2],[-a m1,-a m2,a|m|^2]]
template <typename T>
__device__ __forceinline__ void apply_N(T am1, T am2, T amsq, T q0, T q1, T q2, T& v0, T& v1, T& v2) {
  v0 = q0 - am1 * q2;
  v1 = q1 - am2 * q2;
  v2 = amsq * q2 - am1 * q0 - am2 * q1;
}

// ------------------------------------------------ 3x3 symmetric (pseudo-)inverse
// Moore-Penrose inverse of a symmetric PSD 3x3 block by cyclic Jacobi
// rotations; eigenvalues <= 1e-12 * the largest are treated as zero.
__device__ __forceinline__ void jacobi_rotate(double (&A)[3][3], double (&Q)[3][3], int p, int q, int r) {
  const double apq = A[p][q];
  if (apq == 0.0) return;
  const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
  const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
  A[p][p] -= t * apq;
  A[q][q] += t * apq;
  A[p][q] = A[q][p] = 0.0;
  const double arp = A[r][p], arq = A[r][q];
  A[r][p] = A[p][r] = c * arp - s * arq;
  A[r][q] = A[q][r] = s * arp + c * arq;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double qp = Q[k][p], qq = Q[k][q];
    Q[k][p] = c * qp - s * qq;
    Q[k][q] = s * qp + c * qq;
  }
}

__device__ __noinline__ void sym3_pinv_jacobi(const double (&v)[6], double (&out)[6]) {
  double A[3][3] = {{v[0], v[1], v[2]}, {v[1], v[3], v[4]}, {v[2], v[4], v[5]}};
  double Q[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dg = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (!(off > 1e-40 * dg)) break;
    jacobi_rotate(A, Q, 0, 1, 2);
    jacobi_rotate(A, Q, 0, 2, 1);
    jacobi_rotate(A, Q, 1, 2, 0);
  }
  const double l[3] = {A[0][0], A[1][1], A[2][2]};
  const double lmax = fmax(l[0], fmax(l[1], l[2]));
  const double cut = 1e-12 * lmax;
#pragma unroll
  for (int k = 0; k < 6; ++k) out[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (l[k] > cut && l[k] > 0.0) {
      const double il = 1.0 / l[k];
      out[0] += Q[0][k] * Q[0][k] * il;
      out[1] += Q[0][k] * Q[1][k] * il;
      out[2] += Q[0][k] * Q[2][k] * il;
      out[3] += Q[1][k] * Q[1][k] * il;
      out[4] += Q[1][k] * Q[2][k] * il;
      out[5] += Q[2][k] * Q[2][k] * il;
    }
  }
}

// LDL^T inverse when every pivot exceeds 1e-3 of the largest diagonal entry.
// Every block whose eigenvalue ratio falls below the 1e-12 cutoff fails that
// screen (a 3x3 SPD block has d_min^3 <= lmin lmax^2 and lmax <= 3 max diag),
// so the cutoff decision is always taken by the eigen path.
__device__ __forceinline__ void sym3_pinv(const double (&v)[6], double (&out)[6]) {
  const double maxd = fmax(v[0], fmax(v[3], v[5]));
  if (maxd > 0.0 && maxd < INFINITY) {
    const double thr = 1e-3 * maxd;
    const double d0 = v[0];
    if (d0 > thr) {
      const double l10 = v[1] / d0, l20 = v[2] / d0;
      const double d1 = v[3] - l10 * v[1];
      if (d1 > thr) {
        const double e12 = v[4] - l20 * v[1];
        const double l21 = e12 / d1;
        const double d2 = v[5] - l20 * v[2] - l21 * e12;
        if (d2 > thr) {
          const double a10 = -l10, a21 = -l21, a20 = l10 * l21 - l20;
          const double i0 = 1.0 / d0, i1 = 1.0 / d1, i2 = 1.0 / d2;
          out[0] = i0 + a10 * a10 * i1 + a20 * a20 * i2;
          out[1] = a10 * i1 + a20 * a21 * i2;
          out[2] = a20 * i2;
          out[3] = i1 + a21 * a21 * i2;
          out[4] = a21 * i2;
          out[5] = i2;
          return;
        }
      }
    }
  }
  sym3_pinv_jacobi(v, out);
}

// -------------------------------------------------------- k_landmark_solve
// One lane per landmark, FP64.  V_j = sum J_l^T J_l, h_j = -sum J_l^T r(X=0),
// X_j = V_j^+ h_j (8); then, at X_j, the cost sum ||r||^2 (9) and
// b_l = sum J_l^T r, and z0 = V^+ b_l.  J_l rows: sqrt(a)(R0 - m1 R2),
// sqrt(a)(R1 - m2 R2), sqrt(eta) R0, sqrt(eta) R1 with R_a the rows of Pbar.
// mode 0: initial state (writes the current buffers, cost and cost0);
// mode 1: trial point of a step (other buffers, cost_trial);
// mode 2: re-solve at the current cameras (writes cost).
__global__ void __launch_bounds__(kBlock) k_landmark_solve(Batch B, int mode) {
  int p, s;
  if (!map_wave(B, kUnitSlice, p, s)) return;
  const DevProblem& D = B.probs[p];
  Ctl* ctl = D.ctl;
  const int trial = mode == 1 ? 1 : 0;
  if (trial && ctl->done) return;
  const int pc = ctl->pcur ^ trial, lc = ctl->lcur ^ trial;
  const double* __restrict__ P = D.P64[pc];
  const int lane = lane_id();
  const int j = s * kWave + lane;
  const double eta = D.eta, a = 1.0 - eta;
  const int len = D.sl_len[s];
  const int base = D.sl_off[s];
  const int32_t* __restrict__ ecam = D.e_cam;
  const double2* __restrict__ em = D.e_m64;

  double v[6] = {0, 0, 0, 0, 0, 0};
  double h0 = 0, h1 = 0, h2 = 0;
  for (int t = 0; t < len; ++t) {
    const int e = base + t * kWave + lane;
    const int c = ecam[e];
    if (c < 0) continue;
    const double2 m = em[e];
    double Pc[12];
    load12(P + (size_t)c * kCam, Pc);
    const double D0[3] = {Pc[0] - m.x * Pc[8], Pc[1] - m.x * Pc[9], Pc[2] - m.x * Pc[10]};
    const double D1[3] = {Pc[4] - m.y * Pc[8], Pc[5] - m.y * Pc[9], Pc[6] - m.y * Pc[10]};
    const double R0[3] = {Pc[0], Pc[1], Pc[2]};
    const double R1[3] = {Pc[4], Pc[5], Pc[6]};
    v[0] += a * (D0[0] * D0[0] + D1[0] * D1[0]) + eta * (R0[0] * R0[0] + R1[0] * R1[0]);
    v[1] += a * (D0[0] * D0[1] + D1[0] * D1[1]) + eta * (R0[0] * R0[1] + R1[0] * R1[1]);
    v[2] += a * (D0[0] * D0[2] + D1[0] * D1[2]) + eta * (R0[0] * R0[2] + R1[0] * R1[2]);
    v[3] += a * (D0[1] * D0[1] + D1[1] * D1[1]) + eta * (R0[1] * R0[1] + R1[1] * R1[1]);
    v[4] += a * (D0[1] * D0[2] + D1[1] * D1[2]) + eta * (R0[1] * R0[2] + R1[1] * R1[2]);
    v[5] += a * (D0[2] * D0[2] + D1[2] * D1[2]) + eta * (R0[2] * R0[2] + R1[2] * R1[2]);
    // residual at X = 0 is built from p4 = (Pc[3], Pc[7], Pc[11])
    const double o1 = a * (Pc[3] - m.x * Pc[11]), o2 = a * (Pc[7] - m.y * Pc[11]);
    const double f1 = eta * (Pc[3] - m.x), f2 = eta * (Pc[7] - m.y);
    h0 -= D0[0] * o1 + D1[0] * o2 + R0[0] * f1 + R1[0] * f2;
    h1 -= D0[1] * o1 + D1[1] * o2 + R0[1] * f1 + R1[1] * f2;
    h2 -= D0[2] * o1 + D1[2] * o2 + R0[2] * f1 + R1[2] * f2;
  }
  double vp[6];
  sym3_pinv(v, vp);
  const double X0 = vp[0] * h0 + vp[1] * h1 + vp[2] * h2;
  const double X1 = vp[1] * h0 + vp[3] * h1 + vp[4] * h2;
  const double X2 = vp[2] * h0 + vp[4] * h1 + vp[5] * h2;

  double f = 0, b0 = 0, b1 = 0, b2 = 0;
  for (int t = 0; t < len; ++t) {
    const int e = base + t * kWave + lane;
    const int c = ecam[e];
    if (c < 0) continue;
    const double2 m = em[e];
    double Pc[12];
    load12(P + (size_t)c * kCam, Pc);
    const double u = Pc[0] * X0 + Pc[1] * X1 + Pc[2] * X2 + Pc[3];
    const double vv = Pc[4] * X0 + Pc[5] * X1 + Pc[6] * X2 + Pc[7];
    const double w = Pc[8] * X0 + Pc[9] * X1 + Pc[10] * X2 + Pc[11];
    const double o1 = u - m.x * w, o2 = vv - m.y * w;
    const double f1 = u - m.x, f2 = vv - m.y;
    f += a * (o1 * o1 + o2 * o2) + eta * (f1 * f1 + f2 * f2);
    const double ao1 = a * o1, ao2 = a * o2, ef1 = eta * f1, ef2 = eta * f2;
    b0 += (Pc[0] - m.x * Pc[8]) * ao1 + (Pc[4] - m.y * Pc[8]) * ao2 + Pc[0] * ef1 + Pc[4] * ef2;
    b1 += (Pc[1] - m.x * Pc[9]) * ao1 + (Pc[5] - m.y * Pc[9]) * ao2 + Pc[1] * ef1 + Pc[5] * ef2;
    b2 += (Pc[2] - m.x * Pc[10]) * ao1 + (Pc[6] - m.y * Pc[10]) * ao2 + Pc[2] * ef1 + Pc[6] * ef2;
  }
  if (j < D.n_l) {
    const double z0 = vp[0] * b0 + vp[1] * b1 + vp[2] * b2;
    const double z1 = vp[1] * b0 + vp[3] * b1 + vp[4] * b2;
    const double z2 = vp[2] * b0 + vp[4] * b1 + vp[5] * b2;
    store4(D.X64[lc] + (size_t)j * kLmVec, X0, X1, X2, 1.0);
    store4(D.z064[lc] + (size_t)j * kLmVec, z0, z1, z2, 0.0);
    double* vo = D.Vp64[lc] + (size_t)j * kLmSym;
    store4(vo, vp[0], vp[1], vp[2], vp[3]);
    store4(vo + 4, vp[4], vp[5], 0.0, 0.0);
    store4(D.X32[lc] + (size_t)j * kLmVec, (float)X0, (float)X1, (float)X2, 1.0f);
    store4(D.z032[lc] + (size_t)j * kLmVec, (float)z0, (float)z1, (float)z2, 0.0f);
    float* vo32 = D.Vp32[lc] + (size_t)j * kLmSym;
    store4(vo32, (float)vp[0], (float)vp[1], (float)vp[2], (float)vp[3]);
    store4(vo32 + 4, (float)vp[4], (float)vp[5], 0.0f, 0.0f);
  }
  // deterministic cost: lane tree per slice, then slices in order
  f = wave_sum(f);
  double total = f;
  if (D.n_sl > 1) {
    if (lane == 0) D.cost_part[s] = f;
    if (!arrive_last(D.cost_cnt, (uint32_t)D.n_sl)) return;
    double acc = 0;
    for (int q = lane; q < D.n_sl; q += kWave) acc += ld_coherent(D.cost_part + q);
    total = wave_sum(acc);
    reset_counter(D.cost_cnt);
  }
  if (lane == 0) {
    if (mode == 0) { ctl->cost = total; ctl->cost0 = total; }
    else if (mode == 1) ctl->cost_trial = total;
    else ctl->cost = total;
  }
}

// ------------------------------------------------------------- k_linearize
// One wave per camera chunk.  Accumulates, in FP64, the 40 distinct values
// of U_i = sum N_k (x) x~x~^T (N has fixed entries 1 and 0 in its top-left
// 2x2 block, so U_i is made of sum x~x~^T, sum m1 x~x~^T, sum m2 x~x~^T and
// sum |m|^2 x~x~^T), b_p = sum vec((N y - eta (m,0)) x~^T) and
// sum_k W_k z0_j = sum vec((N Pbar z0) x~^T).  Products in T.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_linearize(Batch B, int force) {
  int p, ch;
  if (!map_wave(B, kUnitChunk, p, ch)) return;
  const DevProblem& D = B.probs[p];
  Ctl* ctl = D.ctl;
  if (ctl->done) return;
  if (!force && !ctl->need_lin) return;
  const int lc = ctl->lcur, pc = ctl->pcur;
  const int lane = lane_id();
  const int cam = D.ch_cam[ch];
  const int beg = D.ch_beg[ch], end = D.ch_beg[ch + 1];
  T Pc[12];
  load12(Prec<T>::P(D, pc) + (size_t)cam * kCam, Pc);
  const T* __restrict__ X = Prec<T>::X(D, lc);
  const T* __restrict__ Z0 = Prec<T>::z0(D, lc);
  const typename Prec<T>::T2* __restrict__ M = Prec<T>::cm_m(D);
  const int32_t* __restrict__ lm = D.cm_lm;
  const T eta = (T)D.eta, a = (T)(1.0 - D.eta);

  double acc[kLinVals];
#pragma unroll
  for (int k = 0; k < kLinVals; ++k) acc[k] = 0.0;
  for (int e = beg + lane; e < end; e += kWave) {
    const int j = lm[e];
    const auto m = M[e];
    T x[4], z[4];
    load4(X + (size_t)j * kLmVec, x[0], x[1], x[2], x[3]);
    load4(Z0 + (size_t)j * kLmVec, z[0], z[1], z[2], z[3]);
    x[3] = (T)1;
    const T am1 = a * m.x, am2 = a * m.y, msq = m.x * m.x + m.y * m.y, amsq = a * msq;
    T y[3], q[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      y[r] = Pc[4 * r] * x[0] + Pc[4 * r + 1] * x[1] + Pc[4 * r + 2] * x[2] + Pc[4 * r + 3];
      q[r] = Pc[4 * r] * z[0] + Pc[4 * r + 1] * z[1] + Pc[4 * r + 2] * z[2];
    }
    T n[3], vq[3];
    apply_N(am1, am2, amsq, y[0], y[1], y[2], n[0], n[1], n[2]);
    apply_N(am1, am2, amsq, q[0], q[1], q[2], vq[0], vq[1], vq[2]);
    n[0] -= eta * m.x;
    n[1] -= eta * m.y;
    int o = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int d = c; d < 4; ++d) {
        const T xx = x[c] * x[d];
        acc[o] += (double)xx;
        acc[10 + o] += (double)(m.x * xx);
        acc[20 + o] += (double)(m.y * xx);
        acc[30 + o] += (double)(msq * xx);
        ++o;
      }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[40 + 4 * r + c] += (double)(n[r] * x[c]);
        acc[52 + 4 * r + c] += (double)(vq[r] * x[c]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kLinVals; ++k) acc[k] = wave_sum(acc[k]);

  const int c0 = D.cam_ch[cam], nch = D.cam_ch[cam + 1] - c0;
  if (nch > 1) {
    if (lane == 0) {
      double* part = D.lin_part + (size_t)ch * kLinVals;
#pragma unroll
      for (int k = 0; k < kLinVals; ++k) part[k] = acc[k];
    }
    if (!arrive_last(D.cam_cnt + cam, (uint32_t)nch)) return;
#pragma unroll
    for (int k = 0; k < kLinVals; ++k) acc[k] = 0.0;
    for (int q = lane; q < nch; q += kWave) {
      const double* part = D.lin_part + (size_t)(c0 + q) * kLinVals;
#pragma unroll
      for (int k = 0; k < kLinVals; ++k) acc[k] += ld_coherent(part + k);
    }
#pragma unroll
    for (int k = 0; k < kLinVals; ++k) acc[k] = wave_sum(acc[k]);
    reset_counter(D.cam_cnt + cam);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 40; ++k) D.U40[(size_t)cam * 40 + k] = acc[k];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      D.bp[(size_t)cam * kCam + k] = acc[40 + k];
      D.wz[(size_t)cam * kCam + k] = acc[52 + k];
    }
  }
}

// ----------------------------------------------------------- k_camera_prep
// One lane per camera, FP64.  U_l = U + lambda diag(U) (floored), then on the
// sphere A = Pi U_l Pi + tau p p^T with Pi = I - p p^T, tau = tr(U_l)/12
// (A restricted to the tangent space is B^T U_l B for any orthonormal basis
// B of p^perp, and A p = tau p).  K = Pi A^-1 Pi = B (B^T U_l B)^-1 B^T is
// stored; x_0 = acc = -K g with g = b_p - sum W_k V^+ b_l.  Euclidean: K = U_l^-1.
__host__ __device__ constexpr int tri(int r, int c) { return r * (r + 1) / 2 + c; }

template <typename T>
__global__ void __launch_bounds__(kWave) k_camera_prep(Batch B) {
  int p, w;
  if (!map_wave(B, kUnitCamWave, p, w)) return;
  const DevProblem& D = B.probs[p];
  Ctl* ctl = D.ctl;
  if (ctl->done) return;
  const int i = w * kWave + lane_id();
  if (i >= D.n_p) return;
  const double lam = ctl->lambda;
  const int pc = ctl->pcur;
  const bool sphere = D.manifold == 0;
  const double a = 1.0 - D.eta;

  double u40[40];
#pragma unroll
  for (int k = 0; k < 40; ++k) u40[k] = D.U40[(size_t)i * 40 + k];
  // 4x4 symmetric packed index of (c, d)
  auto s4 = [](int c, int d) { return c <= d ? (c * 7 - c * c) / 2 + d : (d * 7 - d * d) / 2 + c; };
  double L[78];
#pragma unroll
  for (int r = 0; r < 12; ++r) {
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      const int ar = r >> 2, ac = c >> 2;
      const int k = s4(r & 3, c & 3);
      double val;
      if (ar < 2 && ac < 2) val = (ar == ac) ? u40[k] : 0.0;
      else if (ar == 2 && ac == 2) val = a * u40[30 + k];
      else val = -a * u40[(ar == 1 || ac == 1) ? 20 + k : 10 + k];
      L[tri(r, c)] = val;
    }
  }
  double dmax = 0.0;
#pragma unroll
  for (int r = 0; r < 12; ++r) dmax = fmax(dmax, L[tri(r, r)]);
#pragma unroll
  for (int r = 0; r < 12; ++r) L[tri(r, r)] += lam * fmax(L[tri(r, r)], 1e-12 * dmax);

  double pv[12];
  load12(D.P64[pc] + (size_t)i * kCam, pv);
  if (sphere) {
    double w12[12], tr = 0.0, s = 0.0;
#pragma unroll
    for (int r = 0; r < 12; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < 12; ++c) acc += L[r >= c ? tri(r, c) : tri(c, r)] * pv[c];
      w12[r] = acc;
      tr += L[tri(r, r)];
    }
#pragma unroll
    for (int r = 0; r < 12; ++r) s += pv[r] * w12[r];
    const double st = s + tr / 12.0;
#pragma unroll
    for (int r = 0; r < 12; ++r) {
#pragma unroll
      for (int c = 0; c <= r; ++c) L[tri(r, c)] += -pv[r] * w12[c] - w12[r] * pv[c] + st * pv[r] * pv[c];
    }
  }
  // Cholesky A = L L^T in place
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 12; ++j) {
    double d = L[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[tri(j, k)] * L[tri(j, k)];
    if (!(d > 0.0)) { ok = false; d = 1.0; }
    d = sqrt(d);
    L[tri(j, j)] = d;
    const double inv = 1.0 / d;
#pragma unroll
    for (int r = j + 1; r < 12; ++r) {
      double v = L[tri(r, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[tri(r, k)] * L[tri(j, k)];
      L[tri(r, j)] = v * inv;
    }
  }
  // L^-1 in place, column by column, rows ascending
#pragma unroll
  for (int j = 0; j < 12; ++j) {
    L[tri(j, j)] = 1.0 / L[tri(j, j)];
#pragma unroll
    for (int r = j + 1; r < 12; ++r) {
      double v = 0.0;
#pragma unroll
      for (int k = j; k < r; ++k) v += L[tri(r, k)] * L[tri(k, j)];
      L[tri(r, j)] = -v / L[tri(r, r)];
    }
  }
  double wp[12], sp = 0.0;
  if (sphere) {
    double u[12];
#pragma unroll
    for (int r = 0; r < 12; ++r) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k <= r; ++k) v += L[tri(r, k)] * pv[k];
      u[r] = v;
      sp += v * v;
    }
#pragma unroll
    for (int r = 0; r < 12; ++r) {
      double v = 0.0;
#pragma unroll
      for (int k = r; k < 12; ++k) v += L[tri(k, r)] * u[k];
      wp[r] = v;
    }
  }
  double g[12], x0[12];
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    g[r] = D.bp[(size_t)i * kCam + r] - D.wz[(size_t)i * kCam + r];
    x0[r] = 0.0;
  }
  double* K64 = D.K64 + (size_t)i * kCamMat;
  float* K32 = D.K32 + (size_t)i * kCamMat;
#pragma unroll
  for (int r = 0; r < 12; ++r) {
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      double v = 0.0;
#pragma unroll
      for (int k = r; k < 12; ++k) v += L[tri(k, r)] * L[tri(k, c)];
      if (sphere) v += -pv[r] * wp[c] - wp[r] * pv[c] + sp * pv[r] * pv[c];
      if (!ok) v = 0.0;
      K64[r * 12 + c] = v;
      K64[c * 12 + r] = v;
      K32[r * 12 + c] = (float)v;
      K32[c * 12 + r] = (float)v;
      x0[r] -= v * g[c];
      if (c != r) x0[c] -= v * g[r];
    }
  }
  T* x = static_cast<T*>(D.x) + (size_t)i * kCam;
  T* acc = static_cast<T*>(D.acc) + (size_t)i * kCam;
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    x[r] = (T)x0[r];
    acc[r] = (T)x0[r];
  }
  if (!ok) atomicOr(&ctl->status, 1);
}

// ------------------------------------------------------- k_series_landmark
// z_j = V_j^+ sum_k Pbar_i^T N_k (X_i x~_j), X_i = x_i as a 3x4 matrix.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_series_landmark(Batch B, int t) {
  int p, s;
  if (!map_wave(B, kUnitSlice, p, s)) return;
  const DevProblem& D = B.probs[p];
  const Ctl* ctl = D.ctl;
  if (ctl->done || t > ctl->order) return;
  const int lc = ctl->lcur, pc = ctl->pcur;
  const int lane = lane_id();
  const int j = s * kWave + lane;
  const int len = D.sl_len[s];
  const int base = D.sl_off[s];
  const int32_t* __restrict__ ecam = D.e_cam;
  const typename Prec<T>::T2* __restrict__ em = Prec<T>::e_m(D);
  const T* __restrict__ xs = static_cast<const T*>(D.x);
  const T* __restrict__ Pm = Prec<T>::P(D, pc);
  const T a = (T)(1.0 - D.eta);
  if (j >= D.n_l) return;
  T X0, X1, X2, X3;
  load4(Prec<T>::X(D, lc) + (size_t)j * kLmVec, X0, X1, X2, X3);
  T y0 = 0, y1 = 0, y2 = 0;
  for (int tt = 0; tt < len; ++tt) {
    const int e = base + tt * kWave + lane;
    const int c = ecam[e];
    if (c < 0) break;   // entries of one landmark are contiguous in t; padding only at its end
    const auto m = em[e];
    T xc[12], Pc[12];
    load12(xs + (size_t)c * kCam, xc);
    load12(Pm + (size_t)c * kCam, Pc);
    const T q0 = xc[0] * X0 + xc[1] * X1 + xc[2] * X2 + xc[3];
    const T q1 = xc[4] * X0 + xc[5] * X1 + xc[6] * X2 + xc[7];
    const T q2 = xc[8] * X0 + xc[9] * X1 + xc[10] * X2 + xc[11];
    T v0, v1, v2;
    apply_N(a * m.x, a * m.y, a * (m.x * m.x + m.y * m.y), q0, q1, q2, v0, v1, v2);
    y0 += Pc[0] * v0 + Pc[4] * v1 + Pc[8] * v2;
    y1 += Pc[1] * v0 + Pc[5] * v1 + Pc[9] * v2;
    y2 += Pc[2] * v0 + Pc[6] * v1 + Pc[10] * v2;
  }
  T v[8];
  const T* vp = Prec<T>::Vp(D, lc) + (size_t)j * kLmSym;
  load4(vp, v[0], v[1], v[2], v[3]);
  load4(vp + 4, v[4], v[5], v[6], v[7]);
  const T z0 = v[0] * y0 + v[1] * y1 + v[2] * y2;
  const T z1 = v[1] * y0 + v[3] * y1 + v[4] * y2;
  const T z2 = v[2] * y0 + v[4] * y1 + v[5] * y2;
  store4(static_cast<T*>(D.z) + (size_t)j * kLmVec, z0, z1, z2, (T)0);
}

// --------------------------------------------------------- k_series_camera
// t_i = sum_k vec((N_k Pbar_i z_j) x~_j^T); x_i = K_i t_i; acc_i += x_i.
template <typename T>
__device__ __forceinline__ void camera_finalize(const DevProblem& D, int cam, const T (&tv)[12]) {
  const int r = lane_id();
  if (r >= 12) return;
  const T* K = Prec<T>::K(D) + (size_t)cam * kCamMat + r * 12;
  T kr[12];
  load12(K, kr);
  T xr = 0;
#pragma unroll
  for (int c = 0; c < 12; ++c) xr += kr[c] * tv[c];
  static_cast<T*>(D.x)[(size_t)cam * kCam + r] = xr;
  static_cast<T*>(D.acc)[(size_t)cam * kCam + r] += xr;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_series_camera(Batch B, int t) {
  int p, ch;
  if (!map_wave(B, kUnitChunk, p, ch)) return;
  const DevProblem& D = B.probs[p];
  const Ctl* ctl = D.ctl;
  if (ctl->done || t > ctl->order) return;
  const int lc = ctl->lcur, pc = ctl->pcur;
  const int lane = lane_id();
  const int cam = D.ch_cam[ch];
  const int beg = D.ch_beg[ch], end = D.ch_beg[ch + 1];
  T Pc[12];
  load12(Prec<T>::P(D, pc) + (size_t)cam * kCam, Pc);
  const T* __restrict__ X = Prec<T>::X(D, lc);
  const T* __restrict__ Z = static_cast<const T*>(D.z);
  const typename Prec<T>::T2* __restrict__ M = Prec<T>::cm_m(D);
  const int32_t* __restrict__ lm = D.cm_lm;
  const T a = (T)(1.0 - D.eta);
  T acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0;
  for (int e = beg + lane; e < end; e += kWave) {
    const int j = lm[e];
    const auto m = M[e];
    T x[4], z[4];
    load4(X + (size_t)j * kLmVec, x[0], x[1], x[2], x[3]);
    load4(Z + (size_t)j * kLmVec, z[0], z[1], z[2], z[3]);
    const T q0 = Pc[0] * z[0] + Pc[1] * z[1] + Pc[2] * z[2];
    const T q1 = Pc[4] * z[0] + Pc[5] * z[1] + Pc[6] * z[2];
    const T q2 = Pc[8] * z[0] + Pc[9] * z[1] + Pc[10] * z[2];
    T v[3];
    apply_N(a * m.x, a * m.y, a * (m.x * m.x + m.y * m.y), q0, q1, q2, v[0], v[1], v[2]);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      acc[4 * r + 0] += v[r] * x[0];
      acc[4 * r + 1] += v[r] * x[1];
      acc[4 * r + 2] += v[r] * x[2];
      acc[4 * r + 3] += v[r];
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = wave_sum(acc[k]);
  const int c0 = D.cam_ch[cam], nch = D.cam_ch[cam + 1] - c0;
  if (nch > 1) {
    if (lane == 0) {
      T* part = static_cast<T*>(D.t_part) + (size_t)ch * kCam;
      store4(part, acc[0], acc[1], acc[2], acc[3]);
      store4(part + 4, acc[4], acc[5], acc[6], acc[7]);
      store4(part + 8, acc[8], acc[9], acc[10], acc[11]);
    }
    if (!arrive_last(D.cam_cnt + cam, (uint32_t)nch)) return;
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = 0;
    for (int q = lane; q < nch; q += kWave) {
      const T* part = static_cast<const T*>(D.t_part) + (size_t)(c0 + q) * kCam;
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] += ld_coherent(part + k);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = wave_sum(acc[k]);
    reset_counter(D.cam_cnt + cam);
  }
  camera_finalize<T>(D, cam, acc);
}

// --------------------------------------------------------------- k_retract
template <typename T>
__global__ void __launch_bounds__(kWave) k_retract(Batch B) {
  int p, w;
  if (!map_wave(B, kUnitCamWave, p, w)) return;
  const DevProblem& D = B.probs[p];
  const Ctl* ctl = D.ctl;
  if (ctl->done) return;
  const int i = w * kWave + lane_id();
  if (i >= D.n_p) return;
  const int pc = ctl->pcur;
  double q[12];
  load12(D.P64[pc] + (size_t)i * kCam, q);
  const T* acc = static_cast<const T*>(D.acc) + (size_t)i * kCam;
  double nrm = 0.0;
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    q[r] += (double)acc[r];
    nrm += q[r] * q[r];
  }
  if (D.manifold == 0) {
    const double inv = 1.0 / sqrt(nrm);
#pragma unroll
    for (int r = 0; r < 12; ++r) q[r] *= inv;
  }
  double* o64 = D.P64[pc ^ 1] + (size_t)i * kCam;
  float* o32 = D.P32[pc ^ 1] + (size_t)i * kCam;
#pragma unroll
  for (int r = 0; r < 12; r += 4) {
    store4(o64 + r, q[r], q[r + 1], q[r + 2], q[r + 3]);
    store4(o32 + r, (float)q[r], (float)q[r + 1], (float)q[r + 2], (float)q[r + 3]);
  }
}

// ---------------------------------------------------------------- k_decide
// Strict decrease accepts (NaN rejects); lambda /10 on accept, x10 on reject,
// clamped; relinearise only after an accept; ftol on accepted steps.
__global__ void __launch_bounds__(kWave) k_decide(Batch B) {
  int p, w;
  if (!map_wave(B, kUnitOne, p, w)) return;
  if (lane_id() != 0) return;
  const DevProblem& D = B.probs[p];
  Ctl* ctl = D.ctl;
  if (ctl->done) return;
  const double fn = ctl->cost_trial, f = ctl->cost;
  const bool accept = (fn < f) && (fn - fn == 0.0);
  const int it = ctl->iter;
  if (it < D.trace_cap) {
    D.tr_cost[it] = fn;
    D.tr_lambda[it] = ctl->lambda;
    D.tr_acc[it] = accept ? 1 : 0;
  }
  if (accept) {
    const double rel = (f - fn) / f;
    ctl->cost = fn;
    ctl->lcur ^= 1;
    ctl->pcur ^= 1;
    ctl->lambda = fmax(ctl->lambda / 10.0, D.lambda_min);
    ctl->n_accept += 1;
    if (rel < D.ftol) { ctl->done = 1; ctl->stop_reason = 1; }
  } else {
    ctl->lambda = fmin(ctl->lambda * 10.0, D.lambda_max);
  }
  ctl->need_lin = accept ? 1 : 0;
  ctl->iter = it + 1;
  if (ctl->iter >= ctl->iter_limit) ctl->done = 1;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- launchers
static inline dim3 grid_for(int waves, int waves_per_block) {
  return dim3((unsigned)((waves + waves_per_block - 1) / waves_per_block));
}

hipError_t launch_landmark_solve(const Batch& b, int mode, hipStream_t s) {
  if (b.total[kUnitSlice] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_landmark_solve, grid_for(b.total[kUnitSlice], kWavesPerBlock), dim3(kBlock), 0, s, b, mode);
  return hipGetLastError();
}

hipError_t launch_linearize(const Batch& b, bool fp32, int force, hipStream_t s) {
  if (b.total[kUnitChunk] == 0) return hipSuccess;
  const dim3 g = grid_for(b.total[kUnitChunk], kWavesPerBlock);
  if (fp32) hipLaunchKernelGGL(k_linearize<float>, g, dim3(kBlock), 0, s, b, force);
  else hipLaunchKernelGGL(k_linearize<double>, g, dim3(kBlock), 0, s, b, force);
  return hipGetLastError();
}

hipError_t launch_camera_prep(const Batch& b, bool fp32, hipStream_t s) {
  if (b.total[kUnitCamWave] == 0) return hipSuccess;
  const dim3 g = grid_for(b.total[kUnitCamWave], 1);
  if (fp32) hipLaunchKernelGGL(k_camera_prep<float>, g, dim3(kWave), 0, s, b);
  else hipLaunchKernelGGL(k_camera_prep<double>, g, dim3(kWave), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_series_landmark(const Batch& b, bool fp32, int t, hipStream_t s) {
  if (b.total[kUnitSlice] == 0) return hipSuccess;
  const dim3 g = grid_for(b.total[kUnitSlice], kWavesPerBlock);
  if (fp32) hipLaunchKernelGGL(k_series_landmark<float>, g, dim3(kBlock), 0, s, b, t);
  else hipLaunchKernelGGL(k_series_landmark<double>, g, dim3(kBlock), 0, s, b, t);
  return hipGetLastError();
}

hipError_t launch_series_camera(const Batch& b, bool fp32, int t, hipStream_t s) {
  if (b.total[kUnitChunk] == 0) return hipSuccess;
  const dim3 g = grid_for(b.total[kUnitChunk], kWavesPerBlock);
  if (fp32) hipLaunchKernelGGL(k_series_camera<float>, g, dim3(kBlock), 0, s, b, t);
  else hipLaunchKernelGGL(k_series_camera<double>, g, dim3(kBlock), 0, s, b, t);
  return hipGetLastError();
}

hipError_t launch_retract(const Batch& b, bool fp32, hipStream_t s) {
  if (b.total[kUnitCamWave] == 0) return hipSuccess;
  const dim3 g = grid_for(b.total[kUnitCamWave], 1);
  if (fp32) hipLaunchKernelGGL(k_retract<float>, g, dim3(kWave), 0, s, b);
  else hipLaunchKernelGGL(k_retract<double>, g, dim3(kWave), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_decide(const Batch& b, hipStream_t s) {
  if (b.total[kUnitOne] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_decide, grid_for(b.total[kUnitOne], 1), dim3(kWave), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace povar
