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
// Passes (deterministic: no floating-point atomics, fixed reduction orders):
//   k_landmark_solve       closed-form landmarks (8), V_j^+, b_l, z0 = V^+ b_l, cost (9)
//   k_linearize            U_i, b_p, sum_k W_k z0_j per camera chunk         (10)-(13)
//   k_camera_prep          damping, tangent projection, 12x12 inverse, x_0  (14),(17),(20)-(29)
//   k_series_landmark      z_j = V_j^+ sum_k W_k^T x_i                      (17)
//   k_series_landmark_coop the same, FP32 problems with many cameras, camera
//                          records fetched by whole waves
//   k_series_landmark_coop64  the same for every FP64 problem (two gathers per
//                          record)
//   k_series_camera        x_i = K_i sum_k W_k z_j, acc_i += x_i             (17)
//   k_series_camera_slots  the same sums for landmark-blocked problems, per run
//   k_series_camera_combine  adds a camera's partial sums, applies K_i
//   k_series_check         optional early stop of the series (Sec. 5.2)
//   k_retract              p_i <- (p_i + acc_i) / |p_i + acc_i|             (Sec. 4.3)
//                          (series order 0 only; otherwise in the last camera pass)
//   k_decide               LM accept / reject and damping update            (Sec. 5.2)
// Second stage, objective (7) with both blocks on their spheres (Sec. 4.3):
//   k_refine_landmarks     V_j, b_l, G_j (projected damped inverse), z0, cost
//   k_refine_cameras       U_i, b_p, sum W z0 per camera chunk
//   k_refine_prep          damping, K_i in a Householder tangent basis, x_0
//   k_refine_series_landmark / _camera / _camera_slots / _combine / _check
//                          the series (29) and its optional early stop
//   k_refine_landmark_update  back-substitution and landmark retraction
//   k_refine_retract, k_refine_cost  camera retraction, trial cost
// Landmark-major passes run one lane per observation over 64-entry packet
// slots of whole landmarks and sum each landmark's lanes with a segmented
// scan of DPP lane moves.  The camera-major pass runs one workgroup per chunk
// of <= 2048 observations of one camera while the landmark records fit one
// XCD's L2; larger problems use landmark blocks pinned to XCDs, with 64-lane
// slots of 8 (FP32) or 4 (FP64) observations per lane and one partial per
// (camera, block part), which the combine kernel adds per camera in a fixed
// order.
#include <hip/hip_ext.h>

#include <mutex>
#include <type_traits>

#include "povar_internal.h"

namespace povar {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ bool find_unit(const Batch& B, int kind, int ug, int& p, int& u) {
  if (ug >= B.total[kind]) return false;
  if (B.n_prob == 1) {   // a single problem: no table lookup before the first real load
    p = 0;
    u = ug;
    return true;
  }
  const int32_t* off = B.tables + (size_t)kind * B.tab_stride;
  int lo = 0, hi = B.n_prob;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= ug) lo = mid; else hi = mid;
  }
  p = lo;
  u = ug - off[lo];
  return true;
}

// one unit per wave of a WG-thread workgroup
template <int WG = kBlock>
__device__ __forceinline__ bool map_wave(const Batch& B, int kind, int& p, int& u) {
  const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * (WG / kWave) + (threadIdx.x >> 6));
  return find_unit(B, kind, w, p, u);
}

// one unit per workgroup
__device__ __forceinline__ bool map_block(const Batch& B, int kind, int& p, int& u) {
  return find_unit(B, kind, (int)blockIdx.x, p, u);
}

// ------------------------------------------------- cross-lane primitives
// Built on DPP lane moves (VALU operands, no LDS round trip).  GFX9 DPP
// controls: quad permutes, row (16-lane) shifts and mirrors, and the two row
// broadcasts used by wave-wide scans.  Callers run them with all 64 lanes of
// the wave active.
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]: lane i <- i^1
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]: lane i <- i^2
constexpr int kDppMirror = 0x140;     // lane i <- 15-i within each row
constexpr int kDppHalfMirror = 0x141; // lane i <- 7-i within each half row
constexpr int kDppBcast15 = 0x142;    // rows 1, 3 <- lane 15 of the previous row
constexpr int kDppBcast31 = 0x143;    // rows 2, 3 <- lane 31
constexpr int kDppWaveShl1 = 0x130;   // lane i <- lane i+1 across the wave
constexpr int kDppRowShr = 0x110;     // + d: lane i <- lane i-d within its row

// Lane move: lanes whose source is outside the row (or whose row is not in
// RowMask) keep `old`.
template <int Ctrl, int RowMask = 0xF, typename T>
__device__ __forceinline__ T dpp(T old, T v) {
  return __builtin_amdgcn_update_dpp(old, v, Ctrl, RowMask, 0xF, false);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 16 bytes as a native vector (plain loads and stores in any address space)
typedef float f4v __attribute__((ext_vector_type(4)));

// Wave-cooperative gather of R records of NP 16-byte pieces per lane (record
// src[r] of `base`, stride in bytes; a lane with src[r] < 0 receives record 0
// there, which it must not use).  For each r, piece k of the wave's 64 NP
// pieces is loaded by lane k % 64 and belongs to lane k / NP, so the lanes of
// one load instruction read consecutive pieces of a few records (a cache line
// serves several lanes) instead of one piece of 64 records (up to 64 lines,
// each one lookup in the vector L1).  All loads are issued first; the pieces
// then go to their lanes through `buf` (64 NP pieces of this wave), one r at
// a time.  With Halves = 2 the exchange takes two rounds through half the
// buffer (64 NP / 2 pieces): the first NP / 2 load instructions hold exactly
// the pieces of lanes 0-31, the others those of lanes 32-63, so each round
// delivers all pieces of one half of the wave; the loads and the number of
// cache lines they touch do not change.  All 64 lanes call it.
template <int NP, int R = 1, int Halves = 1>
__device__ __forceinline__ void coop_fetch(const char POVAR_GMEM* base, size_t stride, const int (&src)[R],
                                           f4v POVAR_LDS* buf, f4v (&out)[R][NP]) {
  static_assert(Halves == 1 || (Halves == 2 && NP % 2 == 0), "one round, or two for an even piece count");
  const int lane = lane_id();
  f4v piece[R][NP];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int k = i * kWave + lane, o = k / NP, part = k - o * NP;
      const int so = max(__shfl(src[r], o), 0);
      piece[r][i] = *(const f4v POVAR_GMEM*)(base + (size_t)so * stride + (size_t)part * 16);
    }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if constexpr (Halves == 1) {
#pragma unroll
      for (int i = 0; i < NP; ++i) buf[i * kWave + lane] = piece[r][i];
      wave_sync();
#pragma unroll
      for (int k = 0; k < NP; ++k) out[r][k] = buf[lane * NP + k];
      wave_sync();
    } else {
      constexpr int H = NP / 2;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int i = 0; i < H; ++i) buf[i * kWave + lane] = piece[r][h * H + i];
        wave_sync();
        if ((lane >> 5) == h)
#pragma unroll
          for (int k = 0; k < NP; ++k) out[r][k] = buf[(lane & 31) * NP + k];
        wave_sync();
      }
    }
  }
}

// A 16-byte piece of a cooperative gather as two doubles.
__device__ __forceinline__ void piece_d2(f4v v, double& a, double& b) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  const d2v d = __builtin_bit_cast(d2v, v);
  a = d[0];
  b = d[1];
}

// Value of lane l (a uniform result); the builtin moves 32-bit words.
template <typename T>
__device__ __forceinline__ T read_lane(T v, int l) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
  } else {
    const int2 w = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_readlane(w.x, l);
    r.y = __builtin_amdgcn_readlane(w.y, l);
    return __builtin_bit_cast(T, r);
  }
}

// Wave sum in a fixed order, the same value in every lane: pairs, quads,
// half rows and rows by lane moves (a + b and b + a are the same number), then
// the four row totals as ((r0 + r1) + (r2 + r3)).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp<kDppXor1>(v, v);
  v += dpp<kDppXor2>(v, v);
  v += dpp<kDppHalfMirror>(v, v);
  v += dpp<kDppMirror>(v, v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Reduce-scatter of N values (N a power of two, 2 <= N <= 64) over the wave:
// afterwards lane l holds the wave total of value rs_index<N>(l), each value
// in 64 / N lanes, for about N lane moves per lane instead of the 8 N of N
// separate wave sums.  Step s pairs the lanes that differ in lane bit s (bits
// 0..3 by lane moves: xor 1, xor 2, the half-row and the row mirror; bits 4, 5
// by ds_bpermute: xor 16, xor 32); while values remain to be split, each lane
// keeps one half and adds its partner's copy of it.  The half kept at step s
// is chosen by k_s = b0^b2, b1^b2, b2^b3, b3, b4, b5 (b = lane bits): the two
// lanes of a pair differ in it, and the partners of every later step (the
// mirrors flip all lower bits) agree on it, so they hold the same values.
// Once one value is left, the remaining steps add the partners' copies.  The
// order is fixed: bitwise repeatable.
__device__ __forceinline__ int rs_keep(int lane, int s) {
  const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  switch (s) {
    case 0: return b0 ^ b2;
    case 1: return b1 ^ b2;
    case 2: return b2 ^ b3;
    case 3: return b3;
    default: return (lane >> s) & 1;
  }
}

template <int N>
__device__ __forceinline__ int rs_index(int lane) {
  int idx = 0;
#pragma unroll
  for (int s = 0, w = N >> 1; w > 0; ++s, w >>= 1) idx += rs_keep(lane, s) * w;
  return idx;
}

template <int S, typename T>
__device__ __forceinline__ T rs_partner(T v) {
  if constexpr (S == 0) return dpp<kDppXor1>(v, v);
  else if constexpr (S == 1) return dpp<kDppXor2>(v, v);
  else if constexpr (S == 2) return dpp<kDppHalfMirror>(v, v);
  else if constexpr (S == 3) return dpp<kDppMirror>(v, v);
  else return __shfl_xor(v, 1 << S);
}

template <int S, int N, typename T>
__device__ __forceinline__ void rs_step(T (&v)[N], int n, int lane) {
  if (n > 1) {
    const bool up = rs_keep(lane, S);
    const int h = n >> 1;
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      if (i < h) {
        const T send = up ? v[i] : v[i + h];
        const T keep = up ? v[i + h] : v[i];
        v[i] = keep + rs_partner<S>(send);
      }
    }
  } else {
    v[0] += rs_partner<S>(v[0]);
  }
}

template <int N, typename T>
__device__ __forceinline__ T reduce_scatter(T (&v)[N]) {
  static_assert(N >= 2 && N <= 64 && (N & (N - 1)) == 0, "N a power of two up to 64");
  const int lane = lane_id();
  rs_step<0>(v, N, lane);
  rs_step<1>(v, N >> 1, lane);
  rs_step<2>(v, N >> 2, lane);
  rs_step<3>(v, N >> 3, lane);
  rs_step<4>(v, N >> 4, lane);
  rs_step<5>(v, N >> 5, lane);
  return v[0];
}

// Segmented inclusive scan over lanes whose keys form contiguous runs (each
// key one run).  A scan inside each 16-lane row by shifts of 1, 2, 4, 8, then
// the carries between rows: rows 1 and 3 take lane 15 of the row before,
// rows 2 and 3 take lane 31.  Bit s of `links` (s < 4) says that lane - 2^s is
// in this lane's row and run; bit 4 that the row broadcast source of the
// first carry is in this lane's run, bit 5 the same for lane 31.  After
// seg_sum the last lane of each run holds the run's total.
__device__ __forceinline__ uint32_t seg_links(int key) {
  const int nk = ~key;   // never equal to key
  uint32_t l = 0;
  l |= dpp<kDppRowShr + 1>(nk, key) == key ? 1u : 0u;
  l |= dpp<kDppRowShr + 2>(nk, key) == key ? 2u : 0u;
  l |= dpp<kDppRowShr + 4>(nk, key) == key ? 4u : 0u;
  l |= dpp<kDppRowShr + 8>(nk, key) == key ? 8u : 0u;
  l |= dpp<kDppBcast15, 0xA>(nk, key) == key ? 16u : 0u;
  l |= dpp<kDppBcast31, 0xC>(nk, key) == key ? 32u : 0u;
  return l;
}

// 32-bit values: an add with the lane move folded in, and a select.  64-bit
// values: v += f * t with f = 1 (take) or 0, one multiply-add instead of an
// add and two 32-bit selects; for finite t the result is v + t or v exactly.
template <int Ctrl, int RowMask, int N, typename T>
__device__ __forceinline__ void seg_step(T (&v)[N], bool take) {
  T t[N];
#pragma unroll
  for (int k = 0; k < N; ++k) t[k] = dpp<Ctrl, RowMask>(T(0), v[k]);
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = take ? v[k] + t[k] : v[k];
  } else {
    const T f = take ? T(1) : T(0);
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = __builtin_fma(t[k], f, v[k]);
  }
}

template <int N, typename T>
__device__ __forceinline__ void seg_sum(T (&v)[N], uint32_t links) {
  seg_step<kDppRowShr + 1, 0xF>(v, links & 1u);
  seg_step<kDppRowShr + 2, 0xF>(v, links & 2u);
  seg_step<kDppRowShr + 4, 0xF>(v, links & 4u);
  seg_step<kDppRowShr + 8, 0xF>(v, links & 8u);
  seg_step<kDppBcast15, 0xA>(v, links & 16u);
  seg_step<kDppBcast31, 0xC>(v, links & 32u);
}

// true in the last lane of each run (and in lane 63)
__device__ __forceinline__ bool run_tail(int key) { return dpp<kDppWaveShl1>(~key, key) != key; }

template <typename T>
__device__ __forceinline__ T ld_coherent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T> struct Prec;
template <> struct Prec<float> {
  using T2 = float2;
  __device__ static const float2 POVAR_GMEM* cm_m(const DevProblem& D) { return D.cm_m32; }
  __device__ static const float2 POVAR_GMEM* pk_m(const DevProblem& D) { return D.pk_m32; }
  __device__ static const float2 POVAR_GMEM* cs_m(const DevProblem& D) { return D.cs_m32; }
  // series record of buffer b: P at 0, x at kSerX (stride s_stride)
  __device__ static float POVAR_GMEM* S(const DevProblem& D, int b) { return b ? D.S32[1] : D.S32[0]; }
  __device__ static const float POVAR_GMEM* xs(const DevProblem& D, int b) { return b ? D.xs32[1] : D.xs32[0]; }
};
template <> struct Prec<double> {
  using T2 = double2;
  __device__ static const double2 POVAR_GMEM* cm_m(const DevProblem& D) { return D.cm_m64; }
  __device__ static const double2 POVAR_GMEM* pk_m(const DevProblem& D) { return D.pk_m64; }
  __device__ static const double2 POVAR_GMEM* cs_m(const DevProblem& D) { return D.cs_m64; }
  __device__ static double POVAR_GMEM* S(const DevProblem& D, int b) { return b ? D.S64[1] : D.S64[0]; }
  __device__ static const double POVAR_GMEM* xs(const DevProblem& D, int b) { return b ? D.xs64[1] : D.xs64[0]; }
};

// Two consecutive doubles (16 B aligned).
template <typename Ptr>
__device__ __forceinline__ void load_d2(Ptr p, double& a, double& b) {
  const double2 v = *(const double2 POVAR_GMEM*)(p);
  a = v.x;
  b = v.y;
}

// Vector loads and stores of 4 / 12 consecutive elements of device memory
// (16 B aligned), through global-address-space pointers.
template <typename T, typename Ptr>
__device__ __forceinline__ void load4(Ptr p, T& a, T& b, T& c, T& d) {
  if constexpr (std::is_same<T, float>::value) {
    const float4 v = *(const float4 POVAR_GMEM*)(p);
    a = v.x; b = v.y; c = v.z; d = v.w;
  } else {
    const double2 POVAR_GMEM* q = (const double2 POVAR_GMEM*)(p);
    const double2 v0 = q[0], v1 = q[1];
    a = v0.x; b = v0.y; c = v1.x; d = v1.y;
  }
}

template <typename T, typename Ptr>
__device__ __forceinline__ void store4(Ptr p, T a, T b, T c, T d) {
  if constexpr (std::is_same<T, float>::value) {
    *(float4 POVAR_GMEM*)(p) = make_float4(a, b, c, d);
  } else {
    double2 POVAR_GMEM* q = (double2 POVAR_GMEM*)(p);
    q[0] = make_double2(a, b);
    q[1] = make_double2(c, d);
  }
}

template <typename T, typename Ptr>
__device__ __forceinline__ void load12(Ptr p, T (&v)[12]) {
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

__device__ __forceinline__ void sym3_pinv_jacobi(const double (&v)[6], double (&out)[6]) {
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
      const double i0 = 1.0 / d0;
      const double l10 = v[1] * i0, l20 = v[2] * i0;
      const double d1 = v[3] - l10 * v[1];
      if (d1 > thr) {
        const double i1 = 1.0 / d1;
        const double e12 = v[4] - l20 * v[1];
        const double l21 = e12 * i1;
        const double d2 = v[5] - l20 * v[2] - l21 * e12;
        if (d2 > thr) {
          const double a10 = -l10, a21 = -l21, a20 = l10 * l21 - l20;
          const double i2 = 1.0 / d2;
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
// FP64.  Per observation, J_l has rows sqrt(a)(R0 - m1 R2), sqrt(a)(R1 - m2 R2),
// sqrt(eta) R0, sqrt(eta) R1 (R_a = rows of Pbar), and the residual at X = 0
// is built from p4.  V_j = sum J_l^T J_l, h_j = -sum J_l^T r(X=0),
// X_j = V_j^+ h_j (8); then at X_j the cost sum ||r||^2 (9), b_l = sum J_l^T r
// and z0 = V^+ b_l.
__device__ __forceinline__ void obs_normal(const double (&Pc)[12], double m1, double m2, double a, double eta,
                                           double (&v)[6], double (&h)[3]) {
  const double D0[3] = {Pc[0] - m1 * Pc[8], Pc[1] - m1 * Pc[9], Pc[2] - m1 * Pc[10]};
  const double D1[3] = {Pc[4] - m2 * Pc[8], Pc[5] - m2 * Pc[9], Pc[6] - m2 * Pc[10]};
  const double R0[3] = {Pc[0], Pc[1], Pc[2]};
  const double R1[3] = {Pc[4], Pc[5], Pc[6]};
  v[0] = a * (D0[0] * D0[0] + D1[0] * D1[0]) + eta * (R0[0] * R0[0] + R1[0] * R1[0]);
  v[1] = a * (D0[0] * D0[1] + D1[0] * D1[1]) + eta * (R0[0] * R0[1] + R1[0] * R1[1]);
  v[2] = a * (D0[0] * D0[2] + D1[0] * D1[2]) + eta * (R0[0] * R0[2] + R1[0] * R1[2]);
  v[3] = a * (D0[1] * D0[1] + D1[1] * D1[1]) + eta * (R0[1] * R0[1] + R1[1] * R1[1]);
  v[4] = a * (D0[1] * D0[2] + D1[1] * D1[2]) + eta * (R0[1] * R0[2] + R1[1] * R1[2]);
  v[5] = a * (D0[2] * D0[2] + D1[2] * D1[2]) + eta * (R0[2] * R0[2] + R1[2] * R1[2]);
  const double o1 = a * (Pc[3] - m1 * Pc[11]), o2 = a * (Pc[7] - m2 * Pc[11]);
  const double f1 = eta * (Pc[3] - m1), f2 = eta * (Pc[7] - m2);
#pragma unroll
  for (int k = 0; k < 3; ++k) h[k] = -(D0[k] * o1 + D1[k] * o2 + R0[k] * f1 + R1[k] * f2);
}

// residual cost and J_l^T r of one observation at X
__device__ __forceinline__ double obs_residual(const double (&Pc)[12], double m1, double m2, double a, double eta,
                                              double X0, double X1, double X2, double (&b)[3]) {
  const double u = Pc[0] * X0 + Pc[1] * X1 + Pc[2] * X2 + Pc[3];
  const double v = Pc[4] * X0 + Pc[5] * X1 + Pc[6] * X2 + Pc[7];
  const double w = Pc[8] * X0 + Pc[9] * X1 + Pc[10] * X2 + Pc[11];
  const double o1 = u - m1 * w, o2 = v - m2 * w;
  const double f1 = u - m1, f2 = v - m2;
  const double ao1 = a * o1, ao2 = a * o2, ef1 = eta * f1, ef2 = eta * f2;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    b[k] = (Pc[k] - m1 * Pc[8 + k]) * ao1 + (Pc[4 + k] - m2 * Pc[8 + k]) * ao2 + Pc[k] * ef1 + Pc[4 + k] * ef2;
  return a * (o1 * o1 + o2 * o2) + eta * (f1 * f1 + f2 * f2);
}

__device__ __forceinline__ void store_landmark(DevProblem& D, int lc, int j, const double (&vp)[6], double X0,
                                               double X1, double X2, const double (&bl)[3]) {
  const double z0 = vp[0] * bl[0] + vp[1] * bl[1] + vp[2] * bl[2];
  const double z1 = vp[1] * bl[0] + vp[3] * bl[1] + vp[4] * bl[2];
  const double z2 = vp[2] * bl[0] + vp[4] * bl[1] + vp[5] * bl[2];
  double* r64 = (lc ? D.rec64[1] : D.rec64[0]) + (size_t)j * kRec;
  double* v64 = (lc ? D.Vp64[1] : D.Vp64[0]) + (size_t)j * kLmSym;
  store4(r64, z0, z1, z2, 0.0);
  store4(r64 + 4, X0, X1, X2, 1.0);
  store4((lc ? D.xs64[1] : D.xs64[0]) + (size_t)j * 4, X0, X1, X2, 1.0);
  store4((lc ? D.xs32[1] : D.xs32[0]) + (size_t)j * 4, (float)X0, (float)X1, (float)X2, 1.0f);
  store4(v64, vp[0], vp[1], vp[2], vp[3]);
  *(double2 POVAR_GMEM*)(v64 + 4) = make_double2(vp[4], vp[5]);
}

// mode 0: initial state, 1: trial point of a step (other buffers), 2: re-solve
// at the current cameras.  Writes one cost partial per packet.
__global__ void __launch_bounds__(kBlock) k_landmark_solve(Batch B, int mode) {
  int p, q;
  if (!map_wave(B, kUnitPacket, p, q)) return;
  DevProblem& D = B.probs[p];
  const int trial = mode == 1 ? 1 : 0;
  if (trial && D.ctl.done) return;
  const int pc = D.ctl.pcur ^ trial, lc = D.ctl.lcur ^ trial;
  const double* __restrict__ P = pc ? D.P64[1] : D.P64[0];
  const int lane = lane_id();
  const double eta = D.eta, a = 1.0 - eta;
  const int off = q * kWave;
  // entry loads do not wait for the slot header
  const uint32_t code = D.pk_code[off + lane];
  const double2 mraw = D.pk_m64[off + lane];
  const int2 hdr = D.pk_hdr[q];
  const int n = hdr.x, lm0 = hdr.y;
  double ftot = 0.0, bl2 = 0.0;   // cost and |b_l|^2 of the slot's landmarks
  if (n == 0) {
    // continuation slot of a landmark with more than 64 observations
  } else if (n <= kWave) {
    const bool act = lane < n;
    int key = kWave + lane, c = 0;
    double2 m = make_double2(0.0, 0.0);
    if (act) {
      c = (int)(code & kCamMask);
      key = (int)(code >> kCamBits);
      m = mraw;
    }
    double Pc[12];
    if (act) load12(P + (size_t)c * kCam, Pc);
    else
#pragma unroll
      for (int k = 0; k < 12; ++k) Pc[k] = 0.0;
    double v[6], h[3];
    obs_normal(Pc, m.x, m.y, a, eta, v, h);
    const uint32_t links = seg_links(key);
    double vh[9] = {v[0], v[1], v[2], v[3], v[4], v[5], h[0], h[1], h[2]};
    seg_sum(vh, links);
    const bool tail = act && run_tail(key);
    double vp[6] = {0, 0, 0, 0, 0, 0};
    double X0 = 0, X1 = 0, X2 = 0;
    // the tail lane solves its landmark and hands X to the run through LDS
    __shared__ double bx[kWavesPerBlock][3][kWave];
    const int wv = threadIdx.x >> 6;
    if (tail) {
      const double vs[6] = {vh[0], vh[1], vh[2], vh[3], vh[4], vh[5]};
      sym3_pinv(vs, vp);
      X0 = vp[0] * vh[6] + vp[1] * vh[7] + vp[2] * vh[8];
      X1 = vp[1] * vh[6] + vp[3] * vh[7] + vp[4] * vh[8];
      X2 = vp[2] * vh[6] + vp[4] * vh[7] + vp[5] * vh[8];
      bx[wv][0][key] = X0;
      bx[wv][1][key] = X1;
      bx[wv][2][key] = X2;
    }
    wave_sync();
    double b[3] = {0, 0, 0}, f = 0.0;
    if (act) {
      X0 = bx[wv][0][key];
      X1 = bx[wv][1][key];
      X2 = bx[wv][2][key];
      f = obs_residual(Pc, m.x, m.y, a, eta, X0, X1, X2, b);
    }
    seg_sum(b, links);
    ftot = wave_sum(f);
    bl2 = wave_sum(tail ? b[0] * b[0] + b[1] * b[1] + b[2] * b[2] : 0.0);
    if (tail) store_landmark(D, lc, lm0 + key, vp, X0, X1, X2, b);
  } else {
    // a single landmark with more than 64 observations: lanes stride over it
    double v[6] = {0, 0, 0, 0, 0, 0}, h[3] = {0, 0, 0};
    for (int e = off + lane; e < off + n; e += kWave) {
      const int c = (int)(D.pk_code[e] & kCamMask);
      const double2 m = D.pk_m64[e];
      double Pc[12], vv[6], hh[3];
      load12(P + (size_t)c * kCam, Pc);
      obs_normal(Pc, m.x, m.y, a, eta, vv, hh);
#pragma unroll
      for (int k = 0; k < 6; ++k) v[k] += vv[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) h[k] += hh[k];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) h[k] = wave_sum(h[k]);
    double vp[6];
    sym3_pinv(v, vp);
    const double X0 = vp[0] * h[0] + vp[1] * h[1] + vp[2] * h[2];
    const double X1 = vp[1] * h[0] + vp[3] * h[1] + vp[4] * h[2];
    const double X2 = vp[2] * h[0] + vp[4] * h[1] + vp[5] * h[2];
    double b[3] = {0, 0, 0}, f = 0.0;
    for (int e = off + lane; e < off + n; e += kWave) {
      const int c = (int)(D.pk_code[e] & kCamMask);
      const double2 m = D.pk_m64[e];
      double Pc[12], bb[3];
      load12(P + (size_t)c * kCam, Pc);
      f += obs_residual(Pc, m.x, m.y, a, eta, X0, X1, X2, bb);
#pragma unroll
      for (int k = 0; k < 3; ++k) b[k] += bb[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) b[k] = wave_sum(b[k]);
    ftot = wave_sum(f);
    bl2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    if (lane == 0) store_landmark(D, lc, lm0, vp, X0, X1, X2, b);
  }
  if (lane == 0) {
    D.cost_part[q] = ftot;
    D.bl_part[q] = bl2;
    // the trial landmark solve starts when the step's power series has ended
    if (trial && q == 0 && D.ctl.series_t0 != 0) D.ctl.series_last = wall_clock64() - D.ctl.series_t0;
  }
}

// Cost reduction in two fixed-order levels: k_cost_groups adds kCostGroup
// consecutive packet partials per workgroup, then one workgroup adds the
// groups (thread t adds groups t, t+256, ... in order, then a fixed tree).
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kWavesPerBlock];
  const double s = wave_sum(v);
  if (lane_id() == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void __launch_bounds__(kBlock) k_cost_groups(Batch B, int trial) {
  int p, g;
  if (!map_block(B, kUnitCostGroup, p, g)) return;
  DevProblem& D = B.probs[p];
  if (trial && D.ctl.done) return;
  const int q0 = g * kCostGroup, q1 = min(q0 + kCostGroup, D.n_pk);
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int r = 0; r < kCostGroup / kBlock; ++r) {
    const int q = q0 + r * kBlock + (int)threadIdx.x;
    if (q < q1) {
      a += D.cost_part[q];
      b += D.bl_part[q];
    }
  }
  const double s = block_sum(a);
  __syncthreads();   // block_sum's LDS is reused
  const double sb = block_sum(b);
  if (threadIdx.x == 0) {
    D.cost_group[g] = s;
    D.bl_group[g] = sb;
  }
}

// Cost of all packets: from the group sums, or, for problems with few
// packets (no groups), from the packet partials directly.
__device__ __forceinline__ double packet_sum(const DevProblem& D, const double POVAR_GMEM* part,
                                             const double POVAR_GMEM* group) {
  double a = 0.0;
  if (D.n_cg > 0) {
    for (int q = threadIdx.x; q < D.n_cg; q += kBlock) a += group[q];
  } else {
    // eight independent loads per thread per round, added in a fixed order
    for (int q0 = 0; q0 < D.n_pk; q0 += kBlock * 8) {
      double v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int q = q0 + r * kBlock + (int)threadIdx.x;
        v[r] = q < D.n_pk ? part[q] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) a += v[r];
    }
  }
  return block_sum(a);
}

__device__ __forceinline__ double packet_cost_sum(const DevProblem& D) {
  return packet_sum(D, D.cost_part, D.cost_group);
}

// cost of a landmark solve outside the LM loop, one workgroup per problem:
// mode 0 initial (cost, cost0), 1 trial (cost_trial), 2 reset (cost)
__global__ void __launch_bounds__(kBlock) k_cost_finalize(Batch B, int mode) {
  int p, w;
  if (!map_block(B, kUnitOne, p, w)) return;
  DevProblem& D = B.probs[p];
  const double f = packet_cost_sum(D);
  if (threadIdx.x == 0) {
    if (mode == 1) {
      D.ctl.cost_trial = f;
    } else {
      D.ctl.cost = f;
      if (mode == 0) D.ctl.cost0 = f;
    }
  }
}

// ------------------------------------------------------------- k_linearize
// One workgroup per camera chunk.  Accumulates, in FP64, the 40 distinct
// values of U_i = sum N_k (x) x~x~^T (N has fixed entries 1 and 0 in its
// top-left 2x2 block, so U_i is made of sum x~x~^T, sum m1 x~x~^T, sum m2 x~x~^T
// and sum |m|^2 x~x~^T), b_p = sum vec((N y - eta (m,0)) x~^T) and
// sum_k W_k z0_j = sum vec((N Pbar z0) x~^T).  U_i is formed from the FP64
// landmark copy and the FP64 measurements with FP64 products in both
// precisions: the damped camera block is factored in FP64, and at small
// damping its weakest directions turn the rounding of an FP32-formed U_i
// into steps that fail.  The other products are in T.  Writes one 64-value partial per chunk; k_camera_prep
// adds a camera's chunks in order.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_linearize(Batch B, int force) {
  int p, ch;
  if (!map_block(B, kUnitChunk, p, ch)) return;
  DevProblem& D = B.probs[p];
  // force 0: a running problem after an accept; 1: any running problem;
  // 2: after an accept, also once the problem has finished (report)
  if (force != 2 && D.ctl.done) return;
  if (force != 1 && !D.ctl.need_lin) return;
  const int lc = D.ctl.lcur, pc = D.ctl.pcur;
  const int4 meta = D.ch_meta[ch];
  const int cam = meta.x, beg = meta.y, end = meta.z;
  T Pc[12];
  load12(Prec<T>::S(D, pc) + (size_t)cam * D.s_stride, Pc);
  // landmarks and measurements are read in FP64 in both precisions (U_i is
  // formed from them) and rounded to T for the other sums: the rounded values
  // are the FP32 copies the series passes use
  const double* __restrict__ rec = lc ? D.rec64[1] : D.rec64[0];
  const double2* __restrict__ M = D.cm_m64;
  const int32_t* __restrict__ lm = D.cm_lm;
  const T eta = (T)D.eta, a = (T)(1.0 - D.eta);

  double acc[kLinVals];
#pragma unroll
  for (int k = 0; k < kLinVals; ++k) acc[k] = 0.0;
  // two observations at a time in FP32; in FP64 that would spill the
  // reduction's registers
  constexpr int kUnroll = sizeof(T) == 4 ? 2 : 1;
#pragma unroll kUnroll
  for (int r = 0; r < kPerLane; ++r) {
    const int e = beg + r * kBlock + (int)threadIdx.x;
    if (e >= end) break;
    const int j = lm[e];
    const double2 m64 = M[e];
    double z64[4], X64[4];
    load4(rec + (size_t)j * kRec, z64[0], z64[1], z64[2], z64[3]);
    load4(rec + (size_t)j * kRec + 4, X64[0], X64[1], X64[2], X64[3]);
    T z[4], x[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      z[c] = (T)z64[c];
      x[c] = (T)X64[c];
    }
    struct {
      T x, y;
    } const m = {(T)m64.x, (T)m64.y};
    const T am1 = a * m.x, am2 = a * m.y, msq = m.x * m.x + m.y * m.y, amsq = a * msq;
    T y[3], q[3];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
      y[rr] = Pc[4 * rr] * x[0] + Pc[4 * rr + 1] * x[1] + Pc[4 * rr + 2] * x[2] + Pc[4 * rr + 3];
      q[rr] = Pc[4 * rr] * z[0] + Pc[4 * rr + 1] * z[1] + Pc[4 * rr + 2] * z[2];
    }
    T nv[3], vq[3];
    apply_N(am1, am2, amsq, y[0], y[1], y[2], nv[0], nv[1], nv[2]);
    apply_N(am1, am2, amsq, q[0], q[1], q[2], vq[0], vq[1], vq[2]);
    nv[0] -= eta * m.x;
    nv[1] -= eta * m.y;
    const double mx = m64.x, my = m64.y, ms = mx * mx + my * my;
    int o = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int d = c; d < 4; ++d) {
        const double xx = X64[c] * X64[d];
        acc[o] += xx;
        acc[10 + o] += mx * xx;
        acc[20 + o] += my * xx;
        acc[30 + o] += ms * xx;
        ++o;
      }
    }
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[40 + 4 * rr + c] += (double)(nv[rr] * x[c]);
        acc[52 + 4 * rr + c] += (double)(vq[rr] * x[c]);
      }
    }
  }
  __shared__ double red[kWavesPerBlock][kLinVals];
  const int wv = threadIdx.x >> 6;
  {
    const double s = reduce_scatter<kLinVals>(acc);
    red[wv][rs_index<kLinVals>(lane_id())] = s;
  }
  __syncthreads();
  if (threadIdx.x < kLinVals) {
    const int k = threadIdx.x;
    D.lin_part[(size_t)ch * kLinVals + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
}

// ----------------------------------------------------------- k_camera_prep
// One lane per camera, FP64.  After a linearisation it adds the camera's
// chunk partials in order.  U_l = U + lambda diag(U) (floored).  On the
// sphere the tangent-space inverse B (B^T U_l B)^-1 B^T (B any orthonormal
// basis of p^perp) equals the constrained (KKT) form
//   K = U_l^-1 - w w^T / (p^T w),   w = U_l^-1 p ,
// which needs only the Cholesky factor of U_l.  Euclidean: K = U_l^-1.
// x_0 = acc = -K g with g = b_p - sum W_k V^+ b_l.
__host__ __device__ constexpr int tri(int r, int c) { return r * (r + 1) / 2 + c; }

// -------------------------------------------------------- k_camera_sums
// After an accept, for problems with wave_sums set: each camera's 64
// linearisation sums (the 40 distinct entries of U_i, then the two 12-vectors
// whose difference is the reduced gradient g_i), its chunk partials added in
// chunk order.  One wave per camera, lane k adds value k: a camera seen
// hundreds of thousands of times (hundreds of chunks) costs that many
// coalesced loads of one wave instead of one lane's serial walk over 64
// values per chunk.  The sums are those k_camera_prep forms for the other
// problems, bit for bit.  The second stage (whose partials, recomputed every
// iteration, have the same 40 + 12 + 12 layout) takes its sums from here on
// every iteration for k_refine_prep.  One workgroup per 64 cameras, each
// wave a quarter of them.
static_assert(kLinVals == kWave && kLin2 == kWave, "one linearisation value per lane");
__global__ void __launch_bounds__(kBlock) k_camera_sums(Batch B) {
  int p, w;
  if (!map_block(B, kUnitCamWave, p, w)) return;
  DevProblem& D = B.probs[p];
  const bool stage2 = D.stage == 2;
  if (D.ctl.done || !D.wave_sums || !(stage2 || D.ctl.need_lin)) return;
  const int lane = lane_id();
  const double* __restrict__ part = stage2 ? D.lin2 : D.lin_part;
  for (int c = (int)(threadIdx.x >> 6); c < kWave; c += kWavesPerBlock) {
    const int i = w * kWave + c;
    if (i >= D.n_p) break;
    const int q1 = D.cam_ch[i + 1];
    double s = 0.0;
#pragma unroll 8
    for (int q = D.cam_ch[i]; q < q1; ++q) s += part[(size_t)q * kLinVals + lane];
    const double other = __shfl(s, (lane + 12) & (kWave - 1));   // lane 40 + k receives value 52 + k
    if (lane < 40) D.U40[(size_t)i * 40 + lane] = s;
    else if (lane < 52) D.g64[(size_t)i * kCam + lane - 40] = s - other;
  }
}

template <typename T>
__global__ void __launch_bounds__(kWave) k_camera_prep(Batch B) {
  int p, w;
  if (!map_wave<kWave>(B, kUnitCamWave, p, w)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done) return;
  const int i = w * kWave + lane_id();
  // a new step: all series terms until an early stop says otherwise
  if (i == 0) {
    D.ctl.stop_at = D.ctl.order;
    D.ctl.stopped = 0;
    // device clock of the step's power series (17): from here (the camera
    // blocks' factors and x_0) to the trial landmark solve, which reads it
    D.ctl.series_t0 = wall_clock64();
    D.ctl.series_last = 0;
  }
  if (i >= D.n_p) return;
  const double lam = D.ctl.lambda;
  const int pc = D.ctl.pcur;
  const bool sphere = D.manifold == 0;
  const double a = 1.0 - D.eta;

  // U_i and g_i: after an accept the sums of the chunk partials (here, or in
  // k_camera_sums for problems with wave_sums), else those in place
  double u40[40], g[12];
  if (D.ctl.need_lin && !D.wave_sums) {
    double s[kLinVals];
#pragma unroll
    for (int k = 0; k < kLinVals; ++k) s[k] = 0.0;
    for (int q = D.cam_ch[i]; q < D.cam_ch[i + 1]; ++q) {
      const double* part = D.lin_part + (size_t)q * kLinVals;
#pragma unroll
      for (int k = 0; k < kLinVals; ++k) s[k] += part[k];
    }
#pragma unroll
    for (int k = 0; k < 40; ++k) {
      u40[k] = s[k];
      D.U40[(size_t)i * 40 + k] = s[k];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      g[k] = s[40 + k] - s[52 + k];
      D.g64[(size_t)i * kCam + k] = g[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < 40; ++k) u40[k] = D.U40[(size_t)i * 40 + k];
#pragma unroll
    for (int k = 0; k < 12; ++k) g[k] = D.g64[(size_t)i * kCam + k];
  }
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
  load12(pc ? D.P64[1] + (size_t)i * kCam : D.P64[0] + (size_t)i * kCam, pv);
  // Cholesky U_l = L L^T in place (Marquardt damping keeps the diagonally
  // scaled block well conditioned; Cholesky is insensitive to that scaling)
  bool ok = true;
  double rd[12];   // reciprocals of the diagonal of L
#pragma unroll
  for (int j = 0; j < 12; ++j) {
    double d = L[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[tri(j, k)] * L[tri(j, k)];
    if (!(d > 0.0)) { ok = false; d = 1.0; }
    d = sqrt(d);
    L[tri(j, j)] = d;
    rd[j] = 1.0 / d;
#pragma unroll
    for (int r = j + 1; r < 12; ++r) {
      double v = L[tri(r, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[tri(r, k)] * L[tri(j, k)];
      L[tri(r, j)] = v * rd[j];
    }
  }
  // L^-1 in place, column by column, rows ascending; the one reciprocal per
  // row replaces a division per entry (which dominates this lane's chain)
#pragma unroll
  for (int j = 0; j < 12; ++j) {
    L[tri(j, j)] = rd[j];
#pragma unroll
    for (int r = j + 1; r < 12; ++r) {
      double v = 0.0;
#pragma unroll
      for (int k = j; k < r; ++k) v += L[tri(r, k)] * L[tri(k, j)];
      L[tri(r, j)] = -v * rd[r];
    }
  }
  // sphere: w = U_l^-1 p, h = p^T U_l^-1 p
  double wp[12], ih = 0.0;
  if (sphere) {
    double u[12], h = 0.0;
#pragma unroll
    for (int r = 0; r < 12; ++r) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k <= r; ++k) v += L[tri(r, k)] * pv[k];
      u[r] = v;
      h += v * v;
    }
#pragma unroll
    for (int r = 0; r < 12; ++r) {
      double v = 0.0;
#pragma unroll
      for (int k = r; k < 12; ++k) v += L[tri(k, r)] * u[k];
      wp[r] = v;
    }
    ih = 1.0 / h;
  }
  double x0[12];
#pragma unroll
  for (int r = 0; r < 12; ++r) x0[r] = 0.0;
  double* K64 = D.K64 + (size_t)i * kCamMat;
#pragma unroll
  for (int r = 0; r < 12; ++r) {
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      double v = 0.0;
#pragma unroll
      for (int k = r; k < 12; ++k) v += L[tri(k, r)] * L[tri(k, c)];
      if (sphere) v -= wp[r] * wp[c] * ih;
      if (!ok) v = 0.0;
      K64[r * 12 + c] = v;
      K64[c * 12 + r] = v;
      x0[r] -= v * g[c];
      if (c != r) x0[c] -= v * g[r];
    }
  }
  T POVAR_GMEM* x = Prec<T>::S(D, D.ctl.pcur) + (size_t)i * D.s_stride + kSerX;
  double* acc = D.acc + (size_t)i * kCam;
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    x[r] = (T)x0[r];
    acc[r] = x0[r];
  }
  if (!ok) atomicOr(&D.ctl.status, 1);
}

// ------------------------------------------------------- k_series_landmark
// z_j = V_j^+ y_j with the FP64 pseudo-inverse in both precisions: rounding
// V^+ itself to FP32 would perturb W V^+ W^T by ~eps * cond(V_j) and can push
// the spectrum of M past 1 for the near-singular blocks of random starts;
// applied in FP64 to the FP32 sum y_j the error stays ~eps * sqrt(cond(V_j)).
template <typename T>
__device__ __forceinline__ void store_z(const double (&v)[8], int j, T y0, T y1, T y2, T X0, T X1, T X2, T* zx) {
  const double d0 = y0, d1 = y1, d2 = y2;
  const double z0 = v[0] * d0 + v[1] * d1 + v[2] * d2;
  const double z1 = v[1] * d0 + v[3] * d1 + v[4] * d2;
  const double z2 = v[2] * d0 + v[4] * d1 + v[5] * d2;
  store4(zx + (size_t)j * kRec, (T)z0, (T)z1, (T)z2, (T)0);
  store4(zx + (size_t)j * kRec + 4, X0, X1, X2, (T)1);
}

// Camera series data of the landmark pass: x_i (12 values) and the rows of
// Pbar_i, from the series records in global memory ...
template <typename T>
struct CamFromRecords {
  const T* __restrict__ S;
  int stride;
  __device__ __forceinline__ void operator()(int c, T (&xc)[12], T (&Pc)[12]) const {
    load12(S + (size_t)c * stride + kSerX, xc);
    load12(S + (size_t)c * stride, Pc);
  }
};

// The first loads of a packet slot (this lane's entry and the slot header),
// which depend on nothing else.
template <typename T>
struct SlotHead {
  uint32_t code;
  typename Prec<T>::T2 m;
  int2 hdr;
};

template <typename T>
__device__ __forceinline__ SlotHead<T> slot_head(const DevProblem& D, int q) {
  const int e = q * kWave + lane_id();
  return SlotHead<T>{D.pk_code[e], Prec<T>::pk_m(D)[e], D.pk_hdr[q]};
}

// One packet slot of the landmark pass: z_j = V_j^+ sum_k Pbar_i^T N_k (X_i x~_j),
// X_i = x_i as a 3x4 matrix; the (z_j, X_j) record is written for the camera
// pass.  Wave-uniform; all 64 lanes call it.
template <typename T, typename Cam, bool Coop = false>
__device__ __forceinline__ void landmark_slot(const DevProblem& D, int q, const SlotHead<T>& head, int lc,
                                              const Cam& cam, f4v POVAR_LDS* cbuf = nullptr) {
  const int lane = lane_id();
  const int off = q * kWave;
  const T* __restrict__ xs = Prec<T>::xs(D, lc);
  const typename Prec<T>::T2* __restrict__ em = Prec<T>::pk_m(D);
  const T a = (T)(1.0 - D.eta);
  T* zx = static_cast<T*>(D.zx);
  const uint32_t code = head.code;
  const auto mraw = head.m;
  const int n = head.hdr.x, lm0 = head.hdr.y;
  if (n == 0) return;   // continuation slot of a long landmark
  if (n <= kWave) {
    const bool act = lane < n;
    const int key = act ? (int)(code >> kCamBits) : kWave + lane;
    const bool tail = act && run_tail(key);
    T y0 = 0, y1 = 0, y2 = 0, X0 = 0, X1 = 0, X2 = 0, one;
    double v[8];
    T xc[12], Pc[12];
    if constexpr (Coop) {
      // V^+ and X are requested before the cooperative camera gather
      if (act) {
        if (tail) {
          const double* vp = (lc ? D.Vp64[1] : D.Vp64[0]) + (size_t)(lm0 + key) * kLmSym;
          load4(vp, v[0], v[1], v[2], v[3]);
          load_d2(vp + 4, v[4], v[5]);
        }
        load4(xs + (size_t)(lm0 + key) * 4, X0, X1, X2, one);
      }
      const int src[1] = {act ? (int)(code & kCamMask) : -1};
      if constexpr (sizeof(T) == 4) {
        f4v pc[1][kCoopPieces];
        coop_fetch<kCoopPieces, 1, kCoopHalves>((const char POVAR_GMEM*)cam.S, (size_t)cam.stride * sizeof(T), src,
                                                cbuf, pc);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            Pc[4 * r + k] = pc[0][r][k];
            xc[4 * r + k] = pc[0][3 + r][k];
          }
      } else {
        // P and x (96 bytes each) in two gathers through the same buffer
        f4v pp[1][kCoopPieces], px[1][kCoopPieces];
        const char POVAR_GMEM* base = (const char POVAR_GMEM*)cam.S;
        coop_fetch<kCoopPieces>(base, (size_t)cam.stride * sizeof(T), src, cbuf, pp);
        coop_fetch<kCoopPieces>(base + kSerX * sizeof(T), (size_t)cam.stride * sizeof(T), src, cbuf, px);
#pragma unroll
        for (int i = 0; i < kCoopPieces; ++i) {
          piece_d2(pp[0][i], Pc[2 * i], Pc[2 * i + 1]);
          piece_d2(px[0][i], xc[2 * i], xc[2 * i + 1]);
        }
      }
    }
    if (act) {
      const int c = (int)(code & kCamMask);
      if constexpr (!Coop) {
        // the tail lane fetches V^+ together with the gathers
        if (tail) {
          const double* vp = (lc ? D.Vp64[1] : D.Vp64[0]) + (size_t)(lm0 + key) * kLmSym;
          load4(vp, v[0], v[1], v[2], v[3]);
          load_d2(vp + 4, v[4], v[5]);
        }
        load4(xs + (size_t)(lm0 + key) * 4, X0, X1, X2, one);
        cam(c, xc, Pc);
      }
      const auto m = mraw;
      const T q0 = xc[0] * X0 + xc[1] * X1 + xc[2] * X2 + xc[3];
      const T q1 = xc[4] * X0 + xc[5] * X1 + xc[6] * X2 + xc[7];
      const T q2 = xc[8] * X0 + xc[9] * X1 + xc[10] * X2 + xc[11];
      T v0, v1, v2;
      apply_N(a * m.x, a * m.y, a * (m.x * m.x + m.y * m.y), q0, q1, q2, v0, v1, v2);
      y0 = Pc[0] * v0 + Pc[4] * v1 + Pc[8] * v2;
      y1 = Pc[1] * v0 + Pc[5] * v1 + Pc[9] * v2;
      y2 = Pc[2] * v0 + Pc[6] * v1 + Pc[10] * v2;
    }
    T y[3] = {y0, y1, y2};
    seg_sum(y, seg_links(key));
    if (tail) store_z<T>(v, lm0 + key, y[0], y[1], y[2], X0, X1, X2, zx);
  } else {
    T X0, X1, X2, one;
    load4(xs + (size_t)lm0 * 4, X0, X1, X2, one);
    T y0 = 0, y1 = 0, y2 = 0;
    double v[8];
    const double* vp = (lc ? D.Vp64[1] : D.Vp64[0]) + (size_t)lm0 * kLmSym;
    load4(vp, v[0], v[1], v[2], v[3]);
    load_d2(vp + 4, v[4], v[5]);
    for (int e = off + lane; e < off + n; e += kWave) {
      const int c = (int)(D.pk_code[e] & kCamMask);
      const auto m = em[e];
      T xc[12], Pc[12];
      cam(c, xc, Pc);
      const T q0 = xc[0] * X0 + xc[1] * X1 + xc[2] * X2 + xc[3];
      const T q1 = xc[4] * X0 + xc[5] * X1 + xc[6] * X2 + xc[7];
      const T q2 = xc[8] * X0 + xc[9] * X1 + xc[10] * X2 + xc[11];
      T v0, v1, v2;
      apply_N(a * m.x, a * m.y, a * (m.x * m.x + m.y * m.y), q0, q1, q2, v0, v1, v2);
      y0 += Pc[0] * v0 + Pc[4] * v1 + Pc[8] * v2;
      y1 += Pc[1] * v0 + Pc[5] * v1 + Pc[9] * v2;
      y2 += Pc[2] * v0 + Pc[6] * v1 + Pc[10] * v2;
    }
    y0 = wave_sum(y0);
    y1 = wave_sum(y1);
    y2 = wave_sum(y2);
    if (lane == 0) store_z<T>(v, lm0, y0, y1, y2, X0, X1, X2, zx);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_series_landmark(Batch B, int t) {
  int p, q;
  if (!map_wave(B, kUnitPacket, p, q)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || t > D.ctl.stop_at) return;
  const CamFromRecords<T> cam{Prec<T>::S(D, D.ctl.pcur), D.s_stride};
  landmark_slot<T>(D, q, slot_head<T>(D, q), D.ctl.lcur, cam);
}

// FP32 landmark pass of batches holding problems with 128-byte camera records
// (too many cameras for the vector L1): those problems fetch the records
// cooperatively, through kCoopLdsBytes of dynamic LDS; the others per lane.
__global__ void __launch_bounds__(kBlock) k_series_landmark_coop(Batch B, int t) {
  int p, q;
  if (!map_wave(B, kUnitPacket, p, q)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || t > D.ctl.stop_at) return;
  const CamFromRecords<float> cam{Prec<float>::S(D, D.ctl.pcur), D.s_stride};
  if (D.s_stride == kSerLine) {
    extern __shared__ f4v coop_lds[];
    f4v POVAR_LDS* buf = (f4v POVAR_LDS*)coop_lds + (threadIdx.x >> 6) * (kCoopPieces * kWave / kCoopHalves);
    landmark_slot<float, CamFromRecords<float>, true>(D, q, slot_head<float>(D, q), D.ctl.lcur, cam, buf);
  } else {
    landmark_slot<float>(D, q, slot_head<float>(D, q), D.ctl.lcur, cam);
  }
}

// FP64 landmark pass (every FP64 problem): P and x gathered cooperatively,
// through a 6 KB LDS buffer per wave.  Even 250 cameras' FP64 records (48 KB)
// overflow the vector L1, so per-lane gathers would go to L2 one line per
// lane and piece.
__global__ void __launch_bounds__(kBlock) k_series_landmark_coop64(Batch B, int t) {
  int p, q;
  if (!map_wave(B, kUnitPacket, p, q)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || t > D.ctl.stop_at) return;
  const CamFromRecords<double> cam{Prec<double>::S(D, D.ctl.pcur), D.s_stride};
  __shared__ f4v cbuf[kWavesPerBlock][kCoopPieces * kWave];
  landmark_slot<double, CamFromRecords<double>, true>(D, q, slot_head<double>(D, q), D.ctl.lcur, cam,
                                                      (f4v POVAR_LDS*)cbuf[threadIdx.x >> 6]);
}

// --------------------------------------------------------- k_series_camera
// t_i = sum_k vec((N_k Pbar_i z_j) x~_j^T); x_i = K_i t_i; acc_i += x_i.
// The camera block is applied in FP64 in both precisions.
// Retraction of one camera (Sec. 4.3): q = p + acc, p_trial = q / |q| on the
// sphere (q in Euclidean mode), FP64, into the other camera buffer and the
// series record.  Value k of the camera in thread k of 12 consecutive lanes.
template <typename T>
__device__ __forceinline__ void retract_value(DevProblem& D, int cam, int k, double q, double (&qs)[12]) {
  qs[k] = q;
  wave_sync();
  double nrm = 0.0;
#pragma unroll
  for (int r = 0; r < 12; ++r) nrm += qs[r] * qs[r];
  if (D.manifold == 0) q *= 1.0 / sqrt(nrm);
  const int pc = D.ctl.pcur;
  (pc ? D.P64[0] : D.P64[1])[(size_t)cam * kCam + k] = q;
  Prec<T>::S(D, pc ^ 1)[(size_t)cam * D.s_stride + k] = (T)q;
}

// x_i = K_i t_i in FP64, acc_i += x_i (threads 0..11); after the last order
// the same threads retract the camera, so no separate pass is needed.
template <typename T>
__device__ __forceinline__ void camera_solve(DevProblem& D, int cam, const T* tv, const double (&kr)[12], bool last) {
  __shared__ double qs[12];
  const int k = threadIdx.x;
  if (k >= 12) return;
  double xr = 0.0;
#pragma unroll
  for (int c = 0; c < 12; ++c) xr += kr[c] * (double)tv[c];
  const int pc = D.ctl.pcur;
  Prec<T>::S(D, pc)[(size_t)cam * D.s_stride + kSerX + k] = (T)xr;
  const double a = D.acc[(size_t)cam * kCam + k] + xr;
  D.acc[(size_t)cam * kCam + k] = a;
  if (last) retract_value<T>(D, cam, k, (pc ? D.P64[1] : D.P64[0])[(size_t)cam * kCam + k] + a, qs);
}

constexpr int kCamWG = 1024;   // threads of a camera-chunk workgroup

// Sum of the per-wave partials of value k, in a fixed pairwise order.
template <typename T, int NW>
__device__ __forceinline__ T wg_sum(const T (&red)[NW][12], int k) {
  if constexpr (NW == 4) {
    return ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  } else {
    T v[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) v[w] = red[w][k];
#pragma unroll
    for (int h = NW / 2; h > 0; h >>= 1)
#pragma unroll
      for (int w = 0; w < h; ++w) v[w] = v[w] + v[w + h];
    return v[0];
  }
}

template <typename T, int WG>
__global__ void __launch_bounds__(WG) k_series_camera(Batch B, int t) {
  constexpr int kPL = kChunk / WG;   // observations per lane
  int p, ch;
  if (!map_block(B, kUnitSerChunk, p, ch)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || t > D.ctl.stop_at) return;
  const int pc = D.ctl.pcur;
  const int4 meta = D.ch_meta[ch];
  const int cam = meta.x, beg = meta.y, end = meta.z, nch = meta.w;
  T Pc[12];
  load12(Prec<T>::S(D, pc) + (size_t)cam * D.s_stride, Pc);
  // the camera-block row of this thread, fetched before the reduction needs it
  double kr[12];
  if (nch == 1 && threadIdx.x < 12) load12(D.K64 + (size_t)cam * kCamMat + threadIdx.x * 12, kr);
  const T* __restrict__ zx = static_cast<const T*>(D.zx);
  const typename Prec<T>::T2* __restrict__ M = Prec<T>::cm_m(D);
  const int32_t* __restrict__ lm = D.cm_lm;
  const T a = (T)(1.0 - D.eta);
  // all index and measurement loads, then all record gathers, then the
  // arithmetic: two memory round trips per lane instead of two per
  // observation.  The trip count is uniform over the workgroup.
  const int nr = (end - beg + WG - 1) / WG;
  const int tid = (int)threadIdx.x;
  int jr[kPL];
  typename Prec<T>::T2 mr[kPL];
#pragma unroll
  for (int r = 0; r < kPL; ++r) {
    if (r < nr) {
      const int e = min(beg + r * WG + tid, end - 1);
      jr[r] = lm[e];
      mr[r] = M[e];
    }
  }
  T z[kPL][4], x[kPL][4];
#pragma unroll
  for (int r = 0; r < kPL; ++r) {
    if (r < nr) {
      load4(zx + (size_t)jr[r] * kRec, z[r][0], z[r][1], z[r][2], z[r][3]);
      load4(zx + (size_t)jr[r] * kRec + 4, x[r][0], x[r][1], x[r][2], x[r][3]);
    }
  }
  T acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0;
#pragma unroll
  for (int r = 0; r < kPL; ++r) {
    if (r < nr && beg + r * WG + tid < end) {
      const auto m = mr[r];
      const T q0 = Pc[0] * z[r][0] + Pc[1] * z[r][1] + Pc[2] * z[r][2];
      const T q1 = Pc[4] * z[r][0] + Pc[5] * z[r][1] + Pc[6] * z[r][2];
      const T q2 = Pc[8] * z[r][0] + Pc[9] * z[r][1] + Pc[10] * z[r][2];
      T v[3];
      apply_N(a * m.x, a * m.y, a * (m.x * m.x + m.y * m.y), q0, q1, q2, v[0], v[1], v[2]);
#pragma unroll
      for (int rr = 0; rr < 3; ++rr) {
        acc[4 * rr + 0] += v[rr] * x[r][0];
        acc[4 * rr + 1] += v[rr] * x[r][1];
        acc[4 * rr + 2] += v[rr] * x[r][2];
        acc[4 * rr + 3] += v[rr];
      }
    }
  }
  __shared__ T red[WG / kWave][12];
  __shared__ T tv[12];
  const int wv = threadIdx.x >> 6;
  {
    T v16[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v16[k] = k < 12 ? acc[k] : T(0);
    const T s = reduce_scatter<16>(v16);
    const int idx = rs_index<16>(lane_id());
    if (lane_id() < 16 && idx < 12) red[wv][idx] = s;
  }
  __syncthreads();
  const int k = threadIdx.x;
  if (nch > 1) {
    // finished by k_series_camera_combine after all chunks are written
    if (k < 12) static_cast<T*>(D.t_part)[(size_t)ch * kCam + k] = wg_sum<T, WG / kWave>(red, k);
    return;
  }
  if (k < 12) tv[k] = wg_sum<T, WG / kWave>(red, k);
  __syncthreads();
  camera_solve<T>(D, cam, tv, kr, t == D.ctl.order);
}

// One wave per camera whose series partials need adding (chunks of a camera
// spanning several chunks, or the runs of a blocked problem): adds the
// camera's partials in order (lane-strided, then a fixed tree) and applies
// the camera block.
template <typename T>
__global__ void __launch_bounds__(kWave) k_series_camera_combine(Batch B, int t) {
  int p, u;
  if (!map_wave<kWave>(B, kUnitMultiCam, p, u)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || t > D.ctl.stop_at) return;
  const int cam = D.ser_mc[u];
  const int c0 = D.ser_off[cam], np = D.ser_off[cam + 1] - c0;
  double kr[12];
  if (threadIdx.x < 12) load12(D.K64 + (size_t)cam * kCamMat + threadIdx.x * 12, kr);
  const T* __restrict__ part = static_cast<const T*>(D.ser_part);
  T s[12];
#pragma unroll
  for (int kk = 0; kk < 12; ++kk) s[kk] = 0;
  for (int q = lane_id(); q < np; q += kWave) {
    T v[12];
    load12(part + (size_t)(c0 + q) * kCam, v);
#pragma unroll
    for (int kk = 0; kk < 12; ++kk) s[kk] += v[kk];
  }
  __shared__ T tv[12];
  {
    T v16[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v16[k] = k < 12 ? s[k] : T(0);
    const T r = reduce_scatter<16>(v16);
    const int idx = rs_index<16>(lane_id());
    if (lane_id() < 16 && idx < 12) tv[idx] = r;
  }
  __syncthreads();
  camera_solve<T>(D, cam, tv, kr, t == D.ctl.order);
}

// --------------------------------------------------- k_series_camera_slots
// Blocked problems: one wave per camera slot, cs_per_lane observations per
// lane, all of one run.  t_run = sum_k vec((N_k Pbar_i z_j) x~_j^T) over the
// run's observations; the (z, X) records gathered here belong to the slot's
// landmark block, which the slot order keeps in one XCD's L2.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_series_camera_slots(Batch B, int t) {
  constexpr int kCsPerLane = cs_per_lane(sizeof(T) == 4);
  int p, q;
  if (!map_wave(B, kUnitCSlot, p, q)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || t > D.ctl.stop_at) return;
  const int lane = lane_id();
  const int pc = D.ctl.pcur;
  // entry loads do not wait for the slot header
  const int2 li = D.cs_lane[(size_t)q * kWave + lane];
  int jr[kCsPerLane];
  typename Prec<T>::T2 mr[kCsPerLane];
#pragma unroll
  for (int r = 0; r < kCsPerLane; ++r) {
    const size_t e = ((size_t)q * kCsPerLane + r) * kWave + lane;
    jr[r] = D.cs_lm[e];
    mr[r] = Prec<T>::cs_m(D)[e];
  }
  const int nl = D.cs_hdr[q];
  if (nl == 0) return;   // empty slot (keeps the XCD order)
  const bool act = lane < nl;
  const int cam = li.x & (int)kCamMask;
  const int key = act ? (int)((uint32_t)li.x >> kCamBits) : kWave + lane;
  T Pc[12];
  if (act) load12(Prec<T>::S(D, pc) + (size_t)cam * D.s_stride, Pc);
  else
#pragma unroll
    for (int k = 0; k < 12; ++k) Pc[k] = 0;
  const T* __restrict__ zx = static_cast<const T*>(D.zx);
  T z[kCsPerLane][4], x[kCsPerLane][4];
  if constexpr (sizeof(T) == 4) {
    // the 32-byte records fetched by pairs of lanes (half the L1 lookups)
    __shared__ f4v cbuf[kWavesPerBlock][2 * kWave];
    f4v rz[kCsPerLane][2];
    coop_fetch<2, kCsPerLane>((const char POVAR_GMEM*)zx, kRec * sizeof(T), jr,
                              (f4v POVAR_LDS*)cbuf[threadIdx.x >> 6], rz);
#pragma unroll
    for (int r = 0; r < kCsPerLane; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        z[r][k] = rz[r][0][k];
        x[r][k] = rz[r][1][k];
      }
  } else {
    // the 64-byte records fetched by groups of four lanes (a quarter of the L1 lookups)
    __shared__ f4v cbuf[kWavesPerBlock][4 * kWave];
    f4v rz[kCsPerLane][4];
    coop_fetch<4, kCsPerLane>((const char POVAR_GMEM*)zx, kRec * sizeof(T), jr,
                              (f4v POVAR_LDS*)cbuf[threadIdx.x >> 6], rz);
#pragma unroll
    for (int r = 0; r < kCsPerLane; ++r) {
      piece_d2(rz[r][0], z[r][0], z[r][1]);
      piece_d2(rz[r][1], z[r][2], z[r][3]);
      piece_d2(rz[r][2], x[r][0], x[r][1]);
      piece_d2(rz[r][3], x[r][2], x[r][3]);
    }
  }
  const T a = (T)(1.0 - D.eta);
  T acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0;
#pragma unroll
  for (int r = 0; r < kCsPerLane; ++r) {
    if (jr[r] >= 0) {
      const auto m = mr[r];
      const T q0 = Pc[0] * z[r][0] + Pc[1] * z[r][1] + Pc[2] * z[r][2];
      const T q1 = Pc[4] * z[r][0] + Pc[5] * z[r][1] + Pc[6] * z[r][2];
      const T q2 = Pc[8] * z[r][0] + Pc[9] * z[r][1] + Pc[10] * z[r][2];
      T v[3];
      apply_N(a * m.x, a * m.y, a * (m.x * m.x + m.y * m.y), q0, q1, q2, v[0], v[1], v[2]);
#pragma unroll
      for (int rr = 0; rr < 3; ++rr) {
        acc[4 * rr + 0] += v[rr] * x[r][0];
        acc[4 * rr + 1] += v[rr] * x[r][1];
        acc[4 * rr + 2] += v[rr] * x[r][2];
        acc[4 * rr + 3] += v[rr];
      }
    }
  }
  seg_sum(acc, seg_links(key));
  if (act && run_tail(key)) {
    T* out = static_cast<T*>(D.ser_part) + (size_t)li.y * kCam;
#pragma unroll
    for (int k = 0; k < 12; k += 4) store4(out + k, acc[k], acc[k + 1], acc[k + 2], acc[k + 3]);
  }
}

// ---------------------------------------------------------- k_series_check
// Optional early stop of the series (series_rtol > 0): after term t (1 <= t <
// order), the 2-norms over all cameras of x_t (the stored series term) and of
// acc = x_0 + ... + x_t, summed in FP64 in a fixed order; if ||x_t|| <=
// series_rtol ||acc||, the later terms are skipped and k_retract applies acc.
// One workgroup per problem.
// After term t: ||x_t|| and ||acc|| over all cameras (FP64 sums in a fixed
// order, one workgroup); stop_at = t if ||x_t|| <= series_rtol ||acc||.
// x(i, k) returns value k of camera i's term.
template <typename X>
__device__ __forceinline__ void series_check(DevProblem& D, int t, const X& x) {
  double sx = 0.0, sa = 0.0;
  for (int i = (int)threadIdx.x; i < D.n_p; i += kBlock) {
#pragma unroll
    for (int k = 0; k < kCam; ++k) {
      const double v = x(i, k);
      const double a = D.acc[(size_t)i * kCam + k];
      sx += v * v;
      sa += a * a;
    }
  }
  sx = wave_sum(sx);
  sa = wave_sum(sa);
  __shared__ double red[kWavesPerBlock][2];
  const int wv = threadIdx.x >> 6;
  if (lane_id() == 0) {
    red[wv][0] = sx;
    red[wv][1] = sa;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double nx = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
  const double na = ((red[0][1] + red[1][1]) + red[2][1]) + red[3][1];
  if (sqrt(nx) <= D.series_rtol * sqrt(na)) {
    D.ctl.stop_at = t;
    D.ctl.stopped = 1;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_series_check(Batch B, int t) {
  int p, w;
  if (!map_block(B, kUnitOne, p, w)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || !(D.series_rtol > 0.0) || t > D.ctl.stop_at || t >= D.ctl.order) return;
  const T POVAR_GMEM* S = Prec<T>::S(D, D.ctl.pcur);
  const int ss = D.s_stride;
  series_check(D, t, [&](int i, int k) { return (double)S[(size_t)i * ss + kSerX + k]; });
}

// --------------------------------------------------------------- k_retract
template <typename T>
__global__ void __launch_bounds__(kWave) k_retract(Batch B) {
  int p, w;
  if (!map_wave<kWave>(B, kUnitCamWave, p, w)) return;
  DevProblem& D = B.probs[p];
  // order >= 1: retracted by the camera pass of the last term, unless the
  // series stopped early
  if (D.ctl.done || (D.ctl.order > 0 && !D.ctl.stopped)) return;
  const int i = w * kWave + lane_id();
  if (i >= D.n_p) return;
  const int pc = D.ctl.pcur;
  double q[12];
  load12((pc ? D.P64[1] : D.P64[0]) + (size_t)i * kCam, q);
  const double* acc = D.acc + (size_t)i * kCam;
  double nrm = 0.0;
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    q[r] += acc[r];
    nrm += q[r] * q[r];
  }
  if (D.manifold == 0) {
    const double inv = 1.0 / sqrt(nrm);
#pragma unroll
    for (int r = 0; r < 12; ++r) q[r] *= inv;
  }
  double* o64 = (pc ? D.P64[0] : D.P64[1]) + (size_t)i * kCam;
  T POVAR_GMEM* os = Prec<T>::S(D, pc ^ 1) + (size_t)i * D.s_stride;
#pragma unroll
  for (int r = 0; r < 12; r += 4) {
    store4(o64 + r, q[r], q[r + 1], q[r + 2], q[r + 3]);
    store4(os + r, (T)q[r], (T)q[r + 1], (T)q[r + 2], (T)q[r + 3]);
  }
}

// ------------------------------------------------------------- k_grad_norm
// Riemannian gradient of the reduced cost at the current cameras: by the
// envelope theorem the gradient of f* is 2 b_p (b_p = sum_k J_p,k^T r_k at
// X*(P), Eq. (9)-(10)); on the sphere it is projected onto each camera's
// tangent space.  b_p from the linearisation partials of the current cameras
// (chunks added in order, as in k_camera_prep); one workgroup per problem,
// FP64 sum in a fixed order.
__global__ void __launch_bounds__(kBlock) k_grad_norm(Batch B) {
  int p, w;
  if (!map_block(B, kUnitOne, p, w)) return;
  DevProblem& D = B.probs[p];
  const int pc = D.ctl.pcur;
  double s = 0.0;
  for (int i = (int)threadIdx.x; i < D.n_p; i += kBlock) {
    double b[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) b[k] = 0.0;
    for (int q = D.cam_ch[i]; q < D.cam_ch[i + 1]; ++q) {
#pragma unroll
      for (int k = 0; k < 12; ++k) b[k] += D.lin_part[(size_t)q * kLinVals + 40 + k];
    }
    if (D.manifold == 0) {
      double pv[12], pb = 0.0;
      load12((pc ? D.P64[1] : D.P64[0]) + (size_t)i * kCam, pv);
#pragma unroll
      for (int k = 0; k < 12; ++k) pb += pv[k] * b[k];
#pragma unroll
      for (int k = 0; k < 12; ++k) b[k] -= pb * pv[k];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) s += b[k] * b[k];
  }
  s = block_sum(s);
  if (threadIdx.x == 0) D.ctl.grad_norm = 2.0 * sqrt(s);
}

// ---------------------------------------------------------------- k_decide
// Adds the trial cost partials (packet order), then: strict decrease accepts
// (NaN rejects, and so does a step whose damped camera block could not be
// Cholesky-factored); lambda /10 on accept, x10 on reject, clamped;
// relinearise only after an accept; ftol on accepted steps.  One workgroup
// per problem.
__global__ void __launch_bounds__(kBlock) k_decide(Batch B) {
  int p, w;
  if (!map_block(B, kUnitOne, p, w)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done) return;
  const double fn = packet_cost_sum(D);
  __syncthreads();   // block_sum's LDS is reused
  const double bl2 = packet_sum(D, D.bl_part, D.bl_group);
  if (threadIdx.x != 0) return;
  Ctl& c = D.ctl;
  const double f = c.cost;
  // a step whose damped camera block could not be factored is rejected
  const bool factored = (c.status & 1) == 0;
  c.status &= ~1;
  c.cost_trial = factored ? fn : INFINITY;
  const bool accept = factored && (fn < f) && (fn - fn == 0.0);
  const int it = c.iter;
  if (it < D.trace_cap) {
    D.tr_cost[it] = c.cost_trial;
    D.tr_lambda[it] = c.lambda;
    D.tr_acc[it] = accept ? 1 : 0;
    D.tr_bl[it] = factored ? sqrt(bl2) : NAN;
    D.tr_series[it] = (double)c.series_last;
  }
  c.series_ticks += c.series_last;
  if (accept) {
    const double rel = (f - fn) / f;
    c.cost = fn;
    c.lcur ^= 1;
    c.pcur ^= 1;
    c.lambda = fmax(c.lambda / 10.0, D.lambda_min);
    c.n_accept += 1;
    if (rel < D.ftol) { c.done = 1; c.stop_reason = 1; }
  } else {
    c.lambda = fmin(c.lambda * 10.0, D.lambda_max);
  }
  c.need_lin = accept ? 1 : 0;
  c.iter = it + 1;
  if (c.iter >= c.iter_limit) c.done = 1;
}

// ============================================================ second stage
// Projective refinement (RiPoBA): objective (7), r = pi(P_i X_j) - m with
// pi(y) = (y0 / y2, y1 / y2), P_i on the unit sphere of R^12 and X_j on the
// unit sphere of R^4; the camera update by the power series of the inverse
// Riemannian Schur complement (27)-(29), the landmarks by back-substitution,
// both retracted (Sec. 4.3).  FP64.  With y = P X, iw = 1 / y2 and
// u = (y0 iw, y1 iw):  d pi / d y = iw [[1, 0, -u0], [0, 1, -u1]],
// J_l = (d pi / d y) P (2 x 4) and J_p[r][4a + c] = (d pi / d y)[r][a] X_c.
// Tangent projections in an explicit orthonormal basis of each tangent
// space (the last columns of the Householder reflection that maps the point
// to a coordinate axis): K_i = B (B^T U_l B)^-1 B^T and G_j likewise, applied
// in ambient coordinates.  Both blocks are singular along their own point up
// to the damping, so the constrained (KKT) form through U_l^-1 would cancel
// terms of size 1 / lambda.
struct Proj2 {
  double iw, u0, u1;
  double jl0[4], jl1[4];   // rows of J_l
};

__device__ __forceinline__ Proj2 project2(const double (&P)[12], const double (&X)[4]) {
  Proj2 g;
  const double y0 = P[0] * X[0] + P[1] * X[1] + P[2] * X[2] + P[3] * X[3];
  const double y1 = P[4] * X[0] + P[5] * X[1] + P[6] * X[2] + P[7] * X[3];
  const double y2 = P[8] * X[0] + P[9] * X[1] + P[10] * X[2] + P[11] * X[3];
  g.iw = 1.0 / y2;
  g.u0 = y0 * g.iw;
  g.u1 = y1 * g.iw;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    g.jl0[c] = g.iw * (P[c] - g.u0 * P[8 + c]);
    g.jl1[c] = g.iw * (P[4 + c] - g.u1 * P[8 + c]);
  }
  return g;
}

// (d pi / d y)^T s
__device__ __forceinline__ void dpi_t(const Proj2& g, double s0, double s1, double (&h)[3]) {
  h[0] = g.iw * s0;
  h[1] = g.iw * s1;
  h[2] = -g.iw * (g.u0 * s0 + g.u1 * s1);
}

// J_p x for a camera-space vector x (12 values, row-major 3 x 4)
__device__ __forceinline__ void jp_apply(const Proj2& g, const double (&x)[12], const double (&X)[4], double& s0,
                                         double& s1) {
  const double a0 = x[0] * X[0] + x[1] * X[1] + x[2] * X[2] + x[3] * X[3];
  const double a1 = x[4] * X[0] + x[5] * X[1] + x[6] * X[2] + x[7] * X[3];
  const double a2 = x[8] * X[0] + x[9] * X[1] + x[10] * X[2] + x[11] * X[3];
  s0 = g.iw * (a0 - g.u0 * a2);
  s1 = g.iw * (a1 - g.u1 * a2);
}

__host__ __device__ constexpr int sym4(int a, int b) { return a <= b ? (a * 7 - a * a) / 2 + b : (b * 7 - b * b) / 2 + a; }

// Inverse of a symmetric positive-definite 4x4 block (10 values, sym4 order)
// by Cholesky; false if a pivot is not positive.
__device__ __forceinline__ bool sym4_inv(const double (&v)[10], double (&out)[10]) {
  double L[4][4], Li[4][4], rd[4];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double d = v[sym4(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0)) { ok = false; d = 1.0; }
    d = sqrt(d);
    L[j][j] = d;
    rd[j] = 1.0 / d;
#pragma unroll
    for (int r = j + 1; r < 4; ++r) {
      double t = v[sym4(r, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[r][k] * L[j][k];
      L[r][j] = t * rd[j];
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    Li[j][j] = rd[j];
#pragma unroll
    for (int r = j + 1; r < 4; ++r) {
      double t = 0.0;
#pragma unroll
      for (int k = j; k < r; ++k) t += L[r][k] * Li[k][j];
      Li[r][j] = -t * rd[r];
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      double t = 0.0;
#pragma unroll
      for (int k = b; k < 4; ++k) t += Li[k][a] * Li[k][b];
      out[sym4(a, b)] = t;
    }
  return ok;
}

// V (10) and b_l (4) contributions of one observation
__device__ __forceinline__ void refine_lm_terms(const Proj2& g, double r0, double r1, double (&vb)[14]) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = a; b < 4; ++b) vb[sym4(a, b)] = g.jl0[a] * g.jl0[b] + g.jl1[a] * g.jl1[b];
    vb[10 + a] = g.jl0[a] * r0 + g.jl1[a] * r1;
  }
}

// The damped, projected, inverted landmark block G_j, b_l and z0 = G_j b_l.
__device__ __forceinline__ void refine_lm_finish(DevProblem& D, int j, const double (&vb)[14], const double (&X)[4],
                                                 double lam) {
  double v[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) v[k] = vb[k];
  const double dmax = fmax(fmax(v[0], v[4]), fmax(v[7], v[9]));
  v[0] += lam * fmax(v[0], 1e-12 * dmax);
  v[4] += lam * fmax(v[4], 1e-12 * dmax);
  v[7] += lam * fmax(v[7], 1e-12 * dmax);
  v[9] += lam * fmax(v[9], 1e-12 * dmax);
  // G = B (B^T V_l B)^-1 B^T with B the last three columns of the
  // Householder reflection H = I - beta h h^T that maps X to -+e_0 (an
  // orthonormal basis of the tangent space at X): A = H V_l H, whose lower
  // right 3 x 3 block is inverted (row and column 0 replaced by those of the
  // identity), then G = H diag(0, A_33^-1) H.  V_l is singular along X up to
  // the damping (the landmark's scale does not change the residual), so the
  // inverse of V_l itself would carry 1 / lambda along X; the 3 x 3 block
  // has no such direction.
  double hv[4] = {X[0] + (X[0] >= 0.0 ? 1.0 : -1.0), X[1], X[2], X[3]};
  const double beta = 2.0 / (hv[0] * hv[0] + hv[1] * hv[1] + hv[2] * hv[2] + hv[3] * hv[3]);
  double u[4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
    u[a] = v[sym4(a, 0)] * hv[0] + v[sym4(a, 1)] * hv[1] + v[sym4(a, 2)] * hv[2] + v[sym4(a, 3)] * hv[3];
  const double hu = hv[0] * u[0] + hv[1] * u[1] + hv[2] * u[2] + hv[3] * u[3];
  double A[10];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b)
      A[sym4(a, b)] = v[sym4(a, b)] - beta * (hv[a] * u[b] + u[a] * hv[b]) + beta * beta * hu * hv[a] * hv[b];
  A[sym4(0, 0)] = 1.0;
  A[sym4(0, 1)] = A[sym4(0, 2)] = A[sym4(0, 3)] = 0.0;
  double vi[10];
  const bool ok = sym4_inv(A, vi);
  vi[sym4(0, 0)] = 0.0;   // diag(0, A_33^-1)
  double w[4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
    w[a] = vi[sym4(a, 0)] * hv[0] + vi[sym4(a, 1)] * hv[1] + vi[sym4(a, 2)] * hv[2] + vi[sym4(a, 3)] * hv[3];
  const double hw = hv[0] * w[0] + hv[1] * w[1] + hv[2] * w[2] + hv[3] * w[3];
  double G[10];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b)
      G[sym4(a, b)] = vi[sym4(a, b)] - beta * (hv[a] * w[b] + w[a] * hv[b]) + beta * beta * hw * hv[a] * hv[b];
  double* go = D.g2 + (size_t)j * kG2;
#pragma unroll
  for (int k = 0; k < 10; ++k) go[k] = G[k];
  store4(D.bl2 + (size_t)j * 4, vb[10], vb[11], vb[12], vb[13]);
  // z0 = G_j b_l with X_j: the (z, X) record k_refine_cameras gathers
  double z0[4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
    z0[a] = G[sym4(a, 0)] * vb[10] + G[sym4(a, 1)] * vb[11] + G[sym4(a, 2)] * vb[12] + G[sym4(a, 3)] * vb[13];
  double* zo = static_cast<double*>(D.zx) + (size_t)j * kRec;
  store4(zo, z0[0], z0[1], z0[2], z0[3]);
  store4(zo + 4, X[0], X[1], X[2], X[3]);
  if (!ok) atomicOr(&D.ctl.status, 1);
}

// k_refine_landmarks: per landmark V_j, b_l, G_j and z0 at the current point,
// and the cost partial of each packet (Eq. (7)).
__global__ void __launch_bounds__(kBlock) k_refine_landmarks(Batch B) {
  int p, q;
  if (!map_wave(B, kUnitPacket, p, q)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done) return;
  const double* __restrict__ P = D.ctl.pcur ? D.P64[1] : D.P64[0];
  const double* __restrict__ Xr = D.ctl.lcur ? D.rec64[1] : D.rec64[0];
  const double lam = D.ctl.lambda;
  const int lane = lane_id(), off = q * kWave;
  const uint32_t code = D.pk_code[off + lane];
  const double2 mraw = D.pk_m64[off + lane];
  const int2 hdr = D.pk_hdr[q];
  const int n = hdr.x, lm0 = hdr.y;
  double ftot = 0.0;
  if (n == 0) {
    // continuation slot of a landmark with more than 64 observations
  } else if (n <= kWave) {
    const bool act = lane < n;
    const int key = act ? (int)(code >> kCamBits) : kWave + lane;
    double vb[14], X[4] = {0.0, 0.0, 0.0, 1.0}, f = 0.0;
#pragma unroll
    for (int k = 0; k < 14; ++k) vb[k] = 0.0;
    if (act) {
      double Pc[12];
      load12(P + (size_t)(code & kCamMask) * kCam, Pc);
      load4(Xr + (size_t)(lm0 + key) * kX2, X[0], X[1], X[2], X[3]);
      const Proj2 g = project2(Pc, X);
      const double r0 = g.u0 - mraw.x, r1 = g.u1 - mraw.y;
      refine_lm_terms(g, r0, r1, vb);
      f = r0 * r0 + r1 * r1;
    }
    seg_sum(vb, seg_links(key));
    ftot = wave_sum(f);
    if (act && run_tail(key)) refine_lm_finish(D, lm0 + key, vb, X, lam);
  } else {
    double vb[14], X[4], f = 0.0;
#pragma unroll
    for (int k = 0; k < 14; ++k) vb[k] = 0.0;
    load4(Xr + (size_t)lm0 * kX2, X[0], X[1], X[2], X[3]);
    for (int e = off + lane; e < off + n; e += kWave) {
      double Pc[12], t[14];
      load12(P + (size_t)(D.pk_code[e] & kCamMask) * kCam, Pc);
      const double2 m = D.pk_m64[e];
      const Proj2 g = project2(Pc, X);
      const double r0 = g.u0 - m.x, r1 = g.u1 - m.y;
      refine_lm_terms(g, r0, r1, t);
#pragma unroll
      for (int k = 0; k < 14; ++k) vb[k] += t[k];
      f += r0 * r0 + r1 * r1;
    }
#pragma unroll
    for (int k = 0; k < 14; ++k) vb[k] = wave_sum(vb[k]);
    ftot = wave_sum(f);
    if (lane == 0) refine_lm_finish(D, lm0, vb, X, lam);
  }
  if (lane == 0) D.cost_part[q] = ftot;
}

// k_refine_cameras: per camera chunk, 64 FP64 sums: U_i as 40 sums of
// g (x) X X^T (d pi^T d pi = iw^2 [[1,0,-u0],[0,1,-u1],[-u0,-u1,|u|^2]] has
// the four distinct entries g), b_p = sum J_p^T r and sum W z0 = sum J_p^T J_l z0.
__global__ void __launch_bounds__(kBlock) k_refine_cameras(Batch B) {
  int p, ch;
  if (!map_block(B, kUnitChunk, p, ch)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done) return;
  const int4 meta = D.ch_meta[ch];
  const int cam = meta.x, beg = meta.y, end = meta.z;
  double Pc[12];
  load12((D.ctl.pcur ? D.P64[1] : D.P64[0]) + (size_t)cam * kCam, Pc);
  const double* __restrict__ zx = static_cast<const double*>(D.zx);
  double acc[kLin2];
#pragma unroll
  for (int k = 0; k < kLin2; ++k) acc[k] = 0.0;
#pragma unroll 1
  for (int r = 0; r < kPerLane; ++r) {
    const int e = beg + r * kBlock + (int)threadIdx.x;
    if (e >= end) break;
    const int j = D.cm_lm[e];
    const double2 m = D.cm_m64[e];
    double X[4], z[4];
    load4(zx + (size_t)j * kRec, z[0], z[1], z[2], z[3]);
    load4(zx + (size_t)j * kRec + 4, X[0], X[1], X[2], X[3]);
    const Proj2 g = project2(Pc, X);
    const double r0 = g.u0 - m.x, r1 = g.u1 - m.y;
    const double w2 = g.iw * g.iw;
    const double gg[4] = {w2, -g.u0 * w2, -g.u1 * w2, (g.u0 * g.u0 + g.u1 * g.u1) * w2};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a; b < 4; ++b) {
        const double xx = X[a] * X[b];
#pragma unroll
        for (int gi = 0; gi < 4; ++gi) acc[gi * 10 + sym4(a, b)] += gg[gi] * xx;
      }
    double hb[3], hz[3];
    dpi_t(g, r0, r1, hb);
    const double v0 = g.jl0[0] * z[0] + g.jl0[1] * z[1] + g.jl0[2] * z[2] + g.jl0[3] * z[3];
    const double v1 = g.jl1[0] * z[0] + g.jl1[1] * z[1] + g.jl1[2] * z[2] + g.jl1[3] * z[3];
    dpi_t(g, v0, v1, hz);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[40 + 4 * a + c] += hb[a] * X[c];
        acc[52 + 4 * a + c] += hz[a] * X[c];
      }
  }
  __shared__ double red[kWavesPerBlock][kLin2];
  const int wv = threadIdx.x >> 6;
  {
    const double sv = reduce_scatter<kLin2>(acc);
    red[wv][rs_index<kLin2>(lane_id())] = sv;
  }
  __syncthreads();
  if (threadIdx.x < kLin2) {
    const int k = threadIdx.x;
    D.lin2[(size_t)ch * kLin2 + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
}

// which of the four g sums feeds U[(a, c), (a2, c2)] (rows a, a2 of
// d pi^T d pi); -1 for the zero entries (0, 1)
__device__ __forceinline__ int refine_gsel(int a, int a2) {
  const int lo = a < a2 ? a : a2, hi = a < a2 ? a2 : a;
  if (lo == hi) return lo == 2 ? 3 : 0;
  if (lo == 0 && hi == 1) return -1;
  return hi == 2 ? (lo == 0 ? 1 : 2) : -1;
}

// k_refine_prep: one lane per camera.  U_i from the chunk sums, Marquardt
// damping, the tangent inverse K_i (Householder basis, Cholesky of the 11 x 11
// block), g_i = b_p - sum W z0, x0 = acc = -K_i g_i.
__global__ void __launch_bounds__(kWave) k_refine_prep(Batch B) {
  int p, w;
  if (!map_wave<kWave>(B, kUnitCamWave, p, w)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done) return;
  const int i = w * kWave + lane_id();
  // a new step: all series terms until an early stop says otherwise
  if (i == 0) {
    D.ctl.stop_at = D.ctl.order;
    D.ctl.stopped = 0;
  }
  if (i >= D.n_p) return;
  const double lam = D.ctl.lambda;
  // the chunk partials' sums, here or (problems with wave_sums) from
  // k_camera_sums: s[0..39] in U40, s[40 + k] - s[52 + k] in g64
  double s[kLin2];
  if (D.wave_sums) {
#pragma unroll
    for (int k = 0; k < 40; ++k) s[k] = D.U40[(size_t)i * 40 + k];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      s[40 + k] = D.g64[(size_t)i * kCam + k];
      s[52 + k] = 0.0;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kLin2; ++k) s[k] = 0.0;
    for (int q = D.cam_ch[i]; q < D.cam_ch[i + 1]; ++q) {
      const double* part = D.lin2 + (size_t)q * kLin2;
#pragma unroll
      for (int k = 0; k < kLin2; ++k) s[k] += part[k];
    }
  }
  double L[78];
#pragma unroll
  for (int r = 0; r < 12; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      const int gs = refine_gsel(r >> 2, c >> 2);
      L[tri(r, c)] = gs < 0 ? 0.0 : s[gs * 10 + sym4(r & 3, c & 3)];
    }
  double dmax = 0.0;
#pragma unroll
  for (int r = 0; r < 12; ++r) dmax = fmax(dmax, L[tri(r, r)]);
#pragma unroll
  for (int r = 0; r < 12; ++r) L[tri(r, r)] += lam * fmax(L[tri(r, r)], 1e-12 * dmax);
  // K = B (B^T U_l B)^-1 B^T with B the last eleven columns of the
  // Householder reflection H = I - beta h h^T mapping p to -+e_0: A = H U_l H
  // (a rank-two update of U_l), its lower right 11 x 11 block factored with
  // row and column 0 replaced by those of the identity, then
  // K = H diag(0, A_11^-1) H.  U_l is singular along p up to the damping (a
  // camera's scale does not change the residual), so the inverse of U_l
  // itself would carry 1 / lambda along p; the 11 x 11 block has no such
  // direction.
  double pv[12];
  load12((D.ctl.pcur ? D.P64[1] : D.P64[0]) + (size_t)i * kCam, pv);
  pv[0] += pv[0] >= 0.0 ? 1.0 : -1.0;   // pv is now h (p has unit norm)
  double beta;
  {
    double hh = 0.0;
#pragma unroll
    for (int r = 0; r < 12; ++r) hh += pv[r] * pv[r];
    beta = 2.0 / hh;
    double u[12], hu = 0.0;
#pragma unroll
    for (int r = 0; r < 12; ++r) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < 12; ++k) t += L[r >= k ? tri(r, k) : tri(k, r)] * pv[k];
      u[r] = t;
      hu += pv[r] * t;
    }
#pragma unroll
    for (int r = 0; r < 12; ++r)
#pragma unroll
      for (int c = 0; c <= r; ++c)
        L[tri(r, c)] += -beta * (pv[r] * u[c] + u[r] * pv[c]) + beta * beta * hu * pv[r] * pv[c];
#pragma unroll
    for (int c = 0; c < 12; ++c) L[tri(c, 0)] = c == 0 ? 1.0 : 0.0;
  }
  bool ok = true;
  double rd[12];
#pragma unroll
  for (int j = 0; j < 12; ++j) {
    double d = L[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[tri(j, k)] * L[tri(j, k)];
    if (!(d > 0.0)) { ok = false; d = 1.0; }
    d = sqrt(d);
    L[tri(j, j)] = d;
    rd[j] = 1.0 / d;
#pragma unroll
    for (int r = j + 1; r < 12; ++r) {
      double v = L[tri(r, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[tri(r, k)] * L[tri(j, k)];
      L[tri(r, j)] = v * rd[j];
    }
  }
#pragma unroll
  for (int j = 0; j < 12; ++j) {
    L[tri(j, j)] = rd[j];
#pragma unroll
    for (int r = j + 1; r < 12; ++r) {
      double v = 0.0;
#pragma unroll
      for (int k = j; k < r; ++k) v += L[tri(r, k)] * L[tri(k, j)];
      L[tri(r, j)] = -v * rd[r];
    }
  }
  // w = diag(0, A_11^-1) h = L^-T L^-1 h - h_0 e_0 (the inverse holds 1 at (0, 0))
  double wp[12], hw = 0.0;
  {
    double u[12];
#pragma unroll
    for (int r = 0; r < 12; ++r) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k <= r; ++k) v += L[tri(r, k)] * pv[k];
      u[r] = v;
    }
#pragma unroll
    for (int r = 0; r < 12; ++r) {
      double v = 0.0;
#pragma unroll
      for (int k = r; k < 12; ++k) v += L[tri(k, r)] * u[k];
      wp[r] = v;
    }
    wp[0] -= pv[0];
#pragma unroll
    for (int r = 0; r < 12; ++r) hw += pv[r] * wp[r];
  }
  double gv[12], x0[12];
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    gv[r] = s[40 + r] - s[52 + r];
    D.g64[(size_t)i * kCam + r] = gv[r];
    x0[r] = 0.0;
  }
  double* K64 = D.K64 + (size_t)i * kCamMat;
#pragma unroll
  for (int r = 0; r < 12; ++r) {
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      double v = (r == 0 && c == 0) ? -1.0 : 0.0;   // the (0, 0) entry of diag(0, A_11^-1)
#pragma unroll
      for (int k = r; k < 12; ++k) v += L[tri(k, r)] * L[tri(k, c)];
      v += -beta * (pv[r] * wp[c] + wp[r] * pv[c]) + beta * beta * hw * pv[r] * pv[c];
      if (!ok) v = 0.0;
      K64[r * 12 + c] = v;
      K64[c * 12 + r] = v;
      x0[r] -= v * gv[c];
      if (c != r) x0[c] -= v * gv[r];
    }
  }
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    D.x2[(size_t)i * kCam + r] = x0[r];
    D.acc[(size_t)i * kCam + r] = x0[r];
  }
  if (!ok) atomicOr(&D.ctl.status, 1);
}

// W^T y for one observation of camera vector y (12): J_l^T J_p y
__device__ __forceinline__ void refine_wt(const Proj2& g, const double (&y)[12], const double (&X)[4],
                                          double (&o)[4]) {
  double s0, s1;
  jp_apply(g, y, X, s0, s1);
#pragma unroll
  for (int c = 0; c < 4; ++c) o[c] = g.jl0[c] * s0 + g.jl1[c] * s1;
}

// Landmark pass over packets shared by the series (z_j = G_j sum W^T x_i) and
// the back-substitution (dl_j = -G_j (b_l + sum W^T dp_i), then the landmark
// is retracted into the other buffer).
template <bool Update>
__device__ __forceinline__ void refine_landmark_slot(DevProblem& D, int q, f4v POVAR_LDS* cbuf) {
  const double* __restrict__ P = D.ctl.pcur ? D.P64[1] : D.P64[0];
  const int lc = D.ctl.lcur;
  const double* __restrict__ Xr = lc ? D.rec64[1] : D.rec64[0];
  const double* __restrict__ Y = Update ? D.acc : D.x2;
  const int lane = lane_id(), off = q * kWave;
  const uint32_t code = D.pk_code[off + lane];
  const int2 hdr = D.pk_hdr[q];
  const int n = hdr.x, lm0 = hdr.y;
  if (n == 0) return;
  double wt[4] = {0.0, 0.0, 0.0, 0.0}, X[4] = {0.0, 0.0, 0.0, 1.0};
  int j = lm0;
  bool tail;
  if (n <= kWave) {
    const bool act = lane < n;
    const int key = act ? (int)(code >> kCamBits) : kWave + lane;
    j = lm0 + (act ? key : 0);
    if (act) load4(Xr + (size_t)j * kX2, X[0], X[1], X[2], X[3]);
    // P_i and y_i (96 bytes each) fetched cooperatively: each load
    // instruction covers about eleven consecutive records instead of 64
    // scattered ones, which cuts the vector L1's tag lookups fourfold
    const int src[1] = {act ? (int)(code & kCamMask) : -1};
    f4v pp[1][6], py[1][6];
    coop_fetch<6>((const char POVAR_GMEM*)P, kCam * sizeof(double), src, cbuf, pp);
    coop_fetch<6>((const char POVAR_GMEM*)Y, kCam * sizeof(double), src, cbuf, py);
    if (act) {
      double Pc[12], y[12];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        piece_d2(pp[0][i], Pc[2 * i], Pc[2 * i + 1]);
        piece_d2(py[0][i], y[2 * i], y[2 * i + 1]);
      }
      const Proj2 g = project2(Pc, X);
      refine_wt(g, y, X, wt);
    }
    seg_sum(wt, seg_links(key));
    tail = act && run_tail(key);
  } else {
    load4(Xr + (size_t)lm0 * kX2, X[0], X[1], X[2], X[3]);
    for (int e = off + lane; e < off + n; e += kWave) {
      const int c = (int)(D.pk_code[e] & kCamMask);
      double Pc[12], y[12], t[4];
      load12(P + (size_t)c * kCam, Pc);
      load12(Y + (size_t)c * kCam, y);
      const Proj2 g = project2(Pc, X);
      refine_wt(g, y, X, t);
#pragma unroll
      for (int k = 0; k < 4; ++k) wt[k] += t[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) wt[k] = wave_sum(wt[k]);
    tail = lane == 0;
  }
  if (!tail) return;
  const double* G = D.g2 + (size_t)j * kG2;
  double v[4];
  if (Update) {
    const double* bl = D.bl2 + (size_t)j * 4;
#pragma unroll
    for (int a = 0; a < 4; ++a) v[a] = bl[a] + wt[a];
  } else {
#pragma unroll
    for (int a = 0; a < 4; ++a) v[a] = wt[a];
  }
  double z[4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
    z[a] = G[sym4(a, 0)] * v[0] + G[sym4(a, 1)] * v[1] + G[sym4(a, 2)] * v[2] + G[sym4(a, 3)] * v[3];
  if (Update) {
    double xn[4], nrm = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      xn[a] = X[a] - z[a];
      nrm += xn[a] * xn[a];
    }
    const double inv = 1.0 / sqrt(nrm);
    double* o = (lc ? D.rec64[0] : D.rec64[1]) + (size_t)j * kX2;
    store4(o, xn[0] * inv, xn[1] * inv, xn[2] * inv, xn[3] * inv);
  } else {
    // the (z, X) record the camera pass gathers, one 64-byte line per landmark
    double* o = static_cast<double*>(D.zx) + (size_t)j * kRec;
    store4(o, z[0], z[1], z[2], z[3]);
    store4(o + 4, X[0], X[1], X[2], X[3]);
  }
}

__global__ void __launch_bounds__(kBlock) k_refine_series_landmark(Batch B, int t) {
  int p, q;
  if (!map_wave(B, kUnitPacket, p, q)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || t > D.ctl.stop_at) return;
  __shared__ f4v cbuf[kWavesPerBlock][6 * kWave];
  refine_landmark_slot<false>(D, q, (f4v POVAR_LDS*)cbuf[threadIdx.x >> 6]);
}

__global__ void __launch_bounds__(kBlock) k_refine_landmark_update(Batch B) {
  int p, q;
  if (!map_wave(B, kUnitPacket, p, q)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done) return;
  __shared__ f4v cbuf[kWavesPerBlock][6 * kWave];
  refine_landmark_slot<true>(D, q, (f4v POVAR_LDS*)cbuf[threadIdx.x >> 6]);
}

// W z for one observation, added to the camera's 12 sums:
// J_p^T J_l z = vec((d pi / d y)^T J_l z) X^T (row-major 3 x 4).
__device__ __forceinline__ void refine_w_add(const double (&Pc)[12], const double (&z)[4], const double (&X)[4],
                                             double (&acc)[12]) {
  const Proj2 g = project2(Pc, X);
  const double v0 = g.jl0[0] * z[0] + g.jl0[1] * z[1] + g.jl0[2] * z[2] + g.jl0[3] * z[3];
  const double v1 = g.jl1[0] * z[0] + g.jl1[1] * z[1] + g.jl1[2] * z[2] + g.jl1[3] * z[3];
  double h[3];
  dpi_t(g, v0, v1, h);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[4 * a + c] += h[a] * X[c];
}

// x_i = K_i t_i (rows of K_i in kr, one per thread 0..11), acc_i += x_i.
__device__ __forceinline__ void refine_camera_solve(DevProblem& D, int cam, const double* tv, const double (&kr)[12]) {
  const int k = (int)threadIdx.x;
  if (k >= 12) return;
  double x = 0.0;
#pragma unroll
  for (int c = 0; c < 12; ++c) x += kr[c] * tv[c];
  D.x2[(size_t)cam * kCam + k] = x;
  D.acc[(size_t)cam * kCam + k] += x;
}

// Camera pass of the series over camera-major chunks: t_i = sum_k W_k z_j,
// x_i = K_i t_i, acc_i += x_i.  Index loads, then the (z, X) record gathers,
// then the arithmetic; a camera spanning several chunks leaves one partial
// per chunk for k_refine_series_combine.
__global__ void __launch_bounds__(kCamWG) k_refine_series_camera(Batch B, int t) {
  constexpr int kPL = kChunk / kCamWG;   // observations per lane
  int p, ch;
  if (!map_block(B, kUnitSerChunk, p, ch)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || t > D.ctl.stop_at) return;
  const int4 meta = D.ch_meta[ch];
  const int cam = meta.x, beg = meta.y, end = meta.z, nch = meta.w;
  double Pc[12];
  load12((D.ctl.pcur ? D.P64[1] : D.P64[0]) + (size_t)cam * kCam, Pc);
  double kr[12];
  if (nch == 1 && threadIdx.x < 12) load12(D.K64 + (size_t)cam * kCamMat + threadIdx.x * 12, kr);
  const double* __restrict__ zx = static_cast<const double*>(D.zx);
  const int nr = (end - beg + kCamWG - 1) / kCamWG;
  const int tid = (int)threadIdx.x;
  int jr[kPL];
#pragma unroll
  for (int r = 0; r < kPL; ++r)
    if (r < nr) jr[r] = D.cm_lm[min(beg + r * kCamWG + tid, end - 1)];
  double z[kPL][4], X[kPL][4];
#pragma unroll
  for (int r = 0; r < kPL; ++r) {
    if (r < nr) {
      load4(zx + (size_t)jr[r] * kRec, z[r][0], z[r][1], z[r][2], z[r][3]);
      load4(zx + (size_t)jr[r] * kRec + 4, X[r][0], X[r][1], X[r][2], X[r][3]);
    }
  }
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
#pragma unroll
  for (int r = 0; r < kPL; ++r)
    if (r < nr && beg + r * kCamWG + tid < end) refine_w_add(Pc, z[r], X[r], acc);
  __shared__ double red[kCamWG / kWave][12];
  __shared__ double tv[12];
  const int wv = threadIdx.x >> 6;
  {
    double v16[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v16[k] = k < 12 ? acc[k] : 0.0;
    const double sv = reduce_scatter<16>(v16);
    const int idx = rs_index<16>(lane_id());
    if (lane_id() < 16 && idx < 12) red[wv][idx] = sv;
  }
  __syncthreads();
  const int k = threadIdx.x;
  if (nch > 1) {
    if (k < 12) static_cast<double*>(D.t_part)[(size_t)ch * kCam + k] = wg_sum<double, kCamWG / kWave>(red, k);
    return;
  }
  if (k < 12) tv[k] = wg_sum<double, kCamWG / kWave>(red, k);
  __syncthreads();
  refine_camera_solve(D, cam, tv, kr);
}

// Camera pass of landmark-blocked problems: one wave per camera slot,
// kCsPerLane observations of one run per lane, a partial sum per run; the
// (z, X) records of the slot's landmark block stay in one XCD's L2.
__global__ void __launch_bounds__(kBlock) k_refine_series_camera_slots(Batch B, int t) {
  constexpr int kCsPerLane = cs_per_lane(false);
  int p, q;
  if (!map_wave(B, kUnitCSlot, p, q)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || t > D.ctl.stop_at) return;
  const int lane = lane_id();
  const int2 li = D.cs_lane[(size_t)q * kWave + lane];
  int jr[kCsPerLane];
#pragma unroll
  for (int r = 0; r < kCsPerLane; ++r) jr[r] = D.cs_lm[((size_t)q * kCsPerLane + r) * kWave + lane];
  const int nl = D.cs_hdr[q];
  if (nl == 0) return;
  const bool act = lane < nl;
  const int cam = li.x & (int)kCamMask;
  const int key = act ? (int)((uint32_t)li.x >> kCamBits) : kWave + lane;
  double Pc[12];
  if (act) load12((D.ctl.pcur ? D.P64[1] : D.P64[0]) + (size_t)cam * kCam, Pc);
  else
#pragma unroll
    for (int k = 0; k < 12; ++k) Pc[k] = 0.0;
  const double* __restrict__ zx = static_cast<const double*>(D.zx);
  double z[kCsPerLane][4], X[kCsPerLane][4];
  {
    // (z, X) records fetched by groups of four lanes
    __shared__ f4v cbuf[kWavesPerBlock][4 * kWave];
    f4v rz[kCsPerLane][4];
    coop_fetch<4, kCsPerLane>((const char POVAR_GMEM*)zx, kRec * sizeof(double), jr,
                              (f4v POVAR_LDS*)cbuf[threadIdx.x >> 6], rz);
#pragma unroll
    for (int r = 0; r < kCsPerLane; ++r) {
      piece_d2(rz[r][0], z[r][0], z[r][1]);
      piece_d2(rz[r][1], z[r][2], z[r][3]);
      piece_d2(rz[r][2], X[r][0], X[r][1]);
      piece_d2(rz[r][3], X[r][2], X[r][3]);
    }
  }
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
#pragma unroll
  for (int r = 0; r < kCsPerLane; ++r)
    if (jr[r] >= 0) refine_w_add(Pc, z[r], X[r], acc);
  seg_sum(acc, seg_links(key));
  if (act && run_tail(key)) {
    double* out = static_cast<double*>(D.ser_part) + (size_t)li.y * kCam;
#pragma unroll
    for (int k = 0; k < 12; k += 4) store4(out + k, acc[k], acc[k + 1], acc[k + 2], acc[k + 3]);
  }
}

// One wave per camera with several partial sums (chunks or runs): adds them
// in order (lane-strided, then a fixed tree) and applies K_i.
__global__ void __launch_bounds__(kWave) k_refine_series_combine(Batch B, int t) {
  int p, u;
  if (!map_wave<kWave>(B, kUnitMultiCam, p, u)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || t > D.ctl.stop_at) return;
  const int cam = D.ser_mc[u];
  const int c0 = D.ser_off[cam], np = D.ser_off[cam + 1] - c0;
  double kr[12];
  if (threadIdx.x < 12) load12(D.K64 + (size_t)cam * kCamMat + threadIdx.x * 12, kr);
  const double* __restrict__ part = static_cast<const double*>(D.ser_part);
  double s[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) s[k] = 0.0;
  for (int q = lane_id(); q < np; q += kWave) {
    double v[12];
    load12(part + (size_t)(c0 + q) * kCam, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] += v[k];
  }
  __shared__ double tv[12];
  {
    const double r = reduce_scatter<16>(s);
    const int idx = rs_index<16>(lane_id());
    if (lane_id() < 16 && idx < 12) tv[idx] = r;
  }
  __syncthreads();
  refine_camera_solve(D, cam, tv, kr);
}

// Optional early stop of the second stage's series (series_rtol > 0), on
// the ambient terms x_t (whose norms equal the tangent ones).
__global__ void __launch_bounds__(kBlock) k_refine_series_check(Batch B, int t) {
  int p, w;
  if (!map_block(B, kUnitOne, p, w)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done || !(D.series_rtol > 0.0) || t > D.ctl.stop_at || t >= D.ctl.order) return;
  const double* __restrict__ x2 = D.x2;
  series_check(D, t, [&](int i, int k) { return x2[(size_t)i * kCam + k]; });
}

// Camera retraction of the second stage: p <- (p + acc) / |p + acc|.
__global__ void __launch_bounds__(kWave) k_refine_retract(Batch B) {
  int p, w;
  if (!map_wave<kWave>(B, kUnitCamWave, p, w)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done) return;
  const int i = w * kWave + lane_id();
  if (i >= D.n_p) return;
  const int pc = D.ctl.pcur;
  double q[12], nrm = 0.0;
  load12((pc ? D.P64[1] : D.P64[0]) + (size_t)i * kCam, q);
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    q[r] += D.acc[(size_t)i * kCam + r];
    nrm += q[r] * q[r];
  }
  const double inv = 1.0 / sqrt(nrm);
  double* o = (pc ? D.P64[0] : D.P64[1]) + (size_t)i * kCam;
#pragma unroll
  for (int r = 0; r < 12; r += 4) store4(o + r, q[r] * inv, q[r + 1] * inv, q[r + 2] * inv, q[r + 3] * inv);
}

// Cost (7) at the trial cameras and landmarks, one partial per packet.
__global__ void __launch_bounds__(kBlock) k_refine_cost(Batch B) {
  int p, q;
  if (!map_wave(B, kUnitPacket, p, q)) return;
  DevProblem& D = B.probs[p];
  if (D.ctl.done) return;
  const double* __restrict__ P = D.ctl.pcur ? D.P64[0] : D.P64[1];
  const double* __restrict__ Xr = D.ctl.lcur ? D.rec64[0] : D.rec64[1];
  const int lane = lane_id(), off = q * kWave;
  const int2 hdr = D.pk_hdr[q];
  const int n = hdr.x, lm0 = hdr.y;
  double f = 0.0;
  if (n > 0) {
    // a landmark with more than 64 observations runs over its continuation slots
    for (int e = off + lane; e < off + n; e += kWave) {
      const uint32_t code = D.pk_code[e];
      const int j = n <= kWave ? lm0 + (int)(code >> kCamBits) : lm0;
      double Pc[12], X[4];
      load12(P + (size_t)(code & kCamMask) * kCam, Pc);
      load4(Xr + (size_t)j * kX2, X[0], X[1], X[2], X[3]);
      const double2 m = D.pk_m64[e];
      const Proj2 g = project2(Pc, X);
      const double r0 = g.u0 - m.x, r1 = g.u1 - m.y;
      f += r0 * r0 + r1 * r1;
    }
  }
  f = wave_sum(f);
  if (lane == 0) D.cost_part[q] = f;
}

// ---------------------------------------------------------------- launchers
static inline dim3 blocks_for(int units, int units_per_block) {
  return dim3((unsigned)((units + units_per_block - 1) / units_per_block));
}

hipError_t launch_landmark_solve(const Batch& b, int mode, hipStream_t s) {
  if (b.total[kUnitPacket] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_landmark_solve, blocks_for(b.total[kUnitPacket], kWavesPerBlock), dim3(kBlock), 0, s, b,
                     mode);
  return hipGetLastError();
}

hipError_t launch_cost_finalize(const Batch& b, int mode, hipStream_t s) {
  if (b.total[kUnitOne] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cost_finalize, blocks_for(b.total[kUnitOne], 1), dim3(kBlock), 0, s, b, mode);
  return hipGetLastError();
}

hipError_t launch_linearize(const Batch& b, bool fp32, int force, hipStream_t s) {
  if (b.total[kUnitChunk] == 0) return hipSuccess;
  const dim3 g = blocks_for(b.total[kUnitChunk], 1);
  if (fp32) hipLaunchKernelGGL(k_linearize<float>, g, dim3(kBlock), 0, s, b, force);
  else hipLaunchKernelGGL(k_linearize<double>, g, dim3(kBlock), 0, s, b, force);
  return hipGetLastError();
}

hipError_t launch_camera_prep(const Batch& b, bool fp32, hipStream_t s) {
  if (b.total[kUnitCamWave] == 0) return hipSuccess;
  const dim3 g = blocks_for(b.total[kUnitCamWave], 1);
  if (b.wave_sums) hipLaunchKernelGGL(k_camera_sums, g, dim3(kBlock), 0, s, b);
  if (fp32) hipLaunchKernelGGL(k_camera_prep<float>, g, dim3(kWave), 0, s, b);
  else hipLaunchKernelGGL(k_camera_prep<double>, g, dim3(kWave), 0, s, b);
  return hipGetLastError();
}

// With ev0/ev1 set, the events are recorded by the dispatch itself
// (hipExtLaunchKernelGGL), so their interval is the kernel's execution.
hipError_t launch_series_landmark(const Batch& b, bool fp32, int t, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (b.total[kUnitPacket] == 0) return hipSuccess;
  const dim3 g = blocks_for(b.total[kUnitPacket], kWavesPerBlock);
  if (!fp32) hipExtLaunchKernelGGL(k_series_landmark_coop64, g, dim3(kBlock), 0, s, ev0, ev1, 0, b, t);
  else if (b.coop_cams)
    hipExtLaunchKernelGGL(k_series_landmark_coop, g, dim3(kBlock), kCoopLdsBytes, s, ev0, ev1, 0, b, t);
  else hipExtLaunchKernelGGL(k_series_landmark<float>, g, dim3(kBlock), 0, s, ev0, ev1, 0, b, t);
  return hipGetLastError();
}

// The timing events bracket the whole camera pass of one order: ev0 is
// recorded by the first of its kernels (chunk or slot pass), ev1 by the last
// (the combine kernel when some camera has several partial sums).
hipError_t launch_series_camera(const Batch& b, bool fp32, int t, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  hipError_t e = hipSuccess;
  const bool chunks = b.total[kUnitSerChunk] > 0, slots = b.total[kUnitCSlot] > 0;
  const bool comb = b.total[kUnitMultiCam] > 0;
  if (chunks) {
    const dim3 g = blocks_for(b.total[kUnitSerChunk], 1);
    hipEvent_t e1 = (slots || comb) ? nullptr : ev1;
    if (fp32) hipExtLaunchKernelGGL((k_series_camera<float, kCamWG>), g, dim3(kCamWG), 0, s, ev0, e1, 0, b, t);
    else hipExtLaunchKernelGGL((k_series_camera<double, kCamWG>), g, dim3(kCamWG), 0, s, ev0, e1, 0, b, t);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (slots) {
    const dim3 g = blocks_for(b.total[kUnitCSlot], kWavesPerBlock);
    hipEvent_t e0 = chunks ? nullptr : ev0, e1 = comb ? nullptr : ev1;
    if (fp32) hipExtLaunchKernelGGL(k_series_camera_slots<float>, g, dim3(kBlock), 0, s, e0, e1, 0, b, t);
    else hipExtLaunchKernelGGL(k_series_camera_slots<double>, g, dim3(kBlock), 0, s, e0, e1, 0, b, t);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (!comb) return e;
  const dim3 gm = blocks_for(b.total[kUnitMultiCam], 1);
  if (fp32) hipExtLaunchKernelGGL(k_series_camera_combine<float>, gm, dim3(kWave), 0, s, nullptr, ev1, 0, b, t);
  else hipExtLaunchKernelGGL(k_series_camera_combine<double>, gm, dim3(kWave), 0, s, nullptr, ev1, 0, b, t);
  return hipGetLastError();
}

hipError_t launch_cost_groups(const Batch& b, int trial, hipStream_t s) {
  if (b.total[kUnitCostGroup] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cost_groups, blocks_for(b.total[kUnitCostGroup], 1), dim3(kBlock), 0, s, b, trial);
  return hipGetLastError();
}

hipError_t launch_series_check(const Batch& b, bool fp32, int t, hipStream_t s) {
  if (b.total[kUnitOne] == 0) return hipSuccess;
  const dim3 g = blocks_for(b.total[kUnitOne], 1);
  if (fp32) hipLaunchKernelGGL(k_series_check<float>, g, dim3(kBlock), 0, s, b, t);
  else hipLaunchKernelGGL(k_series_check<double>, g, dim3(kBlock), 0, s, b, t);
  return hipGetLastError();
}

hipError_t launch_retract(const Batch& b, bool fp32, hipStream_t s) {
  if (b.total[kUnitCamWave] == 0) return hipSuccess;
  const dim3 g = blocks_for(b.total[kUnitCamWave], 1);
  if (fp32) hipLaunchKernelGGL(k_retract<float>, g, dim3(kWave), 0, s, b);
  else hipLaunchKernelGGL(k_retract<double>, g, dim3(kWave), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_refine_landmarks(const Batch& b, hipStream_t s) {
  if (b.total[kUnitPacket] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine_landmarks, blocks_for(b.total[kUnitPacket], kWavesPerBlock), dim3(kBlock), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_refine_cameras(const Batch& b, hipStream_t s) {
  if (b.total[kUnitChunk] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine_cameras, blocks_for(b.total[kUnitChunk], 1), dim3(kBlock), 0, s, b);
  return hipGetLastError();
}

// camera blocks through the trial cost (the landmark blocks and the camera
// chunk sums of the current point must be in place)
hipError_t launch_refine_step(const Batch& b, int order, bool check, hipStream_t s) {
  const dim3 gp = blocks_for(b.total[kUnitPacket], kWavesPerBlock);
  const dim3 gw = blocks_for(b.total[kUnitCamWave], 1);
  if (b.wave_sums) hipLaunchKernelGGL(k_camera_sums, gw, dim3(kBlock), 0, s, b);
  hipLaunchKernelGGL(k_refine_prep, gw, dim3(kWave), 0, s, b);
  for (int t = 1; t <= order; ++t) {
    hipLaunchKernelGGL(k_refine_series_landmark, gp, dim3(kBlock), 0, s, b, t);
    if (b.total[kUnitSerChunk] > 0)
      hipLaunchKernelGGL(k_refine_series_camera, blocks_for(b.total[kUnitSerChunk], 1), dim3(kCamWG), 0, s, b, t);
    if (b.total[kUnitCSlot] > 0)
      hipLaunchKernelGGL(k_refine_series_camera_slots, blocks_for(b.total[kUnitCSlot], kWavesPerBlock), dim3(kBlock),
                         0, s, b, t);
    if (b.total[kUnitMultiCam] > 0)
      hipLaunchKernelGGL(k_refine_series_combine, blocks_for(b.total[kUnitMultiCam], 1), dim3(kWave), 0, s, b, t);
    if (check && t < order)
      hipLaunchKernelGGL(k_refine_series_check, blocks_for(b.total[kUnitOne], 1), dim3(kBlock), 0, s, b, t);
  }
  hipLaunchKernelGGL(k_refine_landmark_update, gp, dim3(kBlock), 0, s, b);
  hipLaunchKernelGGL(k_refine_retract, gw, dim3(kWave), 0, s, b);
  hipLaunchKernelGGL(k_refine_cost, gp, dim3(kBlock), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_refine_iteration(const Batch& b, int order, bool check, hipStream_t s) {
  hipError_t e;
  if ((e = launch_refine_landmarks(b, s)) != hipSuccess) return e;
  if ((e = launch_refine_cameras(b, s)) != hipSuccess) return e;
  if ((e = launch_refine_step(b, order, check, s)) != hipSuccess) return e;
  if ((e = launch_cost_groups(b, 1, s)) != hipSuccess) return e;
  return launch_decide(b, s);
}

hipError_t launch_grad_norm(const Batch& b, hipStream_t s) {
  if (b.total[kUnitOne] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_norm, blocks_for(b.total[kUnitOne], 1), dim3(kBlock), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_decide(const Batch& b, hipStream_t s) {
  if (b.total[kUnitOne] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_decide, blocks_for(b.total[kUnitOne], 1), dim3(kBlock), 0, s, b);
  return hipGetLastError();
}

}  // namespace povar
