// Internal data layout of the PoVar HIP library (device structs and launchers).
//
// One problem = one DevProblem record in device memory.  Every kernel is
// launched over a *batch* of problems: the grid is a flat list of waves,
// and each wave finds its (problem, unit) pair from a prefix table of units
// per problem.  A single solve is a batch of one; the server batches every
// admitted problem into the same launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace povar {

constexpr int kWave = 64;                 // CDNA wavefront
constexpr int kBlock = 256;               // 4 independent waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kChunk = 256;               // camera-major observations per wave (4 per lane)
constexpr int kLinVals = 64;              // per-camera linearisation accumulators

// Landmark slot strides (elements) in the per-landmark arrays.
constexpr int kLmVec = 4;                 // X (x,y,z,1), z0, z: 4 values
constexpr int kLmSym = 8;                 // V^+ : 6 values (00,01,02,11,12,22) + 2 pad
constexpr int kCam = 12;                  // one camera / camera vector
constexpr int kCamMat = 144;              // 12 x 12 camera operator

// Per-problem control block.  Only device kernels write it during a solve;
// the host reads it after synchronising and writes it only between launches.
struct Ctl {
  double lambda;        // damping for the next step
  double cost;          // f* at the current cameras
  double cost_trial;    // f* at the trial cameras of the last step
  double cost0;         // f* at the initial cameras
  int32_t lcur;         // landmark buffer holding the current linearisation point
  int32_t pcur;         // camera buffer holding the current cameras
  int32_t need_lin;     // 1: linearise before the next step (after an accept)
  int32_t done;         // 1: finished (ftol, or iteration limit of a served problem)
  int32_t iter;         // LM iterations taken
  int32_t n_accept;
  int32_t iter_limit;   // done when iter reaches it
  int32_t order;        // series order m of the next steps
  int32_t stop_reason;  // 1: ftol
  int32_t status;       // bit 0: a damped camera block was not positive definite
  int32_t pad0, pad1;
};

struct DevProblem {
  int32_t n_p, n_l, n_sl, n_ch;
  int32_t manifold;     // 0 sphere, 1 euclidean
  int32_t trace_cap;
  int32_t pad0, pad1;
  double eta, ftol, lambda_min, lambda_max;

  // landmark-major slices: slice s holds landmarks 64s..64s+63 (internal
  // order = decreasing track length); entry (t, lane) at sl_off[s]+64t+lane
  const int32_t* sl_off;
  const int32_t* sl_len;
  const int32_t* e_cam;     // camera of each entry, -1 = padding
  const float2* e_m32;
  const double2* e_m64;
  // camera-major observations (sorted by camera, then internal landmark)
  const int32_t* cm_lm;     // internal landmark id
  const float2* cm_m32;
  const double2* cm_m64;
  const int32_t* ch_beg;    // n_ch + 1: chunk c covers [ch_beg[c], ch_beg[c+1])
  const int32_t* ch_cam;    // camera of chunk c (a chunk never spans two cameras)
  const int32_t* cam_ch;    // n_p + 1: chunks of camera i are cam_ch[i]..cam_ch[i+1]-1

  // cameras, double-buffered (current / trial), n_p x 12
  double* P64[2];
  float* P32[2];
  // landmarks of the current linearisation / trial point, internal order
  double* X64[2];           // n_l x 4 (X, 1)
  double* Vp64[2];          // n_l x 8 (V^+ packed)
  double* z064[2];          // n_l x 4 (V^+ b_l)
  float* X32[2];
  float* Vp32[2];
  float* z032[2];

  // linearisation per camera
  double* U40;              // n_p x 40: sum x~x~^T, sum m1 x~x~^T, sum m2 x~x~^T, sum |m|^2 x~x~^T
  double* bp;               // n_p x 12
  double* wz;               // n_p x 12: sum_k W_k V^+ b_l
  double* lin_part;         // n_ch x 64 chunk partials
  // damped, projected, inverted camera blocks K_i = Pi (Pi U_l Pi + tau p p^T)^-1 Pi
  double* K64;              // n_p x 144
  float* K32;
  // power-series work vectors (series precision)
  void* x;                  // n_p x 12, current term
  void* acc;                // n_p x 12, partial sum x(m)
  void* z;                  // n_l x 4
  void* t_part;             // n_ch x 12 chunk partials
  uint32_t* cam_cnt;        // n_p arrival counters (reset by the last wave)
  double* cost_part;        // n_sl
  uint32_t* cost_cnt;       // 1
  Ctl* ctl;
  double* tr_cost;          // trace_cap entries
  double* tr_lambda;
  int32_t* tr_acc;
};

// Unit kinds of a launch.
enum UnitKind { kUnitSlice = 0, kUnitChunk = 1, kUnitCamWave = 2, kUnitOne = 3, kNumUnitKinds = 4 };

// A batch of problems: device array of records and, per unit kind, the
// prefix table of waves per problem (n_prob + 1 entries each).
struct Batch {
  const DevProblem* probs;
  const int32_t* off[kNumUnitKinds];
  int32_t n_prob;
  int32_t total[kNumUnitKinds];
};

// Launchers (defined with the kernels).  `fp32` selects the series /
// Jacobian precision; the critical kernels are FP64 in both modes.
hipError_t launch_landmark_solve(const Batch& b, int mode, hipStream_t s);   // mode 0 init, 1 trial, 2 reset
hipError_t launch_linearize(const Batch& b, bool fp32, int force, hipStream_t s);
hipError_t launch_camera_prep(const Batch& b, bool fp32, hipStream_t s);
hipError_t launch_series_landmark(const Batch& b, bool fp32, int t, hipStream_t s);
hipError_t launch_series_camera(const Batch& b, bool fp32, int t, hipStream_t s);
hipError_t launch_retract(const Batch& b, bool fp32, hipStream_t s);
hipError_t launch_decide(const Batch& b, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);

}  // namespace povar
