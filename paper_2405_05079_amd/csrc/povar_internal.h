// Internal data layout of the PoVar HIP library (device structs and launchers).
//
// One problem = one DevProblem record in device memory.  Every kernel is
// launched over a *batch* of problems: the grid is a flat list of work units
// (a wave or a workgroup each), and each unit finds its (problem, local unit)
// pair from a prefix table of units per problem.  A single solve is a batch
// of one; the server batches every admitted problem into the same launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace povar {

// Every pointer of a problem record and a batch addresses global device
// memory.  Device code sees them in the global address space, so loads and
// stores through them compile to global (not flat) memory instructions; the
// host sees plain pointers of the same size and value.
#if defined(__HIP_DEVICE_COMPILE__)
#define POVAR_GMEM __attribute__((address_space(1)))
#define POVAR_LDS __attribute__((address_space(3)))
#else
#define POVAR_GMEM
#define POVAR_LDS
#endif

constexpr int kWave = 64;                 // CDNA wavefront
constexpr int kBlock = 256;               // workgroup of the streaming passes
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPerLane = 8;               // camera-major observations per lane
constexpr int kChunk = kBlock * kPerLane; // camera-major observations per workgroup
constexpr int kLinVals = 64;              // per-camera linearisation accumulators
constexpr int kWaveSumChunks = 8;         // above this many chunks per camera, a wave adds a camera's partials
constexpr int kCamBits = 26;              // packet entry: camera index bits
constexpr uint32_t kCamMask = (1u << kCamBits) - 1u;

// Landmark slot strides (elements) in the per-landmark arrays.
constexpr int kRec = 8;                   // (z0, z1, z2, 0, X0, X1, X2, 1)
constexpr int kLmSym = 6;                 // V^+ : 6 values (00,01,02,11,12,22), 48 bytes
constexpr int kCam = 12;                  // one camera / camera vector
constexpr int kCamMat = 144;              // 12 x 12 camera operator
// Series camera record: P (12 values) then x (12 values).  Packed (stride 24)
// while the records of all cameras fit a 32 KB L1 in FP32; otherwise padded to
// stride 32, one 128-byte line per camera in FP32, so that a gather of a
// camera's P and x touches a single line.
constexpr int kSerX = 12;                 // offset of x in the series record
constexpr int kSerPacked = 24;
constexpr int kSerLine = 32;
__host__ __device__ constexpr int ser_stride(int n_p) {
  return (long long)n_p * kSerPacked * 4 <= 32768 ? kSerPacked : kSerLine;
}

// Per-problem control block (first member of the problem record).  Only
// kernels write it during a solve; the host reads it after synchronising and
// writes it only between launches.
struct Ctl {
  double lambda;        // damping for the next step
  double cost;          // f* at the current cameras
  double cost_trial;    // f* at the trial cameras of the last step
  double cost0;         // f* at the initial cameras
  int32_t lcur;         // landmark buffer holding the current linearisation point
  int32_t pcur;         // camera buffer holding the current cameras
  int32_t need_lin;     // 1: linearise before the next step (after an accept)
  int32_t done;         // 1: finished (ftol, or iteration limit)
  int32_t iter;         // LM iterations taken
  int32_t n_accept;
  int32_t iter_limit;   // done when iter reaches it
  int32_t order;        // series order m of the next steps
  int32_t stop_reason;  // 1: ftol
  int32_t status;       // bit 0: a damped camera block of this step could not be factored
  int32_t stop_at;      // last series term of the current step (order, or earlier on an early stop)
  int32_t stopped;      // 1: the series of the current step stopped early (retraction still to do)
  double grad_norm;     // |2 Pi b_p| at the current cameras (k_grad_norm; report only)
  // device clock (wall_clock64 ticks) of the power series: start of the
  // current step's first series pass (0: none yet), that step's duration, and
  // the sum over all steps
  uint64_t series_t0, series_last, series_ticks;
};

struct DevProblem {
  Ctl ctl;
  int32_t n_p, n_l, n_pk, n_ch;   // n_pk: packet slots
  int32_t manifold;     // 0 sphere, 1 euclidean
  int32_t trace_cap;
  int32_t s_stride;     // series record stride, ser_stride(n_p)
  int32_t wave_sums;    // 1: a camera spans more than kWaveSumChunks chunks; k_camera_sums adds the
                        // linearisation partials (one wave per camera), else k_camera_prep (one lane)
  double eta, ftol, lambda_min, lambda_max;
  double series_rtol;   // early stop of the series (0: off)

  // landmark-major packets on 64-entry slots: slot q holds whole landmarks
  // lm0, lm0+1, ... (internal ids) in entries 64q .. 64q + n - 1 (one lane
  // per entry), with pk_hdr[q] = (n, lm0).  A landmark with more than 64
  // observations fills consecutive slots; its first slot has n = its count
  // and the following ones n = 0.  Entry code = camera | (landmark - lm0) << 26.
  const int2 POVAR_GMEM* pk_hdr;
  const uint32_t POVAR_GMEM* pk_code;
  const float2 POVAR_GMEM* pk_m32;
  const double2 POVAR_GMEM* pk_m64;
  // camera-major observations (sorted by camera, then internal landmark)
  const int32_t POVAR_GMEM* cm_lm;     // internal landmark id
  const float2 POVAR_GMEM* cm_m32;
  const double2 POVAR_GMEM* cm_m64;
  const int4 POVAR_GMEM* ch_meta;      // chunk c: (camera, first obs, end obs, chunks of that camera);
                            // a chunk never spans two cameras
  const int32_t POVAR_GMEM* cam_ch;    // n_p + 1: chunks of camera i are cam_ch[i]..cam_ch[i+1]-1
  const int32_t POVAR_GMEM* mc_cam;    // n_mc cameras whose observations span more than one chunk
  int32_t n_mc, n_cg;       // multi-chunk cameras; cost groups (kCostGroup packets each; 0 up to kCostDirect packets)

  // cameras, double-buffered (current / trial): FP64 n_p x 12, and the
  // series record of each camera in the series precision, n_p x s_stride,
  // holding P and the current series term x
  double POVAR_GMEM* P64[2];
  float POVAR_GMEM* S32[2];    // FP32-bulk problems only
  double POVAR_GMEM* S64[2];   // FP64 problems only
  // landmarks of the current linearisation / trial point, internal order:
  // record (z0 = V^+ b_l, X) per landmark, and V^+
  double POVAR_GMEM* rec64[2];         // n_l x 8
  // (X, 1) of the same records, compact (n_l x 4): what the landmark series
  // pass reads, half the bytes of the full records
  double POVAR_GMEM* xs64[2];
  float POVAR_GMEM* xs32[2];
  double POVAR_GMEM* Vp64[2];          // n_l x 8

  // linearisation per camera
  double POVAR_GMEM* lin_part;         // n_ch x 64 chunk partials: 40 U values, b_p, sum W z0
  // damped, projected, inverted camera blocks K_i = Pi (Pi U_l Pi + tau p p^T)^-1 Pi
  double POVAR_GMEM* K64;              // n_p x 144
  double POVAR_GMEM* g64;              // n_p x 12  b_p - sum W V^+ b_l  (kept for inspection)
  double POVAR_GMEM* U40;              // n_p x 40  combined U values (kept for inspection)
  // power-series work vectors
  double POVAR_GMEM* acc;              // n_p x 12, partial sum x(m) (FP64)
  void POVAR_GMEM* zx;                 // n_l x 8, (z, X) records of the current order
  void POVAR_GMEM* t_part;             // n_ch x 12 chunk partials
  // Series camera pass of blocked problems (landmark records of the series
  // precision larger than one XCD's L2): landmarks fall in blocks of lm_block
  // consecutive internal ids, and each block's observations, by camera then
  // landmark, fill 64-lane slots with kCsPerLane observations per lane.  A run
  // is the part of one camera's observations of one block that lies in one
  // slot; each run gives one partial sum.  Workgroup g (4 slots) runs on XCD
  // g % 8, and the slots are ordered so that all slots of a block go to the
  // XCD that block is assigned to, in block order.
  int32_t blocked, n_cs, n_runs, n_smc;
  int32_t pad2[2];
  const int32_t POVAR_GMEM* cs_hdr;    // n_cs: lanes used (0: empty slot)
  const int2 POVAR_GMEM* cs_lane;      // n_cs x 64: (camera | run key << 26, run id)
  const int32_t POVAR_GMEM* cs_lm;     // entry (q, r, lane) at (q * kCsPerLane + r) * 64 + lane:
                                       // internal landmark, -1 for padding
  const float2 POVAR_GMEM* cs_m32;
  const double2 POVAR_GMEM* cs_m64;
  // partial camera sums of the series camera pass (per chunk, or per run of a
  // blocked problem) and the cameras whose partials are combined
  const int32_t POVAR_GMEM* ser_off;   // n_p + 1: partials of camera i are ser_off[i] .. ser_off[i+1]-1
  const int32_t POVAR_GMEM* ser_mc;    // n_smc cameras
  void POVAR_GMEM* ser_part;           // 12 values per partial, series precision
  double POVAR_GMEM* cost_part;        // n_pk landmark-solve cost partials (one per packet)
  double POVAR_GMEM* cost_group;       // n_cg sums of kCostGroup consecutive packet partials
  double POVAR_GMEM* bl_part;          // n_pk partials of |b_l|^2 (landmark solve), and
  double POVAR_GMEM* bl_group;         // their n_cg group sums
  double POVAR_GMEM* tr_cost;          // trace_cap entries
  double POVAR_GMEM* tr_lambda;
  int32_t POVAR_GMEM* tr_acc;
  double POVAR_GMEM* tr_bl;            // |b_l| at the trial point
  double POVAR_GMEM* tr_series;        // series device clock ticks of the iteration

  // Second stage (projective refinement, Eq. (7), RiPoBA of Sec. 4.3), FP64:
  // landmarks are unit 4-vectors in rec64[b] (first 4 of each record).
  int32_t stage;                       // 1: PoVar on Eq. (6); 2: RiPoBA on Eq. (7)
  int32_t pad3;
  double POVAR_GMEM* g2;               // n_l x kG2: G_j (sym4 order)
  double POVAR_GMEM* bl2;              // n_l x 4: b_l
  double POVAR_GMEM* lin2;             // n_ch x kLin2 chunk partials: 40 sums of g (x) X X^T, b_p, sum W z0
  double POVAR_GMEM* x2;               // n_p x 12 series term (the landmark term goes to zx as (z, X))
};
constexpr int kG2 = 10;
constexpr int kX2 = 4;   // second stage: X_j (unit 4-vector) at stride 4 in rec64
constexpr int kLin2 = 64;

// Unit kinds of a launch.
enum UnitKind {
  kUnitPacket = 0,     // one wave per landmark packet
  kUnitChunk = 1,      // one workgroup per camera chunk (linearisation)
  kUnitCamWave = 2,    // one wave per 64 cameras
  kUnitOne = 3,        // one workgroup per problem
  kUnitMultiCam = 4,   // one wave per camera whose series partials are combined
  kUnitCostGroup = 5,  // one workgroup per kCostGroup packets
  kUnitSerChunk = 6,   // one workgroup per camera chunk, series pass (problems not blocked)
  kUnitCSlot = 7,      // one wave per camera slot, series pass (blocked problems)
  kNumUnitKinds = 8
};
constexpr int kGraphIters = 4;       // iterations per replay of the longer graph
constexpr int kCostGroup = 2048;
constexpr int kCostDirect = 8192;    // up to this many packets, k_decide adds the packet partials itself

// Blocked series camera pass.
// Observations per lane of a camera slot, by series precision: FP32 slots
// hold eight (more loads in flight per lane, and fewer runs split at slot
// ends), FP64 slots four (the same registers).
__host__ __device__ constexpr int cs_per_lane(bool fp32) { return fp32 ? 8 : 4; }
__host__ __device__ constexpr int cs_obs(bool fp32) { return kWave * cs_per_lane(fp32); }
constexpr long long kLmBlockBytes = 2ll << 20;   // landmark records per block (half of one XCD's L2)
constexpr long long kL2Bytes = 4ll << 20;        // L2 of one XCD
constexpr int kXcds = 8;
// landmark records of the series precision do not fit one XCD's L2
__host__ __device__ constexpr bool blocked_layout(long long n_l, bool fp32) {
  return n_l * kRec * (fp32 ? 4 : 8) > kL2Bytes;
}

// A batch of problems: device array of records and, per unit kind, the
// prefix table of units per problem (n_prob + 1 entries each).
struct Batch {
  DevProblem POVAR_GMEM* probs;
  // prefix table of unit kind k: tables + k * tab_stride (n_prob + 1 entries)
  const int32_t POVAR_GMEM* tables;
  int32_t n_prob, tab_stride;
  int32_t total[kNumUnitKinds];
  // 1: the landmark pass gathers camera series records cooperatively: every
  // FP64 batch; an FP32 batch holding problems whose records are kSerLine
  // values (128 bytes) apart (kCoopLdsBytes of LDS per workgroup)
  int32_t coop_cams;
  // 1: some problem of the batch has wave_sums set (k_camera_sums is launched)
  int32_t wave_sums;
};
constexpr int kCoopPieces = 6;   // 16-byte pieces of P and x (FP32), or of each of them (FP64)
constexpr int kCoopHalves = 2;   // FP32 exchange rounds (half the wave each): 3 KB of LDS per wave
constexpr int kCoopLdsBytes = kBlock / kWave * kCoopPieces * kWave * 16 / kCoopHalves;

// Launchers (defined with the kernels).  `fp32` selects the series /
// Jacobian precision; the critical kernels are FP64 in both modes.
hipError_t launch_landmark_solve(const Batch& b, int mode, hipStream_t s);   // mode 0 init, 1 trial, 2 reset
hipError_t launch_cost_finalize(const Batch& b, int mode, hipStream_t s);    // mode 0 init, 1 trial, 2 reset
hipError_t launch_linearize(const Batch& b, bool fp32, int force, hipStream_t s);
hipError_t launch_camera_prep(const Batch& b, bool fp32, hipStream_t s);
hipError_t launch_series_landmark(const Batch& b, bool fp32, int t, hipStream_t s, hipEvent_t ev0 = nullptr,
                                  hipEvent_t ev1 = nullptr);
hipError_t launch_series_camera(const Batch& b, bool fp32, int t, hipStream_t s, hipEvent_t ev0 = nullptr,
                                hipEvent_t ev1 = nullptr);   // chunk or slot pass, + combine (not timed)
hipError_t launch_cost_groups(const Batch& b, int trial, hipStream_t s);
hipError_t launch_series_check(const Batch& b, bool fp32, int t, hipStream_t s);
// second stage (RiPoBA): one LM iteration, and the landmark linearisation with
// the cost at the current point (initial state)
hipError_t launch_refine_iteration(const Batch& b, int order, bool check, hipStream_t s);
hipError_t launch_refine_landmarks(const Batch& b, hipStream_t s);
hipError_t launch_refine_cameras(const Batch& b, hipStream_t s);
hipError_t launch_refine_step(const Batch& b, int order, bool check, hipStream_t s);
hipError_t launch_retract(const Batch& b, bool fp32, hipStream_t s);
hipError_t launch_decide(const Batch& b, hipStream_t s);
// |2 Pi_i b_p,i| over all cameras from the linearisation partials (which must
// be those of the current cameras) into Ctl::grad_norm
hipError_t launch_grad_norm(const Batch& b, hipStream_t s);

}  // namespace povar
