// Host-side objects of the PoVar library (context, problem, layout).
#pragma once

#include <cstddef>
#include <cstdint>
#include <exception>
#include <mutex>
#include <string>
#include <vector>

#include "povar.h"
#include "povar_internal.h"

struct povar_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::mutex err_mu;
  std::string err, err_copy;
  int live_problems = 0;   // problems created on this context and not destroyed
  double clock_hz = 0.0;   // rate of the device clock kernels read (wall_clock64)
};

namespace povar {

// Host image of the observation layout (see DevProblem for the meaning).
struct HostLayout {
  int32_t n_p = 0, n_l = 0;
  int64_t n_obs = 0;
  int32_t n_pk = 0, n_ch = 0;
  std::vector<int32_t> int2ext;        // internal landmark -> caller's index
  std::vector<int32_t> cam_int2ext;    // internal camera -> caller's index
  std::vector<int32_t> pk_hdr;         // 2 per slot: (n, lm0)
  std::vector<uint32_t> pk_code;
  std::vector<float> pk_m32;
  std::vector<double> pk_m64;
  std::vector<int32_t> cm_lm;
  std::vector<float> cm_m32;
  std::vector<double> cm_m64;
  std::vector<int32_t> ch_meta, cam_ch;   // ch_meta: 4 per chunk
  std::vector<int32_t> mc_cam;         // cameras spanning more than one chunk
  int32_t n_mc = 0, n_cg = 0;
  // blocked series camera pass (DevProblem::blocked)
  int32_t blocked = 0, lm_block = 0, n_cs = 0, n_runs = 0;
  std::vector<int32_t> cs_hdr, cs_lane, cs_lm;   // cs_lane: 2 per lane
  std::vector<float> cs_m32;
  std::vector<double> cs_m64;
  std::vector<int32_t> run_off;        // n_p + 1, runs of each camera
  std::vector<int32_t> smc;            // cameras whose series partials are combined
};

// Array sizes that fix a problem's device arena.
struct LayoutSizes {
  int64_t n_p, n_l, n_obs, n_pk, n_ch, n_mc, n_cs, n_runs;
  bool blocked;
};
inline LayoutSizes sizes_of(const HostLayout& L) {
  return LayoutSizes{L.n_p, L.n_l, L.n_obs, L.n_pk, L.n_ch, L.n_mc, L.n_cs, L.n_runs, L.blocked != 0};
}

// Byte offsets of every buffer inside a problem's device arena
// (SIZE_MAX = not allocated for this precision).
struct ArenaOffsets {
  size_t pk_hdr, pk_code, pk_m32, pk_m64, cm_lm, cm_m32, cm_m64, ch_meta, cam_ch, mc_cam;
  size_t cs_hdr, cs_lane, cs_lm, cs_m32, cs_m64, run_off, smc, t_run;
  size_t P64[2], S32[2], S64[2], rec64[2], xs64[2], xs32[2], Vp64[2];
  size_t lin_part, K64, g64, U40, acc, zx, t_part, cost_part, cost_group, bl_part, bl_group;
  size_t tr_cost, tr_lambda, tr_acc, tr_bl, tr_series, rec, tables;
  size_t init_end;   // buffers with initial values lie below this offset
};

size_t arena_bytes(const LayoutSizes& z, bool fp32, int64_t trace_cap, ArenaOffsets* o);
povar_status build_layout(povar_ctx ctx, int32_t n_p, int32_t n_l, int64_t n_obs, const int32_t* cam,
                          const int32_t* pt, const double* meas, bool fp32, HostLayout& L);
povar_status check_options(povar_ctx ctx, const povar_options* o);
void set_error(povar_ctx ctx, const char* fmt, ...);

// Turns a host exception (host memory or threads exhausted) into an error
// status.  The C entry points that allocate host memory end with it as the
// handler of a function-try-block, so that no exception leaves the C ABI.
#define POVAR_HOST_CATCH(ctxexpr)                                                \
  catch (const std::exception& povar_ex_) {                                     \
    povar::set_error((ctxexpr), "host resources exhausted: %s", povar_ex_.what()); \
    return POVAR_ENOMEM;                                                        \
  }                                                                             \
  catch (...) {                                                                 \
    povar::set_error((ctxexpr), "unexpected host exception");                   \
    return POVAR_EDEVICE;                                                       \
  }

struct TimedPair {
  hipEvent_t start, stop;
  int kind;   // 0 landmark pass, 1 camera pass
};

}  // namespace povar

struct povar_problem_s {
  povar_ctx ctx = nullptr;
  bool owned_by_ctx = false;   // counted in ctx->live_problems
  povar_options opt{};
  bool fp32 = false;
  hipStream_t stream = nullptr;
  int trace_cap = 0;
  povar::HostLayout L;
  povar::ArenaOffsets off{};
  size_t bytes = 0;
  void* arena = nullptr;
  void* arena2 = nullptr;      // second-stage buffers (RiPoBA problems only)
  povar::DevProblem rec{};    // host copy of the device record
  povar::Batch batch{};       // batch of one
  hipGraphExec_t graph_exec = nullptr;     // one iteration
  hipGraphExec_t graph_exec_k = nullptr;   // kGraphIters iterations
  bool graph_failed = false;
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> events;
  size_t event_next = 0;
  std::vector<povar::TimedPair> pending;
  double ms_kernel[2] = {0.0, 0.0};
  int64_t n_kernel[2] = {0, 0};

  hipEvent_t event_pool_get();
  hipError_t drain_timing();
};

namespace povar {
// Allocates and fills the device state of a problem and solves its initial
// landmarks.  rec_dev: where the problem record lives (NULL: in its arena).
povar_status problem_init(povar_ctx ctx, HostLayout&& L, const double* cams0, const povar_options* o,
                          hipStream_t stream, povar_problem_s* pb, DevProblem* rec_dev, int32_t iter_limit, const double* pts0 = nullptr);
size_t layout_footprint(const HostLayout& L, bool fp32);
void unit_counts(const HostLayout& L, int32_t* units);
// width values per camera, internal order -> caller's order
void cams_to_caller(const HostLayout& L, const double* in, double* out, int width);   // kNumUnitKinds units per kind
povar_status copy_points(povar_problem_s* pb, int lcur, double* out);
hipError_t read_ctl(povar_problem_s* pb, Ctl* out);
hipError_t write_ctl(povar_problem_s* pb, const Ctl* in);
hipError_t enqueue_iteration(povar_problem_s* pb, bool timed);
hipError_t enqueue_iterations(povar_problem_s* pb, int n);
// grad_norm: the report's grad_norm_final (NaN when not computed)
void fill_report(const povar_problem_s* pb, const Ctl& c, double seconds, double grad_norm, povar_report* r);
// Device address of the no-allocation metric upgrade's scratch array on
// ctx's device, looked up once per device (povar_ctx_create calls it with
// that device current).
povar_status metric_scratch_init(povar_ctx ctx);
// Seeded initial cameras (the init_seed field of povar_options): n x 12,
// caller's order, unit norm.
void seeded_cameras(uint64_t seed, int32_t n, double* out);
}  // namespace povar
