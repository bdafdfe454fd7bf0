// Continuous-batching server: many bundle-adjustment problems resident on one
// GPU, advanced together.
//
// submit() validates a request and builds its observation layout on the
// caller's thread, so its exact device footprint is known before admission.
// One worker thread runs the batched iterations.  It admits queued requests
// in FIFO order whenever a slot is free and the summed footprint of resident
// problems stays within the budget; an admission thread initialises them
// (device allocation, upload, initial landmark solve) on a stream of its own
// into staging records, so the worker keeps relaunching groups meanwhile, and
// an initialised problem's record is copied into its group while the group
// is idle, before its next launch.  Resident problems form groups by precision and by size
// (up to kLargeObs observations, or more).  A group advances with one batched
// launch sequence per LM iteration (each kernel's grid covers the work units
// of all its problems) on a stream of its own, so the small problems iterate
// at their own pace beside the large ones instead of waiting for every large
// problem's kernels.  After a few iterations the group's control blocks are
// copied back (an event marks their arrival), and finished problems are
// retired: their results are copied to the host at once, their device memory
// is freed later, when no group has work in flight (freeing memory
// synchronises the whole device).  New requests thus join their group while
// others are mid-solve.  Every reduction stays inside one
// problem's own units in a fixed order, so a problem's result does not depend
// on which others shared the launches.
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <system_error>
#include <thread>
#include <utility>
#include <vector>

#include "povar.h"
#include "povar_host.h"

namespace povar {

struct Request {
  uint64_t ticket = 0;
  HostLayout layout;
  std::vector<double> cams0;
  povar_options opt{};
  bool fp32 = false;
  bool budget_waited = false;   // counted once among the requests that waited for budget
  size_t footprint = 0;
  int64_t n_obs = 0;
  int32_t n_p = 0, n_l = 0;
  double t_submit = 0.0, t_admit = -1.0, t_finish = -1.0;
  bool finished = false;
  povar_status status = POVAR_OK;
  std::string error;
  povar_report report{};
  std::vector<double> cams, pts;
};

struct Resident {
  std::shared_ptr<Request> req;
  povar_problem_s* pb = nullptr;
  int32_t left = 1;   // iterations before the problem reaches its limit (as of the last read-back)
};

// An initialised problem waiting to join its group.
struct Ready {
  std::shared_ptr<Request> req;
  povar_problem_s* pb = nullptr;
  int stage = 0;   // its staging record
};

constexpr int kServerItersPerSync = 4;   // batched iterations between control-block read-backs, at most
// Problems of more than this many observations form the large class of their
// precision: each precision's small problems iterate beside its large ones on
// a stream of their own.  (Serving 20-400-camera requests, this bound cut the
// median latency by a quarter against one group per precision.)
constexpr int64_t kLargeObs = 250000;
constexpr int kNumGroups = 4;   // {FP32-bulk, FP64} x {small, large}

inline int group_index(bool fp32, int64_t n_obs) { return (fp32 ? 0 : 2) + (n_obs > kLargeObs ? 1 : 0); }

// The problems of one group share one batch: their records sit contiguously
// in `recs`, in the order of `res`.
struct Group {
  bool fp32 = false;
  hipStream_t stream = nullptr;        // the group's iterations, read-backs and retirements
  hipEvent_t ready = nullptr;          // recorded after the control-block read-back
  DevProblem* recs = nullptr;          // device, max_slots records
  int32_t* tables = nullptr;           // device, kNumUnitKinds x (max_slots + 1)
  DevProblem* host_recs = nullptr;     // pinned read-back buffer, max_slots records
  std::vector<Resident> res;
  int n_flight = 0;                    // residents covered by the batch in flight (0: nothing in flight)
  int it_flight = 0;                   // its iterations
  Batch batch{};
  int max_order = 0, min_order = 0;
  bool any_rtol = false;               // a problem of the group may stop its series early
  bool dirty = true;
};

}  // namespace povar

using namespace povar;

struct povar_server_s {
  povar_ctx ctx = nullptr;
  hipStream_t admit_stream = nullptr;   // the admission thread's initialisations
  uint64_t budget = 0;
  int32_t max_slots = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> tickets;   // submitted and not yet collected
  uint64_t next_ticket = 1;
  bool stop = false;
  uint64_t used = 0;                    // footprints of resident and retired-but-not-freed problems
  int32_t n_resident = 0;
  int64_t n_finished = 0, batch_iters = 0;
  int64_t syncs = 0, budget_waits = 0;
  // time (seconds) of the admission thread initialising requests, and of the
  // worker enqueueing launches, waiting for the GPU while no read-back has
  // arrived, retiring finished problems and freeing their memory
  double t_admit = 0.0, t_launch = 0.0, t_wait = 0.0, t_retire = 0.0;
  // admission: requests admitted and waiting for initialisation, problems
  // initialised and waiting to join their group, admitted problems not yet in
  // their group (per group), and the staging records not in use
  std::condition_variable admit_cv;
  std::deque<std::shared_ptr<Request>> to_init;
  std::vector<Ready> ready;
  int pending[kNumGroups] = {};
  std::vector<int> free_stage;
  DevProblem* stage_recs = nullptr;     // device, max_slots records
  Group groups[kNumGroups];
  // worker only: finished problems whose device memory is not yet freed
  std::vector<std::pair<povar_problem_s*, size_t>> retired;
  uint64_t retired_bytes = 0;
  std::thread worker, admitter;
  std::chrono::steady_clock::time_point t0;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

void fail_request(povar_server_s* sv, const std::shared_ptr<Request>& r, povar_status st, const std::string& msg) {
  std::lock_guard<std::mutex> g(sv->mu);
  r->status = st;
  r->error = msg;
  r->finished = true;
  r->t_finish = sv->now();
  sv->n_finished += 1;
}

hipError_t upload_tables(povar_server_s* sv, Group& G) {
  const int n = (int)G.res.size();
  const int stride = sv->max_slots + 1;
  std::vector<int32_t> tab((size_t)kNumUnitKinds * stride, 0);
  G.max_order = 0;
  G.min_order = INT_MAX;
  G.any_rtol = false;
  for (int p = 0; p < n; ++p) {
    const HostLayout& L = G.res[p].pb->L;
    int32_t units[kNumUnitKinds];
    unit_counts(L, units);
    for (int k = 0; k < kNumUnitKinds; ++k) tab[(size_t)k * stride + p + 1] = tab[(size_t)k * stride + p] + units[k];
    G.max_order = std::max(G.max_order, G.res[p].pb->opt.series_order);
    G.min_order = std::min(G.min_order, G.res[p].pb->opt.series_order);
    if (G.res[p].pb->opt.series_rtol > 0.0) G.any_rtol = true;
  }
  hipError_t e = hipMemcpyAsync(G.tables, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, G.stream);
  if (e != hipSuccess) return e;
  G.batch.probs = G.recs;
  G.batch.n_prob = n;
  G.batch.coop_cams = G.fp32 ? 0 : 1;   // FP64: always cooperative
  G.batch.wave_sums = 0;
  for (int p = 0; p < n; ++p) {
    if (G.res[p].pb->rec.s_stride == kSerLine) G.batch.coop_cams = 1;
    if (G.res[p].pb->rec.wave_sums) G.batch.wave_sums = 1;
  }
  G.batch.tables = G.tables;
  G.batch.tab_stride = stride;
  for (int k = 0; k < kNumUnitKinds; ++k) G.batch.total[k] = tab[(size_t)k * stride + n];
  G.dirty = false;
  // the host table must outlive the asynchronous copy
  return hipStreamSynchronize(G.stream);
}

hipError_t launch_iteration(Group& G) {
  hipError_t e;
  const Batch& B = G.batch;
  hipStream_t s = G.stream;
  if ((e = launch_linearize(B, G.fp32, 0, s)) != hipSuccess) return e;
  if ((e = launch_camera_prep(B, G.fp32, s)) != hipSuccess) return e;
  for (int t = 1; t <= G.max_order; ++t) {
    if ((e = launch_series_landmark(B, G.fp32, t, s)) != hipSuccess) return e;
    if ((e = launch_series_camera(B, G.fp32, t, s)) != hipSuccess) return e;
    if (G.any_rtol && t < G.max_order && (e = launch_series_check(B, G.fp32, t, s)) != hipSuccess) return e;
  }
  if ((G.min_order == 0 || G.any_rtol) && (e = launch_retract(B, G.fp32, s)) != hipSuccess) return e;
  if ((e = launch_landmark_solve(B, 1, s)) != hipSuccess) return e;
  if ((e = launch_cost_groups(B, 1, s)) != hipSuccess) return e;
  return launch_decide(B, s);
}

// Every resident of the group fails with the device error.
void fail_group(povar_server_s* sv, Group& G, hipError_t e) {
  for (auto& R : G.res) {
    povar_problem_destroy(R.pb);
    {
      std::lock_guard<std::mutex> g(sv->mu);
      sv->used -= R.req->footprint;
      sv->n_resident -= 1;
    }
    fail_request(sv, R.req, POVAR_EDEVICE, hipGetErrorString(e));
  }
  G.res.clear();
  G.dirty = true;
  G.n_flight = 0;
}

std::string error_text(povar_ctx ctx) {
  std::lock_guard<std::mutex> g(ctx->err_mu);
  return ctx->err;
}

// Initialises admitted requests, in admission order, into staging records.
// Every admitted request holds a slot until it finishes, and a staging record
// only until it joins its group, so a staging record is free for each.
void admitter_loop(povar_server_s* sv) {
  (void)hipSetDevice(sv->ctx->device);
  for (;;) {
    std::shared_ptr<Request> r;
    int k = -1;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->admit_cv.wait(lk, [&] { return sv->stop || !sv->to_init.empty(); });
      if (sv->stop) return;
      r = sv->to_init.front();
      sv->to_init.pop_front();
      if (!sv->free_stage.empty()) {
        k = sv->free_stage.back();
        sv->free_stage.pop_back();
      }
    }
    const double t0 = sv->now();
    const int g = group_index(r->fp32, r->n_obs);
    auto* pb = new povar_problem_s();
    povar_status st = POVAR_ESTATE;
    std::string msg = "no staging record free";
    if (k >= 0) {
      try {
        st = problem_init(sv->ctx, std::move(r->layout), r->cams0.data(), &r->opt, sv->admit_stream, pb,
                          sv->stage_recs + k, r->opt.max_iters);
        if (st != POVAR_OK) msg = error_text(sv->ctx);
      } catch (const std::exception& ex) {
        st = POVAR_ENOMEM;
        msg = std::string("host resources exhausted: ") + ex.what();
      }
    }
    r->cams0.clear();
    r->cams0.shrink_to_fit();
    if (st != POVAR_OK) {
      povar_problem_destroy(pb);
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->used -= r->footprint;
        sv->n_resident -= 1;
        sv->pending[g] -= 1;
        if (k >= 0) sv->free_stage.push_back(k);
        sv->t_admit += sv->now() - t0;
      }
      fail_request(sv, r, st, msg);
      continue;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    r->t_admit = sv->now();
    sv->ready.push_back({r, pb, k});
    sv->t_admit += r->t_admit - t0;
  }
}

// Initialised problems whose group is idle join it: the staging record is
// copied behind the group's records, and released once the copy is done.
// Returns whether any joined.
bool join_ready(povar_server_s* sv) {
  std::vector<Ready> joining;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    std::vector<Ready> keep;
    for (auto& x : sv->ready) {
      if (sv->groups[group_index(x.req->fp32, x.req->n_obs)].n_flight == 0) joining.push_back(x);
      else keep.push_back(x);
    }
    sv->ready.swap(keep);
  }
  if (joining.empty()) return false;
  bool copied[kNumGroups] = {};
  for (auto& x : joining) {
    const int g = group_index(x.req->fp32, x.req->n_obs);
    Group& G = sv->groups[g];
    const int pos = (int)G.res.size();
    const hipError_t e = hipMemcpyAsync(G.recs + pos, sv->stage_recs + x.stage, sizeof(DevProblem),
                                        hipMemcpyDeviceToDevice, G.stream);
    x.pb->batch.probs = G.recs + pos;
    x.pb->stream = G.stream;
    G.res.push_back({x.req, x.pb, x.req->opt.max_iters});
    G.dirty = true;
    copied[g] = true;
    if (e != hipSuccess) fail_group(sv, G, e);
  }
  for (int g = 0; g < kNumGroups; ++g)
    if (copied[g]) (void)hipStreamSynchronize(sv->groups[g].stream);
  std::lock_guard<std::mutex> lk(sv->mu);
  for (auto& x : joining) {
    sv->free_stage.push_back(x.stage);
    sv->pending[group_index(x.req->fp32, x.req->n_obs)] -= 1;
  }
  return true;
}

// Copies the result of resident problem `idx` out, moves the last record into
// its place, and keeps the problem for freeing (its footprint stays counted
// until then).  The group has nothing in flight.
hipError_t retire(povar_server_s* sv, Group& G, int idx, const Ctl& c) {
  Resident R = G.res[idx];
  auto& r = R.req;
  povar_problem_s* pb = R.pb;
  std::vector<double> cams, pts, cin;
  hipError_t e = hipSuccess;
  povar_status st = POVAR_OK;
  try {
    cams.resize((size_t)r->n_p * kCam);
    pts.resize((size_t)r->n_l * 3);
    cin.resize((size_t)r->n_p * kCam);
  } catch (const std::exception&) {
    st = POVAR_ENOMEM;   // the request fails; the problem still leaves its group
  }
  if (st == POVAR_OK) {
    e = hipMemcpyAsync(cin.data(), pb->rec.P64[c.pcur], cin.size() * 8, hipMemcpyDeviceToHost, G.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(G.stream);
    if (e == hipSuccess) cams_to_caller(pb->L, cin.data(), cams.data(), kCam);
    st = e == hipSuccess ? copy_points(pb, c.lcur, pts.data()) : POVAR_EDEVICE;
  }
  povar_report rep;
  fill_report(pb, c, 0.0, NAN, &rep);
  const int last = (int)G.res.size() - 1;
  if (idx != last) {
    hipError_t e2 = hipMemcpyAsync(G.recs + idx, G.recs + last, sizeof(DevProblem), hipMemcpyDeviceToDevice,
                                   G.stream);
    if (e2 != hipSuccess && e == hipSuccess) e = e2;
    G.res[idx] = G.res[last];
    G.res[idx].pb->batch.probs = G.recs + idx;
  }
  G.res.pop_back();
  G.dirty = true;
  sv->retired.push_back({pb, r->footprint});
  sv->retired_bytes += r->footprint;
  std::lock_guard<std::mutex> g(sv->mu);
  rep.seconds_total = sv->now() - r->t_admit;
  r->report = rep;
  r->cams = std::move(cams);
  r->pts = std::move(pts);
  r->status = st == POVAR_ENOMEM ? POVAR_ENOMEM : (e != hipSuccess || st != POVAR_OK) ? POVAR_EDEVICE : POVAR_OK;
  if (r->status != POVAR_OK)
    r->error = st == POVAR_ENOMEM ? "host memory for the result exhausted"
               : e != hipSuccess  ? hipGetErrorString(e)
                                  : "result copy failed";
  r->finished = true;
  r->t_finish = sv->now();
  sv->n_resident -= 1;
  sv->n_finished += 1;
  return e;
}

// Frees the device memory of retired problems (each free synchronises the
// device, so this runs only while no group has work in flight).
void free_retired(povar_server_s* sv) {
  for (auto& pr : sv->retired) povar_problem_destroy(pr.first);
  sv->retired.clear();
  std::lock_guard<std::mutex> g(sv->mu);
  sv->used -= sv->retired_bytes;
  sv->retired_bytes = 0;
}

void worker_loop(povar_server_s* sv) {
  (void)hipSetDevice(sv->ctx->device);
  bool drain = false;   // launches held until no group is in flight, to free retired problems' memory
  double quiet_since = -1.0;   // start of the current run of passes without progress
  for (;;) {
    const double t_pass = sv->now();
    bool idle = true;
    for (Group& G : sv->groups) idle = idle && G.n_flight == 0;
    double d_retire = 0.0;
    if (idle && !sv->retired.empty()) {
      free_retired(sv);
      d_retire += sv->now() - t_pass;
    }
    if (idle) drain = false;
    bool progressed = false;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (sv->n_resident == 0 && idle) sv->cv.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
      if (sv->stop) return;
      // FIFO admission by slot and footprint; the admission thread
      // initialises the admitted requests
      while (!sv->queue.empty()) {
        auto& r = sv->queue.front();
        const bool slot = sv->n_resident < sv->max_slots;
        const bool fits = sv->used + r->footprint <= sv->budget;
        if (slot && !fits) {
          if (!r->budget_waited) {
            r->budget_waited = true;
            sv->budget_waits += 1;
          }
          // the memory of retired problems would make room: free it as soon
          // as the groups in flight have finished their batches
          if (sv->retired_bytes > 0 && sv->used - sv->retired_bytes + r->footprint <= sv->budget) drain = true;
        }
        if (!slot || !fits) break;
        sv->used += r->footprint;
        sv->n_resident += 1;
        sv->pending[group_index(r->fp32, r->n_obs)] += 1;
        sv->to_init.push_back(r);
        sv->queue.pop_front();
        progressed = true;
      }
    }
    if (progressed) sv->admit_cv.notify_one();
    // Idle groups take in their initialised newcomers and launch their next
    // iterations.
    //
    // Iterations per read-back: a problem's iteration count is known exactly
    // (each batched iteration advances every running problem of the group by
    // one), so as long as no problem can reach its limit and no admitted
    // request waits to join the group, several iterations are enqueued before
    // the control blocks are read.  A problem that stops earlier by ftol has
    // its remaining kernels return at once (they check its done flag).
    const double t1 = sv->now();
    if (!drain && join_ready(sv)) progressed = true;
    int pending[kNumGroups];
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      for (int g = 0; g < kNumGroups; ++g) pending[g] = sv->pending[g];
    }
    for (int g = 0; g < kNumGroups && !drain; ++g) {
      Group& G = sv->groups[g];
      if (G.n_flight > 0 || G.res.empty()) continue;
      int n_it = pending[g] > 0 ? 1 : kServerItersPerSync;
      for (auto& R : G.res) n_it = std::min(n_it, std::max(1, R.left));
      hipError_t e = G.dirty ? upload_tables(sv, G) : hipSuccess;
      for (int i = 0; i < n_it && e == hipSuccess; ++i) e = launch_iteration(G);
      const size_t n = G.res.size();
      if (e == hipSuccess)
        e = hipMemcpyAsync(G.host_recs, G.recs, n * sizeof(DevProblem), hipMemcpyDeviceToHost, G.stream);
      if (e == hipSuccess) e = hipEventRecord(G.ready, G.stream);
      if (e != hipSuccess) {
        fail_group(sv, G, e);
        continue;
      }
      G.n_flight = (int)n;
      G.it_flight = n_it;
      progressed = true;
    }
    const double t2 = sv->now();
    // read-backs that have arrived (nothing joins a group in flight, so the
    // read-back covers all of its residents)
    int64_t iters = 0, readbacks = 0;
    for (Group& G : sv->groups) {
      if (G.n_flight == 0) continue;
      const hipError_t q = hipEventQuery(G.ready);
      if (q == hipErrorNotReady) continue;
      const double tr = sv->now();
      const int n = G.n_flight;
      G.n_flight = 0;
      iters += G.it_flight;
      readbacks += 1;
      progressed = true;
      if (q != hipSuccess) {
        fail_group(sv, G, q);
        continue;
      }
      for (int idx = n - 1; idx >= 0; --idx) {
        const Ctl& c = G.host_recs[idx].ctl;
        G.res[idx].left = c.iter_limit - c.iter;
        if (c.done) (void)retire(sv, G, idx, c);
      }
      d_retire += sv->now() - tr;
    }
    // Without progress the worker polls again at once for 2 ms (batches of
    // serving-sized problems come back every millisecond or so, and a sleep
    // between polls measured 3-5% longer median latency), then at 20 us
    // intervals, so that long batches do not keep a core spinning.
    if (progressed) {
      quiet_since = -1.0;
    } else {
      if (quiet_since < 0.0) quiet_since = t_pass;
      if (t_pass - quiet_since < 2e-3) std::this_thread::yield();
      else std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    const double t3 = sv->now();
    std::lock_guard<std::mutex> g(sv->mu);
    if (progressed) sv->t_launch += t2 - t1;
    else sv->t_wait += t3 - t_pass - d_retire;
    sv->t_retire += d_retire;
    sv->batch_iters += iters;
    sv->syncs += readbacks;
  }
}

void free_server(povar_server_s* sv) {
  for (Group& G : sv->groups) {
    if (G.stream) (void)hipStreamSynchronize(G.stream);
    for (auto& R : G.res) povar_problem_destroy(R.pb);
    G.res.clear();
  }
  for (auto& pr : sv->retired) povar_problem_destroy(pr.first);
  sv->retired.clear();
  for (auto& x : sv->ready) povar_problem_destroy(x.pb);
  sv->ready.clear();
  if (sv->stage_recs) (void)hipFree(sv->stage_recs);
  for (Group& G : sv->groups) {
    if (G.recs) (void)hipFree(G.recs);
    if (G.tables) (void)hipFree(G.tables);
    if (G.host_recs) (void)hipHostFree(G.host_recs);
    if (G.ready) (void)hipEventDestroy(G.ready);
    if (G.stream) (void)hipStreamDestroy(G.stream);
  }
  if (sv->admit_stream) (void)hipStreamDestroy(sv->admit_stream);
}

}  // namespace

extern "C" {

povar_status povar_server_create(povar_ctx ctx, uint64_t hbm_budget_bytes, int32_t max_slots, povar_server* out) try {
  if (!out) return POVAR_EINVAL;
  *out = nullptr;
  if (!ctx || max_slots <= 0 || hbm_budget_bytes == 0) {
    set_error(ctx, "server needs a context, max_slots > 0 and a positive budget");
    return POVAR_EINVAL;
  }
  (void)hipSetDevice(ctx->device);
  auto* sv = new povar_server_s();
  sv->ctx = ctx;
  sv->budget = hbm_budget_bytes;
  sv->max_slots = max_slots;
  sv->t0 = std::chrono::steady_clock::now();
  // streams in the order of use: the FP32-bulk groups and the admissions
  // first, so that they take distinct hardware queues where few exist
  hipError_t e = hipSuccess;
  for (int g = 0; g < kNumGroups && e == hipSuccess; ++g) {
    Group& G = sv->groups[g];
    G.fp32 = g < 2;
    e = hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking);
    if (e == hipSuccess && g == 1) e = hipStreamCreateWithFlags(&sv->admit_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&G.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&G.recs, sizeof(DevProblem) * max_slots);
    if (e == hipSuccess) e = hipMalloc(&G.tables, sizeof(int32_t) * kNumUnitKinds * (max_slots + 1));
    if (e == hipSuccess) e = hipHostMalloc(&G.host_recs, sizeof(DevProblem) * max_slots, hipHostMallocDefault);
  }
  if (e == hipSuccess) e = hipMalloc(&sv->stage_recs, sizeof(DevProblem) * max_slots);
  for (int k = max_slots - 1; k >= 0; --k) sv->free_stage.push_back(k);
  if (e != hipSuccess) {
    set_error(ctx, "server allocation failed: %s", hipGetErrorString(e));
    free_server(sv);
    delete sv;
    return POVAR_ENOMEM;
  }
  try {
    sv->worker = std::thread(worker_loop, sv);
    sv->admitter = std::thread(admitter_loop, sv);
  } catch (const std::system_error& ex) {
    {
      std::lock_guard<std::mutex> g(sv->mu);
      sv->stop = true;
    }
    sv->cv.notify_all();
    sv->admit_cv.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    free_server(sv);
    delete sv;
    set_error(ctx, "server threads could not start: %s", ex.what());
    return POVAR_ENOMEM;
  }
  ctx->live_problems += 1;
  *out = sv;
  return POVAR_OK;
} POVAR_HOST_CATCH(ctx)

povar_status povar_server_submit(povar_server sv, int32_t n_cams, int32_t n_pts, int64_t n_obs,
                                 const int32_t* cam_idx, const int32_t* pt_idx, const double* meas,
                                 const double* cams0, const povar_options* opts, uint64_t* ticket) try {
  if (!sv || !ticket) return POVAR_EINVAL;
  const double t_call = sv->now();   // the request's latency includes its layout build
  povar_ctx ctx = sv->ctx;
  povar_status st = check_options(ctx, opts);
  if (st != POVAR_OK) return st;
  if (n_cams <= 0) {
    set_error(ctx, "n_cams must be positive");
    return POVAR_EINVAL;
  }
  auto r = std::make_shared<Request>();
  r->opt = *opts;
  r->fp32 = opts->precision == POVAR_PREC_FP32_BULK;
  st = build_layout(ctx, n_cams, n_pts, n_obs, cam_idx, pt_idx, meas, r->fp32, r->layout);
  if (st != POVAR_OK) return st;
  r->footprint = layout_footprint(r->layout, r->fp32);
  if (r->footprint > sv->budget) {
    set_error(ctx, "request needs %zu device bytes, more than the server budget %llu", r->footprint,
              (unsigned long long)sv->budget);
    return POVAR_ENOMEM;
  }
  r->n_p = n_cams;
  r->n_l = n_pts;
  r->n_obs = n_obs;
  if (cams0) {
    r->cams0.assign(cams0, cams0 + (size_t)n_cams * kCam);
  } else {   // seeded unit-norm Gaussian cameras, as for povar_problem_create
    r->cams0.resize((size_t)n_cams * kCam);
    seeded_cameras(opts->init_seed, n_cams, r->cams0.data());
  }
  {
    std::lock_guard<std::mutex> g(sv->mu);
    r->ticket = sv->next_ticket++;
    r->t_submit = t_call;
    sv->tickets[r->ticket] = r;
    sv->queue.push_back(r);
    *ticket = r->ticket;
  }
  sv->cv.notify_one();
  return POVAR_OK;
} POVAR_HOST_CATCH(sv ? sv->ctx : nullptr)

povar_status povar_server_poll(povar_server sv, uint64_t ticket, povar_report* report, double* cams_out,
                               double* pts_out, double* times) {
  if (!sv) return POVAR_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) {
    set_error(sv->ctx, "unknown ticket %llu", (unsigned long long)ticket);
    return POVAR_EINVAL;
  }
  auto r = it->second;
  if (!r->finished) return POVAR_EAGAIN;
  if (times) {
    times[0] = r->t_submit;
    times[1] = r->t_admit;
    times[2] = r->t_finish;
  }
  if (report) *report = r->report;
  if (r->status == POVAR_OK) {
    if (cams_out) std::memcpy(cams_out, r->cams.data(), r->cams.size() * 8);
    if (pts_out) std::memcpy(pts_out, r->pts.data(), r->pts.size() * 8);
  } else {
    set_error(sv->ctx, "request %llu failed: %s", (unsigned long long)ticket, r->error.c_str());
  }
  const povar_status st = r->status;
  sv->tickets.erase(it);
  return st;
}

povar_status povar_server_stats(povar_server sv, int32_t* queued, int32_t* active, int64_t* finished,
                                int64_t* batch_iters) {
  if (!sv) return POVAR_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  if (queued) *queued = (int32_t)sv->queue.size();
  if (active) *active = sv->n_resident;
  if (finished) *finished = sv->n_finished;
  if (batch_iters) *batch_iters = sv->batch_iters;
  return POVAR_OK;
}

povar_status povar_server_profile(povar_server sv, double* seconds, int64_t* counts) {
  if (!sv) return POVAR_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  if (seconds) {
    seconds[0] = sv->t_admit;
    seconds[1] = sv->t_launch;
    seconds[2] = sv->t_wait;
    seconds[3] = sv->t_retire;
  }
  if (counts) {
    counts[0] = sv->batch_iters;
    counts[1] = sv->syncs;
    counts[2] = sv->budget_waits;
  }
  return POVAR_OK;
}

povar_status povar_server_destroy(povar_server sv) {
  if (!sv) return POVAR_EINVAL;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  sv->admit_cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  if (sv->admitter.joinable()) sv->admitter.join();
  (void)hipSetDevice(sv->ctx->device);
  free_server(sv);
  sv->ctx->live_problems -= 1;
  delete sv;
  return POVAR_OK;
}

}  // extern "C"
