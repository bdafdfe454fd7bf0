// Host side of the PoVar library: validation, observation layout, device
// state, the LM driver (device-side decisions, graph replay) and the per-step
// hooks.  Implements the single-problem part of include/povar.h; the server
// lives in povar_server.hip.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <system_error>
#include <thread>
#include <tuple>
#include <vector>

#include "povar.h"
#include "povar_host.h"

namespace povar {

constexpr int kTraceCapacity = 4096;   // per-iteration trace entries kept per problem

thread_local std::string g_noctx_error;

void set_error(povar_ctx ctx, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) {
    std::lock_guard<std::mutex> g(ctx->err_mu);
    ctx->err = buf;
  } else {
    g_noctx_error = buf;
  }
}

static inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Byte plan of one problem's device arena.  Used both to allocate and to
// answer povar_problem_footprint, so admission accounting matches exactly.
struct ArenaPlan {
  size_t total = 0;
  size_t take(size_t bytes) {
    const size_t off = total;
    total += align_up(bytes);
    return off;
  }
};

size_t arena_bytes(const LayoutSizes& z, bool fp32, int64_t trace_cap, ArenaOffsets* o) {
  const int64_t n_p = z.n_p, n_l = z.n_l, n_obs = z.n_obs, n_pk = z.n_pk, n_ch = z.n_ch, n_mc = z.n_mc;
  ArenaPlan a;
  ArenaOffsets tmp;
  ArenaOffsets& r = o ? *o : tmp;
  const size_t ts = fp32 ? 4 : 8;
  const int64_t n_ent = n_pk * kWave;   // packet slots of 64 entries
  r.pk_hdr = a.take(n_pk * 8);
  r.pk_code = a.take(n_ent * 4);
  r.pk_m32 = fp32 ? a.take(n_ent * 8) : SIZE_MAX;
  r.pk_m64 = a.take(n_ent * 16);
  r.cm_lm = a.take(n_obs * 4);
  r.cm_m32 = fp32 ? a.take(n_obs * 8) : SIZE_MAX;
  r.cm_m64 = a.take(n_obs * 16);   // FP32-bulk too: its linearisation forms U_i in FP64
  r.ch_meta = a.take(n_ch * 16);
  r.cam_ch = a.take((n_p + 1) * 4);
  r.mc_cam = a.take(n_mc * 4);
  const int64_t n_cs = z.blocked ? z.n_cs : 0, n_runs = z.blocked ? z.n_runs : 0;
  r.cs_hdr = a.take(n_cs * 4);
  r.cs_lane = a.take(n_cs * kWave * 8);
  r.cs_lm = a.take(n_cs * cs_obs(fp32) * 4);
  r.cs_m32 = fp32 ? a.take(n_cs * cs_obs(fp32) * 8) : SIZE_MAX;
  r.cs_m64 = fp32 ? SIZE_MAX : a.take(n_cs * cs_obs(fp32) * 16);
  r.run_off = a.take((n_p + 1) * 4);
  r.smc = a.take((z.blocked ? n_p : n_mc) * 4);
  // the other buffers with initial values (current cameras and series
  // records, second-stage landmarks, the problem record, unit tables) end the
  // prefix that problem creation copies from the host; the rest is cleared
  // on the device
  r.P64[0] = a.take(n_p * kCam * 8);
  r.S32[0] = fp32 ? a.take(n_p * ser_stride((int)n_p) * 4) : SIZE_MAX;
  r.S64[0] = fp32 ? SIZE_MAX : a.take(n_p * ser_stride((int)n_p) * 8);
  r.rec64[0] = a.take(n_l * kRec * 8);
  r.rec = a.take(sizeof(DevProblem));
  r.tables = a.take(kNumUnitKinds * 2 * 4);
  r.init_end = a.total;
  r.t_run = a.take(n_runs * kCam * ts);
  for (int b = 0; b < 2; ++b) {
    if (b == 1) {
      r.P64[b] = a.take(n_p * kCam * 8);
      r.S32[b] = fp32 ? a.take(n_p * ser_stride((int)n_p) * 4) : SIZE_MAX;
      r.S64[b] = fp32 ? SIZE_MAX : a.take(n_p * ser_stride((int)n_p) * 8);
      r.rec64[b] = a.take(n_l * kRec * 8);
    }
    r.xs64[b] = a.take(n_l * 4 * 8);
    r.xs32[b] = a.take(n_l * 4 * 4);
    r.Vp64[b] = a.take(n_l * kLmSym * 8);
  }
  r.lin_part = a.take(n_ch * kLinVals * 8);
  r.K64 = a.take(n_p * kCamMat * 8);
  r.g64 = a.take(n_p * kCam * 8);
  r.U40 = a.take(n_p * 40 * 8);
  r.acc = a.take(n_p * kCam * 8);
  r.zx = a.take(n_l * kRec * ts);
  r.t_part = a.take(n_ch * kCam * ts);
  r.cost_part = a.take(n_pk * 8);
  r.cost_group = a.take((n_pk + kCostGroup - 1) / kCostGroup * 8);
  r.bl_part = a.take(n_pk * 8);
  r.bl_group = a.take((n_pk + kCostGroup - 1) / kCostGroup * 8);
  r.tr_cost = a.take(trace_cap * 8);
  r.tr_lambda = a.take(trace_cap * 8);
  r.tr_acc = a.take(trace_cap * 4);
  r.tr_bl = a.take(trace_cap * 8);
  r.tr_series = a.take(trace_cap * 8);
  return a.total;
}

void cams_to_caller(const HostLayout& L, const double* in, double* out, int width) {
  for (int32_t i = 0; i < L.n_p; ++i)
    std::memcpy(out + (size_t)L.cam_int2ext[i] * width, in + (size_t)i * width, sizeof(double) * width);
}

void unit_counts(const HostLayout& L, int32_t* units) {
  units[kUnitPacket] = L.n_pk;
  units[kUnitChunk] = L.n_ch;
  units[kUnitCamWave] = (L.n_p + kWave - 1) / kWave;
  units[kUnitOne] = 1;
  units[kUnitMultiCam] = (int32_t)L.smc.size();
  units[kUnitCostGroup] = L.n_cg;
  units[kUnitSerChunk] = L.blocked ? 0 : L.n_ch;
  units[kUnitCSlot] = L.blocked ? L.n_cs : 0;
}

size_t layout_footprint(const HostLayout& L, bool fp32) {
  return arena_bytes(sizes_of(L), fp32, kTraceCapacity, nullptr);
}

// ------------------------------------------------------------------ layout
// Number of landmark blocks of a blocked problem: records of at most
// kLmBlockBytes per block, a multiple of kXcds blocks of equal size.
static int64_t landmark_blocks(int64_t n_l, bool fp32) {
  const int64_t lb_max = kLmBlockBytes / (kRec * (fp32 ? 4 : 8));
  const int64_t nb = (n_l + lb_max - 1) / lb_max;
  return (nb + kXcds - 1) / kXcds * kXcds;
}

// XCD of landmark block b: blocks go round the XCDs forwards, then
// backwards, so that each XCD receives a mix of early (denser) and later
// blocks of the min-camera landmark order.
static int xcd_of_block(int64_t b) {
  const int64_t g = b / kXcds, r = b % kXcds;
  return (int)((g & 1) ? kXcds - 1 - r : r);
}

// Slots of the blocked series camera pass, from the camera-major order
// (camera, then internal landmark) already in L.cm_lm / L.cm_m*.
static povar_status build_camera_slots(povar_ctx ctx, HostLayout& L, const std::vector<int64_t>& cstart,
                                       bool fp32) {
  const int kCsPerLane = cs_per_lane(fp32), kCsObs = cs_obs(fp32);
  const int32_t n_p = L.n_p, n_l = L.n_l;
  const int64_t nb = landmark_blocks(n_l, fp32);
  const int64_t lb = (n_l + nb - 1) / nb;
  L.blocked = 1;
  L.lm_block = (int32_t)lb;
  // one run per (block, camera) segment part that lies in one slot
  struct Run {
    int32_t cam, lslot, lane0, nlanes, key;
    int64_t beg, cnt;   // camera-major observation range
  };
  std::vector<std::vector<std::pair<int64_t, int64_t>>> segs_cam(nb);   // (camera, begin) per block
  std::vector<std::vector<int64_t>> segs_end(nb);
  for (int32_t c = 0; c < n_p; ++c) {
    int64_t pos = cstart[c];
    while (pos < cstart[c + 1]) {
      const int64_t b = L.cm_lm[pos] / lb;
      int64_t end = pos;
      while (end < cstart[c + 1] && L.cm_lm[end] / lb == b) ++end;
      segs_cam[b].push_back({c, pos});
      segs_end[b].push_back(end);
      pos = end;
    }
  }
  std::vector<std::vector<Run>> runs(nb);
  std::vector<int32_t> nslots(nb, 0);
  std::vector<std::vector<int32_t>> slot_lanes(nb);
  for (int64_t b = 0; b < nb; ++b) {
    int32_t used = kWave, key = 0;
    for (size_t k = 0; k < segs_cam[b].size(); ++k) {
      int64_t beg = segs_cam[b][k].second;
      const int64_t end = segs_end[b][k];
      while (beg < end) {
        if (used == kWave) {
          slot_lanes[b].push_back(0);
          ++nslots[b];
          used = 0;
          key = 0;
        }
        const int64_t want = (end - beg + kCsPerLane - 1) / kCsPerLane;   // lanes
        const int32_t nl = (int32_t)std::min<int64_t>(kWave - used, want);
        const int64_t cnt = std::min<int64_t>(end - beg, (int64_t)nl * kCsPerLane);
        runs[b].push_back(Run{(int32_t)segs_cam[b][k].first, nslots[b] - 1, used, nl, key, beg, cnt});
        used += nl;
        ++key;
        slot_lanes[b].back() = used;
        beg += cnt;
      }
    }
  }
  // dispatch order: rounds of one workgroup (4 slots) per XCD while every
  // XCD has slots left, then the remaining slots in block order
  std::vector<std::vector<std::pair<int64_t, int32_t>>> xl(kXcds);   // (block, local slot)
  for (int64_t b = 0; b < nb; ++b)
    for (int32_t q = 0; q < nslots[b]; ++q) xl[xcd_of_block(b)].push_back({b, q});
  std::vector<std::vector<int64_t>> gslot(nb);
  for (int64_t b = 0; b < nb; ++b) gslot[b].assign(nslots[b], -1);
  int64_t g = 0;
  std::vector<size_t> next(kXcds, 0);
  auto all_left = [&]() {
    for (int x = 0; x < kXcds; ++x)
      if (next[x] >= xl[x].size()) return false;
    return true;
  };
  while (all_left()) {
    for (int x = 0; x < kXcds; ++x) {
      for (int w = 0; w < kWavesPerBlock; ++w, ++g) {
        if (next[x] < xl[x].size()) {
          const auto bq = xl[x][next[x]++];
          gslot[bq.first][bq.second] = g;
        }   // else: empty slot keeps the XCD alignment
      }
    }
  }
  for (int x = 0; x < kXcds; ++x)
    for (; next[x] < xl[x].size(); ++next[x], ++g) gslot[xl[x][next[x]].first][xl[x][next[x]].second] = g;
  g = (g + kXcds * kWavesPerBlock - 1) / (kXcds * kWavesPerBlock) * (kXcds * kWavesPerBlock);
  if (g * (int64_t)kCsObs >= (int64_t)INT_MAX) {
    set_error(ctx, "camera slot layout exceeds 2^31 entries");
    return POVAR_EINVAL;
  }
  L.n_cs = (int32_t)g;
  // run ids camera-major (each camera's runs in block order)
  L.run_off.assign(n_p + 1, 0);
  for (int64_t b = 0; b < nb; ++b)
    for (const Run& r : runs[b]) ++L.run_off[r.cam + 1];
  for (int32_t c = 0; c < n_p; ++c) L.run_off[c + 1] += L.run_off[c];
  L.n_runs = L.run_off[n_p];
  std::vector<int32_t> fill(L.run_off.begin(), L.run_off.end() - 1);
  L.cs_hdr.assign(L.n_cs, 0);
  L.cs_lane.assign((size_t)L.n_cs * kWave * 2, 0);
  L.cs_lm.assign((size_t)L.n_cs * kCsObs, -1);
  if (fp32) L.cs_m32.assign((size_t)L.n_cs * kCsObs * 2, 0.0f);
  else L.cs_m64.assign((size_t)L.n_cs * kCsObs * 2, 0.0);
  for (int64_t b = 0; b < nb; ++b) {
    for (int32_t q = 0; q < nslots[b]; ++q) L.cs_hdr[gslot[b][q]] = slot_lanes[b][q];
    for (const Run& r : runs[b]) {
      const int64_t gs = gslot[b][r.lslot];
      const int32_t id = fill[r.cam]++;
      for (int32_t l = r.lane0; l < r.lane0 + r.nlanes; ++l) {
        L.cs_lane[2 * ((size_t)gs * kWave + l)] = r.cam | (r.key << kCamBits);
        L.cs_lane[2 * ((size_t)gs * kWave + l) + 1] = id;
      }
      for (int64_t o = 0; o < r.cnt; ++o) {
        const int32_t lane = r.lane0 + (int32_t)(o / kCsPerLane), rr = (int32_t)(o % kCsPerLane);
        const size_t e = ((size_t)gs * kCsPerLane + rr) * kWave + lane;
        const int64_t src = r.beg + o;
        L.cs_lm[e] = L.cm_lm[src];
        if (fp32) {
          L.cs_m32[2 * e] = L.cm_m32[2 * src];
          L.cs_m32[2 * e + 1] = L.cm_m32[2 * src + 1];
        } else {
          L.cs_m64[2 * e] = L.cm_m64[2 * src];
          L.cs_m64[2 * e + 1] = L.cm_m64[2 * src + 1];
        }
      }
    }
  }
  L.smc.resize(n_p);
  for (int32_t c = 0; c < n_p; ++c) L.smc[c] = c;
  return POVAR_OK;
}

// Runs fn(t, begin, end) over T contiguous parts of [0, n) on T threads (the
// caller's included).  Large layouts use up to four: the parts write
// disjoint entries, so the result does not depend on T.
template <typename F>
static void parallel_parts(int T, int64_t n, F fn) {
  if (T <= 1) {
    fn(0, (int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  int t = 1;
  try {
    for (; t < T; ++t) th.emplace_back(fn, t, n * t / T, n * (t + 1) / T);
  } catch (const std::system_error&) {
    // no thread to be had: the caller takes the parts left over
  }
  for (int u = t; u < T; ++u) fn(u, n * u / T, n * (u + 1) / T);
  fn(0, (int64_t)0, n / T);
  for (auto& x : th) x.join();
}

static int layout_threads(int64_t n_obs) {
  if (n_obs < (1 << 17)) return 1;
  const unsigned hw = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(4u, hw));
}

povar_status build_layout(povar_ctx ctx, int32_t n_p, int32_t n_l, int64_t n_obs, const int32_t* cam,
                          const int32_t* pt, const double* meas, bool fp32, HostLayout& L) {
  if (n_p <= 0 || n_l <= 0 || n_obs <= 0) {
    set_error(ctx, "n_cams, n_pts and n_obs must be positive (got %d, %d, %lld)", n_p, n_l, (long long)n_obs);
    return POVAR_EINVAL;
  }
  if (n_obs >= (int64_t)INT_MAX / 2) {
    set_error(ctx, "n_obs = %lld exceeds the supported maximum", (long long)n_obs);
    return POVAR_EINVAL;
  }
  if (!cam || !pt || !meas) {
    set_error(ctx, "cam_idx, pt_idx and meas must not be NULL");
    return POVAR_EINVAL;
  }
  L.n_p = n_p;
  L.n_l = n_l;
  L.n_obs = n_obs;
  std::vector<int32_t> cnt_l(n_l, 0), cnt_c(n_p, 0);
  for (int64_t k = 0; k < n_obs; ++k) {
    const int32_t c = cam[k], j = pt[k];
    if (c < 0 || c >= n_p || j < 0 || j >= n_l) {
      set_error(ctx, "observation %lld has camera %d / point %d out of range", (long long)k, c, j);
      return POVAR_EINVAL;
    }
    if (!std::isfinite(meas[2 * k]) || !std::isfinite(meas[2 * k + 1])) {
      set_error(ctx, "observation %lld has a non-finite measurement", (long long)k);
      return POVAR_EINVAL;
    }
    ++cnt_l[j];
    ++cnt_c[c];
  }
  for (int32_t i = 0; i < n_p; ++i)
    if (cnt_c[i] == 0) {
      set_error(ctx, "camera %d has no observation", i);
      return POVAR_EINVAL;
    }
  for (int32_t j = 0; j < n_l; ++j)
    if (cnt_l[j] == 0) {
      set_error(ctx, "point %d has no observation", j);
      return POVAR_EINVAL;
    }
  // internal camera order: most observed first (the landmark pass of large
  // problems keeps the first cameras' series data in LDS), then caller's index;
  // everything below works on internal camera ids
  L.cam_int2ext.resize(n_p);
  std::iota(L.cam_int2ext.begin(), L.cam_int2ext.end(), 0);
  std::stable_sort(L.cam_int2ext.begin(), L.cam_int2ext.end(),
                   [&](int32_t a, int32_t b) { return cnt_c[a] > cnt_c[b]; });
  std::vector<int32_t> cam_ext2int(n_p);
  for (int32_t i = 0; i < n_p; ++i) cam_ext2int[L.cam_int2ext[i]] = i;
  std::vector<int32_t> cam_in(n_obs);
  for (int64_t k = 0; k < n_obs; ++k) cam_in[k] = cam_ext2int[cam[k]];
  {
    std::vector<int32_t> cnt(n_p);
    for (int32_t i = 0; i < n_p; ++i) cnt[i] = cnt_c[L.cam_int2ext[i]];
    cnt_c.swap(cnt);
  }
  cam = cam_in.data();
  // internal landmark order: by the set of XCDs that read the landmark's
  // series record in the chunked camera pass, then by the smallest camera that
  // sees it, then caller's index.  Chunk q runs on XCD q % 8 (round-robin
  // dispatch; in a batch every XCD index shifts by the same amount), so a
  // landmark's record is fetched into the L2 of each XCD holding one of its
  // cameras' chunks; grouping landmarks with equal XCD sets keeps a 128-byte
  // line of records from being fetched into more L2s than its landmarks need
  // (about half the fetches at 250 cameras).  Within a group, landmarks that
  // share their first camera sit together, which helps the camera-major
  // gathers.  Blocked problems have their own XCD order and use the second
  // key alone.
  std::vector<int32_t> minc(n_l, INT_MAX);
  for (int64_t k = 0; k < n_obs; ++k) minc[pt[k]] = std::min(minc[pt[k]], cam[k]);
  std::vector<uint32_t> sig(n_l, 0);
  if (!blocked_layout(n_l, fp32)) {
    std::vector<uint32_t> cmask(n_p, 0);
    int64_t ch0 = 0;
    for (int32_t i = 0; i < n_p; ++i) {
      const int64_t nch = (cnt_c[i] + kChunk - 1) / kChunk;
      for (int64_t q = ch0; q < ch0 + nch && q < ch0 + kXcds; ++q) cmask[i] |= 1u << (q % kXcds);
      ch0 += nch;
    }
    for (int64_t k = 0; k < n_obs; ++k) sig[pt[k]] |= cmask[cam[k]];
  }
  // (the order of a stable sort by (sig, minc), built as two stable counting
  // sorts: by minc, then by sig)
  L.int2ext.resize(n_l);
  {
    std::vector<int32_t> by_minc(n_l);
    std::vector<int64_t> start((size_t)n_p + 1, 0);
    for (int32_t j = 0; j < n_l; ++j) ++start[(size_t)minc[j] + 1];
    for (int32_t i = 0; i < n_p; ++i) start[i + 1] += start[i];
    for (int32_t j = 0; j < n_l; ++j) by_minc[start[minc[j]]++] = j;
    int64_t sstart[(1 << kXcds) + 1] = {0};
    for (int32_t j = 0; j < n_l; ++j) ++sstart[sig[j] + 1];
    for (int s = 0; s < (1 << kXcds); ++s) sstart[s + 1] += sstart[s];
    for (int32_t j : by_minc) L.int2ext[sstart[sig[j]]++] = j;
  }
  // observations grouped by caller's landmark, then sorted by camera
  std::vector<int64_t> lstart(n_l + 1, 0);
  for (int32_t j = 0; j < n_l; ++j) lstart[j + 1] = lstart[j] + cnt_l[j];
  std::vector<int64_t> lobs(n_obs);
  {
    std::vector<int64_t> fill(lstart.begin(), lstart.end() - 1);
    for (int64_t k = 0; k < n_obs; ++k) lobs[fill[pt[k]]++] = k;
  }
  // each landmark's observations by camera, stable (insertion sort for the
  // usual short tracks, merge sort for long ones)
  const int T = layout_threads(n_obs);
  parallel_parts(T, n_l, [&](int, int64_t j0, int64_t j1) {
    for (int64_t j = j0; j < j1; ++j) {
      int64_t* o = lobs.data() + lstart[j];
      const int64_t m = lstart[j + 1] - lstart[j];
      if (m > 32) {
        std::stable_sort(o, o + m, [&](int64_t a, int64_t b) { return cam[a] < cam[b]; });
        continue;
      }
      for (int64_t u = 1; u < m; ++u) {
        const int64_t x = o[u];
        const int32_t cx = cam[x];
        int64_t v = u;
        for (; v > 0 && cam[o[v - 1]] > cx; --v) o[v] = o[v - 1];
        o[v] = x;
      }
    }
  });
  if (n_p > (int32_t)kCamMask) {
    set_error(ctx, "n_cams exceeds the supported maximum");
    return POVAR_EINVAL;
  }
  // landmark-major packets on 64-entry slots: greedy runs of whole landmarks
  // with <= 64 observations; a landmark with more than 64 observations fills
  // consecutive slots of its own
  std::vector<int32_t> slot_of(n_l), pos_in_slot(n_l);
  {
    int32_t slot = -1, used = kWave;
    for (int32_t jj = 0; jj < n_l; ++jj) {
      const int32_t len = cnt_l[L.int2ext[jj]];
      if (len > kWave) {
        slot += 1;
        slot_of[jj] = slot;
        pos_in_slot[jj] = 0;
        L.pk_hdr.push_back(len);
        L.pk_hdr.push_back(jj);
        const int32_t extra = (len + kWave - 1) / kWave - 1;
        for (int32_t x = 0; x < extra; ++x) {
          L.pk_hdr.push_back(0);
          L.pk_hdr.push_back(jj);
        }
        slot += extra;
        used = kWave;   // closed
      } else {
        if (used + len > kWave) {
          slot += 1;
          used = 0;
          L.pk_hdr.push_back(0);
          L.pk_hdr.push_back(jj);
        }
        slot_of[jj] = slot;
        pos_in_slot[jj] = used;
        used += len;
        L.pk_hdr[2 * slot] = used;
      }
    }
    L.n_pk = slot + 1;
  }
  const int64_t n_ent = (int64_t)L.n_pk * kWave;
  if (n_ent >= (int64_t)INT_MAX) {
    set_error(ctx, "packet layout exceeds 2^31 entries");
    return POVAR_EINVAL;
  }
  L.pk_code.assign(n_ent, 0u);
  L.pk_m64.assign(2 * n_ent, 0.0);
  if (fp32) L.pk_m32.assign(2 * n_ent, 0.0f);
  // filled in the caller's landmark order, so that the observation data are
  // read in (usually) their own order and each landmark's entries written
  // where its slot puts them
  {
    std::vector<int32_t> lm_ext2int(n_l);
    for (int32_t jj = 0; jj < n_l; ++jj) lm_ext2int[L.int2ext[jj]] = jj;
    parallel_parts(T, n_l, [&](int, int64_t j0, int64_t j1) {
      for (int64_t j = j0; j < j1; ++j) {
        const int32_t jj = lm_ext2int[j];
        const int32_t slot = slot_of[jj];
        const int32_t local = jj - L.pk_hdr[2 * slot + 1];
        int64_t e = (int64_t)slot * kWave + pos_in_slot[jj];
        for (int64_t q = lstart[j]; q < lstart[j + 1]; ++q, ++e) {
          const int64_t k = lobs[q];
          L.pk_code[e] = (uint32_t)cam[k] | ((uint32_t)local << kCamBits);
          L.pk_m64[2 * e] = meas[2 * k];
          L.pk_m64[2 * e + 1] = meas[2 * k + 1];
          if (fp32) {
            L.pk_m32[2 * e] = (float)meas[2 * k];
            L.pk_m32[2 * e + 1] = (float)meas[2 * k + 1];
          }
        }
      }
    });
  }
  // camera-major order: by camera, then internal landmark, then the order
  // within the landmark, which is the order of the packet entries (read
  // from them in sequence)
  std::vector<int64_t> cstart(n_p + 1, 0);
  for (int32_t i = 0; i < n_p; ++i) cstart[i + 1] = cstart[i] + cnt_c[i];
  L.cm_lm.resize(n_obs);
  if (fp32) L.cm_m32.resize(2 * n_obs);
  L.cm_m64.resize(2 * n_obs);
  {
    // with several threads, each takes a contiguous range of slots and
    // starts each camera after the entries the earlier ranges put there
    // (counted first), so the order is the sequential one
    const int Tc = (int64_t)n_p * 64 <= n_obs ? T : 1;
    std::vector<int64_t> fill((size_t)Tc * n_p);
    auto walk = [&](int64_t q0, int64_t q1, auto&& visit) {
      for (int64_t q = q0; q < q1; ++q) {
        const int32_t n = L.pk_hdr[2 * q], lm0 = L.pk_hdr[2 * q + 1];
        // continuation slots (n = 0) hold the tail of the landmark started before
        for (int64_t e = q * kWave; e < q * kWave + n; ++e) visit(e, lm0);
      }
    };
    if (Tc > 1) {
      std::vector<int64_t> cnt((size_t)Tc * n_p, 0);
      parallel_parts(Tc, L.n_pk, [&](int t, int64_t q0, int64_t q1) {
        int64_t* c = cnt.data() + (size_t)t * n_p;
        walk(q0, q1, [&](int64_t e, int32_t) { ++c[L.pk_code[e] & kCamMask]; });
      });
      for (int32_t i = 0; i < n_p; ++i) {
        int64_t at = cstart[i];
        for (int t = 0; t < Tc; ++t) {
          fill[(size_t)t * n_p + i] = at;
          at += cnt[(size_t)t * n_p + i];
        }
      }
    } else {
      for (int32_t i = 0; i < n_p; ++i) fill[i] = cstart[i];
    }
    parallel_parts(Tc, L.n_pk, [&](int t, int64_t q0, int64_t q1) {
      int64_t* f = fill.data() + (size_t)t * n_p;
      walk(q0, q1, [&](int64_t e, int32_t lm0) {
        const uint32_t code = L.pk_code[e];
        const int64_t pos = f[code & kCamMask]++;
        L.cm_lm[pos] = lm0 + (int32_t)(code >> kCamBits);
        if (fp32) {
          L.cm_m32[2 * pos] = L.pk_m32[2 * e];
          L.cm_m32[2 * pos + 1] = L.pk_m32[2 * e + 1];
        }
        L.cm_m64[2 * pos] = L.pk_m64[2 * e];
        L.cm_m64[2 * pos + 1] = L.pk_m64[2 * e + 1];
      });
    });
  }
  // chunks of <= kChunk observations, never spanning two cameras
  L.cam_ch.resize(n_p + 1);
  L.cam_ch[0] = 0;
  for (int32_t i = 0; i < n_p; ++i) L.cam_ch[i + 1] = L.cam_ch[i] + (cnt_c[i] + kChunk - 1) / kChunk;
  L.n_ch = L.cam_ch[n_p];
  L.ch_meta.resize((size_t)4 * L.n_ch);
  for (int32_t i = 0; i < n_p; ++i) {
    const int32_t nch = L.cam_ch[i + 1] - L.cam_ch[i];
    for (int32_t q = L.cam_ch[i]; q < L.cam_ch[i + 1]; ++q) {
      const int64_t b = cstart[i] + (int64_t)(q - L.cam_ch[i]) * kChunk;
      L.ch_meta[4 * (size_t)q + 0] = i;
      L.ch_meta[4 * (size_t)q + 1] = (int32_t)b;
      L.ch_meta[4 * (size_t)q + 2] = (int32_t)std::min<int64_t>(b + kChunk, cstart[i + 1]);
      L.ch_meta[4 * (size_t)q + 3] = nch;
    }
  }
  for (int32_t i = 0; i < n_p; ++i)
    if (L.cam_ch[i + 1] - L.cam_ch[i] > 1) L.mc_cam.push_back(i);
  L.n_mc = (int32_t)L.mc_cam.size();
  L.n_cg = L.n_pk > kCostDirect ? (L.n_pk + kCostGroup - 1) / kCostGroup : 0;
  if (!blocked_layout(n_l, fp32)) {
    L.smc = L.mc_cam;
    return POVAR_OK;
  }
  return build_camera_slots(ctx, L, cstart, fp32);
}

// Checks the invariants of a built layout that the kernels rely on (the
// properties are listed with povar_debug_layout_check).
static povar_status check_layout(const HostLayout& L, const int32_t* cam, const int32_t* pt, const double* meas,
                                 bool fp32, int64_t* out) {
  const int kCsPerLane = cs_per_lane(fp32);
  auto fail = [](const char* what, long long a, long long b) {
    set_error(nullptr, "layout check: %s (%lld, %lld)", what, a, b);
    return POVAR_EINVAL;
  };
  const int32_t n_p = L.n_p, n_l = L.n_l;
  const int64_t n_obs = L.n_obs;
  std::vector<int32_t> cam_ext2int(n_p), lm_ext2int(n_l);
  for (int32_t i = 0; i < n_p; ++i) cam_ext2int[L.cam_int2ext[i]] = i;
  for (int32_t j = 0; j < n_l; ++j) lm_ext2int[L.int2ext[j]] = j;
  // each observation as (internal camera, internal landmark, u, v), the
  // measurement in FP64 and in the bulk precision
  using Obs = std::tuple<int32_t, int32_t, double, double>;
  std::vector<Obs> want64(n_obs), want(n_obs);
  for (int64_t k = 0; k < n_obs; ++k) {
    const int32_t c = cam_ext2int[cam[k]], j = lm_ext2int[pt[k]];
    want64[k] = Obs(c, j, meas[2 * k], meas[2 * k + 1]);
    want[k] = fp32 ? Obs(c, j, (double)(float)meas[2 * k], (double)(float)meas[2 * k + 1]) : want64[k];
  }
  std::sort(want64.begin(), want64.end());
  std::sort(want.begin(), want.end());
  // landmark-major packets: a slot holds whole landmarks in internal order, or
  // starts a landmark of more than 64 observations whose continuation slots
  // carry n = 0 and the same first landmark
  {
    if ((int64_t)L.pk_hdr.size() != 2LL * L.n_pk) return fail("packet header count", L.pk_hdr.size(), L.n_pk);
    std::vector<Obs> got;
    int32_t next_lm = 0;
    for (int32_t q = 0; q < L.n_pk;) {
      const int32_t n = L.pk_hdr[2 * q], lm0 = L.pk_hdr[2 * q + 1];
      if (n <= 0 || lm0 != next_lm) return fail("packet header", q, n);
      const int32_t slots = n > kWave ? (n + kWave - 1) / kWave : 1;
      if (q + slots > L.n_pk) return fail("long landmark past the last slot", q, n);
      for (int32_t x = 1; x < slots; ++x)
        if (L.pk_hdr[2 * (q + x)] != 0 || L.pk_hdr[2 * (q + x) + 1] != lm0) return fail("continuation slot", q + x, n);
      int32_t prev = 0;
      for (int32_t e = 0; e < n; ++e) {
        const size_t idx = (size_t)q * kWave + e;
        const int32_t c = (int32_t)(L.pk_code[idx] & kCamMask), key = (int32_t)(L.pk_code[idx] >> kCamBits);
        if (key < prev || key > prev + 1 || (e == 0 && key != 0) || (n > kWave && key != 0) || c >= n_p)
          return fail("packet entry", q, e);
        prev = key;
        if (fp32 && (double)L.pk_m32[2 * idx] != (double)(float)L.pk_m64[2 * idx]) return fail("packet FP32 copy", q, e);
        got.push_back(Obs(c, lm0 + key, L.pk_m64[2 * idx], L.pk_m64[2 * idx + 1]));
      }
      next_lm = lm0 + prev + 1;
      q += slots;
    }
    if (next_lm != n_l) return fail("packets do not cover every landmark", next_lm, n_l);
    std::sort(got.begin(), got.end());
    if (got != want64) return fail("packets do not hold every observation once", (long long)got.size(), n_obs);
  }
  // camera-major chunks: consecutive, at most kChunk observations, one camera each
  {
    if ((int64_t)L.cm_lm.size() != n_obs) return fail("camera-major size", L.cm_lm.size(), n_obs);
    if ((int64_t)L.cm_m64.size() != 2 * n_obs) return fail("camera-major FP64 size", L.cm_m64.size(), n_obs);
    std::vector<Obs> got, got64;
    int64_t pos = 0;
    for (int32_t i = 0; i < n_p; ++i) {
      if (L.cam_ch[i + 1] <= L.cam_ch[i]) return fail("camera without a chunk", i, L.cam_ch[i]);
      for (int32_t ch = L.cam_ch[i]; ch < L.cam_ch[i + 1]; ++ch) {
        const int32_t* m = &L.ch_meta[4 * (size_t)ch];
        if (m[0] != i || m[1] != pos || m[2] <= m[1] || m[2] - m[1] > kChunk || m[3] != L.cam_ch[i + 1] - L.cam_ch[i])
          return fail("chunk metadata", ch, m[0]);
        int32_t prev = -1;
        for (int64_t e = m[1]; e < m[2]; ++e) {
          if (L.cm_lm[e] < prev) return fail("camera-major landmarks out of order", i, e);
          prev = L.cm_lm[e];
          got.push_back(Obs(i, L.cm_lm[e], fp32 ? L.cm_m32[2 * e] : L.cm_m64[2 * e],
                            fp32 ? L.cm_m32[2 * e + 1] : L.cm_m64[2 * e + 1]));
          // the FP64 measurements beside the bulk ones (FP32-bulk forms U_i from them)
          if (fp32 && ((float)L.cm_m64[2 * e] != L.cm_m32[2 * e] || (float)L.cm_m64[2 * e + 1] != L.cm_m32[2 * e + 1]))
            return fail("camera-major FP64 measurement", i, e);
          if (fp32) got64.push_back(Obs(i, L.cm_lm[e], L.cm_m64[2 * e], L.cm_m64[2 * e + 1]));
        }
        pos = m[2];
      }
    }
    if (pos != n_obs) return fail("chunks end early", pos, n_obs);
    std::sort(got.begin(), got.end());
    if (got != want) return fail("chunks do not hold every observation once", (long long)got.size(), n_obs);
    std::sort(got64.begin(), got64.end());
    if (fp32 && got64 != want64) return fail("camera-major FP64 measurements", (long long)got64.size(), n_obs);
    int32_t n_mc = 0;
    for (int32_t i = 0; i < n_p; ++i)
      if (L.cam_ch[i + 1] - L.cam_ch[i] > 1 && (n_mc >= L.n_mc || L.mc_cam[n_mc++] != i))
        return fail("multi-chunk camera list", i, n_mc);
    if (n_mc != L.n_mc) return fail("multi-chunk camera count", n_mc, L.n_mc);
  }
  // camera slots of a landmark-blocked problem
  if (L.blocked) {
    const int64_t nb = landmark_blocks(n_l, fp32), lb = L.lm_block;
    if (lb <= 0 || lb * nb < n_l || (int64_t)L.lm_block * kRec * (fp32 ? 4 : 8) > kLmBlockBytes)
      return fail("landmark block size", lb, nb);
    if (L.n_cs % (kXcds * kWavesPerBlock) != 0) return fail("camera slots not a multiple of 32", L.n_cs, 0);
    if ((int32_t)L.run_off.size() != n_p + 1 || L.run_off[0] != 0 || L.run_off[n_p] != L.n_runs)
      return fail("run offsets", L.run_off.size(), L.n_runs);
    std::vector<Obs> got;
    std::vector<int32_t> run_tails(L.n_runs, 0);
    std::vector<int64_t> slot_block(L.n_cs, -1), per_xcd(kXcds, 0);
    for (int32_t q = 0; q < L.n_cs; ++q) {
      const int32_t nl = L.cs_hdr[q];
      if (nl < 0 || nl > kWave) return fail("slot header", q, nl);
      int32_t prev_key = -1, prev_code = -1, prev_id = -1;
      for (int32_t lane = 0; lane < kWave; ++lane) {
        const size_t li = (size_t)q * kWave + lane;
        const int32_t code = L.cs_lane[2 * li], id = L.cs_lane[2 * li + 1];
        if (lane >= nl) {
          for (int32_t r = 0; r < kCsPerLane; ++r)
            if (L.cs_lm[((size_t)q * kCsPerLane + r) * kWave + lane] != -1) return fail("entry in an unused lane", q, lane);
          continue;
        }
        const int32_t c = code & (int32_t)kCamMask, key = (int32_t)((uint32_t)code >> kCamBits);
        if (c >= n_p || id < L.run_off[c] || id >= L.run_off[c + 1]) return fail("run id outside its camera", q, lane);
        if (code == prev_code ? id != prev_id : key != prev_key + 1) return fail("run keys", q, lane);
        prev_key = key;
        prev_code = code;
        prev_id = id;
        if (lane == nl - 1 || L.cs_lane[2 * (li + 1)] != code) run_tails[id] += 1;
        for (int32_t r = 0; r < kCsPerLane; ++r) {
          const size_t e = ((size_t)q * kCsPerLane + r) * kWave + lane;
          const int32_t j = L.cs_lm[e];
          if (j == -1) {
            if (r == 0) return fail("empty lane inside a run", q, lane);
            continue;
          }
          if (j < 0 || j >= n_l) return fail("slot landmark", q, j);
          if (slot_block[q] < 0) slot_block[q] = j / lb;
          if (j / lb != slot_block[q]) return fail("slot spans two landmark blocks", q, j);
          got.push_back(Obs(c, j, fp32 ? L.cs_m32[2 * e] : L.cs_m64[2 * e], fp32 ? L.cs_m32[2 * e + 1] : L.cs_m64[2 * e + 1]));
        }
      }
      if ((nl > 0) != (slot_block[q] >= 0)) return fail("slot header and entries disagree", q, nl);
      if (slot_block[q] >= 0) ++per_xcd[xcd_of_block(slot_block[q])];
    }
    for (int32_t id = 0; id < L.n_runs; ++id)
      if (run_tails[id] != 1) return fail("run without exactly one tail lane", id, run_tails[id]);
    std::sort(got.begin(), got.end());
    if (got != want) return fail("camera slots do not hold every observation once", (long long)got.size(), n_obs);
    // workgroup g (slots 4g..4g+3) runs on XCD g % 8: while every XCD has
    // slots left, rounds of 32 slots give each XCD four slots of its blocks
    const int64_t rounds = (*std::min_element(per_xcd.begin(), per_xcd.end()) + kWavesPerBlock - 1) / kWavesPerBlock;
    for (int64_t q = 0; q < rounds * kXcds * kWavesPerBlock; ++q)
      if (slot_block[q] >= 0 && xcd_of_block(slot_block[q]) != (int)((q / kWavesPerBlock) % kXcds))
        return fail("slot off its XCD in an aligned round", q, slot_block[q]);
  }
  // footprint from sizes alone
  const size_t exact = layout_footprint(L, fp32);
  uint64_t bound = 0;
  if (povar_problem_footprint(n_p, n_l, n_obs, fp32 ? POVAR_PREC_FP32_BULK : POVAR_PREC_FP64, &bound) != POVAR_OK ||
      exact > bound)
    return fail("footprint bound below the built layout", (long long)exact, (long long)bound);
  if (out) {
    out[0] = L.blocked;
    out[1] = L.n_pk;
    out[2] = L.n_ch;
    out[3] = L.n_cs;
    out[4] = L.n_runs;
    out[5] = L.lm_block;
    out[6] = (int64_t)exact;
    out[7] = (int64_t)bound;
  }
  return POVAR_OK;
}

}  // namespace povar

using namespace povar;

#define HIP_TRY(ctx, expr)                                                          \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess) {                                                         \
      set_error((ctx), "%s failed: %s", #expr, hipGetErrorString(_e));              \
      return POVAR_EDEVICE;                                                         \
    }                                                                               \
  } while (0)

namespace povar {


povar_status check_options(povar_ctx ctx, const povar_options* o) {
  if (!o) {
    set_error(ctx, "options must not be NULL");
    return POVAR_EINVAL;
  }
  if (o->struct_size != sizeof(povar_options)) {
    set_error(ctx, "povar_options.struct_size is %u, expected %zu", o->struct_size, sizeof(povar_options));
    return POVAR_EINVAL;
  }
  if (!(o->eta >= 0.0 && o->eta <= 1.0)) {
    set_error(ctx, "eta must lie in [0, 1]");
    return POVAR_EINVAL;
  }
  if (o->series_order < 0 || o->series_order > 100000) {
    set_error(ctx, "series_order must lie in [0, 100000]");
    return POVAR_EINVAL;
  }
  if (o->max_iters < 0) {
    set_error(ctx, "max_iters must be >= 0");
    return POVAR_EINVAL;
  }
  if (!(o->ftol >= 0.0) || !(o->lambda0 > 0.0) || !(o->lambda_min > 0.0) ||
      !(o->lambda_max >= o->lambda_min) || !std::isfinite(o->lambda_max)) {
    set_error(ctx, "need ftol >= 0 and 0 < lambda_min <= lambda_max < inf, lambda0 > 0");
    return POVAR_EINVAL;
  }
  if (o->precision != POVAR_PREC_FP64 && o->precision != POVAR_PREC_FP32_BULK) {
    set_error(ctx, "unknown precision %d", o->precision);
    return POVAR_EINVAL;
  }
  if (o->manifold != POVAR_MANIFOLD_SPHERE && o->manifold != POVAR_MANIFOLD_EUCLIDEAN) {
    set_error(ctx, "unknown manifold %d", o->manifold);
    return POVAR_EINVAL;
  }
  if (!(o->series_rtol >= 0.0 && o->series_rtol < 1.0)) {
    set_error(ctx, "series_rtol must lie in [0, 1)");
    return POVAR_EINVAL;
  }
  return POVAR_OK;
}

template <typename T>
static bool upload(std::vector<char>& staging, size_t off, const std::vector<T>& v) {
  // every buffer with an initial value lies in the staged prefix
  if (v.empty()) return true;
  if (off > staging.size() || v.size() * sizeof(T) > staging.size() - off) return false;
  std::memcpy(staging.data() + off, v.data(), v.size() * sizeof(T));
  return true;
}

// Builds the device state of a problem from a host layout and initial
// cameras: one arena allocation, filled from a single host staging image.
povar_status problem_init(povar_ctx ctx, HostLayout&& L, const double* cams0, const povar_options* o,
                          hipStream_t stream, povar_problem_s* pb, DevProblem* rec_dev, int32_t iter_limit,
                          const double* pts0) {
  pb->ctx = ctx;
  pb->opt = *o;
  pb->fp32 = o->precision == POVAR_PREC_FP32_BULK;
  pb->stream = stream;
  pb->trace_cap = kTraceCapacity;
  pb->L = std::move(L);
  HostLayout& H = pb->L;
  ArenaOffsets& A = pb->off;
  pb->bytes = arena_bytes(sizes_of(H), pb->fp32, pb->trace_cap, &A);
  hipError_t e = hipMalloc(&pb->arena, pb->bytes);
  if (e != hipSuccess) {
    pb->arena = nullptr;
    set_error(ctx, "hipMalloc of %zu bytes failed: %s", pb->bytes, hipGetErrorString(e));
    return POVAR_ENOMEM;
  }
  char* base = static_cast<char*>(pb->arena);
  auto dp = [&](size_t off) -> void* { return off == SIZE_MAX ? nullptr : base + off; };

  // cameras (normalised on the sphere)
  std::vector<double> P64((size_t)H.n_p * kCam);
  const int ss = ser_stride(H.n_p);
  std::vector<float> S32(pb->fp32 ? (size_t)H.n_p * ss : 0, 0.0f);
  std::vector<double> S64(pb->fp32 ? 0 : (size_t)H.n_p * ss, 0.0);
  for (int32_t i = 0; i < H.n_p; ++i) {
    const int32_t e = H.cam_int2ext[i];
    double nrm = 0.0;
    for (int r = 0; r < kCam; ++r) {
      const double v = cams0[(size_t)e * kCam + r];
      if (!std::isfinite(v)) {
        set_error(ctx, "initial camera %d is not finite", e);
        return POVAR_EINVAL;
      }
      nrm += v * v;
    }
    if (!(nrm > 0.0)) {
      set_error(ctx, "initial camera %d is zero", e);
      return POVAR_EINVAL;
    }
    const double s = o->manifold == POVAR_MANIFOLD_SPHERE ? 1.0 / std::sqrt(nrm) : 1.0;
    for (int r = 0; r < kCam; ++r) {
      const double v = cams0[(size_t)e * kCam + r] * s;
      P64[(size_t)i * kCam + r] = v;
      if (pb->fp32) S32[(size_t)i * ss + r] = (float)v;
      else S64[(size_t)i * ss + r] = v;
    }
  }

  DevProblem& R = pb->rec;
  std::memset(&R, 0, sizeof(R));
  R.n_p = H.n_p;
  R.n_l = H.n_l;
  R.n_pk = H.n_pk;
  R.n_mc = H.n_mc;
  R.n_cg = H.n_cg;
  R.n_ch = H.n_ch;
  R.manifold = o->manifold;
  R.s_stride = ser_stride(H.n_p);
  R.wave_sums = 0;
  for (int32_t i = 0; i < H.n_p; ++i)
    if (H.cam_ch[i + 1] - H.cam_ch[i] > kWaveSumChunks) R.wave_sums = 1;
  R.trace_cap = pb->trace_cap;
  R.eta = o->eta;
  R.ftol = o->ftol;
  R.lambda_min = o->lambda_min;
  R.lambda_max = o->lambda_max;
  R.series_rtol = o->series_rtol;
  R.pk_hdr = (const int2*)dp(A.pk_hdr);
  R.pk_code = (const uint32_t*)dp(A.pk_code);
  R.pk_m32 = (const float2*)dp(A.pk_m32);
  R.pk_m64 = (const double2*)dp(A.pk_m64);
  R.cm_lm = (const int32_t*)dp(A.cm_lm);
  R.cm_m32 = (const float2*)dp(A.cm_m32);
  R.cm_m64 = (const double2*)dp(A.cm_m64);
  R.ch_meta = (const int4*)dp(A.ch_meta);
  R.cam_ch = (const int32_t*)dp(A.cam_ch);
  R.mc_cam = (const int32_t*)dp(A.mc_cam);
  R.blocked = H.blocked;
  R.n_cs = H.blocked ? H.n_cs : 0;
  R.n_runs = H.blocked ? H.n_runs : 0;
  R.n_smc = (int32_t)H.smc.size();
  R.cs_hdr = (const int32_t*)dp(A.cs_hdr);
  R.cs_lane = (const int2*)dp(A.cs_lane);
  R.cs_lm = (const int32_t*)dp(A.cs_lm);
  R.cs_m32 = (const float2*)dp(A.cs_m32);
  R.cs_m64 = (const double2*)dp(A.cs_m64);
  R.ser_off = H.blocked ? (const int32_t*)dp(A.run_off) : (const int32_t*)dp(A.cam_ch);
  R.ser_mc = (const int32_t*)dp(A.smc);
  for (int b = 0; b < 2; ++b) {
    R.P64[b] = (double*)dp(A.P64[b]);
    R.S32[b] = (float*)dp(A.S32[b]);
    R.S64[b] = (double*)dp(A.S64[b]);
    R.rec64[b] = (double*)dp(A.rec64[b]);
    R.xs64[b] = (double*)dp(A.xs64[b]);
    R.xs32[b] = (float*)dp(A.xs32[b]);
    R.Vp64[b] = (double*)dp(A.Vp64[b]);
  }
  R.lin_part = (double*)dp(A.lin_part);
  R.K64 = (double*)dp(A.K64);
  R.g64 = (double*)dp(A.g64);
  R.U40 = (double*)dp(A.U40);
  R.acc = (double*)dp(A.acc);
  R.zx = dp(A.zx);
  R.t_part = dp(A.t_part);
  R.ser_part = H.blocked ? dp(A.t_run) : dp(A.t_part);
  R.cost_part = (double*)dp(A.cost_part);
  R.cost_group = (double*)dp(A.cost_group);
  R.bl_part = (double*)dp(A.bl_part);
  R.bl_group = (double*)dp(A.bl_group);
  R.tr_cost = (double*)dp(A.tr_cost);
  R.tr_lambda = (double*)dp(A.tr_lambda);
  R.tr_acc = (int32_t*)dp(A.tr_acc);
  R.tr_bl = (double*)dp(A.tr_bl);
  R.tr_series = (double*)dp(A.tr_series);

  // second stage: initial landmarks (unit 4-vectors) and its own buffers
  R.stage = pts0 ? 2 : 1;
  std::vector<double> X4;
  if (pts0) {
    X4.assign((size_t)H.n_l * kX2, 0.0);
    for (int32_t jj = 0; jj < H.n_l; ++jj) {
      const int32_t e = H.int2ext[jj];
      double nrm = 0.0;
      for (int k = 0; k < 4; ++k) {
        const double v = pts0[(size_t)e * 4 + k];
        if (!std::isfinite(v)) {
          set_error(ctx, "initial point %d is not finite", e);
          return POVAR_EINVAL;
        }
        nrm += v * v;
      }
      if (!(nrm > 0.0)) {
        set_error(ctx, "initial point %d is zero", e);
        return POVAR_EINVAL;
      }
      for (int k = 0; k < 4; ++k) X4[(size_t)jj * kX2 + k] = pts0[(size_t)e * 4 + k] / std::sqrt(nrm);
    }
    const size_t b_g2 = align_up((size_t)H.n_l * kG2 * 8), b_bl2 = align_up((size_t)H.n_l * 4 * 8);
    const size_t b_lin2 = align_up((size_t)H.n_ch * kLin2 * 8), b_x2 = align_up((size_t)H.n_p * kCam * 8);
    e = hipMalloc(&pb->arena2, b_g2 + b_bl2 + b_lin2 + b_x2);
    if (e != hipSuccess) {
      pb->arena2 = nullptr;
      set_error(ctx, "hipMalloc of the second-stage buffers failed: %s", hipGetErrorString(e));
      return POVAR_ENOMEM;
    }
    char* b2 = static_cast<char*>(pb->arena2);
    R.g2 = (double*)b2;
    R.bl2 = (double*)(b2 + b_g2);
    R.lin2 = (double*)(b2 + b_g2 + b_bl2);
    R.x2 = (double*)(b2 + b_g2 + b_bl2 + b_lin2);
  }

  Ctl& c = R.ctl;
  c.lambda = o->lambda0;
  c.need_lin = 1;
  c.iter_limit = iter_limit;
  c.order = o->series_order;
  c.stop_at = o->series_order;

  // batch of one: prefix tables of waves per unit kind
  int32_t units[kNumUnitKinds];
  unit_counts(H, units);
  int32_t tables[kNumUnitKinds * 2];
  for (int k = 0; k < kNumUnitKinds; ++k) {
    tables[2 * k] = 0;
    tables[2 * k + 1] = units[k];
  }

  // one staging image of the arena's prefix with initial values; the rest is
  // cleared on the device
  std::vector<char> img(A.init_end, 0);
  bool staged = true;
  staged &= upload(img, A.pk_hdr, H.pk_hdr);
  staged &= upload(img, A.pk_code, H.pk_code);
  if (A.pk_m32 != SIZE_MAX) staged &= upload(img, A.pk_m32, H.pk_m32);
  staged &= upload(img, A.pk_m64, H.pk_m64);
  staged &= upload(img, A.cm_lm, H.cm_lm);
  if (A.cm_m32 != SIZE_MAX) staged &= upload(img, A.cm_m32, H.cm_m32);
  if (A.cm_m64 != SIZE_MAX) staged &= upload(img, A.cm_m64, H.cm_m64);
  staged &= upload(img, A.ch_meta, H.ch_meta);
  staged &= upload(img, A.cam_ch, H.cam_ch);
  staged &= upload(img, A.mc_cam, H.mc_cam);
  staged &= upload(img, A.smc, H.smc);
  if (H.blocked) {
    staged &= upload(img, A.cs_hdr, H.cs_hdr);
    staged &= upload(img, A.cs_lane, H.cs_lane);
    staged &= upload(img, A.cs_lm, H.cs_lm);
    if (A.cs_m32 != SIZE_MAX) staged &= upload(img, A.cs_m32, H.cs_m32);
    if (A.cs_m64 != SIZE_MAX) staged &= upload(img, A.cs_m64, H.cs_m64);
    staged &= upload(img, A.run_off, H.run_off);
  }
  staged &= upload(img, A.P64[0], P64);
  if (pts0) staged &= upload(img, A.rec64[0], X4);
  if (pb->fp32) staged &= upload(img, A.S32[0], S32);
  else staged &= upload(img, A.S64[0], S64);
  if (!staged || A.rec + sizeof(R) > A.init_end || A.tables + sizeof(int32_t) * kNumUnitKinds * 2 > A.init_end) {
    set_error(ctx, "internal: a buffer with an initial value lies outside the staged prefix");
    return POVAR_EDEVICE;
  }
  std::memcpy(img.data() + A.rec, &R, sizeof(R));
  std::memcpy(img.data() + A.tables, tables, sizeof(tables));
  HIP_TRY(ctx, hipMemcpyAsync(pb->arena, img.data(), A.init_end, hipMemcpyHostToDevice, stream));
  HIP_TRY(ctx, hipMemsetAsync(static_cast<char*>(pb->arena) + A.init_end, 0, pb->bytes - A.init_end, stream));
  HIP_TRY(ctx, hipStreamSynchronize(stream));   // the staging image is freed on return

  Batch& B = pb->batch;
  B.probs = (DevProblem*)dp(A.rec);
  if (rec_dev) {   // the record lives in a caller-owned array (server slots)
    HIP_TRY(ctx, hipMemcpyAsync(rec_dev, &R, sizeof(R), hipMemcpyHostToDevice, stream));
    B.probs = rec_dev;
  }
  B.tables = (const int32_t*)dp(A.tables);
  B.tab_stride = 2;
  for (int k = 0; k < kNumUnitKinds; ++k) B.total[k] = units[k];
  B.n_prob = 1;
  B.coop_cams = (!pb->fp32 || R.s_stride == kSerLine) ? 1 : 0;
  B.wave_sums = R.wave_sums;
  if (pts0) {
    // second stage: the cost (7) at the given cameras and landmarks
    HIP_TRY(ctx, launch_refine_landmarks(B, stream));
  } else {
    // initial landmarks and cost, Eq. (8)-(9)
    HIP_TRY(ctx, launch_landmark_solve(B, 0, stream));
  }
  HIP_TRY(ctx, launch_cost_groups(B, 0, stream));
  HIP_TRY(ctx, launch_cost_finalize(B, 0, stream));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  // free the host copies of what only the device needs
  HostLayout keep;
  keep.n_p = H.n_p;
  keep.n_l = H.n_l;
  keep.n_obs = H.n_obs;
  keep.n_pk = H.n_pk;
  keep.n_ch = H.n_ch;
  keep.n_mc = H.n_mc;
  keep.n_cg = H.n_cg;
  keep.blocked = H.blocked;
  keep.lm_block = H.lm_block;
  keep.n_cs = H.n_cs;
  keep.n_runs = H.n_runs;
  keep.smc = std::move(H.smc);
  keep.int2ext = std::move(H.int2ext);
  keep.cam_int2ext = std::move(H.cam_int2ext);
  keep.cam_ch = std::move(H.cam_ch);
  H = std::move(keep);
  Ctl now;
  HIP_TRY(ctx, read_ctl(pb, &now));
  if (!std::isfinite(now.cost)) {
    set_error(ctx, "initial cost is not finite");
    return POVAR_ENUMERIC;
  }
  return POVAR_OK;
}

hipError_t read_ctl(povar_problem_s* pb, Ctl* out) {
  hipError_t e = hipMemcpyAsync(out, pb->batch.probs, sizeof(Ctl), hipMemcpyDeviceToHost, pb->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(pb->stream);
}

hipError_t write_ctl(povar_problem_s* pb, const Ctl* in) {
  hipError_t e = hipMemcpyAsync(pb->batch.probs, in, sizeof(Ctl), hipMemcpyHostToDevice, pb->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(pb->stream);
}

// Series kernels; when timed, each series kernel carries a start/stop event
// pair recorded by its own dispatch.
static hipError_t enqueue_series(povar_problem_s* pb, int order, bool timed) {
  hipError_t e;
  for (int t = 1; t <= order; ++t) {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (timed)
      for (int q = 0; q < 4; ++q) {
        ev[q] = pb->event_pool_get();
        if (!ev[q]) return hipErrorOutOfMemory;
      }
    if ((e = launch_series_landmark(pb->batch, pb->fp32, t, pb->stream, ev[0], ev[1])) != hipSuccess) return e;
    if ((e = launch_series_camera(pb->batch, pb->fp32, t, pb->stream, ev[2], ev[3])) != hipSuccess) return e;
    if (pb->opt.series_rtol > 0.0 && t < order &&
        (e = launch_series_check(pb->batch, pb->fp32, t, pb->stream)) != hipSuccess)
      return e;
    if (timed) {
      pb->pending.push_back({ev[0], ev[1], 0});
      pb->pending.push_back({ev[2], ev[3], 1});
    }
  }
  return hipSuccess;
}

hipError_t enqueue_iteration(povar_problem_s* pb, bool timed) {
  hipError_t e;
  const Batch& B = pb->batch;
  if (pb->rec.stage == 2)
    return launch_refine_iteration(B, pb->opt.series_order, pb->opt.series_rtol > 0.0, pb->stream);
  if ((e = launch_linearize(B, pb->fp32, 0, pb->stream)) != hipSuccess) return e;
  if ((e = launch_camera_prep(B, pb->fp32, pb->stream)) != hipSuccess) return e;
  if ((e = enqueue_series(pb, pb->opt.series_order, timed)) != hipSuccess) return e;
  // order 0, or a series that may stop early: the retraction is a kernel of its own
  if ((pb->opt.series_order == 0 || pb->opt.series_rtol > 0.0) &&
      (e = launch_retract(B, pb->fp32, pb->stream)) != hipSuccess)
    return e;
  if ((e = launch_landmark_solve(B, 1, pb->stream)) != hipSuccess) return e;
  if ((e = launch_cost_groups(B, 1, pb->stream)) != hipSuccess) return e;
  return launch_decide(B, pb->stream);
}

// Graphs of one and of kGraphIters iterations: replaying a graph costs a few
// microseconds between graphs, which the longer graph pays once per
// kGraphIters iterations.
static hipError_t capture_iterations(povar_problem_s* pb, int iters, hipGraphExec_t* out) {
  hipError_t e = hipStreamBeginCapture(pb->stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return e;
  for (int i = 0; i < iters && e == hipSuccess; ++i) e = enqueue_iteration(pb, false);
  hipGraph_t captured = nullptr;
  const hipError_t e2 = hipStreamEndCapture(pb->stream, &captured);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (captured) (void)hipGraphDestroy(captured);
    return e != hipSuccess ? e : e2;
  }
  e = hipGraphInstantiate(out, captured, nullptr, nullptr, 0);
  (void)hipGraphDestroy(captured);
  if (e != hipSuccess) *out = nullptr;
  return e;
}

static hipError_t ensure_graph(povar_problem_s* pb) {
  if (pb->graph_exec && pb->graph_exec_k) return hipSuccess;
  hipError_t e = hipSuccess;
  if (!pb->graph_exec) e = capture_iterations(pb, 1, &pb->graph_exec);
  if (e == hipSuccess && !pb->graph_exec_k) e = capture_iterations(pb, kGraphIters, &pb->graph_exec_k);
  return e;
}

// Problems above this many observations launch their kernels directly: each
// kernel then runs for tens of microseconds or more, so the host enqueues
// far ahead of the GPU and a graph saves nothing.  (A first-stage solve of
// the 13,700-camera workload once ended in a host segmentation fault inside
// the runtime's graph-launch path while it ran under a profiler, with no
// cause found in this library; large problems do not take that path.)
constexpr int64_t kGraphMaxObs = 2000000;

hipError_t enqueue_iterations(povar_problem_s* pb, int n) {
  hipError_t e = hipSuccess;
  const bool timed = pb->timing;
  if (!timed && pb->opt.use_graph && !pb->graph_failed && pb->L.n_obs <= kGraphMaxObs) {
    e = ensure_graph(pb);
    if (e != hipSuccess) {
      pb->graph_failed = true;   // fall back to direct launches
      (void)hipGetLastError();
    }
  }
  const bool graphs = !timed && !pb->graph_failed && pb->graph_exec && pb->graph_exec_k &&
                      pb->L.n_obs <= kGraphMaxObs;
  int it = 0;
  if (graphs)
    for (; it + kGraphIters <= n; it += kGraphIters)
      if ((e = hipGraphLaunch(pb->graph_exec_k, pb->stream)) != hipSuccess) return e;
  for (; it < n; ++it) {
    if (graphs) e = hipGraphLaunch(pb->graph_exec, pb->stream);
    else e = enqueue_iteration(pb, timed);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace povar

hipEvent_t povar_problem_s::event_pool_get() {
  if (event_next < events.size()) return events[event_next++];
  hipEvent_t ev;
  if (hipEventCreate(&ev) != hipSuccess) return nullptr;
  events.push_back(ev);
  ++event_next;
  return ev;
}

hipError_t povar_problem_s::drain_timing() {
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return e;
  for (const auto& p : pending) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, p.start, p.stop);
    if (e != hipSuccess) return e;
    ms_kernel[p.kind] += ms;
    n_kernel[p.kind] += 1;
  }
  pending.clear();
  event_next = 0;
  return hipSuccess;
}

namespace povar {

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): ten rounds of two 64x64 -> 128-bit products
// with the published multipliers, the key bumped by the published Weyl
// constants between rounds.
static void philox4x64(const uint64_t (&ctr_in)[4], const uint64_t (&key_in)[2], uint64_t (&out)[4]) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
  uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const unsigned __int128 p0 = (unsigned __int128)kM0 * c[0];
    const unsigned __int128 p1 = (unsigned __int128)kM1 * c[2];
    const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    c[0] = hi1 ^ c[1] ^ k0;
    c[1] = lo1;
    c[2] = hi0 ^ c[3] ^ k1;
    c[3] = lo0;
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

void seeded_cameras(uint64_t seed, int32_t n, double* out) {
  constexpr double kTwoPi = 6.283185307179586476925286766559;
  const uint64_t key[2] = {seed, 0};
  for (int32_t cam = 0; cam < n; ++cam) {
    double* v = out + (size_t)cam * kCam;
    for (uint64_t b = 0; b < 3; ++b) {
      const uint64_t ctr[4] = {(uint64_t)cam, b, 0, 0};
      uint64_t w[4];
      philox4x64(ctr, key, w);
      for (int h = 0; h < 2; ++h) {
        // uniforms in (0, 1): the top 53 bits, offset by half a unit
        const double u0 = ((double)(w[2 * h] >> 11) + 0.5) * 0x1p-53;
        const double u1 = ((double)(w[2 * h + 1] >> 11) + 0.5) * 0x1p-53;
        const double rho = std::sqrt(-2.0 * std::log(u0));   // Box-Muller
        v[4 * b + 2 * h] = rho * std::cos(kTwoPi * u1);
        v[4 * b + 2 * h + 1] = rho * std::sin(kTwoPi * u1);
      }
    }
    double nrm = 0.0;
    for (int r = 0; r < kCam; ++r) nrm += v[r] * v[r];
    const double inv = 1.0 / std::sqrt(nrm);
    for (int r = 0; r < kCam; ++r) v[r] *= inv;
  }
}

void fill_report(const povar_problem_s* pb, const Ctl& c, double seconds, double grad_norm, povar_report* r) {
  if (!r) return;
  std::memset(r, 0, sizeof(*r));
  r->cost_initial = c.cost0;
  r->cost_final = c.cost;
  r->lambda_final = c.lambda;
  r->grad_norm_final = grad_norm;
  r->seconds_total = seconds;
  r->seconds_series = pb->ctx->clock_hz > 0.0 ? (double)c.series_ticks / pb->ctx->clock_hz : NAN;
  r->iters = c.iter;
  r->accepted = c.n_accept;
  r->stop_reason = c.stop_reason;
}

}  // namespace povar

static povar_status copy_landmark_vec(povar_problem_s* pb, const double* dev, int stride, int offset, int width,
                                      double* out) {
  std::vector<double> tmp((size_t)pb->L.n_l * stride);
  HIP_TRY(pb->ctx, hipMemcpyAsync(tmp.data(), dev, tmp.size() * 8, hipMemcpyDeviceToHost, pb->stream));
  HIP_TRY(pb->ctx, hipStreamSynchronize(pb->stream));
  for (int32_t jj = 0; jj < pb->L.n_l; ++jj) {
    const int32_t j = pb->L.int2ext[jj];
    for (int k = 0; k < width; ++k) out[(size_t)j * width + k] = tmp[(size_t)jj * stride + offset + k];
  }
  return POVAR_OK;
}

namespace povar {
povar_status copy_points(povar_problem_s* pb, int lcur, double* out) {
  return copy_landmark_vec(pb, pb->rec.rec64[lcur], kRec, 4, 3, out);
}
}  // namespace povar

// ==================================================================== C ABI
extern "C" {

povar_status povar_options_default(povar_options* o) {
  if (!o) return POVAR_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(povar_options);
  o->eta = 0.01;
  o->series_order = 20;
  o->max_iters = 50;
  o->ftol = 1e-6;
  o->lambda0 = 1e-4;
  o->lambda_min = 1e-12;
  o->lambda_max = 1e12;
  o->precision = POVAR_PREC_FP64;
  o->manifold = POVAR_MANIFOLD_SPHERE;
  o->use_graph = 1;
  return POVAR_OK;
}

povar_status povar_ctx_create(int device, void* hip_stream, povar_ctx* out) try {
  if (!out) return POVAR_EINVAL;
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) {
    set_error(nullptr, "no HIP device available (%s)", hipGetErrorString(e));
    return POVAR_EDEVICE;
  }
  if (device < 0 || device >= n) {
    set_error(nullptr, "device %d out of range [0, %d)", device, n);
    return POVAR_EINVAL;
  }
  e = hipSetDevice(device);
  if (e != hipSuccess) {
    set_error(nullptr, "hipSetDevice(%d): %s", device, hipGetErrorString(e));
    return POVAR_EDEVICE;
  }
  auto* c = new povar_ctx_s();
  c->device = device;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    c->clock_hz = 1e3 * khz;
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->own_stream = false;
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      set_error(nullptr, "hipStreamCreate: %s", hipGetErrorString(e));
      delete c;
      return POVAR_EDEVICE;
    }
    c->own_stream = true;
  }
  const povar_status st = metric_scratch_init(c);
  if (st != POVAR_OK) {
    set_error(nullptr, "%s", povar_last_error(c));
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return st;
  }
  *out = c;
  return POVAR_OK;
} POVAR_HOST_CATCH(nullptr)

povar_status povar_ctx_destroy(povar_ctx ctx) {
  if (!ctx) return POVAR_EINVAL;
  if (ctx->live_problems > 0) {
    set_error(ctx, "%d problem(s) of this context are still alive", ctx->live_problems);
    return POVAR_ESTATE;
  }
  (void)hipSetDevice(ctx->device);
  if (ctx->own_stream) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
  return POVAR_OK;
}

const char* povar_last_error(povar_ctx ctx) {
  if (!ctx) return g_noctx_error.c_str();
  std::lock_guard<std::mutex> g(ctx->err_mu);
  ctx->err_copy = ctx->err;
  return ctx->err_copy.c_str();
}

povar_status povar_problem_footprint(int32_t n_cams, int32_t n_pts, int64_t n_obs, int32_t precision,
                                     uint64_t* bytes) {
  if (!bytes || n_cams <= 0 || n_pts <= 0 || n_obs <= 0) return POVAR_EINVAL;
  if (precision != POVAR_PREC_FP64 && precision != POVAR_PREC_FP32_BULK) return POVAR_EINVAL;
  // upper bounds on the packet slots: (a) every slot starts a landmark or
  // continues one with more than 64 observations; (b) two consecutive slots of
  // short landmarks hold more than 64 observations together, a run of them
  // starts after each long landmark, and a long landmark of L observations
  // takes ceil(L/64) slots.  Chunk rounding adds at most one chunk per camera.
  const int64_t n_pk = std::min<int64_t>(n_pts + n_obs / kWave + 1, n_obs / kWave + 2 * n_obs / (kWave + 1) + 3);
  const int64_t n_ch = n_obs / kChunk + n_cams;
  const bool fp32 = precision == POVAR_PREC_FP32_BULK;
  LayoutSizes z{n_cams, n_pts, n_obs, n_pk, n_ch, n_cams, 0, 0, blocked_layout(n_pts, fp32)};
  if (z.blocked) {
    // segments (block, camera) <= min(n_obs, n_cams * blocks); a slot holds
    // 64 lanes, a run wastes less than one lane, and a slot boundary splits
    // at most one run; plus one partial slot per block and the dispatch padding
    const int64_t nb = landmark_blocks(n_pts, fp32);
    const int64_t segs = std::min<int64_t>(n_obs, (int64_t)n_cams * nb);
    z.n_cs = (n_obs / cs_per_lane(fp32) + segs) / (kWave - 1) + 2 * nb + 2 * kXcds * kWavesPerBlock;
    z.n_runs = segs + z.n_cs;
  }
  *bytes = arena_bytes(z, fp32, kTraceCapacity, nullptr);
  return POVAR_OK;
}

povar_status povar_problem_create(povar_ctx ctx, int32_t n_cams, int32_t n_pts, int64_t n_obs,
                                  const int32_t* cam_idx, const int32_t* pt_idx, const double* meas,
                                  const double* cams0, const povar_options* opts, povar_problem* out) try {
  if (!ctx || !out) return POVAR_EINVAL;
  *out = nullptr;
  povar_status st = check_options(ctx, opts);
  if (st != POVAR_OK) return st;
  if (n_cams <= 0) {
    set_error(ctx, "n_cams must be positive");
    return POVAR_EINVAL;
  }
  std::vector<double> seeded;
  if (!cams0) {   // seeded unit-norm Gaussian cameras
    seeded.resize((size_t)n_cams * kCam);
    seeded_cameras(opts->init_seed, n_cams, seeded.data());
    cams0 = seeded.data();
  }
  (void)hipSetDevice(ctx->device);
  HostLayout L;
  st = build_layout(ctx, n_cams, n_pts, n_obs, cam_idx, pt_idx, meas,
                    opts->precision == POVAR_PREC_FP32_BULK, L);
  if (st != POVAR_OK) return st;
  auto* pb = new povar_problem_s();
  pb->ctx = ctx;
  pb->owned_by_ctx = true;
  ctx->live_problems += 1;
  st = problem_init(ctx, std::move(L), cams0, opts, ctx->stream, pb, nullptr, INT_MAX);
  if (st != POVAR_OK) {
    povar_problem_destroy(pb);
    return st;
  }
  *out = pb;
  return POVAR_OK;
} POVAR_HOST_CATCH(ctx)

povar_status povar_problem_create_device(povar_ctx ctx, int32_t n_cams, int32_t n_pts, int64_t n_obs,
                                         const int32_t* cam_idx, const int32_t* pt_idx, const double* meas,
                                         const double* cams0, const povar_options* opts, povar_problem* out) try {
  if (!ctx || !out) return POVAR_EINVAL;
  if (n_cams <= 0 || n_pts <= 0 || n_obs <= 0 || !cam_idx || !pt_idx || !meas) {
    set_error(ctx, "invalid sizes or NULL device pointers");
    return POVAR_EINVAL;
  }
  (void)hipSetDevice(ctx->device);
  std::vector<int32_t> c(n_obs), p(n_obs);
  std::vector<double> m(2 * n_obs), q(cams0 ? (size_t)n_cams * kCam : 0);
  HIP_TRY(ctx, hipMemcpyAsync(c.data(), cam_idx, n_obs * 4, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(p.data(), pt_idx, n_obs * 4, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(m.data(), meas, n_obs * 16, hipMemcpyDeviceToHost, ctx->stream));
  if (cams0) HIP_TRY(ctx, hipMemcpyAsync(q.data(), cams0, q.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return povar_problem_create(ctx, n_cams, n_pts, n_obs, c.data(), p.data(), m.data(),
                              cams0 ? q.data() : nullptr, opts, out);
} POVAR_HOST_CATCH(ctx)

povar_status povar_problem_destroy(povar_problem pb) {
  if (!pb) return POVAR_EINVAL;
  if (pb->ctx) (void)hipSetDevice(pb->ctx->device);
  if (pb->stream) (void)hipStreamSynchronize(pb->stream);
  if (pb->graph_exec) (void)hipGraphExecDestroy(pb->graph_exec);
  if (pb->graph_exec_k) (void)hipGraphExecDestroy(pb->graph_exec_k);
  for (auto ev : pb->events) (void)hipEventDestroy(ev);
  if (pb->arena) (void)hipFree(pb->arena);
  if (pb->arena2) (void)hipFree(pb->arena2);
  if (pb->ctx && pb->owned_by_ctx) pb->ctx->live_problems -= 1;
  delete pb;
  return POVAR_OK;
}

// Gradient norm of the report at the current cameras: the linearisation
// partials are those of the current cameras unless an accepted step has made
// them stale (then one linearisation pass refreshes them; the next step
// linearises again as it would have).  First stage only.
static povar_status report_grad_norm(povar_problem pb, double* out) {
  *out = NAN;
  if (pb->rec.stage != 1) return POVAR_OK;
  HIP_TRY(pb->ctx, launch_linearize(pb->batch, pb->fp32, 2, pb->stream));
  HIP_TRY(pb->ctx, launch_grad_norm(pb->batch, pb->stream));
  Ctl c;
  HIP_TRY(pb->ctx, read_ctl(pb, &c));
  *out = c.grad_norm;
  return POVAR_OK;
}

static povar_status run_iters(povar_problem pb, int32_t n, bool check_done, povar_report* report) {
  povar_ctx ctx = pb->ctx;
  (void)hipSetDevice(ctx->device);
  const auto t0 = std::chrono::steady_clock::now();
  Ctl c;
  HIP_TRY(ctx, read_ctl(pb, &c));
  int left = n;
  while (left > 0 && !c.done) {
    const int batch = check_done ? std::min(left, 4) : left;
    HIP_TRY(ctx, enqueue_iterations(pb, batch));
    left -= batch;
    HIP_TRY(ctx, read_ctl(pb, &c));
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (!report) return POVAR_OK;
  double gn;
  const povar_status st = report_grad_norm(pb, &gn);
  if (st != POVAR_OK) return st;
  fill_report(pb, c, secs, gn, report);
  return POVAR_OK;
}

povar_status povar_solve(povar_problem pb, povar_report* report) {
  if (!pb) return POVAR_EINVAL;
  Ctl c;
  HIP_TRY(pb->ctx, read_ctl(pb, &c));
  const int left = std::max(0, pb->opt.max_iters - c.iter);
  return run_iters(pb, left, pb->opt.ftol > 0.0, report);
}

povar_status povar_step(povar_problem pb, int32_t n_iters, povar_report* report) {
  if (!pb || n_iters < 0) return POVAR_EINVAL;
  return run_iters(pb, n_iters, pb->opt.ftol > 0.0, report);
}

povar_status povar_enqueue(povar_problem pb, int32_t n_iters) {
  if (!pb || n_iters < 0) return POVAR_EINVAL;
  (void)hipSetDevice(pb->ctx->device);
  HIP_TRY(pb->ctx, enqueue_iterations(pb, n_iters));
  return POVAR_OK;
}

povar_status povar_get_report(povar_problem pb, povar_report* report) {
  if (!pb || !report) return POVAR_EINVAL;
  (void)hipSetDevice(pb->ctx->device);
  double gn;
  const povar_status st = report_grad_norm(pb, &gn);
  if (st != POVAR_OK) return st;
  Ctl c;
  HIP_TRY(pb->ctx, read_ctl(pb, &c));
  fill_report(pb, c, 0.0, gn, report);
  return POVAR_OK;
}

povar_status povar_get_cameras(povar_problem pb, double* out) try {
  if (!pb || !out) return POVAR_EINVAL;
  Ctl c;
  HIP_TRY(pb->ctx, read_ctl(pb, &c));
  std::vector<double> tmp((size_t)pb->L.n_p * kCam);
  HIP_TRY(pb->ctx, hipMemcpyAsync(tmp.data(), pb->rec.P64[c.pcur], tmp.size() * 8, hipMemcpyDeviceToHost,
                                  pb->stream));
  HIP_TRY(pb->ctx, hipStreamSynchronize(pb->stream));
  cams_to_caller(pb->L, tmp.data(), out, kCam);
  return POVAR_OK;
} POVAR_HOST_CATCH(pb ? pb->ctx : nullptr)

povar_status povar_get_points(povar_problem pb, double* out) try {
  if (!pb || !out) return POVAR_EINVAL;
  Ctl c;
  HIP_TRY(pb->ctx, read_ctl(pb, &c));
  if (pb->rec.stage != 2) return copy_landmark_vec(pb, pb->rec.rec64[c.lcur], kRec, 4, 3, out);
  std::vector<double> h((size_t)pb->L.n_l * 4);
  const povar_status st = copy_landmark_vec(pb, pb->rec.rec64[c.lcur], kX2, 0, 4, h.data());
  if (st != POVAR_OK) return st;
  for (int32_t j = 0; j < pb->L.n_l; ++j)
    for (int k = 0; k < 3; ++k) out[(size_t)j * 3 + k] = h[(size_t)j * 4 + k] / h[(size_t)j * 4 + 3];
  return POVAR_OK;
} POVAR_HOST_CATCH(pb ? pb->ctx : nullptr)

povar_status povar_get_points_h(povar_problem pb, double* out) try {
  if (!pb || !out) return POVAR_EINVAL;
  Ctl c;
  HIP_TRY(pb->ctx, read_ctl(pb, &c));
  if (pb->rec.stage == 2) return copy_landmark_vec(pb, pb->rec.rec64[c.lcur], kX2, 0, 4, out);
  return copy_landmark_vec(pb, pb->rec.rec64[c.lcur], kRec, 4, 4, out);
} POVAR_HOST_CATCH(pb ? pb->ctx : nullptr)

povar_status povar_refine_create(povar_ctx ctx, int32_t n_cams, int32_t n_pts, int64_t n_obs,
                                 const int32_t* cam_idx, const int32_t* pt_idx, const double* meas,
                                 const double* cams0, const double* pts0, const povar_options* opts,
                                 povar_problem* out) try {
  if (!ctx || !out) return POVAR_EINVAL;
  *out = nullptr;
  povar_status st = check_options(ctx, opts);
  if (st != POVAR_OK) return st;
  if (!cams0 || !pts0) {
    set_error(ctx, "cams0 and pts0 must not be NULL");
    return POVAR_EINVAL;
  }
  if (opts->precision != POVAR_PREC_FP64 || opts->manifold != POVAR_MANIFOLD_SPHERE) {
    set_error(ctx, "the second stage runs in FP64 on the spheres");
    return POVAR_EINVAL;
  }
  (void)hipSetDevice(ctx->device);
  HostLayout L;
  st = build_layout(ctx, n_cams, n_pts, n_obs, cam_idx, pt_idx, meas, false, L);
  if (st != POVAR_OK) return st;
  auto* pb = new povar_problem_s();
  pb->ctx = ctx;
  pb->owned_by_ctx = true;
  ctx->live_problems += 1;
  st = problem_init(ctx, std::move(L), cams0, opts, ctx->stream, pb, nullptr, INT_MAX, pts0);
  if (st != POVAR_OK) {
    povar_problem_destroy(pb);
    return st;
  }
  *out = pb;
  return POVAR_OK;
} POVAR_HOST_CATCH(ctx)



povar_status povar_get_trace(povar_problem pb, int32_t n, double* cost, double* lam, int32_t* acc) {
  if (!pb || n < 0) return POVAR_EINVAL;
  Ctl c;
  HIP_TRY(pb->ctx, read_ctl(pb, &c));
  const int m = std::min(std::min(n, c.iter), pb->trace_cap);
  if (m == 0) return POVAR_OK;
  if (cost) HIP_TRY(pb->ctx, hipMemcpyAsync(cost, pb->rec.tr_cost, m * 8, hipMemcpyDeviceToHost, pb->stream));
  if (lam) HIP_TRY(pb->ctx, hipMemcpyAsync(lam, pb->rec.tr_lambda, m * 8, hipMemcpyDeviceToHost, pb->stream));
  if (acc) HIP_TRY(pb->ctx, hipMemcpyAsync(acc, pb->rec.tr_acc, m * 4, hipMemcpyDeviceToHost, pb->stream));
  HIP_TRY(pb->ctx, hipStreamSynchronize(pb->stream));
  return POVAR_OK;
}

povar_status povar_get_trace_diag(povar_problem pb, int32_t n, double* bl_norm, double* series_seconds) {
  if (!pb || n < 0) return POVAR_EINVAL;
  if (pb->rec.stage != 1) {
    set_error(pb->ctx, "povar_get_trace_diag is for first-stage problems");
    return POVAR_ESTATE;
  }
  Ctl c;
  HIP_TRY(pb->ctx, read_ctl(pb, &c));
  const int m = std::min(std::min(n, c.iter), pb->trace_cap);
  if (m == 0) return POVAR_OK;
  if (bl_norm) HIP_TRY(pb->ctx, hipMemcpyAsync(bl_norm, pb->rec.tr_bl, m * 8, hipMemcpyDeviceToHost, pb->stream));
  std::vector<double> ticks(m);
  HIP_TRY(pb->ctx, hipMemcpyAsync(ticks.data(), pb->rec.tr_series, m * 8, hipMemcpyDeviceToHost, pb->stream));
  HIP_TRY(pb->ctx, hipStreamSynchronize(pb->stream));
  if (series_seconds)
    for (int i = 0; i < m; ++i)
      series_seconds[i] = pb->ctx->clock_hz > 0.0 ? ticks[i] / pb->ctx->clock_hz : NAN;
  return POVAR_OK;
}

povar_status povar_get_state(povar_problem pb, double* cams, double* lambda, int32_t* iter, double* cost) try {
  if (!pb) return POVAR_EINVAL;
  Ctl c;
  HIP_TRY(pb->ctx, read_ctl(pb, &c));
  if (cams) {
    povar_status st = povar_get_cameras(pb, cams);
    if (st != POVAR_OK) return st;
  }
  if (lambda) *lambda = c.lambda;
  if (iter) *iter = c.iter;
  if (cost) *cost = c.cost;
  return POVAR_OK;
} POVAR_HOST_CATCH(pb ? pb->ctx : nullptr)

povar_status povar_set_state(povar_problem pb, const double* cams, double lambda, int32_t iter) try {
  if (!pb || !cams || !(lambda > 0.0) || iter < 0) return POVAR_EINVAL;
  if (pb->rec.stage == 2) {
    set_error(pb->ctx, "povar_set_state restores first-stage problems (their landmarks follow from the cameras)");
    return POVAR_ESTATE;
  }
  povar_ctx ctx = pb->ctx;
  (void)hipSetDevice(ctx->device);
  Ctl c;
  HIP_TRY(ctx, read_ctl(pb, &c));
  const int32_t n_p = pb->L.n_p;
  std::vector<double> P64((size_t)n_p * kCam);
  const int ss = ser_stride(n_p);
  std::vector<float> S32(pb->fp32 ? (size_t)n_p * ss : 0, 0.0f);
  std::vector<double> S64(pb->fp32 ? 0 : (size_t)n_p * ss, 0.0);
  for (int32_t i = 0; i < n_p; ++i) {
    const double* ci = cams + (size_t)pb->L.cam_int2ext[i] * kCam;   // caller's order
    double nrm = 0.0;
    for (int r = 0; r < kCam; ++r) nrm += ci[r] * ci[r];
    if (!(nrm > 0.0) || !std::isfinite(nrm)) {
      set_error(ctx, "camera %d is zero or not finite", pb->L.cam_int2ext[i]);
      return POVAR_EINVAL;
    }
    // cameras already on the sphere (to 1e-14) are taken bit-exactly, so a
    // state read by povar_get_state resumes bit-exactly
    const bool renorm = pb->opt.manifold == POVAR_MANIFOLD_SPHERE && std::fabs(nrm - 1.0) > 1e-14;
    const double s = renorm ? 1.0 / std::sqrt(nrm) : 1.0;
    for (int r = 0; r < kCam; ++r) {
      const double v = ci[r] * s;
      P64[(size_t)i * kCam + r] = v;
      if (pb->fp32) S32[(size_t)i * ss + r] = (float)v;
      else S64[(size_t)i * ss + r] = v;
    }
  }
  HIP_TRY(ctx, hipMemcpyAsync(pb->rec.P64[c.pcur], P64.data(), P64.size() * 8, hipMemcpyHostToDevice, pb->stream));
  if (pb->fp32)
    HIP_TRY(ctx, hipMemcpyAsync(pb->rec.S32[c.pcur], S32.data(), S32.size() * 4, hipMemcpyHostToDevice, pb->stream));
  else
    HIP_TRY(ctx, hipMemcpyAsync(pb->rec.S64[c.pcur], S64.data(), S64.size() * 8, hipMemcpyHostToDevice, pb->stream));
  HIP_TRY(ctx, hipStreamSynchronize(pb->stream));   // host buffers are freed on return
  c.lambda = lambda;
  c.iter = iter;
  c.need_lin = 1;
  c.done = 0;
  c.stop_reason = 0;
  c.status = 0;
  HIP_TRY(ctx, write_ctl(pb, &c));
  HIP_TRY(ctx, launch_landmark_solve(pb->batch, 2, pb->stream));
  HIP_TRY(ctx, launch_cost_groups(pb->batch, 0, pb->stream));
  HIP_TRY(ctx, launch_cost_finalize(pb->batch, 2, pb->stream));
  HIP_TRY(ctx, read_ctl(pb, &c));
  if (!std::isfinite(c.cost)) {
    set_error(ctx, "cost at the given cameras is not finite");
    return POVAR_ENUMERIC;
  }
  return POVAR_OK;
} POVAR_HOST_CATCH(pb ? pb->ctx : nullptr)

povar_status povar_debug_linearize(povar_problem pb, double* U, double* bp, double* g, double* Vp, double* X,
                                   double* z0, double* cost) try {
  if (!pb) return POVAR_EINVAL;
  if (pb->rec.stage == 2) {
    set_error(pb->ctx, "povar_debug_linearize is for first-stage problems; use povar_refine_debug_blocks");
    return POVAR_ESTATE;
  }
  povar_ctx ctx = pb->ctx;
  (void)hipSetDevice(ctx->device);
  Ctl c;
  HIP_TRY(ctx, read_ctl(pb, &c));
  if (c.done) {
    set_error(ctx, "problem has finished; linearisation hooks need a running problem");
    return POVAR_ESTATE;
  }
  HIP_TRY(ctx, launch_linearize(pb->batch, pb->fp32, 1, pb->stream));
  HIP_TRY(ctx, hipStreamSynchronize(pb->stream));
  const int32_t n_p = pb->L.n_p;
  std::vector<double> part((size_t)pb->L.n_ch * kLinVals);
  HIP_TRY(ctx, hipMemcpyAsync(part.data(), pb->rec.lin_part, part.size() * 8, hipMemcpyDeviceToHost, pb->stream));
  HIP_TRY(ctx, hipStreamSynchronize(pb->stream));
  const double a = 1.0 - pb->opt.eta;
  auto s4 = [](int c0, int d0) {
    const int lo = std::min(c0, d0), hi = std::max(c0, d0);
    return (lo * 7 - lo * lo) / 2 + hi;
  };
  for (int32_t i = 0; i < n_p; ++i) {
    const size_t e = (size_t)pb->L.cam_int2ext[i];   // caller's index of internal camera i
    // chunk partials of camera i added in chunk order, as the kernels do
    double q[kLinVals] = {0};
    for (int32_t ch = pb->L.cam_ch[i]; ch < pb->L.cam_ch[i + 1]; ++ch)
      for (int k = 0; k < kLinVals; ++k) q[k] += part[(size_t)ch * kLinVals + k];
    if (U)
      for (int r = 0; r < 12; ++r)
        for (int cc = 0; cc < 12; ++cc) {
          const int ar = r / 4, ac = cc / 4, k = s4(r % 4, cc % 4);
          double v;
          if (ar < 2 && ac < 2) v = ar == ac ? q[k] : 0.0;
          else if (ar == 2 && ac == 2) v = a * q[30 + k];
          else v = -a * q[(ar == 1 || ac == 1) ? 20 + k : 10 + k];
          U[e * 144 + r * 12 + cc] = v;
        }
    for (int r = 0; r < kCam; ++r) {
      if (bp) bp[e * kCam + r] = q[40 + r];
      if (g) g[e * kCam + r] = q[40 + r] - q[52 + r];
    }
  }
  if (Vp) {
    std::vector<double> v((size_t)pb->L.n_l * kLmSym);
    HIP_TRY(ctx, hipMemcpyAsync(v.data(), pb->rec.Vp64[c.lcur], v.size() * 8, hipMemcpyDeviceToHost, pb->stream));
    HIP_TRY(ctx, hipStreamSynchronize(pb->stream));
    static const int map9[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
    for (int32_t jj = 0; jj < pb->L.n_l; ++jj) {
      const int32_t j = pb->L.int2ext[jj];
      for (int k = 0; k < 9; ++k) Vp[(size_t)j * 9 + k] = v[(size_t)jj * kLmSym + map9[k]];
    }
  }
  if (X) {
    povar_status st = copy_landmark_vec(pb, pb->rec.rec64[c.lcur], kRec, 4, 3, X);
    if (st != POVAR_OK) return st;
  }
  if (z0) {
    povar_status st = copy_landmark_vec(pb, pb->rec.rec64[c.lcur], kRec, 0, 3, z0);
    if (st != POVAR_OK) return st;
  }
  if (cost) *cost = c.cost;
  return POVAR_OK;
} POVAR_HOST_CATCH(pb ? pb->ctx : nullptr)

povar_status povar_debug_step(povar_problem pb, double lambda, int32_t order, double* dp, double* p_trial,
                              double* cost_trial) try {
  if (!pb || !(lambda > 0.0) || order < 0) return POVAR_EINVAL;
  if (pb->rec.stage == 2) {
    set_error(pb->ctx, "povar_debug_step is for first-stage problems; use povar_refine_debug_step");
    return POVAR_ESTATE;
  }
  povar_ctx ctx = pb->ctx;
  (void)hipSetDevice(ctx->device);
  Ctl c;
  HIP_TRY(ctx, read_ctl(pb, &c));
  if (c.done) {
    set_error(ctx, "problem has finished; step hooks need a running problem");
    return POVAR_ESTATE;
  }
  const Ctl saved = c;
  c.lambda = lambda;
  c.order = order;
  c.status = 0;
  HIP_TRY(ctx, write_ctl(pb, &c));
  const Batch& B = pb->batch;
  HIP_TRY(ctx, launch_linearize(B, pb->fp32, 0, pb->stream));
  HIP_TRY(ctx, launch_camera_prep(B, pb->fp32, pb->stream));
  for (int t = 1; t <= order; ++t) {
    HIP_TRY(ctx, launch_series_landmark(B, pb->fp32, t, pb->stream));
    HIP_TRY(ctx, launch_series_camera(B, pb->fp32, t, pb->stream));
    if (pb->opt.series_rtol > 0.0 && t < order) HIP_TRY(ctx, launch_series_check(B, pb->fp32, t, pb->stream));
  }
  if (order == 0 || pb->opt.series_rtol > 0.0) HIP_TRY(ctx, launch_retract(B, pb->fp32, pb->stream));
  HIP_TRY(ctx, launch_landmark_solve(B, 1, pb->stream));
  HIP_TRY(ctx, launch_cost_groups(B, 1, pb->stream));
  HIP_TRY(ctx, launch_cost_finalize(B, 1, pb->stream));
  Ctl after;
  HIP_TRY(ctx, read_ctl(pb, &after));
  const int32_t n_p = pb->L.n_p;
  std::vector<double> tdp((size_t)n_p * kCam), tpt((size_t)n_p * kCam);
  HIP_TRY(ctx, hipMemcpyAsync(tdp.data(), pb->rec.acc, tdp.size() * 8, hipMemcpyDeviceToHost, pb->stream));
  HIP_TRY(ctx, hipMemcpyAsync(tpt.data(), pb->rec.P64[c.pcur ^ 1], tpt.size() * 8, hipMemcpyDeviceToHost,
                              pb->stream));
  HIP_TRY(ctx, hipStreamSynchronize(pb->stream));
  if (dp) cams_to_caller(pb->L, tdp.data(), dp, kCam);
  if (p_trial) cams_to_caller(pb->L, tpt.data(), p_trial, kCam);
  if (cost_trial) *cost_trial = after.cost_trial;
  Ctl restore = saved;
  restore.need_lin = 0;   // the linearisation at the current cameras is now in place
  restore.cost_trial = after.cost_trial;
  restore.status = saved.status;   // a failed hook step does not reject the next real step
  HIP_TRY(ctx, write_ctl(pb, &restore));
  if (after.status & 1) {
    set_error(ctx, "a damped camera block could not be factored at this damping");
    return POVAR_ENUMERIC;
  }
  return POVAR_OK;
} POVAR_HOST_CATCH(pb ? pb->ctx : nullptr)

povar_status povar_debug_camera_blocks(povar_problem pb, double lambda, double* K) try {
  if (!pb || !K || !(lambda > 0.0)) return POVAR_EINVAL;
  if (pb->rec.stage == 2) {
    set_error(pb->ctx, "povar_debug_camera_blocks is for first-stage problems; use povar_refine_debug_blocks");
    return POVAR_ESTATE;
  }
  povar_ctx ctx = pb->ctx;
  (void)hipSetDevice(ctx->device);
  Ctl c;
  HIP_TRY(ctx, read_ctl(pb, &c));
  if (c.done) {
    set_error(ctx, "problem has finished; camera-block hooks need a running problem");
    return POVAR_ESTATE;
  }
  const Ctl saved = c;
  c.lambda = lambda;
  c.status = 0;
  HIP_TRY(ctx, write_ctl(pb, &c));
  HIP_TRY(ctx, launch_linearize(pb->batch, pb->fp32, 0, pb->stream));
  HIP_TRY(ctx, launch_camera_prep(pb->batch, pb->fp32, pb->stream));
  Ctl after;
  HIP_TRY(ctx, read_ctl(pb, &after));
  std::vector<double> k((size_t)pb->L.n_p * kCamMat);
  HIP_TRY(ctx, hipMemcpyAsync(k.data(), pb->rec.K64, k.size() * 8, hipMemcpyDeviceToHost, pb->stream));
  HIP_TRY(ctx, hipStreamSynchronize(pb->stream));
  cams_to_caller(pb->L, k.data(), K, kCamMat);
  Ctl restore = saved;
  restore.need_lin = 0;   // the linearisation at the current cameras is in place
  HIP_TRY(ctx, write_ctl(pb, &restore));
  if (after.status & 1) {
    set_error(ctx, "a damped camera block could not be factored at this damping");
    return POVAR_ENUMERIC;
  }
  return POVAR_OK;
} POVAR_HOST_CATCH(pb ? pb->ctx : nullptr)

povar_status povar_debug_series(povar_problem pb, const double* x0, int32_t order, double* x_out) try {
  if (!pb || !x0 || !x_out || order < 0) return POVAR_EINVAL;
  if (pb->rec.stage == 2) {
    set_error(pb->ctx, "povar_debug_series is for first-stage problems");
    return POVAR_ESTATE;
  }
  povar_ctx ctx = pb->ctx;
  (void)hipSetDevice(ctx->device);
  Ctl c;
  HIP_TRY(ctx, read_ctl(pb, &c));
  if (c.done) {
    set_error(ctx, "problem has finished; series hooks need a running problem");
    return POVAR_ESTATE;
  }
  const int32_t n_p = pb->L.n_p;
  for (size_t k = 0; k < (size_t)n_p * kCam; ++k)
    if (!std::isfinite(x0[k])) {
      set_error(ctx, "x0 is not finite");
      return POVAR_EINVAL;
    }
  const Ctl saved = c;
  c.order = order;
  c.status = 0;
  HIP_TRY(ctx, write_ctl(pb, &c));
  const Batch& B = pb->batch;
  // the camera blocks K_i at the problem's damping (x_0 = -K g is replaced below)
  HIP_TRY(ctx, launch_linearize(B, pb->fp32, 0, pb->stream));
  HIP_TRY(ctx, launch_camera_prep(B, pb->fp32, pb->stream));
  // term 0: the caller's x0, in internal camera order, into the series
  // records (series precision) and the FP64 partial sum
  std::vector<double> xin((size_t)n_p * kCam);
  for (int32_t i = 0; i < n_p; ++i)
    std::memcpy(&xin[(size_t)i * kCam], x0 + (size_t)pb->L.cam_int2ext[i] * kCam, sizeof(double) * kCam);
  const size_t ss = (size_t)ser_stride(n_p);
  if (pb->fp32) {
    std::vector<float> xf(xin.size());
    for (size_t k = 0; k < xin.size(); ++k) xf[k] = (float)xin[k];
    HIP_TRY(ctx, hipMemcpy2DAsync(pb->rec.S32[c.pcur] + kSerX, ss * 4, xf.data(), kCam * 4, kCam * 4, n_p,
                                  hipMemcpyHostToDevice, pb->stream));
    HIP_TRY(ctx, hipStreamSynchronize(pb->stream));   // xf is freed at the end of this block
  } else {
    HIP_TRY(ctx, hipMemcpy2DAsync(pb->rec.S64[c.pcur] + kSerX, ss * 8, xin.data(), kCam * 8, kCam * 8, n_p,
                                  hipMemcpyHostToDevice, pb->stream));
  }
  HIP_TRY(ctx, hipMemcpyAsync(pb->rec.acc, xin.data(), xin.size() * 8, hipMemcpyHostToDevice, pb->stream));
  for (int t = 1; t <= order; ++t) {
    HIP_TRY(ctx, launch_series_landmark(B, pb->fp32, t, pb->stream));
    HIP_TRY(ctx, launch_series_camera(B, pb->fp32, t, pb->stream));
  }
  Ctl after;
  HIP_TRY(ctx, read_ctl(pb, &after));   // synchronises: xin may go
  std::vector<double> acc((size_t)n_p * kCam);
  HIP_TRY(ctx, hipMemcpyAsync(acc.data(), pb->rec.acc, acc.size() * 8, hipMemcpyDeviceToHost, pb->stream));
  HIP_TRY(ctx, hipStreamSynchronize(pb->stream));
  cams_to_caller(pb->L, acc.data(), x_out, kCam);
  Ctl restore = saved;
  restore.need_lin = 0;   // the linearisation at the current cameras is in place
  HIP_TRY(ctx, write_ctl(pb, &restore));
  if (after.status & 1) {
    set_error(ctx, "a damped camera block could not be factored at this damping");
    return POVAR_ENUMERIC;
  }
  return POVAR_OK;
} POVAR_HOST_CATCH(pb ? pb->ctx : nullptr)

// Second stage: the blocks at the current point for damping lambda.
povar_status povar_refine_debug_blocks(povar_problem pb, double lambda, double* U, double* bp, double* G,
                                       double* bl, double* cost) try {
  if (!pb || !(lambda > 0.0)) return POVAR_EINVAL;
  if (pb->rec.stage != 2) {
    set_error(pb->ctx, "povar_refine_debug_blocks needs a second-stage problem");
    return POVAR_ESTATE;
  }
  povar_ctx ctx = pb->ctx;
  (void)hipSetDevice(ctx->device);
  Ctl c;
  HIP_TRY(ctx, read_ctl(pb, &c));
  if (c.done) {
    set_error(ctx, "problem has finished; debug hooks need a running problem");
    return POVAR_ESTATE;
  }
  Ctl t = c;
  t.lambda = lambda;
  t.status = 0;
  HIP_TRY(ctx, write_ctl(pb, &t));
  const Batch& B = pb->batch;
  HIP_TRY(ctx, launch_refine_landmarks(B, pb->stream));
  HIP_TRY(ctx, launch_refine_cameras(B, pb->stream));
  HIP_TRY(ctx, launch_cost_groups(B, 0, pb->stream));
  HIP_TRY(ctx, launch_cost_finalize(B, 2, pb->stream));
  const int32_t n_p = pb->L.n_p, n_l = pb->L.n_l, n_ch = pb->L.n_ch;
  std::vector<double> lin((size_t)n_ch * kLin2), g2((size_t)n_l * kG2), bl2((size_t)n_l * 4);
  HIP_TRY(ctx, hipMemcpyAsync(lin.data(), pb->rec.lin2, lin.size() * 8, hipMemcpyDeviceToHost, pb->stream));
  HIP_TRY(ctx, hipMemcpyAsync(g2.data(), pb->rec.g2, g2.size() * 8, hipMemcpyDeviceToHost, pb->stream));
  HIP_TRY(ctx, hipMemcpyAsync(bl2.data(), pb->rec.bl2, bl2.size() * 8, hipMemcpyDeviceToHost, pb->stream));
  HIP_TRY(ctx, hipStreamSynchronize(pb->stream));
  Ctl after;
  HIP_TRY(ctx, read_ctl(pb, &after));
  // U_i (undamped) and b_p from the chunk sums: U[(a, c), (a2, c2)] is the
  // sum for the entry of d pi^T d pi in rows a, a2 times X_c X_c2
  auto sym = [](int a, int b) { return a <= b ? (a * 7 - a * a) / 2 + b : (b * 7 - b * b) / 2 + a; };
  auto gsel = [](int a, int b) {
    const int lo = std::min(a, b), hi = std::max(a, b);
    if (lo == hi) return lo == 2 ? 3 : 0;
    if (lo == 0 && hi == 1) return -1;
    return lo == 0 ? 1 : 2;
  };
  std::vector<double> Ui((size_t)n_p * kCamMat), bpi((size_t)n_p * kCam);
  for (int32_t i = 0; i < n_p; ++i) {
    double sum[kLin2] = {0};
    for (int32_t q = pb->L.cam_ch[i]; q < pb->L.cam_ch[i + 1]; ++q)
      for (int k = 0; k < kLin2; ++k) sum[k] += lin[(size_t)q * kLin2 + k];
    for (int r = 0; r < 12; ++r) {
      for (int cc = 0; cc < 12; ++cc) {
        const int gs = gsel(r >> 2, cc >> 2);
        Ui[(size_t)i * kCamMat + r * 12 + cc] = gs < 0 ? 0.0 : sum[gs * 10 + sym(r & 3, cc & 3)];
      }
      bpi[(size_t)i * kCam + r] = sum[40 + r];
    }
  }
  if (U) cams_to_caller(pb->L, Ui.data(), U, kCamMat);
  if (bp) cams_to_caller(pb->L, bpi.data(), bp, kCam);
  for (int32_t jj = 0; jj < n_l; ++jj) {
    const int32_t j = pb->L.int2ext[jj];
    const double* o = g2.data() + (size_t)jj * kG2;
    for (int a = 0; a < 4; ++a) {
      for (int b = 0; b < 4; ++b)
        if (G) G[(size_t)j * 16 + a * 4 + b] = o[sym(a, b)];
      if (bl) bl[(size_t)j * 4 + a] = bl2[(size_t)jj * 4 + a];
    }
  }
  if (cost) *cost = after.cost;
  Ctl restore = c;
  HIP_TRY(ctx, write_ctl(pb, &restore));
  return POVAR_OK;
} POVAR_HOST_CATCH(pb ? pb->ctx : nullptr)

// Second stage: one step at damping lambda and series order `order`.
povar_status povar_refine_debug_step(povar_problem pb, double lambda, int32_t order, double* dp, double* p_trial,
                                     double* x_trial, double* cost_trial) try {
  if (!pb || !(lambda > 0.0) || order < 0) return POVAR_EINVAL;
  if (pb->rec.stage != 2) {
    set_error(pb->ctx, "povar_refine_debug_step needs a second-stage problem");
    return POVAR_ESTATE;
  }
  povar_ctx ctx = pb->ctx;
  (void)hipSetDevice(ctx->device);
  Ctl c;
  HIP_TRY(ctx, read_ctl(pb, &c));
  if (c.done) {
    set_error(ctx, "problem has finished; debug hooks need a running problem");
    return POVAR_ESTATE;
  }
  Ctl t = c;
  t.lambda = lambda;
  t.order = order;
  t.status = 0;
  HIP_TRY(ctx, write_ctl(pb, &t));
  const Batch& B = pb->batch;
  HIP_TRY(ctx, launch_refine_landmarks(B, pb->stream));
  HIP_TRY(ctx, launch_refine_cameras(B, pb->stream));
  HIP_TRY(ctx, launch_refine_step(B, order, pb->opt.series_rtol > 0.0, pb->stream));
  HIP_TRY(ctx, launch_cost_groups(B, 1, pb->stream));
  HIP_TRY(ctx, launch_cost_finalize(B, 1, pb->stream));
  Ctl after;
  HIP_TRY(ctx, read_ctl(pb, &after));
  const int32_t n_p = pb->L.n_p;
  std::vector<double> tdp((size_t)n_p * kCam), tpt((size_t)n_p * kCam);
  HIP_TRY(ctx, hipMemcpyAsync(tdp.data(), pb->rec.acc, tdp.size() * 8, hipMemcpyDeviceToHost, pb->stream));
  HIP_TRY(ctx, hipMemcpyAsync(tpt.data(), pb->rec.P64[c.pcur ^ 1], tpt.size() * 8, hipMemcpyDeviceToHost,
                              pb->stream));
  HIP_TRY(ctx, hipStreamSynchronize(pb->stream));
  if (dp) cams_to_caller(pb->L, tdp.data(), dp, kCam);
  if (p_trial) cams_to_caller(pb->L, tpt.data(), p_trial, kCam);
  if (x_trial) {
    const povar_status st = copy_landmark_vec(pb, pb->rec.rec64[c.lcur ^ 1], kX2, 0, 4, x_trial);
    if (st != POVAR_OK) return st;
  }
  if (cost_trial) *cost_trial = after.cost_trial;
  Ctl restore = c;
  restore.cost_trial = after.cost_trial;
  restore.status = c.status;   // a failed hook step does not reject the next real step
  HIP_TRY(ctx, write_ctl(pb, &restore));
  if (after.status & 1) {
    set_error(ctx, "a damped block could not be factored at this damping");
    return POVAR_ENUMERIC;
  }
  return POVAR_OK;
} POVAR_HOST_CATCH(pb ? pb->ctx : nullptr)

povar_status povar_kernel_timing(povar_problem pb, int32_t enable) {
  if (!pb) return POVAR_EINVAL;
  (void)hipSetDevice(pb->ctx->device);
  if (!enable) HIP_TRY(pb->ctx, pb->drain_timing());
  pb->timing = enable != 0;
  return POVAR_OK;
}

povar_status povar_kernel_times(povar_problem pb, double* ms_l, int64_t* n_l, double* ms_c, int64_t* n_c) {
  if (!pb) return POVAR_EINVAL;
  (void)hipSetDevice(pb->ctx->device);
  HIP_TRY(pb->ctx, pb->drain_timing());
  if (ms_l) *ms_l = pb->ms_kernel[0];
  if (n_l) *n_l = pb->n_kernel[0];
  if (ms_c) *ms_c = pb->ms_kernel[1];
  if (n_c) *n_c = pb->n_kernel[1];
  pb->ms_kernel[0] = pb->ms_kernel[1] = 0.0;
  pb->n_kernel[0] = pb->n_kernel[1] = 0;
  return POVAR_OK;
}

povar_status povar_problem_info(povar_problem pb, int64_t* n_obs, int64_t* n_packets, int32_t* n_chunks,
                                uint64_t* device_bytes) {
  if (!pb) return POVAR_EINVAL;
  if (n_obs) *n_obs = pb->L.n_obs;
  if (n_packets) *n_packets = pb->L.n_pk;
  if (n_chunks) *n_chunks = pb->L.n_ch;
  if (device_bytes) *device_bytes = pb->bytes;
  return POVAR_OK;
}

povar_status povar_debug_layout_check(int32_t n_cams, int32_t n_pts, int64_t n_obs, const int32_t* cam_idx,
                                      const int32_t* pt_idx, const double* meas, int32_t precision,
                                      int64_t* out) try {
  if (precision != POVAR_PREC_FP64 && precision != POVAR_PREC_FP32_BULK) {
    set_error(nullptr, "precision must be POVAR_PREC_FP64 or POVAR_PREC_FP32_BULK");
    return POVAR_EINVAL;
  }
  const bool fp32 = precision == POVAR_PREC_FP32_BULK;
  HostLayout L;
  const povar_status st = build_layout(nullptr, n_cams, n_pts, n_obs, cam_idx, pt_idx, meas, fp32, L);
  if (st != POVAR_OK) return st;
  return check_layout(L, cam_idx, pt_idx, meas, fp32, out);
} POVAR_HOST_CATCH(nullptr)

povar_status povar_problem_layout(povar_problem pb, int32_t* blocked, int32_t* lm_block, int64_t* n_slots,
                                  int64_t* n_runs, int32_t* coop_gather) {
  if (!pb) return POVAR_EINVAL;
  if (coop_gather) *coop_gather = pb->batch.coop_cams;
  if (blocked) *blocked = pb->L.blocked;
  if (lm_block) *lm_block = pb->L.lm_block;
  if (n_slots) *n_slots = pb->L.blocked ? pb->L.n_cs : 0;
  if (n_runs) *n_runs = pb->L.blocked ? pb->L.n_runs : 0;
  return POVAR_OK;
}

}  // extern "C"
