// Serving runtime for many live acquisitions on one GPU.
//
// Each acquisition is a plan whose spectrum stays resident in HBM.  Acquisitions are
// admitted while the sum of their plans' device memory fits the budget.  Frames are
// submitted as device addresses and queued per acquisition; every scheduling step
// takes whatever frames have arrived (continuous batching), pushes them in batches
// on the acquisition's own stream - so the work of different acquisitions overlaps on
// the device - and then snapshots the acquisitions that are due, with the Wiener
// reduction fused into the last push where the update allows it.  Every frame's
// submit-to-snapshot latency is recorded.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "wdd_internal.h"

namespace {

double now_us() {
  using namespace std::chrono;
  return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

struct Pending {
  uint64_t addr;
  int32_t y, x;
  double t_submit;
};

struct Acq {
  int32_t id = 0;
  wdd_plan_t plan = nullptr;
  int64_t bytes = 0;
  int32_t batch = 0;
  size_t frame_bytes = 0;
  std::deque<Pending> pending;
  std::vector<double> awaiting;  // submit times of frames pushed but not yet in a snapshot
  double last_snapshot = -1e300;
  uint64_t frames_done = 0;
};

}  // namespace

// Host tables keyed by everything they depend on; acquisitions of a repeated geometry
// skip the FP64 table build.
struct TableKey {
  double radius, center_y, center_x, defocus, amplitude, step, eps_rel, sigma;
  int32_t sy, sx, ny, nx, dtype, k, precision, basis;
  bool operator<(const TableKey& o) const {
    return std::memcmp(this, &o, sizeof(TableKey)) < 0;
  }
};

struct wdd_server_s {
  wdd_server_options opts;
  std::map<TableKey, std::shared_ptr<wdd_tables_s>> tables;
  size_t table_bytes = 0;
  int64_t used = 0;
  int32_t next_id = 1;
  std::map<int32_t, Acq*> acqs;
  std::vector<double> latency_us;  // one entry per frame that reached a snapshot
  uint64_t frames = 0, batches = 0, snapshots = 0, steps = 0;
  std::vector<uint64_t> addr_buf;
  std::vector<int32_t> pos_buf;
};

namespace {

wdd_status find(wdd_server_s* s, int32_t id, Acq** a) {
  if (!s) return wdd::fail(WDD_EINVAL, "null server");
  auto it = s->acqs.find(id);
  if (it == s->acqs.end()) return wdd::fail(WDD_EINVAL, "no open acquisition %d", id);
  *a = it->second;
  return WDD_OK;
}

// Pushes every pending frame of `a` in batches of at most a->batch; the last batch
// carries the fused Wiener reduction when `snapshot_due`.  Returns whether that happened.
wdd_status drain(wdd_server_s* s, Acq* a, bool snapshot_due, bool* fused) {
  *fused = false;
  while (!a->pending.empty()) {
    const int32_t n = (int32_t)std::min<size_t>(a->pending.size(), (size_t)a->batch);
    s->addr_buf.resize(n);
    s->pos_buf.resize(2 * (size_t)n);
    for (int32_t i = 0; i < n; ++i) {
      const Pending& pf = a->pending[i];
      s->addr_buf[i] = pf.addr;
      s->pos_buf[2 * i] = pf.y;
      s->pos_buf[2 * i + 1] = pf.x;
    }
    const bool last = (size_t)n == a->pending.size();
    bool f = false;
    wdd_status st = wdd::push_table(a->plan, s->addr_buf.data(), s->pos_buf.data(), n, last && snapshot_due, &f);
    if (st != WDD_OK) return st;
    for (int32_t i = 0; i < n; ++i) {
      a->awaiting.push_back(a->pending.front().t_submit);
      a->pending.pop_front();
    }
    a->frames_done += (uint64_t)n;
    s->frames += (uint64_t)n;
    s->batches += 1;
    if (last) *fused = f;
  }
  return WDD_OK;
}

}  // namespace

extern "C" {

wdd_status wdd_server_default_options(wdd_server_options* o) {
  if (!o) return wdd::fail(WDD_EINVAL, "null options");
  o->hbm_budget_bytes = (int64_t)1 << 30;
  o->snapshot_interval_us = 1000.0;
  o->batch_frames = 256;
  return WDD_OK;
}

wdd_status wdd_server_create(const wdd_server_options* opts, wdd_server_t* out) {
  if (!out) return wdd::fail(WDD_EINVAL, "null output handle");
  *out = nullptr;
  wdd_server_s* s = new (std::nothrow) wdd_server_s();
  if (!s) return wdd::fail(WDD_ENOMEM, "out of host memory");
  wdd_server_default_options(&s->opts);
  if (opts) s->opts = *opts;
  if (s->opts.batch_frames < 1 || !(s->opts.snapshot_interval_us >= 0)) {
    delete s;
    return wdd::fail(WDD_EINVAL, "batch_frames must be >= 1 and the snapshot interval >= 0");
  }
  *out = s;
  return WDD_OK;
}

wdd_status wdd_server_open(wdd_server_t s, const wdd_probe* probe, const wdd_scan* scan, const wdd_detector* det,
                           int32_t K, const wdd_options* opts_in, int32_t* acq_id) {
  if (!s || !acq_id) return wdd::fail(WDD_EINVAL, "null argument");
  *acq_id = 0;
  wdd_options opts;
  wdd_default_options(&opts);
  if (opts_in) opts = *opts_in;
  opts.max_batch = std::max(opts.max_batch, s->opts.batch_frames);
  wdd_status st = wdd::check_plan_options(det, opts);
  if (st != WDD_OK) return st;
  TableKey key;
  std::memset(&key, 0, sizeof(key));
  key.radius = probe->radius_px; key.defocus = probe->defocus_edge_rad; key.amplitude = probe->amplitude;
  key.center_y = probe->center_y; key.center_x = probe->center_x; key.basis = opts.basis;
  key.step = scan->step_px; key.eps_rel = opts.eps_rel; key.sigma = opts.sigma_px;
  key.sy = scan->sy; key.sx = scan->sx; key.ny = det->ny; key.nx = det->nx; key.dtype = det->dtype; key.k = K;
  key.precision = opts.precision;
  std::shared_ptr<wdd_tables_s> tp;
  auto it = s->tables.find(key);
  if (it != s->tables.end()) {
    tp = it->second;
  } else {
    try {
      tp = std::make_shared<wdd_tables_s>();
      if ((st = wdd::build_tables(probe, scan, det, K, &opts, tp.get())) != WDD_OK) return st;
    } catch (const std::bad_alloc&) {
      return wdd::fail(WDD_ENOMEM, "out of host memory");
    }
    const size_t tb = tp->w.size() * sizeof(double) + tp->freqs.size() * sizeof(int32_t);
    if (s->table_bytes + tb > ((size_t)4 << 30)) {  // keep at most 4 GiB of cached host tables
      s->tables.clear();
      s->table_bytes = 0;
    }
    s->tables[key] = tp;
    s->table_bytes += tb;
  }
  const wdd_tables_s& t = *tp;
  const int64_t need = wdd::plan_device_bytes(t, opts, det->dtype);
  if (s->opts.hbm_budget_bytes > 0 && s->used + need > s->opts.hbm_budget_bytes)
    return wdd::fail(WDD_EBUSY, "acquisition needs %lld bytes; %lld of %lld in use", (long long)need,
                     (long long)s->used, (long long)s->opts.hbm_budget_bytes);
  Acq* a = new (std::nothrow) Acq();
  if (!a) return wdd::fail(WDD_ENOMEM, "out of host memory");
  st = wdd::plan_create_from_tables(tp, probe, scan, det, opts, nullptr, &a->plan);
  if (st != WDD_OK) {
    delete a;
    return st;
  }
  wdd_plan_info info;
  wdd_plan_get_info(a->plan, &info);
  a->id = s->next_id++;
  a->bytes = std::max<int64_t>(need, info.device_bytes);
  a->batch = s->opts.batch_frames;
  a->frame_bytes = (size_t)det->ny * det->nx * (det->dtype == WDD_U16 ? 2 : 4);
  s->used += a->bytes;
  s->acqs[a->id] = a;
  *acq_id = a->id;
  return WDD_OK;
}

wdd_status wdd_server_submit(wdd_server_t s, int32_t acq, const void* frames, const int32_t* pos_yx, int32_t n) {
  Acq* a = nullptr;
  wdd_status st = find(s, acq, &a);
  if (st != WDD_OK) return st;
  if (n < 0) return wdd::fail(WDD_EINVAL, "n < 0");
  if (n == 0) return WDD_OK;
  if (!frames || !pos_yx) return wdd::fail(WDD_EINVAL, "null frames or positions");
  if (reinterpret_cast<uintptr_t>(frames) % 16 != 0) return wdd::fail(WDD_EINVAL, "frames must be 16-byte aligned");
  int32_t sy = 0, sx = 0;
  if ((st = wdd::plan_scan_shape(a->plan, &sy, &sx)) != WDD_OK) return st;
  for (int32_t i = 0; i < n; ++i) {
    const int32_t y = pos_yx[2 * i], x = pos_yx[2 * i + 1];
    if (y < 0 || y >= sy || x < 0 || x >= sx)
      return wdd::fail(WDD_ERANGE, "position %d = (%d, %d) outside the %d x %d raster", i, y, x, sy, sx);
  }
  const double t = now_us();
  const uint64_t base = reinterpret_cast<uint64_t>(frames);
  for (int32_t i = 0; i < n; ++i)
    a->pending.push_back({base + (uint64_t)i * a->frame_bytes, pos_yx[2 * i], pos_yx[2 * i + 1], t});
  return WDD_OK;
}

wdd_status wdd_server_step(wdd_server_t s, int32_t* frames_processed) {
  if (!s) return wdd::fail(WDD_EINVAL, "null server");
  const uint64_t before = s->frames;
  const double t = now_us();
  std::vector<std::pair<Acq*, bool>> snap;  // acquisitions to snapshot, and whether the reduction was fused
  for (auto& kv : s->acqs) {
    Acq* a = kv.second;
    const bool due = (t - a->last_snapshot) >= s->opts.snapshot_interval_us;
    const bool had = !a->pending.empty();
    bool fused = false;
    wdd_status st = drain(s, a, due, &fused);
    if (st != WDD_OK) return st;
    if (due && (had || !a->awaiting.empty())) snap.emplace_back(a, fused);
  }
  for (auto& sp : snap) {
    wdd_status st = wdd::snapshot_enqueue(sp.first->plan, !sp.second);
    if (st != WDD_OK) return st;
  }
  for (auto& sp : snap) {
    Acq* a = sp.first;
    wdd_status st = wdd::snapshot_finish(a->plan, nullptr);
    if (st != WDD_OK) return st;
    const double done = now_us();
    for (double ts : a->awaiting) s->latency_us.push_back(done - ts);
    a->awaiting.clear();
    a->last_snapshot = done;
    s->snapshots += 1;
  }
  s->steps += 1;
  if (frames_processed) *frames_processed = (int32_t)(s->frames - before);
  return WDD_OK;
}

wdd_status wdd_server_snapshot(wdd_server_t s, int32_t acq, float* out, uint64_t* frames_seen) {
  Acq* a = nullptr;
  wdd_status st = find(s, acq, &a);
  if (st != WDD_OK) return st;
  if (!out) return wdd::fail(WDD_EINVAL, "null output");
  bool fused = false;
  if ((st = drain(s, a, true, &fused)) != WDD_OK) return st;
  if ((st = wdd::snapshot_enqueue(a->plan, !fused)) != WDD_OK) return st;
  if ((st = wdd::snapshot_finish(a->plan, frames_seen)) != WDD_OK) return st;
  const double done = now_us();
  for (double ts : a->awaiting) s->latency_us.push_back(done - ts);
  a->awaiting.clear();
  a->last_snapshot = done;
  s->snapshots += 1;
  float* buf = nullptr;
  if ((st = wdd_snapshot_buffer(a->plan, &buf)) != WDD_OK) return st;
  int32_t sy = 0, sx = 0;
  if ((st = wdd::plan_scan_shape(a->plan, &sy, &sx)) != WDD_OK) return st;
  std::memcpy(out, buf, (size_t)sy * sx * 2 * sizeof(float));
  return WDD_OK;
}

wdd_status wdd_server_acq_shape(wdd_server_t s, int32_t acq, int32_t* sy, int32_t* sx) {
  Acq* a = nullptr;
  wdd_status st = find(s, acq, &a);
  if (st != WDD_OK) return st;
  return wdd::plan_scan_shape(a->plan, sy, sx);
}

wdd_status wdd_server_close(wdd_server_t s, int32_t acq) {
  Acq* a = nullptr;
  wdd_status st = find(s, acq, &a);
  if (st != WDD_OK) return st;
  wdd_destroy(a->plan);
  s->used -= a->bytes;
  s->acqs.erase(acq);
  delete a;
  return WDD_OK;
}

wdd_status wdd_server_get_stats(wdd_server_t s, wdd_server_stats* out) {
  if (!s || !out) return wdd::fail(WDD_EINVAL, "null argument");
  *out = wdd_server_stats{};
  out->frames = s->frames;
  out->batches = s->batches;
  out->snapshots = s->snapshots;
  out->steps = s->steps;
  out->open = (int32_t)s->acqs.size();
  out->device_bytes = s->used;
  int64_t pending = 0;
  for (auto& kv : s->acqs) pending += (int64_t)kv.second->pending.size();
  out->pending_frames = pending;
  out->latency_samples = (int64_t)s->latency_us.size();
  if (!s->latency_us.empty()) {
    std::vector<double> v = s->latency_us;
    auto pct = [&v](double q) {
      const size_t k = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
      std::nth_element(v.begin(), v.begin() + k, v.end());
      return v[k];
    };
    out->latency_p50_us = pct(0.50);
    out->latency_p99_us = pct(0.99);
    out->latency_max_us = *std::max_element(v.begin(), v.end());
  }
  return WDD_OK;
}

wdd_status wdd_server_destroy(wdd_server_t s) {
  if (!s) return WDD_OK;
  for (auto& kv : s->acqs) {
    wdd_destroy(kv.second->plan);
    delete kv.second;
  }
  delete s;
  return WDD_OK;
}

}  // extern "C"
