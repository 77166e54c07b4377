// Serving runtime for many live acquisitions on one GPU.
//
// Each acquisition is a plan whose spectrum stays resident in HBM.  Acquisitions are
// admitted while the sum of their plans' device memory fits the budget; the FP64 tables,
// the plan's allocations and the upload of W are made on a worker thread, so that opening
// a large acquisition does not stall the scheduling of the others.  Frames are submitted
// as device addresses and queued per acquisition; every scheduling step takes whatever
// frames have arrived (continuous batching) and snapshots the acquisitions that are due.
//
// Hermite-Gauss acquisitions are pushed together: one round takes up to one batch of every
// such acquisition and projects all of them in one launch (per frame type and arithmetic);
// per row pass, one launch updates every object-order spectrum (the live form of the
// modified-WDD algorithm, D updated per frame; its work list covers every (acquisition,
// row pass, chunk of kept frequencies)), and two launches (row DFTs, then A updates) every
// spectrum-order one.  That projection launch also brings the round's descriptors to the
// device from pinned host memory.  Optionally the round's launches are captured once as a
// HIP graph and replayed with updated arguments.  Fourier-basis acquisitions are pushed
// through their plans on their own streams.  Every frame's submit-to-snapshot latency is
// recorded.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "plan.h"

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
  wdd_plan_t plan = nullptr;  // set once the worker has finished (ready)
  int64_t bytes = 0;
  int32_t batch = 0;
  size_t frame_bytes = 0;
  int32_t sy = 0, sx = 0;
  bool grouped = false;  // pushed in the grouped launches on the server's stream
  std::deque<Pending> pending;
  std::vector<double> awaiting;  // submit times of frames pushed but not yet in a snapshot
  double last_snapshot = -1e300;
  bool fused = false;  // grouped spectrum order: the last round reduced D (no Wiener launch needed)
  // a scheduled snapshot still running on the device (wdd_server_step does not wait for
  // it; a later call sees its event complete and records the latencies of its frames)
  hipEvent_t snap_ev = nullptr;
  bool snap_inflight = false;
  std::vector<double> inflight;
  uint64_t frames_done = 0;
  // opening on a worker thread
  std::thread worker;
  std::atomic<bool> done{false};
  wdd_status open_status = WDD_OK;
  std::string open_error;
  wdd_plan_t made = nullptr;
};

constexpr int kRing = 4;  // pinned descriptor blocks of grouped rounds in flight

size_t align16(size_t n) { return (n + 15) / 16 * 16; }

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

// The cache is shared by every server of the process (and their workers).
struct TableCache {
  std::mutex mu;
  std::map<TableKey, std::shared_ptr<wdd_tables_s>> tables;
  size_t bytes = 0;
};
TableCache& table_cache() {
  static TableCache c;
  return c;
}

// An acquisition being closed on a worker thread (freeing a plan's memory waits for the
// device and takes milliseconds); its bytes stay counted against the budget until it is done.
struct Closer {
  std::thread th;
  std::atomic<bool> done{false};
  int64_t bytes = 0;
};

struct wdd_server_s {
  wdd_server_options opts;
  int device = 0;
  std::vector<std::unique_ptr<Closer>> closers;
  hipStream_t stream = nullptr;  // the grouped acquisitions' stream
  int64_t used = 0;
  int32_t next_id = 1;
  std::map<int32_t, Acq*> acqs;
  std::vector<double> latency_us;  // one entry per frame that reached a snapshot
  uint64_t frames = 0, batches = 0, snapshots = 0, steps = 0, group_rounds = 0, graph_replays = 0;
  std::vector<uint64_t> addr_buf;
  std::vector<int32_t> pos_buf;
  // grouped rounds: pinned descriptor blocks (ring) and their device copy
  char* pin[kRing] = {};
  size_t pin_cap[kRing] = {};
  hipEvent_t ring_ev[kRing] = {};
  bool ring_live[kRing] = {};
  int ring = 0;
  char* blk = nullptr;
  size_t blk_cap = 0;
  // the captured round and the shape it was captured for
  hipGraphExec_t exec = nullptr;
  // held by a closer thread while it frees device memory: a round is captured only while the
  // scheduling thread can take it at once, so that no free runs during a capture
  std::mutex free_mu;
  bool failed = false;
};

namespace {

wdd_status hip_fail(wdd_server_s* s, hipError_t e, const char* what) {
  s->failed = true;
  (void)hipGetLastError();
  return wdd::fail(WDD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SRV_HIP(s, call)                                 \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail((s), e_, #call); \
  } while (0)

wdd_status find(wdd_server_s* s, int32_t id, Acq** a) {
  if (!s) return wdd::fail(WDD_EINVAL, "null server");
  if (s->failed) return wdd::fail(WDD_ESTATE, "server is unusable after an earlier device error");
  auto it = s->acqs.find(id);
  if (it == s->acqs.end()) return wdd::fail(WDD_EINVAL, "no open acquisition %d", id);
  *a = it->second;
  return WDD_OK;
}

// Takes the result of a finished worker (wait: join it first even if it has not finished).
// An acquisition whose opening failed reports that error from then on.
wdd_status settle_open(wdd_server_s* s, Acq* a, bool wait) {
  if (a->worker.joinable()) {
    if (!wait && !a->done.load(std::memory_order_acquire)) return WDD_OK;
    a->worker.join();
    if (a->open_status == WDD_OK) {
      a->plan = a->made;
      wdd_plan_info info;
      wdd_plan_get_info(a->plan, &info);
      const int64_t b = std::max<int64_t>(a->bytes, info.device_bytes);
      s->used += b - a->bytes;
      a->bytes = b;
    }
  }
  if (a->open_status != WDD_OK) return wdd::fail(a->open_status, "opening acquisition %d failed: %s", a->id,
                                                 a->open_error.c_str());
  return WDD_OK;
}

bool ready(const Acq* a) { return a->plan != nullptr; }

// Pushes every pending frame of `a` through its plan in batches of at most a->batch; the
// last batch carries the fused Wiener reduction when `snapshot_due`.  Returns whether
// that happened.
wdd_status drain_plan(wdd_server_s* s, Acq* a, bool snapshot_due, bool* fused) {
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

// One member of a grouped round: its frames (up to one batch) grouped by scan row.
struct Member {
  Acq* a;
  wdd_plan_s* p;
  int32_t n;
  bool spectrum;            // spectrum order (A resident): row DFT + A update per pass
  bool display;             // a snapshot follows: object order leaves the display's first pass
                            // in the partial rows, spectrum order fuses the Wiener reduction
  size_t first_frame;       // offset of its frames in the round's order / xs / address arrays
  size_t first_row;         // offset of its rows in the round's row array
  int32_t nrows;
  bool in_order;
};

// A grouped round ready to launch: the descriptors in a pinned ring slot, and where its
// pieces sit in the device copy.
struct Round {
  struct PassRef {
    int32_t member, k, row0, nrows;
  };
  std::vector<PassRef> passes;   // object-order passes, sorted by k
  std::vector<size_t> item0;     // first work item of each pass
  std::vector<PassRef> spasses;  // spectrum-order passes, sorted by k
  std::vector<int32_t> dft_first, upd_first;  // first workgroup of each within its k's launch
  std::vector<int32_t> dft_total, upd_total;  // per k: workgroups of its launches
  char* hb = nullptr;            // pinned block
  char* db = nullptr;            // its device copy
  size_t dev_bytes = 0, off_items = 0, off_spass = 0, off_dft = 0, off_upd = 0;
  const uint64_t* ftab = nullptr;  // frame addresses (pinned)
  int slot = 0;
};

// Builds the descriptors of one grouped round (every member's frames, up to one batch,
// grouped by scan row; row passes of at most kFactorRows rows; one work item per pass and
// chunk of kept frequencies) in the next pinned ring slot, growing the device block when
// needed.  No launch: it may wait for the stream, so it runs before any capture.
wdd_status prepare_round(wdd_server_s* s, std::vector<Member>& ms, Round* rd) {
  std::vector<int4> rows;
  std::vector<int32_t> order, xs;
  std::vector<uint64_t> addrs;
  try {
    for (int32_t mi = 0; mi < (int32_t)ms.size(); ++mi) {
      Member& m = ms[mi];
      m.first_frame = order.size();
      m.first_row = rows.size();
      std::vector<int32_t> idx(m.n);
      for (int32_t i = 0; i < m.n; ++i) idx[i] = i;
      const std::deque<Pending>& q = m.a->pending;
      std::stable_sort(idx.begin(), idx.end(), [&q](int32_t u, int32_t v) { return q[u].y < q[v].y; });
      m.in_order = true;
      for (int32_t i = 0; i < m.n; ++i) {
        const Pending& pf = q[idx[i]];
        m.in_order = m.in_order && idx[i] == i;
        if (rows.size() == m.first_row || rows.back().x != pf.y) rows.push_back(make_int4(pf.y, i, 0, 0));
        rows.back().z += 1;
        order.push_back(idx[i]);
        xs.push_back(pf.x);
      }
      for (int32_t i = 0; i < m.n; ++i) addrs.push_back(q[i].addr);
      m.nrows = (int32_t)(rows.size() - m.first_row);
      std::vector<Round::PassRef>& list = m.spectrum ? rd->spasses : rd->passes;
      for (int32_t r = 0, k = 0; r < m.nrows; r += wdd::kFactorRows, ++k)
        list.push_back({mi, k, r, std::min<int32_t>(wdd::kFactorRows, m.nrows - r)});
    }
  } catch (const std::bad_alloc&) {
    return wdd::fail(WDD_ENOMEM, "out of host memory");
  }
  auto by_k = [](const Round::PassRef& u, const Round::PassRef& v) { return u.k < v.k; };
  std::vector<Round::PassRef>& passes = rd->passes;
  std::stable_sort(passes.begin(), passes.end(), by_k);
  std::vector<Round::PassRef>& spasses = rd->spasses;
  std::stable_sort(spasses.begin(), spasses.end(), by_k);
  rd->item0.assign(passes.size() + 1, 0);
  for (size_t i = 0; i < passes.size(); ++i) rd->item0[i + 1] = rd->item0[i] + ms[passes[i].member].p->host_chunks.size();
  const size_t nitems = rd->item0.back();
  // spectrum-order passes: workgroup offsets within the launch of their k
  const int32_t kmax_s = spasses.empty() ? -1 : spasses.back().k;
  rd->dft_first.assign(spasses.size(), 0);
  rd->upd_first.assign(spasses.size(), 0);
  rd->dft_total.assign((size_t)(kmax_s + 1), 0);
  rd->upd_total.assign((size_t)(kmax_s + 1), 0);
  for (size_t i = 0; i < spasses.size(); ++i) {
    const wdd_plan_s* p = ms[spasses[i].member].p;
    const int32_t k = spasses[i].k;
    rd->dft_first[i] = rd->dft_total[k];
    rd->upd_first[i] = rd->upd_total[k];
    rd->dft_total[k] += wdd::row_dft_blocks(p->sx, p->kpad, spasses[i].nrows);
    rd->upd_total[k] += wdd::row_update_blocks(p->n_freq_pad, p->kpad);
  }
  // block: [passes][items][spectrum passes][their first workgroups (row DFT, update)][rows]
  // [order][xs] (copied to the device) then the frame addresses
  const size_t off_items = align16(passes.size() * sizeof(wdd::ObjPass));
  const size_t off_spass = off_items + align16(nitems * sizeof(int4));
  const size_t off_dft = off_spass + align16(spasses.size() * sizeof(wdd::SpecPass));
  const size_t off_upd = off_dft + align16(spasses.size() * sizeof(int32_t));
  const size_t off_rows = off_upd + align16(spasses.size() * sizeof(int32_t));
  const size_t off_order = off_rows + align16(rows.size() * sizeof(int4));
  const size_t off_xs = off_order + align16(order.size() * sizeof(int32_t));
  const size_t dev_bytes = off_xs + align16(xs.size() * sizeof(int32_t));
  const size_t bytes = dev_bytes + addrs.size() * sizeof(uint64_t);
  if (dev_bytes > s->blk_cap) {  // grown after the stream has drained
    SRV_HIP(s, hipStreamSynchronize(s->stream));
    if (s->blk) SRV_HIP(s, hipFree(s->blk));
    s->blk = nullptr;
    const size_t cap = std::max(dev_bytes * 2, (size_t)1 << 16);
    hipError_t e = hipMalloc((void**)&s->blk, cap);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      s->blk_cap = 0;
      return wdd::fail(WDD_ENOMEM, "device allocation of %zu bytes failed", cap);
    }
    s->blk_cap = cap;
  }
  const int slot = s->ring;
  s->ring = (s->ring + 1) % kRing;
  if (s->ring_live[slot]) SRV_HIP(s, hipEventSynchronize(s->ring_ev[slot]));
  s->ring_live[slot] = false;
  if (bytes > s->pin_cap[slot]) {
    if (s->pin[slot]) SRV_HIP(s, hipHostFree(s->pin[slot]));
    s->pin[slot] = nullptr;
    s->pin_cap[slot] = 0;
    const size_t cap = std::max(bytes * 2, (size_t)1 << 16);
    SRV_HIP(s, hipHostMalloc((void**)&s->pin[slot], cap, hipHostMallocDefault));
    s->pin_cap[slot] = cap;
  }
  char* hb = s->pin[slot];
  char* db = s->blk;
  std::memcpy(hb + off_rows, rows.data(), rows.size() * sizeof(int4));
  std::memcpy(hb + off_order, order.data(), order.size() * sizeof(int32_t));
  std::memcpy(hb + off_xs, xs.data(), xs.size() * sizeof(int32_t));
  uint64_t* ftab = reinterpret_cast<uint64_t*>(hb + dev_bytes);
  std::memcpy(ftab, addrs.data(), addrs.size() * sizeof(uint64_t));
  wdd::ObjPass* op = reinterpret_cast<wdd::ObjPass*>(hb);
  int4* items = reinterpret_cast<int4*>(hb + off_items);
  std::vector<int32_t> last_pass(ms.size(), 0);
  for (const Round::PassRef& pr : passes) last_pass[pr.member] = std::max(last_pass[pr.member], pr.k);
  for (size_t i = 0; i < passes.size(); ++i) {
    const Round::PassRef& pr = passes[i];
    const Member& m = ms[pr.member];
    wdd_plan_s* p = m.p;
    wdd::ObjPass o;
    std::memset(&o, 0, sizeof(o));
    o.h = p->h;
    o.order = reinterpret_cast<const int*>(db + off_order) + m.first_frame;
    o.xs = reinterpret_cast<const int*>(db + off_xs) + m.first_frame;
    o.jv = p->jv;
    o.w = p->w;
    o.d = p->d;
    o.dlo = p->dlo;
    o.z = p->z;
    const bool disp = m.display && p->up && pr.k == last_pass[pr.member];
    o.up = disp ? p->up : nullptr;
    o.rows = reinterpret_cast<const int4*>(db + off_rows) + m.first_row + pr.row0;
    o.kpad = p->kpad;
    o.nrows = pr.nrows;
    o.sx = p->sx;
    o.sy = p->sy;
    o.max_chunk = p->max_chunk;
    o.nslot = p->nslot;
    int lg = 0;
    while ((1 << lg) < p->sy) ++lg;
    o.log2sy = lg;
    o.in_order = m.in_order ? 1 : 0;
    o.tscale = p->tscale;
    op[i] = o;
    for (size_t c = 0; c < p->host_chunks.size(); ++c) {
      const int4 ch = p->host_chunks[c];
      items[rd->item0[i] + c] = make_int4((int32_t)i, ch.x, ch.y, ch.z | (ch.w << 16));
    }
  }
  std::vector<int32_t> last_spass(ms.size(), 0);
  for (const Round::PassRef& pr : spasses) last_spass[pr.member] = std::max(last_spass[pr.member], pr.k);
  wdd::SpecPass* sp = reinterpret_cast<wdd::SpecPass*>(hb + off_spass);
  for (size_t i = 0; i < spasses.size(); ++i) {
    const Round::PassRef& pr = spasses[i];
    const Member& m = ms[pr.member];
    wdd_plan_s* p = m.p;
    wdd::SpecPass o;
    std::memset(&o, 0, sizeof(o));
    o.h = p->h;
    o.xs = reinterpret_cast<const int*>(db + off_xs) + m.first_frame;
    o.order = reinterpret_cast<const int*>(db + off_order) + m.first_frame;
    o.rows = reinterpret_cast<const int4*>(db + off_rows) + m.first_row + pr.row0;
    o.tx = p->tx;
    o.ty = p->ty;
    o.t = p->t;
    o.acc = p->acc;
    o.freqs = p->freqs;
    o.w = p->w;
    o.d = p->d;
    o.z = p->z;
    o.n_freq = p->n_freq;
    o.nrows = pr.nrows;
    o.sx = p->sx;
    o.sy = p->sy;
    o.kpad = p->kpad;
    o.fuse = m.display && pr.k == last_spass[pr.member] ? 1 : 0;  // D current for the snapshot
    sp[i] = o;
  }
  std::memcpy(hb + off_dft, rd->dft_first.data(), rd->dft_first.size() * sizeof(int32_t));
  std::memcpy(hb + off_upd, rd->upd_first.data(), rd->upd_first.size() * sizeof(int32_t));
  rd->off_spass = off_spass;
  rd->off_dft = off_dft;
  rd->off_upd = off_upd;
  rd->hb = hb;
  rd->db = db;
  rd->dev_bytes = dev_bytes;
  rd->off_items = off_items;
  rd->ftab = ftab;
  rd->slot = slot;
  return WDD_OK;
}

// Queues a prepared round: the projections of every member's batch (one launch per frame
// type and arithmetic, at most kProjectGroupMax members each; the first also brings the
// descriptors to the device), then the updates, one launch per row-pass index k (passes k
// of different acquisitions write different spectra; passes of one acquisition add to the
// same D, so the launches order them).  Launches only (captured in graph mode).
wdd_status launch_round(wdd_server_s* s, const std::vector<Member>& ms, const Round& rd) {
  bool sent = false;
  std::vector<bool> done(ms.size(), false);
  for (size_t i0 = 0; i0 < ms.size(); ++i0) {
    if (done[i0]) continue;
    std::vector<wdd::ProjectLaunch> pls;
    for (size_t i = i0; i < ms.size() && (int)pls.size() < wdd::kProjectGroupMax; ++i) {
      wdd_plan_s* p = ms[i].p;
      if (done[i] || p->dtype != ms[i0].p->dtype || p->precision != ms[i0].p->precision) continue;
      wdd::ProjectLaunch pl;
      std::memset(&pl, 0, sizeof(pl));
      pl.dtype = p->dtype;
      pl.precision = p->precision;
      pl.frames = nullptr;
      pl.n = ms[i].n;
      pl.ny = p->ny;
      pl.nx = p->nx;
      pl.psi = p->psi;
      pl.psix_lp = p->psix_lp;
      pl.psi_unscale = p->psi_unscale;
      pl.kmap = p->kmap;
      pl.kpad = p->kpad;
      pl.h = p->h;
      pl.fptr = rd.ftab + ms[i].first_frame;
      pls.push_back(pl);
      done[i] = true;
    }
    SRV_HIP(s, wdd::launch_project_group(pls.data(), (int)pls.size(), sent ? nullptr : rd.hb,
                                         sent ? nullptr : rd.db, sent ? 0 : rd.dev_bytes, s->stream));
    sent = true;
  }
  for (size_t i0 = 0; i0 < rd.passes.size();) {
    size_t i1 = i0;
    size_t lds = 0;
    while (i1 < rd.passes.size() && rd.passes[i1].k == rd.passes[i0].k) {
      const wdd_plan_s* p = ms[rd.passes[i1].member].p;
      lds = std::max(lds, wdd::row_fused_lds_bytes(p->kpad, rd.passes[i1].nrows, p->max_chunk));
      ++i1;
    }
    SRV_HIP(s, wdd::launch_row_fused_obj_group(reinterpret_cast<const wdd::ObjPass*>(rd.db),
                                               reinterpret_cast<const int4*>(rd.db + rd.off_items) + rd.item0[i0],
                                               (int)(rd.item0[i1] - rd.item0[i0]), lds, s->stream));
    i0 = i1;
  }
  // spectrum order: per pass index, the row DFTs of every such member, then their A updates
  // (a member's passes share its T and A, so the launches order them)
  const wdd::SpecPass* sp = reinterpret_cast<const wdd::SpecPass*>(rd.db + rd.off_spass);
  const int32_t* dft_first = reinterpret_cast<const int32_t*>(rd.db + rd.off_dft);
  const int32_t* upd_first = reinterpret_cast<const int32_t*>(rd.db + rd.off_upd);
  for (size_t i0 = 0; i0 < rd.spasses.size();) {
    const int32_t k = rd.spasses[i0].k;
    size_t i1 = i0;
    size_t lds = 0;
    while (i1 < rd.spasses.size() && rd.spasses[i1].k == k) {
      lds = std::max(lds, wdd::row_dft_lds_bytes(ms[rd.spasses[i1].member].p->sx));
      ++i1;
    }
    SRV_HIP(s, wdd::launch_row_dft_group(sp + i0, dft_first + i0, (int)(i1 - i0), rd.dft_total[k], lds, s->stream));
    SRV_HIP(s, wdd::launch_row_update_group(sp + i0, upd_first + i0, (int)(i1 - i0), rd.upd_total[k], s->stream));
    i0 = i1;
  }
  return WDD_OK;
}

// The ring slot of a round just queued is free again once the stream passes this point.
wdd_status mark_round(wdd_server_s* s, int slot) {
  SRV_HIP(s, hipEventRecord(s->ring_ev[slot], s->stream));
  s->ring_live[slot] = true;
  return WDD_OK;
}

// Queues grouped rounds until none of `acqs` has pending frames (with `until`: until that
// one has none); an acquisition in `due` gets the display's first pass left by its last
// round.
wdd_status drain_grouped(wdd_server_s* s, const std::vector<Acq*>& acqs, const std::vector<bool>& due,
                         const Acq* until = nullptr) {
  for (;;) {
    if (until && until->pending.empty()) return WDD_OK;
    std::vector<Member> ms;
    for (size_t i = 0; i < acqs.size(); ++i) {
      Acq* a = acqs[i];
      if (a->pending.empty()) continue;
      Member m;
      std::memset(&m, 0, sizeof(m));
      m.a = a;
      m.p = static_cast<wdd_plan_s*>(a->plan);
      m.n = (int32_t)std::min<size_t>(a->pending.size(), (size_t)a->batch);
      m.spectrum = m.p->order_mode == WDD_ORDER_SPECTRUM;
      m.display = due[i] && (size_t)m.n == a->pending.size();
      if (m.p->failed) return wdd::fail(WDD_ESTATE, "acquisition %d is unusable after an earlier device error", a->id);
      ms.push_back(m);
    }
    if (ms.empty()) return WDD_OK;
    Round rd;
    wdd_status st = prepare_round(s, ms, &rd);
    if (st != WDD_OK) return st;
    // (a round while a closer thread frees memory is launched directly instead of captured)
    std::unique_lock<std::mutex> no_frees(s->free_mu, std::defer_lock);
    if (s->opts.launch_mode == WDD_SERVE_GRAPH && no_frees.try_lock()) {
      // capture the round, then replay it (updating the instantiated graph's arguments when
      // the shape is the one captured before)
      SRV_HIP(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
      st = launch_round(s, ms, rd);
      hipGraph_t g = nullptr;
      const hipError_t ce = hipStreamEndCapture(s->stream, &g);
      if (st != WDD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (ce != hipSuccess) return hip_fail(s, ce, "hipStreamEndCapture");
      bool updated = false;
      if (s->exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        const hipError_t ue = hipGraphExecUpdate(s->exec, g, &err_node, &res);
        updated = ue == hipSuccess && res == hipGraphExecUpdateSuccess;
        if (!updated) {
          (void)hipGetLastError();
          (void)hipGraphExecDestroy(s->exec);
          s->exec = nullptr;
        }
      }
      if (!updated) {
        const hipError_t ie = hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
          (void)hipGraphDestroy(g);
          s->exec = nullptr;
          return hip_fail(s, ie, "hipGraphInstantiate");
        }
      }
      (void)hipGraphDestroy(g);
      SRV_HIP(s, hipGraphLaunch(s->exec, s->stream));
      s->graph_replays += updated ? 1 : 0;
    } else if ((st = launch_round(s, ms, rd)) != WDD_OK) {
      return st;
    }
    if ((st = mark_round(s, rd.slot)) != WDD_OK) return st;
    s->group_rounds += 1;
    for (Member& m : ms) {
      Acq* a = m.a;
      wdd_plan_s* p = m.p;
      for (int32_t i = 0; i < m.n; ++i) {
        a->awaiting.push_back(a->pending.front().t_submit);
        a->pending.pop_front();
      }
      p->frames_seen += (uint64_t)m.n;
      p->last_batch = m.n;
      p->up_valid = m.display && p->up;  // D changed: the partial rows are current only if written now
      a->fused = m.spectrum && m.display;  // spectrum order: D reduced in the round's last pass
      a->frames_done += (uint64_t)m.n;
      s->frames += (uint64_t)m.n;
      s->batches += 1;
    }
  }
}

// Whether D is current for a snapshot: object order always; spectrum order when the last
// push (plan path: `fused_push`) or round (grouped) carried the Wiener reduction.
bool current_d(const Acq* a, bool fused_push) {
  const wdd_plan_s* p = static_cast<const wdd_plan_s*>(a->plan);
  if (p->order_mode == WDD_ORDER_OBJECT) return true;
  return a->grouped ? a->fused : fused_push;
}

void record_snapshot(wdd_server_s* s, Acq* a) {
  const double done = now_us();
  for (double ts : a->awaiting) s->latency_us.push_back(done - ts);
  a->awaiting.clear();
  a->last_snapshot = done;
  s->snapshots += 1;
}

// Records a scheduled snapshot that has completed (its image is in the plan's pinned buffer).
void complete_inflight(wdd_server_s* s, Acq* a, double done) {
  for (double ts : a->inflight) s->latency_us.push_back(done - ts);
  a->inflight.clear();
  a->snap_inflight = false;
  s->snapshots += 1;
}

// Checks the scheduled snapshots still running, without waiting.
wdd_status poll_snapshots(wdd_server_s* s) {
  for (auto& kv : s->acqs) {
    Acq* a = kv.second;
    if (!a->snap_inflight) continue;
    const hipError_t e = hipEventQuery(a->snap_ev);
    if (e == hipSuccess) {
      complete_inflight(s, a, now_us());
    } else if (e != hipErrorNotReady) {
      return hip_fail(s, e, "hipEventQuery");
    } else {
      (void)hipGetLastError();
    }
  }
  return WDD_OK;
}

// The worker that opens an acquisition: tables (unless cached), plan, upload of W; a grouped
// acquisition then moves to the server's stream.
void open_worker(wdd_server_s* s, Acq* a, TableKey key, std::shared_ptr<wdd_tables_s> tp, wdd_probe probe,
                 wdd_scan scan, wdd_detector det, int32_t K, wdd_options opts) {
  wdd_status st = WDD_OK;
  if (hipSetDevice(s->device) != hipSuccess) {
    (void)hipGetLastError();
    st = wdd::fail(WDD_EDEVICE, "hipSetDevice(%d) failed", s->device);
  }
  if (st == WDD_OK && !tp) {
    try {
      tp = std::make_shared<wdd_tables_s>();
      st = wdd::build_tables(&probe, &scan, &det, K, &opts, tp.get());
    } catch (const std::bad_alloc&) {
      st = wdd::fail(WDD_ENOMEM, "out of host memory");
    }
    if (st == WDD_OK) {
      TableCache& c = table_cache();
      std::lock_guard<std::mutex> lock(c.mu);
      const size_t tb = tp->w.size() * sizeof(double) + tp->freqs.size() * sizeof(int32_t);
      if (c.bytes + tb > ((size_t)4 << 30)) {  // keep at most 4 GiB of cached host tables
        c.tables.clear();
        c.bytes = 0;
      }
      c.tables[key] = tp;
      c.bytes += tb;
    }
  }
  wdd_plan_t plan = nullptr;
  if (st == WDD_OK) st = wdd::plan_create_from_tables(tp, &probe, &scan, &det, opts, nullptr, &plan);
  if (st == WDD_OK && a->grouped) st = wdd::plan_set_stream(plan, s->stream);
  if (st == WDD_OK && !a->grouped) st = wdd_sync(plan);
  if (st != WDD_OK) {
    a->open_error = wdd_last_error();
    if (plan) wdd_destroy(plan);
    plan = nullptr;
  }
  a->open_status = st;
  a->made = plan;
  a->done.store(true, std::memory_order_release);
}

// Frees an acquisition that is no longer in the server's map (on a closer thread, or on the
// calling thread when the server is destroyed).  Touches no server counters.
void free_acq(wdd_server_s* s, Acq* a) {
  (void)hipSetDevice(s->device);
  if (a->worker.joinable()) a->worker.join();
  wdd_plan_t plan = a->plan ? a->plan : (a->open_status == WDD_OK ? a->made : nullptr);
  if (plan) {
    // The server's stream is not waited on here: the scheduling thread may be capturing it
    // (WDD_SERVE_GRAPH), and a wait on a capturing stream from another thread invalidates the
    // capture.  A plan with rounds behind it was synchronised by wdd_server_close or by the
    // server's destruction; one that never ran a round has no work there.
    if (a->grouped) wdd::plan_drop_stream(plan);
    std::lock_guard<std::mutex> g(s->free_mu);
    wdd_destroy(plan);
  }
  if (a->snap_ev) (void)hipEventDestroy(a->snap_ev);
  delete a;
}

// Joins the closers that have finished (wait: all of them) and returns their bytes to the budget.
void reap_closers(wdd_server_s* s, bool wait) {
  for (size_t i = 0; i < s->closers.size();) {
    Closer* c = s->closers[i].get();
    if (!wait && !c->done.load(std::memory_order_acquire)) {
      ++i;
      continue;
    }
    c->th.join();
    s->used -= c->bytes;
    s->closers.erase(s->closers.begin() + (std::ptrdiff_t)i);
  }
}

}  // namespace

extern "C" {

wdd_status wdd_server_default_options(wdd_server_options* o) {
  if (!o) return wdd::fail(WDD_EINVAL, "null options");
  o->hbm_budget_bytes = (int64_t)1 << 30;
  o->snapshot_interval_us = 1000.0;
  o->batch_frames = 256;
  o->launch_mode = WDD_SERVE_GROUPED;
  return WDD_OK;
}

wdd_status wdd_server_create(const wdd_server_options* opts, wdd_server_t* out) {
  if (!out) return wdd::fail(WDD_EINVAL, "null output handle");
  *out = nullptr;
  wdd_server_s* s = new (std::nothrow) wdd_server_s();
  if (!s) return wdd::fail(WDD_ENOMEM, "out of host memory");
  wdd_server_default_options(&s->opts);
  if (opts) s->opts = *opts;
  if (s->opts.batch_frames < 1 || !(s->opts.snapshot_interval_us >= 0) || s->opts.launch_mode < WDD_SERVE_STREAMS ||
      s->opts.launch_mode > WDD_SERVE_GRAPH) {
    delete s;
    return wdd::fail(WDD_EINVAL, "batch_frames must be >= 1, the snapshot interval >= 0 and launch_mode known");
  }
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = wdd::prepare_group_kernels();
  for (int i = 0; i < kRing && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&s->ring_ev[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    for (int i = 0; i < kRing; ++i)
      if (s->ring_ev[i]) (void)hipEventDestroy(s->ring_ev[i]);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return wdd::fail(WDD_EDEVICE, "server stream: %s", hipGetErrorString(e));
  }
  *out = s;
  return WDD_OK;
}

wdd_status wdd_server_open(wdd_server_t s, const wdd_probe* probe, const wdd_scan* scan, const wdd_detector* det,
                           int32_t K, const wdd_options* opts_in, int32_t* acq_id) {
  if (!s || !acq_id || !probe || !scan || !det) return wdd::fail(WDD_EINVAL, "null argument");
  *acq_id = 0;
  if (s->failed) return wdd::fail(WDD_ESTATE, "server is unusable after an earlier device error");
  wdd_options opts;
  wdd_default_options(&opts);
  if (opts_in) opts = *opts_in;
  opts.max_batch = std::max(opts.max_batch, s->opts.batch_frames);
  opts.pipeline = 0;  // the server orders each acquisition's launches itself
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
  {
    TableCache& c = table_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    auto it = c.tables.find(key);
    if (it != c.tables.end()) tp = it->second;
  }
  // admission needs only the kept frequencies: the full tables are built by the worker
  int64_t need = 0;
  if (tp) {
    need = wdd::plan_device_bytes(*tp, opts, det->dtype);
  } else {
    try {
      wdd_tables_s kept;
      if ((st = wdd::build_tables(probe, scan, det, K, &opts, &kept, true)) != WDD_OK) return st;
      need = wdd::plan_device_bytes(kept, opts, det->dtype);
    } catch (const std::bad_alloc&) {
      return wdd::fail(WDD_ENOMEM, "out of host memory");
    }
  }
  reap_closers(s, false);
  // memory of closed acquisitions still being freed is waited for before refusing
  if (s->opts.hbm_budget_bytes > 0 && s->used + need > s->opts.hbm_budget_bytes) reap_closers(s, true);
  if (s->opts.hbm_budget_bytes > 0 && s->used + need > s->opts.hbm_budget_bytes)
    return wdd::fail(WDD_EBUSY, "acquisition needs %lld bytes; %lld of %lld in use", (long long)need,
                     (long long)s->used, (long long)s->opts.hbm_budget_bytes);
  Acq* a = new (std::nothrow) Acq();
  if (!a) return wdd::fail(WDD_ENOMEM, "out of host memory");
  a->id = s->next_id++;
  a->bytes = need;
  a->batch = s->opts.batch_frames;
  a->frame_bytes = (size_t)det->ny * det->nx * (det->dtype == WDD_U16 ? 2 : 4);
  a->sy = scan->sy;
  a->sx = scan->sx;
  a->grouped = s->opts.launch_mode != WDD_SERVE_STREAMS && opts.basis == WDD_BASIS_HERMITE_GAUSS;
  try {
    a->worker = std::thread(open_worker, s, a, key, tp, *probe, *scan, *det, K, opts);
  } catch (const std::system_error&) {
    delete a;
    return wdd::fail(WDD_ENOMEM, "could not start the opening thread");
  }
  s->used += a->bytes;
  s->acqs[a->id] = a;
  *acq_id = a->id;
  return WDD_OK;
}

wdd_status wdd_server_wait_open(wdd_server_t s, int32_t acq) {
  Acq* a = nullptr;
  wdd_status st = find(s, acq, &a);
  if (st != WDD_OK) return st;
  return settle_open(s, a, true);
}

wdd_status wdd_server_submit(wdd_server_t s, int32_t acq, const void* frames, const int32_t* pos_yx, int32_t n) {
  Acq* a = nullptr;
  wdd_status st = find(s, acq, &a);
  if (st != WDD_OK) return st;
  if ((st = settle_open(s, a, false)) != WDD_OK) return st;
  if (n < 0) return wdd::fail(WDD_EINVAL, "n < 0");
  if (n == 0) return WDD_OK;
  if (!frames || !pos_yx) return wdd::fail(WDD_EINVAL, "null frames or positions");
  if (reinterpret_cast<uintptr_t>(frames) % 16 != 0) return wdd::fail(WDD_EINVAL, "frames must be 16-byte aligned");
  for (int32_t i = 0; i < n; ++i) {
    const int32_t y = pos_yx[2 * i], x = pos_yx[2 * i + 1];
    if (y < 0 || y >= a->sy || x < 0 || x >= a->sx)
      return wdd::fail(WDD_ERANGE, "position %d = (%d, %d) outside the %d x %d raster", i, y, x, a->sy, a->sx);
  }
  const double t = now_us();
  const uint64_t base = reinterpret_cast<uint64_t>(frames);
  for (int32_t i = 0; i < n; ++i)
    a->pending.push_back({base + (uint64_t)i * a->frame_bytes, pos_yx[2 * i], pos_yx[2 * i + 1], t});
  return WDD_OK;
}

wdd_status wdd_server_step(wdd_server_t s, int32_t* frames_processed) {
  if (!s) return wdd::fail(WDD_EINVAL, "null server");
  if (s->failed) return wdd::fail(WDD_ESTATE, "server is unusable after an earlier device error");
  const uint64_t before = s->frames;
  reap_closers(s, false);
  wdd_status st = poll_snapshots(s);
  if (st != WDD_OK) return st;
  const double t = now_us();
  std::vector<std::pair<Acq*, bool>> snap;  // acquisitions to snapshot, and whether the reduction was fused
  std::vector<Acq*> grouped;
  std::vector<bool> grouped_due;
  for (auto& kv : s->acqs) {
    Acq* a = kv.second;
    if (settle_open(s, a, false) != WDD_OK || !ready(a)) continue;  // failed or still opening: skipped
    // due once the interval has passed and its previous scheduled snapshot is done
    const bool due = (t - a->last_snapshot) >= s->opts.snapshot_interval_us && !a->snap_inflight;
    const bool had = !a->pending.empty();
    bool fused = false;
    if (a->grouped) {
      a->fused = false;
      grouped.push_back(a);
      grouped_due.push_back(due);
    } else {
      wdd_status st = drain_plan(s, a, due, &fused);
      if (st != WDD_OK) return st;
    }
    if (due && (had || !a->awaiting.empty())) snap.emplace_back(a, fused);
  }
  if ((st = drain_grouped(s, grouped, grouped_due)) != WDD_OK) return st;
  // the due snapshots are queued, not waited for
  for (auto& sp : snap) {
    Acq* a = sp.first;
    // object order keeps D current; a grouped spectrum-order acquisition has D current if its
    // last round reduced it
    if ((st = wdd::snapshot_enqueue(a->plan, !current_d(a, sp.second))) != WDD_OK) return st;
    if (!a->snap_ev) SRV_HIP(s, hipEventCreateWithFlags(&a->snap_ev, hipEventDisableTiming));
    SRV_HIP(s, hipEventRecord(a->snap_ev, static_cast<wdd_plan_s*>(a->plan)->stream));
    a->inflight.swap(a->awaiting);
    a->awaiting.clear();
    a->snap_inflight = true;
    a->last_snapshot = t;
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
  if ((st = settle_open(s, a, true)) != WDD_OK) return st;
  bool fused = false;
  if (a->grouped) {
    // rounds over every ready grouped acquisition with frames waiting, until this one's are in
    a->fused = false;
    std::vector<Acq*> acqs;
    std::vector<bool> due;
    for (auto& kv : s->acqs) {
      Acq* b = kv.second;
      if (!b->grouped || settle_open(s, b, false) != WDD_OK || !ready(b)) continue;
      acqs.push_back(b);
      due.push_back(b == a);
    }
    if ((st = drain_grouped(s, acqs, due, a)) != WDD_OK) return st;
  } else if ((st = drain_plan(s, a, true, &fused)) != WDD_OK) {
    return st;
  }
  if ((st = wdd::snapshot_enqueue(a->plan, !current_d(a, fused))) != WDD_OK) return st;
  if ((st = wdd::snapshot_finish(a->plan, frames_seen)) != WDD_OK) return st;
  if (a->snap_inflight) complete_inflight(s, a, now_us());  // queued earlier on the same stream
  record_snapshot(s, a);
  float* buf = nullptr;
  if ((st = wdd_snapshot_buffer(a->plan, &buf)) != WDD_OK) return st;
  std::memcpy(out, buf, (size_t)a->sy * a->sx * 2 * sizeof(float));
  return WDD_OK;
}

wdd_status wdd_server_acq_state(wdd_server_t s, int32_t acq, int32_t* is_ready, int64_t* pending_frames) {
  Acq* a = nullptr;
  wdd_status st = find(s, acq, &a);
  if (st != WDD_OK) return st;
  if ((st = settle_open(s, a, false)) != WDD_OK) return st;
  if (is_ready) *is_ready = ready(a) ? 1 : 0;
  if (pending_frames) *pending_frames = (int64_t)a->pending.size();
  return WDD_OK;
}

wdd_status wdd_server_acq_shape(wdd_server_t s, int32_t acq, int32_t* sy, int32_t* sx) {
  Acq* a = nullptr;
  wdd_status st = find(s, acq, &a);
  if (st != WDD_OK) return st;
  if (!sy || !sx) return wdd::fail(WDD_EINVAL, "null argument");
  *sy = a->sy;
  *sx = a->sx;
  return WDD_OK;
}

wdd_status wdd_server_close(wdd_server_t s, int32_t acq) {
  if (!s) return wdd::fail(WDD_EINVAL, "null server");
  auto it = s->acqs.find(acq);
  if (it == s->acqs.end()) return wdd::fail(WDD_EINVAL, "no open acquisition %d", acq);
  Acq* a = it->second;
  // the caller may reuse the acquisition's frames once this returns: wait for the work that
  // reads them (the frees, which wait for the whole device, go to the closer thread)
  if (a->plan) {
    const hipError_t e = hipStreamSynchronize(static_cast<wdd_plan_s*>(a->plan)->stream);
    if (e != hipSuccess) return hip_fail(s, e, "hipStreamSynchronize");
  }
  s->acqs.erase(it);
  bool listed = false;
  try {
    s->closers.push_back(std::unique_ptr<Closer>(new Closer()));
    listed = true;
    Closer* cp = s->closers.back().get();
    cp->bytes = a->bytes;
    cp->th = std::thread([s, a, cp]() {
      free_acq(s, a);
      cp->done.store(true, std::memory_order_release);
    });
    return WDD_OK;
  } catch (const std::exception&) {
    if (listed) s->closers.pop_back();
  }
  const int64_t bytes = a->bytes;
  free_acq(s, a);  // no thread: free it here
  s->used -= bytes;
  return WDD_OK;
}

wdd_status wdd_server_get_stats(wdd_server_t s, wdd_server_stats* out) {
  if (!s || !out) return wdd::fail(WDD_EINVAL, "null argument");
  *out = wdd_server_stats{};
  out->frames = s->frames;
  out->batches = s->batches;
  out->snapshots = s->snapshots;
  out->steps = s->steps;
  reap_closers(s, false);
  out->open = (int32_t)s->acqs.size();
  int32_t opening = 0;
  for (auto& kv : s->acqs) {
    (void)settle_open(s, kv.second, false);
    opening += (kv.second->worker.joinable() ? 1 : 0);
  }
  out->opening = opening;
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
  out->group_rounds = s->group_rounds;
  out->graph_replays = s->graph_replays;
  return WDD_OK;
}

wdd_status wdd_server_destroy(wdd_server_t s) {
  if (!s) return WDD_OK;
  reap_closers(s, true);
  if (s->stream) (void)hipStreamSynchronize(s->stream);  // the open acquisitions' last rounds
  for (auto& kv : s->acqs) free_acq(s, kv.second);
  s->acqs.clear();
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  for (int i = 0; i < kRing; ++i) {
    if (s->pin[i]) (void)hipHostFree(s->pin[i]);
    if (s->ring_ev[i]) (void)hipEventDestroy(s->ring_ev[i]);
  }
  if (s->blk) (void)hipFree(s->blk);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return WDD_OK;
}

}  // extern "C"
