// Device and host state of a live plan (shared by the plan ABI and the field-of-view patch
// set, which drives a plan's projection and tables for all its patches).
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "kernels.h"
#include "wdd_internal.h"

namespace wdd {

// Pinned upload blocks (positions, row grouping, frame-address table) form a ring that the
// projection kernel reads when it runs; a block is refilled only after the push that last
// used it has been read.  Stream markers follow every mark_every-th push (an event per push
// costs several microseconds of host time on a pipelined step).
constexpr int kUploadSlots = WDD_MAX_PUSHES_IN_FLIGHT;  // most upload blocks in the ring
constexpr size_t kUploadPinBudget = (size_t)8 << 20;    // pinned bytes the ring may take
constexpr int kFrameSlots = 4;                          // pinned staging slots for host frames
constexpr int kFactorRows = 16;  // batches touching at most this many scan rows use the row-factored update
static_assert(kFactorRows <= wdd::kRowSetMax, "a row pass must fit the kernel-argument row set");
constexpr int kMinChunk = 16, kMaxChunk = 512;  // kept frequencies per workgroup of the row-factored update

struct wdd_plan_impl {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool failed = false;
  int32_t sy = 0, sx = 0, ny = 0, nx = 0, k = 0, kpad = 0, l = 0, dtype = 0, max_batch = 0;
  int64_t n_freq = 0, n_freq_pad = 0;
  double sigma = 0, eps_abs = 0;
  uint64_t frames_seen = 0;
  int32_t last_batch = 0;
  int64_t device_bytes = 0;
  size_t frame_bytes = 0;

  float* psi = nullptr;
  uint16_t* psix_lp = nullptr;  // [2][16][nx] bf16/fp16 hi and lo parts (reduced-precision projection)
  float psi_unscale = 1.f;
  int32_t precision = WDD_FP32;
  int32_t order_mode = WDD_ORDER_SPECTRUM;
  bool fourier = false;  // full Fourier basis: K = ny nx, complex projections
  wdd_probe probe = {};
  wdd_scan scan = {};
  wdd_detector det = {};
  wdd_options opts = {};
  std::shared_ptr<const wdd_tables_s> tables;  // the FP64 tables uploaded (wdd_plan_export)
  int32_t* kmap = nullptr;
  int2* freqs = nullptr;
  float2* w = nullptr;
  float2* acc = nullptr;
  float2 *ty = nullptr, *tx = nullptr, *ey = nullptr, *ex = nullptr;
  float2 *fy = nullptr, *fx = nullptr;
  float* h = nullptr;
  char* upload = nullptr;  // pos, order, rows
  int2* pos = nullptr;
  int32_t* order = nullptr;
  int32_t* xs = nullptr;
  int4* rows = nullptr;
  size_t upload_bytes = 0;
  float2* t = nullptr;
  int2* jv = nullptr;  // (j, v_y) of the kept frequencies grouped by v_x (object order)
  float tscale = 1.f;  // 1 / sqrt(sy sx), the unitary scan DFT's factor
  int4* chunks = nullptr;
  int32_t nchunks = 0, max_chunk = 0;
  // object order: the update also leaves the display's first pass as nslot partial rows per
  // v_x in `up` (sx * nslot * sy values); up_valid while they match the current D
  float2* up = nullptr;
  int32_t nslot = 1;
  bool up_valid = false;
  // detectors of more than 128 rows: a deferred column pass rides in the next push's first
  // update launch, which reads the partial rows and D[0] of the previous push while writing
  // new ones.  So they are double-buffered: up / up_alt swap on every push that writes
  // partial rows, d0w (a copy of D[0] that the last pass of such a push stores) with them.
  float2* up_alt = nullptr;
  float2 *d0w = nullptr, *d0w_alt = nullptr;
  bool deferred_in_update = false;  // the pending column pass goes with the update, not the projection
  const float2* deferred_d0 = nullptr;
  // a display's column pass left to the next push (WDD_OUT_DEVICE_DEFERRED): destination
  // and source (the partial rows in `up`, or the first pass's grid `u`)
  float2* deferred_dst = nullptr;
  const float2* deferred_src = nullptr;
  int32_t deferred_sr = 0, deferred_sm = 0, deferred_nslot = 1, deferred_slot_stride = 0;
  // pipelined pushes (wdd_options.pipeline): the update of the last pushed batch is held
  // (`held`) and runs in the next push's launch beside that push's projection, which writes
  // the next batch's projections and upload block to h_alt / upload_alt (swapped with h /
  // upload after each push: h and upload always hold the held batch's)
  bool pipeline = false;
  float* h_alt = nullptr;
  char* upload_alt = nullptr;
  struct Held {
    bool live = false;
    bool in_order = true;
    std::vector<int4> rows;       // the batch's scan rows (y, first, count), row-sorted order
    bool display = false;         // a deferred snapshot follows the batch
    float2* display_dst = nullptr;
  } held;
  // two-stage pipelined pushes (pipeline = 2): `held` is the last pushed batch (projected), and
  // held2 the one before it, whose x-DFT (one row set per kept v_x, xcols) is in t_cur; each
  // push's launch updates held2, forms the x-DFT of `held` into t_next and projects the new
  // batch; t_cur and t_next then swap
  bool two_stage = false;
  Held held2;
  float4 *t_cur = nullptr, *t_next = nullptr;
  int32_t* xcols = nullptr;
  int32_t ncols = 0;       // kept v_x columns (object order)
  void* frames = nullptr;
  float2 *d = nullptr, *z = nullptr, *u = nullptr;
  float2* dlo = nullptr;  // object order: the rounding remainder of D (D = d + dlo, compensated sum)

  int up_ring = 4, mark_every = 1;   // upload blocks in the ring; marker spacing in pushes
  char* pin_ring = nullptr;          // the ring's pinned memory
  std::vector<char*> pin_up;         // [up_ring] blocks in pin_ring
  std::vector<hipEvent_t> marks;     // [up_ring / mark_every + 2]
  std::vector<int64_t> mark_at;      // the push each marker follows (-1: none yet)
  int64_t pushes = 0;                // pushes that carried frames
  int64_t drained = -1;              // every push up to this one is known to have run
  void* pin_frames[kFrameSlots] = {};
  hipEvent_t fev[kFrameSlots] = {};
  bool fev_live[kFrameSlots] = {};
  int fslot = 0;
  float2* pin_out = nullptr;
  std::vector<void*> allocs;
  wdd_alloc_fn alloc_fn = nullptr;  // the caller's device allocator when the plan was created
  wdd_release_fn release_fn = nullptr;
  void* alloc_ctx = nullptr;

  // stage timing (wdd_profile_*): events around launches, harvested when the stream is idle
  int32_t profile_mask = 0;  // bit i: time stage i (Stage enum)
  int32_t profile_period = 1;  // time one push (and its snapshot) in every profile_period
  int64_t profile_tick = 0;    // pushes since profiling was (re)configured
  bool profile_now = true;     // the current push is sampled
  std::vector<hipEvent_t> ev_pool;
  struct Pending { int stage; hipEvent_t e0, e1; };
  std::vector<Pending> pending;
  double stage_ms[5] = {0, 0, 0, 0, 0};
  int64_t stage_n[5] = {0, 0, 0, 0, 0};
  int64_t factored_n = 0;  // timed accumulate launches that were row-factored
  std::vector<int32_t> host_order;
  std::vector<int4> host_rows;
  std::vector<int4> host_chunks;  // the object-order update's chunks (also device `chunks`)
};

}  // namespace wdd

struct wdd_plan_s : wdd::wdd_plan_impl {};
