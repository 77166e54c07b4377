// C ABI of the live WDD plan: device state, push and snapshot.
//
// Device layout of a plan (all on the plan's device):
//   psi     float  [(ny + nx) * 16]     sampled Hermite functions, columns >= L zero
//   kmap    int32  [kpad]               16 n_y(k) + n_x(k); -1 for padding columns
//                                       (kpad = K rounded up to a power of two >= 32)
//   freqs   int2   [n_freq_pad]         kept (v_y, v_x); padding rows (0, 0)
//   w       float2 [n_freq_pad][kpad]   Wiener filter (padding rows/columns zero)
//   acc     float2 [n_freq_pad][kpad]   accumulated spectrum A (spectrum order only)
//   ty, tx  float2 [sy], [sx]           exp(-2 pi i m / S); tx carries 1/sqrt(sy sx)
//   ey, ex  float2 [sy], [sx]           exp(-2 pi i m / S) for the display DFT
//   h       float  [max_batch][kpad]    projections of the current batch (float2 for the
//                                       Fourier basis, whose projections are complex)
//   fy, fx  float2 [ny/2], [nx/2]       exp(+2 pi i m / n) (Fourier basis only)
//   upload  bytes                       per batch: pos int2 [max_batch], order int32 [max_batch],
//                                       xs int32 [max_batch] (scan x of frame order[i]), rows int4
//                                       [max_batch] (brought over by the projection kernel)
//   jv      int2   [n_freq]             (j, v_y) of the kept frequencies grouped by v_x (ascending
//                                       v_x, v_y; object order only)
//   chunks  int4   [nchunks]            (v_x, first jv index, count <= max_chunk, 0): the
//                                       workgroups of the object-order update (object order only)
//   t       float2 [kFactorRows][sx][kpad]  per-row x-DFTs (spectrum order, fused Wiener reduction)
//   frames  staging for host frames     [max_batch][ny][nx]
//   d       float2 [n_freq_pad]         Wiener-reduced spectrum D
//   z, u    float2 [sx][sy], [sx][sy]   conj(D) grid (transposed), grid transformed along y
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "plan.h"

using wdd::kFactorRows;
using wdd::kFrameSlots;
using wdd::kMaxChunk;
using wdd::kMinChunk;
using wdd::kUploadPinBudget;
using wdd::kUploadSlots;

namespace {

wdd_status dev_fail(wdd_plan_s* p, hipError_t e, const char* what) {
  if (p) p->failed = true;
  return wdd::fail(WDD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define WDD_HIP(p, call)                                   \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return dev_fail((p), e_, #call); \
  } while (0)

template <typename T>
wdd_status dalloc(wdd_plan_s* p, T** ptr, size_t count) {
  *ptr = nullptr;
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  if (p->alloc_fn) {
    void* m = p->alloc_fn(bytes, p->alloc_ctx);
    if (!m) return wdd::fail(WDD_ENOMEM, "the caller's allocator returned no memory for %zu bytes", bytes);
    if (reinterpret_cast<uintptr_t>(m) % 256 != 0) {
      p->release_fn(m, p->alloc_ctx);
      return wdd::fail(WDD_EINVAL, "the caller's allocator returned memory not aligned to 256 bytes");
    }
    *ptr = static_cast<T*>(m);
    p->allocs.push_back(m);
    p->device_bytes += (int64_t)bytes;
    return WDD_OK;
  }
  hipError_t e = hipMalloc((void**)ptr, bytes);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    return wdd::fail(WDD_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  if (e != hipSuccess) return dev_fail(p, e, "hipMalloc");
  p->allocs.push_back(*ptr);
  p->device_bytes += (int64_t)bytes;
  return WDD_OK;
}

enum Stage { kProject = 0, kAccumulate = 1, kWiener = 2, kDisplay = 3, kRowDft = 4 };

// Opens a timed stage: returns the end event to record after the launches (or null).
hipError_t stage_begin(wdd_plan_s* p, int stage, hipEvent_t* end) {
  *end = nullptr;
  if (!(p->profile_mask & (1 << stage)) || !p->profile_now) return hipSuccess;
  hipEvent_t e[2];
  for (int i = 0; i < 2; ++i) {
    if (!p->ev_pool.empty()) {
      e[i] = p->ev_pool.back();
      p->ev_pool.pop_back();
    } else {
      hipError_t err = hipEventCreate(&e[i]);
      if (err != hipSuccess) return err;
    }
  }
  hipError_t err = hipEventRecord(e[0], p->stream);
  if (err != hipSuccess) return err;
  p->pending.push_back({stage, e[0], e[1]});
  *end = e[1];
  return hipSuccess;
}

hipError_t stage_end(wdd_plan_s* p, hipEvent_t end) {
  if (!end) return hipSuccess;
  return hipEventRecord(end, p->stream);
}

// Adds the durations of all recorded stages; the stream must be idle.
hipError_t harvest(wdd_plan_s* p) {
  for (auto& x : p->pending) {
    float ms = 0.f;
    hipError_t err = hipEventElapsedTime(&ms, x.e0, x.e1);
    if (err != hipSuccess) return err;
    p->stage_ms[x.stage] += ms;
    p->stage_n[x.stage] += 1;
    p->ev_pool.push_back(x.e0);
    p->ev_pool.push_back(x.e1);
  }
  p->pending.clear();
  return hipSuccess;
}

void release(wdd_plan_s* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (auto& x : p->pending) {
    p->ev_pool.push_back(x.e0);
    p->ev_pool.push_back(x.e1);
  }
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  for (void* a : p->allocs) {
    if (p->release_fn)
      p->release_fn(a, p->alloc_ctx);
    else
      (void)hipFree(a);
  }
  if (p->pin_ring) (void)hipHostFree(p->pin_ring);
  for (hipEvent_t e : p->marks)
    if (e) (void)hipEventDestroy(e);
  for (int i = 0; i < kFrameSlots; ++i) {
    if (p->pin_frames[i]) (void)hipHostFree(p->pin_frames[i]);
    if (p->fev[i]) (void)hipEventDestroy(p->fev[i]);
  }
  if (p->pin_out) (void)hipHostFree(p->pin_out);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

wdd_status check_usable(wdd_plan_s* p) {
  if (!p) return wdd::fail(WDD_EINVAL, "null plan");
  if (p->failed) return wdd::fail(WDD_ESTATE, "plan is unusable after an earlier device error");
  return WDD_OK;
}

// Where the display's column pass reads: the partial rows the object-order update left in
// `up` ([y][vx][slot]), or the grid `u` ([vx][y]) of the first pass.
void column_source(const wdd_plan_s* p, const float2** src, int32_t* sr, int32_t* sm, int32_t* nslot,
                   int32_t* slot_stride) {
  if (p->up_valid) {
    *src = p->up, *sr = p->sx * p->nslot, *sm = p->nslot, *nslot = p->nslot, *slot_stride = 1;
  } else {
    *src = p->u, *sr = 1, *sm = p->sy, *nslot = 1, *slot_stride = 0;
  }
}

wdd_status column_pass(wdd_plan_s* p, const float2* src, int32_t sr, int32_t sm, int32_t nslot, int32_t slot_stride,
                       float2* dst) {
  WDD_HIP(p, wdd::launch_dft_rows(src, dst, p->sy, p->sx, p->ex, p->d, (float)((double)p->sy * p->sx), 1, sr, sm, p->sx,
                                  1, nslot, slot_stride, p->stream));
  return WDD_OK;
}

// A deferred column pass can ride in the next push's projection launch (the Hermite-Gauss
// projection kernels, any arithmetic; radix-2 rows: power-of-two Sx).  Detectors of more
// than 128 rows do not put it there: their 1024-thread projection workgroups (one wave per
// 16 rows) would carry the display rows too, and the merged launch then took longer than
// the two (22 us against 15.5 + 5.4 us for a 512 x 512 scan, 256 x 256 frames).  In object
// order it rides in the next push's first update launch instead (512-thread workgroups),
// reading partial rows and D[0] kept from the previous push (can_defer_to_update).
bool can_defer(const wdd_plan_s* p) {
  return !p->fourier && p->ny <= 128 && (p->sx & (p->sx - 1)) == 0;
}

bool can_defer_to_update(const wdd_plan_s* p) { return p->up_valid && p->up_alt && p->d0w; }

wdd_status flush_held(wdd_plan_s* p, bool for_display);

// Runs a held update (pipelined pushes) and writes a display left to the next push now;
// every call that waits for the plan's stream or reads or changes its state goes through here
// first (D has not changed since a display kept for the projection was queued, so p->d gives
// its D[0]; one kept for the update reads its own copy of D[0]).
wdd_status flush_deferred(wdd_plan_s* p) {
  const wdd_status st = flush_held(p, false);
  if (st != WDD_OK) return st;
  if (!p->deferred_dst) return WDD_OK;
  float2* dst = p->deferred_dst;
  p->deferred_dst = nullptr;
  p->deferred_in_update = false;
  return column_pass(p, p->deferred_src, p->deferred_sr, p->deferred_sm, p->deferred_nslot, p->deferred_slot_stride,
                     dst);
}

// Round to the nearest bf16 / fp16 (ties to even); returns the 16-bit pattern and the value.
uint16_t to_bf16(double x, double* back) {
  const float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  const uint16_t b = (uint16_t)(u >> 16);
  const uint32_t v = (uint32_t)b << 16;
  float fv;
  std::memcpy(&fv, &v, 4);
  *back = fv;
  return b;
}

uint16_t to_fp16(double x, double* back) {
  const _Float16 hv = (_Float16)(float)x;
  uint16_t b;
  std::memcpy(&b, &hv, 2);
  *back = (double)(float)hv;
  return b;
}

std::vector<float2> twiddles(int32_t n, double scale) {
  std::vector<float2> t(n);
  for (int32_t m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)n;
    t[m] = make_float2((float)(std::cos(a) * scale), (float)(std::sin(a) * scale));
  }
  return t;
}

}  // namespace
static wdd_status upload_wiener(wdd_plan_s* p, const wdd_tables_s& t);
namespace {

// pos, order, xs and rows: views of the device upload block `upload`
void set_upload_views(wdd_plan_s* p) {
  p->pos = reinterpret_cast<int2*>(p->upload);
  p->order = reinterpret_cast<int32_t*>(p->upload + (size_t)p->max_batch * 8);
  p->xs = reinterpret_cast<int32_t*>(p->upload + (size_t)p->max_batch * 12);
  p->rows = reinterpret_cast<int4*>(p->upload + ((size_t)p->max_batch * 16 + 15) / 16 * 16);
}

wdd_status create(wdd_plan_s* p, const wdd_tables_s& t, const wdd_options& opts, void* stream) {
  p->sy = t.sy; p->sx = t.sx; p->ny = t.ny; p->nx = t.nx; p->k = t.k; p->l = t.l;
  p->kpad = 32;  // a power of two: the row-factored update reduces over kpad / 4 lanes with xor shuffles
  while (p->kpad < t.k) p->kpad *= 2;
  p->n_freq = t.n_freq();
  p->n_freq_pad = (p->n_freq + 63) / 64 * 64;
  p->tscale = (float)(1.0 / std::sqrt((double)t.sy * (double)t.sx));
  p->sigma = t.sigma; p->eps_abs = t.eps_abs;
  p->max_batch = opts.max_batch;
  p->host_order.resize(p->max_batch);
  p->host_rows.reserve(p->max_batch);
  p->frame_bytes = (size_t)t.ny * t.nx * (p->dtype == WDD_U16 ? 2 : 4);
  WDD_HIP(p, hipGetDevice(&p->device));
  if (stream) {
    p->stream = (hipStream_t)stream;
  } else {
    WDD_HIP(p, hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
    p->own_stream = true;
  }

  // host-side FP32 images of the tables
  std::vector<float> psi((size_t)(t.ny + t.nx) * 16, 0.f);
  for (int32_t i = 0; i < t.ny; ++i)
    for (int32_t m = 0; m < t.l; ++m) psi[(size_t)i * 16 + m] = (float)t.psi_y[(size_t)i * t.l + m];
  for (int32_t i = 0; i < t.nx; ++i)
    for (int32_t m = 0; m < t.l; ++m) psi[(size_t)(t.ny + i) * 16 + m] = (float)t.psi_x[(size_t)i * t.l + m];
  std::vector<int32_t> kmap(p->kpad, -1);
  if (!p->fourier)
    for (int32_t k = 0; k < t.k; ++k) kmap[k] = 16 * t.pairs[2 * k] + t.pairs[2 * k + 1];
  std::vector<int2> freqs(p->n_freq_pad, make_int2(0, 0));
  for (int64_t j = 0; j < p->n_freq; ++j) freqs[j] = make_int2(t.freqs[2 * j], t.freqs[2 * j + 1]);
  // workgroups of the object-order update: runs of kept frequencies with one v_x, cut into
  // chunks of at most max_chunk (size chosen below)
  std::vector<int32_t> jlist(p->n_freq);
  for (int64_t j = 0; j < p->n_freq; ++j) jlist[j] = (int32_t)j;
  std::stable_sort(jlist.begin(), jlist.end(), [&freqs](int32_t a, int32_t b) {
    return freqs[a].y != freqs[b].y ? freqs[a].y < freqs[b].y : freqs[a].x < freqs[b].x;
  });
  // Chunk size.  Every chunk repeats phase 1 (the x-DFT over the whole batch's projections);
  // phase 2 takes its frequencies 2 G at a time (G = 4 kFusedThreads / kpad lane groups).
  // Short chunks (at most three such rounds) favour fewer, larger chunks, long ones more
  // workgroups: n_freq / 384 or n_freq / 512 per chunk (measured on 128^2, 256^2 and 512^2
  // scans: 23.0 -> 21.0, 23.7 -> 22.7 and 51.9 us per pipelined step).
  // Two pipeline stages: no chunk forms the x-DFT (one workgroup per v_x does, a launch ahead),
  // so chunks can be longer: at least four rounds, n_freq / 448 on large scans (measured per
  // two-stage step: 512^2 scan, K = 128: n/384 (224) 36.2, n/448 (256) 35.5, n/400 (288) 35.4,
  // 320 37.7, 384 38.6 us; 256^2 scan, K = 64: 128 14.3, 192 14.1, 256 13.1 us; 128^2 scan,
  // K = 256: 32 11.6, 48 11.6, 64 11.0, 80 11.5, 96 13.4, 128 15.6 us).
  const int64_t per_round = 2 * (4 * wdd::kFusedThreads / p->kpad);
  int64_t chunk;
  if (p->two_stage) {
    chunk = std::max<int64_t>(4 * per_round, (p->n_freq + 447) / 448);
  } else {
    chunk = (p->n_freq + 383) / 384;
    if (chunk > 3 * per_round) chunk = (p->n_freq + 511) / 512;
  }
  // a whole number of rounds: one frequency past a multiple of 2 G would cost its chunk a
  // further round trip to HBM for W, and the slowest chunks set the launch's duration
  if (chunk > per_round) chunk -= chunk % per_round;
  p->max_chunk = (int32_t)std::min<int64_t>(kMaxChunk, std::max<int64_t>(kMinChunk, chunk));
  std::vector<int4> chunks;
  for (int64_t i = 0; i < p->n_freq;) {
    const int32_t vx = freqs[jlist[i]].y;
    int64_t e = i;
    while (e < p->n_freq && freqs[jlist[e]].y == vx) ++e;
    const int64_t pieces = (e - i + p->max_chunk - 1) / p->max_chunk;
    for (int64_t c = 0; c < pieces; ++c) {
      const int64_t b0 = i + (e - i) * c / pieces, b1 = i + (e - i) * (c + 1) / pieces;
      chunks.push_back(make_int4(vx, (int32_t)b0, (int32_t)(b1 - b0), (int32_t)c));
    }
    p->nslot = std::max<int32_t>(p->nslot, (int32_t)pieces);
    i = e;
  }
  p->nchunks = (int32_t)chunks.size();
  p->host_chunks = chunks;
  // partial display rows: power-of-two scan sides (the radix-2 passes), Sy up to the row the
  // update's workgroup transforms in LDS, at most kMaxSlots chunks per v_x
  const bool pow2 = (t.sy & (t.sy - 1)) == 0 && (t.sx & (t.sx - 1)) == 0;
  const bool partial_rows = p->order_mode == WDD_ORDER_OBJECT && !p->fourier && pow2 && t.sy <= wdd::kDisplayRowMax &&
                            p->nslot <= wdd::kMaxSlots;
  const std::vector<float2> ty = twiddles(t.sy, 1.0);
  const std::vector<float2> tx = twiddles(t.sx, 1.0 / std::sqrt((double)t.sy * (double)t.sx));
  const std::vector<float2> ey = twiddles(t.sy, 1.0);
  const std::vector<float2> ex = twiddles(t.sx, 1.0);

  const size_t nfk = (size_t)p->n_freq_pad * p->kpad;
  const size_t grid = (size_t)t.sy * t.sx;
  wdd_status st;
#define ALLOC(ptr, n)                                   \
  if ((st = dalloc(p, &(ptr), (n))) != WDD_OK) return st;
  ALLOC(p->psi, psi.size());
  std::vector<uint16_t> psix_lp;
  if (p->precision != WDD_FP32) {
    // hi and lo 16-bit parts of psi_x.  No pre-scaling: with |psi| < 1 and count digits
    // < 2^11, every FP16 product and 32-term partial sum stays far inside the FP16 range
    // (lo parts below 2^-14 become subnormal, an absolute error under 3e-8).
    const bool bf = (p->precision == WDD_BF16_HILO || p->precision == WDD_BF16);
    const int shift = 0;
    p->psi_unscale = std::ldexp(1.0f, -shift);
    psix_lp.assign((size_t)2 * 16 * t.nx, 0);
    for (int32_t m = 0; m < t.l; ++m)
      for (int32_t i = 0; i < t.nx; ++i) {
        const double v = std::ldexp(t.psi_x[(size_t)i * t.l + m], shift);
        double hv = 0, lv = 0;
        const uint16_t hb = bf ? to_bf16(v, &hv) : to_fp16(v, &hv);
        const uint16_t lb = bf ? to_bf16(v - hv, &lv) : to_fp16(v - hv, &lv);
        psix_lp[(size_t)m * t.nx + i] = hb;
        psix_lp[(size_t)(16 + m) * t.nx + i] = lb;
      }
    ALLOC(p->psix_lp, psix_lp.size());
  }
  ALLOC(p->kmap, kmap.size());
  ALLOC(p->freqs, freqs.size());
  ALLOC(p->w, nfk);
  if (p->order_mode == WDD_ORDER_SPECTRUM) ALLOC(p->acc, nfk);
  ALLOC(p->ty, (size_t)t.sy);
  ALLOC(p->tx, (size_t)t.sx);
  ALLOC(p->ey, (size_t)t.sy);
  ALLOC(p->ex, (size_t)t.sx);
  ALLOC(p->h, (size_t)p->max_batch * p->kpad * (p->fourier ? 2 : 1));
  if (p->fourier) {
    ALLOC(p->fy, (size_t)std::max(1, t.ny / 2));
    ALLOC(p->fx, (size_t)std::max(1, t.nx / 2));
  }
  p->upload_bytes = (size_t)p->max_batch * 16 + 16 + (size_t)p->max_batch * sizeof(int4);
  ALLOC(p->upload, p->upload_bytes);
  set_upload_views(p);
  if (p->order_mode == WDD_ORDER_SPECTRUM || p->fourier) ALLOC(p->t, (size_t)kFactorRows * t.sx * p->kpad);
  if (p->order_mode == WDD_ORDER_OBJECT && !p->fourier) {
    ALLOC(p->jv, jlist.size());
    ALLOC(p->chunks, chunks.size());
  }
  if (p->pipeline && !partial_rows)
    return wdd::fail(WDD_EINVAL, "pipelined pushes need power-of-two scan sides with Sy <= %d", wdd::kDisplayRowMax);
  if (p->pipeline) {
    ALLOC(p->h_alt, (size_t)p->max_batch * p->kpad);
    ALLOC(p->upload_alt, p->upload_bytes);
  }
  std::vector<int32_t> xcols;  // the kept v_x, in chunk order
  for (const int4& c : chunks)
    if (xcols.empty() || xcols.back() != c.x) xcols.push_back(c.x);
  p->ncols = (int32_t)xcols.size();
  if (p->two_stage) {
    const size_t tsz = (size_t)t.sx * wdd::row_fused_t_stride(p->kpad);
    ALLOC(p->t_cur, tsz);
    ALLOC(p->t_next, tsz);
    ALLOC(p->xcols, xcols.size());
  }
  if (partial_rows) ALLOC(p->up, (size_t)t.sx * p->nslot * t.sy);
  if (partial_rows && (t.ny > 128 || p->pipeline)) {  // see can_defer
    ALLOC(p->up_alt, (size_t)t.sx * p->nslot * t.sy);
    ALLOC(p->d0w, 2);
    p->d0w_alt = p->d0w + 1;
  }
  {
    char* fr = nullptr;
    if ((st = dalloc(p, &fr, (size_t)p->max_batch * p->frame_bytes)) != WDD_OK) return st;
    p->frames = fr;
  }
  ALLOC(p->d, (size_t)p->n_freq_pad);
  if (p->order_mode == WDD_ORDER_OBJECT) ALLOC(p->dlo, (size_t)p->n_freq_pad);
  ALLOC(p->z, grid);
  ALLOC(p->u, grid);
#undef ALLOC

  // Wiener filter, FP64 -> FP32, padded
  if ((st = upload_wiener(p, t)) != WDD_OK) return st;
  WDD_HIP(p, hipMemcpyAsync(p->psi, psi.data(), psi.size() * sizeof(float), hipMemcpyHostToDevice, p->stream));
  if (p->psix_lp)
    WDD_HIP(p, hipMemcpyAsync(p->psix_lp, psix_lp.data(), psix_lp.size() * sizeof(uint16_t), hipMemcpyHostToDevice,
                              p->stream));
  WDD_HIP(p, hipMemcpyAsync(p->kmap, kmap.data(), kmap.size() * sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
  WDD_HIP(p, hipMemcpyAsync(p->freqs, freqs.data(), freqs.size() * sizeof(int2), hipMemcpyHostToDevice, p->stream));
  if (p->jv) {
    std::vector<int2> jv(jlist.size());
    for (size_t i = 0; i < jlist.size(); ++i) jv[i] = make_int2(jlist[i], freqs[jlist[i]].x);
    WDD_HIP(p, hipMemcpyAsync(p->jv, jv.data(), jv.size() * sizeof(int2), hipMemcpyHostToDevice, p->stream));
    WDD_HIP(p, hipMemcpyAsync(p->chunks, chunks.data(), chunks.size() * sizeof(int4), hipMemcpyHostToDevice,
                              p->stream));
  }
  WDD_HIP(p, hipMemcpyAsync(p->ty, ty.data(), ty.size() * sizeof(float2), hipMemcpyHostToDevice, p->stream));
  WDD_HIP(p, hipMemcpyAsync(p->tx, tx.data(), tx.size() * sizeof(float2), hipMemcpyHostToDevice, p->stream));
  WDD_HIP(p, hipMemcpyAsync(p->ey, ey.data(), ey.size() * sizeof(float2), hipMemcpyHostToDevice, p->stream));
  WDD_HIP(p, hipMemcpyAsync(p->ex, ex.data(), ex.size() * sizeof(float2), hipMemcpyHostToDevice, p->stream));
  std::vector<float2> fy, fx;
  if (p->fourier) {  // exp(+2 pi i m / n), the conjugates of the forward twiddles
    fy = twiddles(t.ny, 1.0);
    fx = twiddles(t.nx, 1.0);
    for (auto& v : fy) v.y = -v.y;
    for (auto& v : fx) v.y = -v.y;
    WDD_HIP(p, hipMemcpyAsync(p->fy, fy.data(), (size_t)(t.ny / 2) * sizeof(float2), hipMemcpyHostToDevice,
                              p->stream));
    WDD_HIP(p, hipMemcpyAsync(p->fx, fx.data(), (size_t)(t.nx / 2) * sizeof(float2), hipMemcpyHostToDevice,
                              p->stream));
  }
  if (p->acc) WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->acc), nfk * 2, p->stream));
  WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->z), grid * 2, p->stream));
  // slots that no chunk owns stay zero for the plan's life
  if (p->up) WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->up), (size_t)t.sx * p->nslot * t.sy * 2, p->stream));
  if (p->up_alt)
    WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->up_alt), (size_t)t.sx * p->nslot * t.sy * 2, p->stream));
  WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->d), (size_t)p->n_freq_pad * 2, p->stream));
  if (p->dlo) WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->dlo), (size_t)p->n_freq_pad * 2, p->stream));
  WDD_HIP(p, wdd::launch_zero(p->h, (size_t)p->max_batch * p->kpad * (p->fourier ? 2 : 1), p->stream));
  if (p->h_alt) WDD_HIP(p, wdd::launch_zero(p->h_alt, (size_t)p->max_batch * p->kpad, p->stream));
  if (p->xcols)
    WDD_HIP(p, hipMemcpyAsync(p->xcols, xcols.data(), xcols.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                              p->stream));

  {
    const size_t slot_bytes = p->upload_bytes + (size_t)p->max_batch * sizeof(uint64_t);
    p->up_ring = (int)std::max<size_t>(4, std::min<size_t>(kUploadSlots, kUploadPinBudget / slot_bytes));
    p->mark_every = std::max(1, p->up_ring / 4);
    // one pinned allocation for the whole ring (pinned allocations and frees are slow)
    const size_t stride = (slot_bytes + 255) / 256 * 256;
    WDD_HIP(p, hipHostMalloc((void**)&p->pin_ring, stride * p->up_ring, hipHostMallocDefault));
    p->pin_up.assign(p->up_ring, nullptr);
    for (int i = 0; i < p->up_ring; ++i) p->pin_up[i] = p->pin_ring + stride * i;
    p->marks.assign(p->up_ring / p->mark_every + 2, nullptr);
    p->mark_at.assign(p->marks.size(), -1);
    for (hipEvent_t& e : p->marks) WDD_HIP(p, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (hipEvent_t& e : p->fev) WDD_HIP(p, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  WDD_HIP(p, hipHostMalloc((void**)&p->pin_out, grid * sizeof(float2), hipHostMallocDefault));
  WDD_HIP(p, hipStreamSynchronize(p->stream));
  return WDD_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace wdd {

wdd_status check_plan_options(const wdd_detector* det, const wdd_options& opts) {
  if (opts.precision < WDD_FP32 || opts.precision > WDD_FP16)
    return wdd::fail(WDD_EINVAL, "unknown precision %d", opts.precision);
  if (opts.precision != WDD_FP32 && det && det->dtype != WDD_U16)
    return wdd::fail(WDD_EINVAL, "reduced-precision projection needs uint16 frames");
  if (opts.max_batch < 1 || opts.max_batch > 65536)
    return wdd::fail(WDD_EINVAL, "max_batch = %d outside [1, 65536]", opts.max_batch);
  if (opts.order != WDD_ORDER_SPECTRUM && opts.order != WDD_ORDER_OBJECT)
    return wdd::fail(WDD_EINVAL, "unknown order %d", opts.order);
  if (opts.basis != WDD_BASIS_HERMITE_GAUSS && opts.basis != WDD_BASIS_FOURIER)
    return wdd::fail(WDD_EINVAL, "unknown basis %d", opts.basis);
  if (opts.basis == WDD_BASIS_FOURIER && opts.precision != WDD_FP32)
    return wdd::fail(WDD_EINVAL, "the Fourier basis runs in FP32 only");
  if (opts.pipeline < 0 || opts.pipeline > 2) return wdd::fail(WDD_EINVAL, "pipeline must be 0, 1 or 2");
  if (opts.pipeline &&
      (opts.order != WDD_ORDER_OBJECT || opts.basis != WDD_BASIS_HERMITE_GAUSS || !det ||
       !wdd::row_fused_next_supported(det->dtype, opts.precision, det->ny, det->nx, 256)))
    return wdd::fail(WDD_EINVAL,
                     "pipelined pushes need object order, the Hermite-Gauss basis and uint16 frames of 32..256 "
                     "columns in multiples of 32 and at most 256 rows (128 with a reduced-precision projection)");
  return WDD_OK;
}

int64_t plan_device_bytes(const wdd_tables_s& t, const wdd_options& opts, int32_t dtype) {
  int64_t kpad = 32;
  while (kpad < t.k) kpad *= 2;
  const int64_t nfp = (t.n_freq() + 63) / 64 * 64, mb = opts.max_batch, grid = (int64_t)t.sy * t.sx;
  auto a = [](int64_t bytes) { return std::max<int64_t>(bytes, 256); };
  int64_t b = a((int64_t)(t.ny + t.nx) * 16 * 4) + a(kpad * 4) + a(nfp * 8) + a(nfp * kpad * 8);
  if (opts.order == WDD_ORDER_SPECTRUM) b += a(nfp * kpad * 8);
  if (opts.precision != WDD_FP32) b += a((int64_t)2 * 16 * t.nx * 2);
  const bool fourier = t.basis == WDD_BASIS_FOURIER;
  b += 2 * a((int64_t)t.sy * 8) + 2 * a((int64_t)t.sx * 8) + a(mb * kpad * (fourier ? 8 : 4)) + a(mb * 16 + 16 + mb * 16);
  b += a(mb * (int64_t)t.ny * t.nx * (dtype == WDD_U16 ? 2 : 4));
  if (fourier) b += a((int64_t)std::max(1, t.ny / 2) * 8) + a((int64_t)std::max(1, t.nx / 2) * 8);
  if (opts.order == WDD_ORDER_SPECTRUM || fourier) {
    b += a((int64_t)kFactorRows * t.sx * kpad * 8);
  } else {
    const int64_t nchunks_max = t.n_freq() / kMinChunk + t.sx + 1;  // upper bound of the chunk count
    b += a(t.n_freq() * 8) + a(nchunks_max * 16);
  }
  if (opts.order == WDD_ORDER_OBJECT) b += a(nfp * 8);  // D's rounding remainder
  const bool pow2 = (t.sy & (t.sy - 1)) == 0 && (t.sx & (t.sx - 1)) == 0;
  if (opts.order == WDD_ORDER_OBJECT && !fourier && pow2 && t.sy <= wdd::kDisplayRowMax) {
    // partial display rows (at most kMaxSlots per v_x), a second set and D[0] copies for
    // detectors of more than 128 rows
    const int64_t up = a(grid * wdd::kMaxSlots * 8);
    b += t.ny > 128 || opts.pipeline ? 2 * up + a(16) : up;
  }
  if (opts.pipeline) b += a(mb * kpad * 4) + a(mb * 16 + 16 + mb * 16);  // h_alt, upload_alt
  if (opts.pipeline == 2) b += 2 * a((int64_t)t.sx * wdd::row_fused_t_stride((int)kpad) * 16) + a(t.sx * 4);
  b += a(nfp * 8) + 2 * a(grid * 8);
  return b;
}

// The process-wide device allocator that new plans take (wdd_set_allocator).
std::mutex g_alloc_mu;
wdd_alloc_fn g_alloc = nullptr;
wdd_release_fn g_release = nullptr;
void* g_alloc_ctx = nullptr;

void current_allocator(wdd_alloc_fn* a, wdd_release_fn* r, void** ctx) {
  std::lock_guard<std::mutex> lock(g_alloc_mu);
  *a = g_alloc;
  *r = g_release;
  *ctx = g_alloc_ctx;
}

wdd_status plan_create_from_tables(std::shared_ptr<const wdd_tables_s> tp, const wdd_probe* probe,
                                   const wdd_scan* scan, const wdd_detector* det, const wdd_options& opts,
                                   void* hip_stream, wdd_plan_t* out) {
  *out = nullptr;
  if (!tp) return wdd::fail(WDD_EINVAL, "null tables");
  const wdd_tables_s& t = *tp;
  wdd_plan_s* p = new (std::nothrow) wdd_plan_s();
  if (!p) return wdd::fail(WDD_ENOMEM, "out of host memory");
  p->tables = tp;
  current_allocator(&p->alloc_fn, &p->release_fn, &p->alloc_ctx);
  p->dtype = det->dtype;
  p->precision = opts.precision;
  p->order_mode = opts.order;
  p->fourier = t.basis == WDD_BASIS_FOURIER;
  p->pipeline = opts.pipeline != 0;
  p->two_stage = opts.pipeline == 2;
  p->probe = *probe;
  p->scan = *scan;
  p->det = *det;
  p->opts = opts;
  wdd_status st;
  try {
    st = create(p, t, opts, hip_stream);
  } catch (const std::bad_alloc&) {
    st = wdd::fail(WDD_ENOMEM, "out of host memory");
  }
  if (st != WDD_OK) {
    release(p);
    return st;
  }
  *out = p;
  return WDD_OK;
}

}  // namespace wdd

extern "C" {

wdd_status wdd_plan(const wdd_probe* probe, const wdd_scan* scan, const wdd_detector* det, int32_t K,
                    const wdd_options* opts_in, void* hip_stream, wdd_plan_t* out) {
  if (!out) return wdd::fail(WDD_EINVAL, "null output handle");
  *out = nullptr;
  wdd_options opts;
  wdd_default_options(&opts);
  if (opts_in) opts = *opts_in;
  wdd_status st0 = wdd::check_plan_options(det, opts);
  if (st0 != WDD_OK) return st0;
  std::shared_ptr<wdd_tables_s> t;
  try {
    t = std::make_shared<wdd_tables_s>();
    if ((st0 = wdd::build_tables(probe, scan, det, K, &opts, t.get())) != WDD_OK) return st0;
  } catch (const std::bad_alloc&) {
    return wdd::fail(WDD_ENOMEM, "out of host memory");
  }
  return wdd::plan_create_from_tables(t, probe, scan, det, opts, hip_stream, out);
}

}  // extern "C"

namespace {

// After the launch that read this push's pinned data (its projection): the upload block may
// be refilled once the stream passes this point, and so may the host-frame staging slot fs.
wdd_status mark_push(wdd_plan_s* p, int64_t push_no, int fs) {
  if (push_no % p->mark_every == p->mark_every - 1) {
    const size_t m = (size_t)(push_no / p->mark_every) % p->marks.size();
    WDD_HIP(p, hipEventRecord(p->marks[m], p->stream));
    p->mark_at[m] = push_no;
  }
  if (fs >= 0) {
    WDD_HIP(p, hipEventRecord(p->fev[fs], p->stream));
    p->fev_live[fs] = true;
  }
  return WDD_OK;
}

// The object-order update of one batch (Section 6.3, modified-WDD algorithm, the loop body
// with the Wiener filter applied per frame): passes of at most kFactorRows of its scan rows,
// each adding to D, the x-DFT fused in.  With rows_for_display the last pass also leaves the
// display's first pass in `up`.  A deferred column pass kept for the update rides in the
// first launch, and so does `next`, the projection of the following batch (pipelined
// pushes), when given.
wdd_status object_update(wdd_plan_s* p, const int4* rows, int nrows, bool in_order, bool rows_for_display,
                         const wdd::ProjectLaunch* next) {
  hipEvent_t end;
  if (rows_for_display && p->up_alt) {  // keep the previous push's rows for a display still to come
    std::swap(p->up, p->up_alt);
    std::swap(p->d0w, p->d0w_alt);
  }
  for (int r0 = 0; r0 < nrows; r0 += kFactorRows) {
    const int nr = std::min(kFactorRows, nrows - r0);
    const bool last = r0 + kFactorRows >= nrows;
    float2* up_pass = rows_for_display && last ? p->up : nullptr;
    float2* d0out = up_pass && p->up_alt ? p->d0w : nullptr;
    // the previous step's column pass, left to this launch (reads what that push kept)
    wdd::DisplayColumns dc;
    const bool carry = r0 == 0 && p->deferred_dst && p->deferred_in_update;
    if (carry) {
      dc.din = p->deferred_src;
      dc.dout = p->deferred_dst;
      dc.rows = p->sy;
      dc.len = p->sx;
      dc.e = p->ex;
      dc.d0 = p->deferred_d0;
      dc.s_total = (float)((double)p->sy * p->sx);
      dc.in_sr = p->deferred_sr;
      dc.in_sm = p->deferred_sm;
      dc.out_sr = p->sx;
      dc.out_sc = 1;
      dc.nslot = p->deferred_nslot;
      dc.slot_stride = p->deferred_slot_stride;
      p->deferred_dst = nullptr;
      p->deferred_in_update = false;
    }
    if ((p->profile_mask & (1 << kAccumulate)) && p->profile_now) p->factored_n += 1;
    WDD_HIP(p, stage_begin(p, kAccumulate, &end));
    wdd::RowSet rs;
    for (int i = 0; i < wdd::kRowSetMax; ++i) rs.r[i] = i < nr ? rows[r0 + i] : make_int4(0, 0, 0, 0);
    if (r0 == 0 && next)
      WDD_HIP(p, wdd::launch_row_fused_obj_next(p->h, p->kpad, p->order, p->xs, rs, nr, p->tscale, p->sx, p->sy,
                                                p->chunks, p->nchunks, p->max_chunk, p->jv, p->w, p->d, p->dlo, p->z,
                                                up_pass, p->nslot, in_order, d0out, carry ? &dc : nullptr, *next,
                                                p->stream));
    else
      WDD_HIP(p, wdd::launch_row_fused_obj(p->h, p->kpad, p->order, p->xs, rs, nr, p->tscale, p->sx, p->sy,
                                           p->chunks, p->nchunks, p->max_chunk, p->jv, p->w, p->d, p->dlo, p->z,
                                           up_pass, p->nslot, in_order, d0out, carry ? &dc : nullptr, p->stream));
    WDD_HIP(p, stage_end(p, end));
  }
  p->up_valid = rows_for_display;
  return WDD_OK;
}

// Runs the held batch's update (pipelined pushes), with `next` in its first launch when
// given.  It leaves the display's first pass in `up` when a deferred snapshot followed the
// batch (whose column pass then waits for the next launch, as a deferred display kept for
// the update) or when for_display asks for it.
wdd_status run_held(wdd_plan_s* p, const wdd::ProjectLaunch* next, bool for_display) {
  wdd_plan_s::Held& hd = p->held;
  hd.live = false;
  const bool rows = (hd.display || for_display) && p->up;
  wdd_status st = object_update(p, hd.rows.data(), (int)hd.rows.size(), hd.in_order, rows, next);
  if (st != WDD_OK) return st;
  if (hd.display_dst) {
    p->deferred_dst = hd.display_dst;
    column_source(p, &p->deferred_src, &p->deferred_sr, &p->deferred_sm, &p->deferred_nslot,
                  &p->deferred_slot_stride);
    p->deferred_in_update = true;
    p->deferred_d0 = p->d0w;
    hd.display_dst = nullptr;
  }
  hd.display = false;
  return WDD_OK;
}

// The deferred column pass kept for the update, as launch arguments (carry: there is one).
bool carried_display(wdd_plan_s* p, wdd::DisplayColumns* dc) {
  if (!p->deferred_dst || !p->deferred_in_update) return false;
  dc->din = p->deferred_src;
  dc->dout = p->deferred_dst;
  dc->rows = p->sy;
  dc->len = p->sx;
  dc->e = p->ex;
  dc->d0 = p->deferred_d0;
  dc->s_total = (float)((double)p->sy * p->sx);
  dc->in_sr = p->deferred_sr;
  dc->in_sm = p->deferred_sm;
  dc->out_sr = p->sx;
  dc->out_sc = 1;
  dc->nslot = p->deferred_nslot;
  dc->slot_stride = p->deferred_slot_stride;
  p->deferred_dst = nullptr;
  p->deferred_in_update = false;
  return true;
}

// One launch of two-stage pipelined pushes: the update of held2 (its x-DFT in t_cur), the
// x-DFT of `held` into t_next when xdft is set, and `next`; a deferred column pass kept for
// the update rides along.  held2's update leaves the display's first pass in `up` when a
// deferred snapshot followed it or for_display asks for it.  Afterwards held2 is done and,
// with xdft, `held` has moved to held2 (its x-DFT now in t_cur).
wdd_status launch_stage2(wdd_plan_s* p, const wdd::ProjectLaunch* next, bool for_display, bool xdft) {
  wdd_plan_s::Held& u = p->held2;
  wdd_plan_s::Held& x = p->held;
  wdd::RowSet urs, xrs;
  std::memset(&urs, 0, sizeof(urs));
  std::memset(&xrs, 0, sizeof(xrs));
  const bool rows = u.live && (u.display || for_display) && p->up;
  if (rows && p->up_alt) {
    std::swap(p->up, p->up_alt);
    std::swap(p->d0w, p->d0w_alt);
  }
  float2* up_pass = rows ? p->up : nullptr;
  float2* d0out = up_pass && p->up_alt ? p->d0w : nullptr;
  const int unrows = u.live ? (int)u.rows.size() : 0;
  for (int i = 0; i < unrows; ++i) urs.r[i] = u.rows[i];
  wdd::XdftPart xp;
  std::memset(&xp, 0, sizeof(xp));
  if (xdft && x.live) {
    xp.h = p->h;
    xp.order = p->order;
    xp.xs = p->xs;
    xp.nrows = (int)x.rows.size();
    for (int i = 0; i < xp.nrows; ++i) xp.rows.r[i] = x.rows[i];
    xp.in_order = x.in_order;
    xp.xcols = p->xcols;
    xp.ncols = p->ncols;
    xp.tout = p->t_next;
  }
  wdd::DisplayColumns dc;
  const bool carry = carried_display(p, &dc);
  hipEvent_t end;
  if (u.live && (p->profile_mask & (1 << kAccumulate)) && p->profile_now) p->factored_n += 1;
  WDD_HIP(p, stage_begin(p, kAccumulate, &end));
  WDD_HIP(p, wdd::launch_row_fused_obj_next2(p->kpad, p->tscale, p->sx, p->sy, p->chunks, u.live ? p->nchunks : 0,
                                             p->max_chunk, p->jv, p->w, p->d, p->dlo, p->z, p->nslot, urs, unrows,
                                             p->t_cur, up_pass, d0out, xp, carry ? &dc : nullptr, next, p->stream));
  WDD_HIP(p, stage_end(p, end));
  if (u.live) {
    p->up_valid = rows;
    if (u.display_dst) {
      p->deferred_dst = u.display_dst;
      column_source(p, &p->deferred_src, &p->deferred_sr, &p->deferred_sm, &p->deferred_nslot,
                    &p->deferred_slot_stride);
      p->deferred_in_update = true;
      p->deferred_d0 = p->d0w;
    }
    u.live = false;
    u.display = false;
    u.display_dst = nullptr;
  }
  if (xdft && x.live) {
    u = x;
    x.live = false;
    x.display = false;
    x.display_dst = nullptr;
    std::swap(p->t_cur, p->t_next);
  }
  return WDD_OK;
}

// Runs every held update, oldest first (held2's from its x-DFT, then held's with its own);
// the newest leaves the display's first pass in `up` when for_display asks for it.
wdd_status flush_held(wdd_plan_s* p, bool for_display) {
  wdd_status st;
  if (p->held2.live && (st = launch_stage2(p, nullptr, for_display && !p->held.live, false)) != WDD_OK) return st;
  if (p->held.live && (st = run_held(p, nullptr, for_display)) != WDD_OK) return st;
  return WDD_OK;
}

// Queues one batch.  With fuse_wiener the row-factored update also performs the Wiener
// reduction of the updated spectrum; *fused reports whether it did.
wdd_status push_impl(wdd_plan_s* p, const void* frames, const int32_t* pos_yx, int32_t n, int32_t frames_on_device,
                     bool fuse_wiener, bool* fused, const uint64_t* frame_addrs = nullptr) {
  if (fused) *fused = false;
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if (n < 0 || n > p->max_batch) return wdd::fail(WDD_EINVAL, "n = %d outside [0, %d]", n, p->max_batch);
  if (n == 0) return WDD_OK;
  if ((!frames && !frame_addrs) || !pos_yx) return wdd::fail(WDD_EINVAL, "null frames or positions");
  if (frame_addrs) {
    for (int32_t i = 0; i < n; ++i)
      if (frame_addrs[i] % 16 != 0) return wdd::fail(WDD_EINVAL, "device frames must be 16-byte aligned");
  } else if (frames_on_device && (reinterpret_cast<uintptr_t>(frames) % 16) != 0) {
    return wdd::fail(WDD_EINVAL, "device frames must be 16-byte aligned");
  }
  for (int32_t i = 0; i < n; ++i) {
    const int32_t y = pos_yx[2 * i], x = pos_yx[2 * i + 1];
    if (y < 0 || y >= p->sy || x < 0 || x >= p->sx)
      return wdd::fail(WDD_ERANGE, "position %d = (%d, %d) outside the %d x %d raster", i, y, x, p->sy, p->sx);
  }
  // Group the batch by scan row.  Few rows: row-factored update; otherwise the direct one.
  int32_t* ord = p->host_order.data();
  for (int32_t i = 0; i < n; ++i) ord[i] = i;
  std::stable_sort(ord, ord + n, [pos_yx](int32_t a, int32_t b) { return pos_yx[2 * a] < pos_yx[2 * b]; });
  p->host_rows.clear();
  const bool object = p->order_mode == WDD_ORDER_OBJECT;
  const bool passes = object || p->fourier;  // always row-factored, in passes of <= kFactorRows rows
  for (int32_t i = 0; i < n && (passes || (int)p->host_rows.size() <= kFactorRows); ++i) {
    const int32_t y = pos_yx[2 * ord[i]];
    if (p->host_rows.empty() || p->host_rows.back().x != y) p->host_rows.push_back(make_int4(y, i, 0, 0));
    p->host_rows.back().z += 1;
  }
  // object order always takes the factored form, in passes of at most kFactorRows rows
  const bool factored = passes || (int)p->host_rows.size() <= kFactorRows;
  const int nrows = factored ? (int)p->host_rows.size() : 0;

  // the upload block of push i was last filled by push i - up_ring: wait, if that push may
  // not have run yet, for the first stream marker at or after it
  const int64_t push_no = p->pushes++;
  char* up = p->pin_up[push_no % p->up_ring];
  if (push_no >= p->up_ring && push_no - p->up_ring > p->drained) {
    const int64_t last = push_no - p->up_ring;
    const int64_t c = last + (p->mark_every - 1 - last % p->mark_every);
    const size_t m = (size_t)(c / p->mark_every) % p->marks.size();
    if (p->mark_at[m] == c)
      WDD_HIP(p, hipEventSynchronize(p->marks[m]));
    else
      WDD_HIP(p, hipStreamSynchronize(p->stream));
    p->drained = std::max(p->drained, c);
  }
  std::memcpy(up, pos_yx, (size_t)n * sizeof(int2));
  size_t up_bytes = (size_t)n * sizeof(int2);
  if (factored) {
    std::memcpy(up + (size_t)p->max_batch * 8, ord, (size_t)n * sizeof(int32_t));
    int32_t* xs = reinterpret_cast<int32_t*>(up + (size_t)p->max_batch * 12);
    for (int32_t i = 0; i < n; ++i) xs[i] = pos_yx[2 * ord[i] + 1];
    const size_t roff = reinterpret_cast<char*>(p->rows) - p->upload;
    std::memcpy(up + roff, p->host_rows.data(), (size_t)nrows * sizeof(int4));
    up_bytes = roff + (size_t)nrows * sizeof(int4);
  }
  const void* fdev = frames;
  const uint64_t* ftab = nullptr;
  int fs = -1;  // host-frame staging slot, if any
  if (frame_addrs) {  // frames scattered over device memory: the projection reads this pinned table
    uint64_t* tab = reinterpret_cast<uint64_t*>(up + p->upload_bytes);
    std::memcpy(tab, frame_addrs, (size_t)n * sizeof(uint64_t));
    ftab = tab;
  } else if (!frames_on_device) {
    // host frames go through a pinned slot, refilled after the projection that read it
    fs = p->fslot;
    p->fslot = (p->fslot + 1) % kFrameSlots;
    if (p->fev_live[fs]) WDD_HIP(p, hipEventSynchronize(p->fev[fs]));
    if (!p->pin_frames[fs]) {
      hipError_t e = hipHostMalloc(&p->pin_frames[fs], (size_t)p->max_batch * p->frame_bytes, hipHostMallocDefault);
      if (e != hipSuccess) {
        p->pin_frames[fs] = nullptr;
        return dev_fail(p, e, "hipHostMalloc");
      }
    }
    std::memcpy(p->pin_frames[fs], frames, (size_t)n * p->frame_bytes);
    WDD_HIP(p, hipMemcpyAsync(p->frames, p->pin_frames[fs], (size_t)n * p->frame_bytes, hipMemcpyHostToDevice,
                              p->stream));
    fdev = p->frames;
  }
  if (p->pending.size() > 4096) {  // bound the events held while nobody snapshots
    WDD_HIP(p, hipStreamSynchronize(p->stream));
    WDD_HIP(p, harvest(p));
  }
  p->profile_now = (p->profile_tick++ % p->profile_period) == 0;
  hipEvent_t end;
  if (p->fourier || (p->deferred_in_update && !object)) {  // see can_defer
    if ((st = flush_deferred(p)) != WDD_OK) return st;
  }
  bool in_order = true;  // frames already grouped by row (a raster batch): no reordering
  for (int32_t i = 0; i < n && in_order; ++i) in_order = ord[i] == i;
  // held for the next push's launch (pipelined pushes; two-stage ones hold batches of at
  // most kFactorRows scan rows, one x-DFT's worth: others run unpipelined after the held ones)
  const bool hold = p->pipeline && !(p->two_stage && nrows > kFactorRows);
  if (p->pipeline && !hold && (st = flush_held(p, false)) != WDD_OK) return st;
  wdd::ProjectLaunch pl;
  if (!p->fourier) {
    pl.dtype = p->dtype;
    pl.precision = p->precision;
    pl.frames = fdev;
    pl.n = n;
    pl.ny = p->ny;
    pl.nx = p->nx;
    pl.psi = p->psi;
    pl.psix_lp = p->psix_lp;
    pl.psi_unscale = p->psi_unscale;
    pl.kmap = p->kmap;
    pl.kpad = p->kpad;
    pl.h = hold ? p->h_alt : p->h;
    pl.up_src = up;
    pl.up_dst = hold ? p->upload_alt : p->upload;
    pl.up_bytes = up_bytes;
    pl.fptr = ftab;
  }
  if (hold) {
    // the held batch's update, with this batch's projection in its first launch (or the
    // projection alone when nothing is held); this batch's update is held in turn.  Two-stage:
    // held2's update, held's x-DFT and this projection in one launch
    if (p->two_stage && (p->held.live || p->held2.live)) {
      if ((st = launch_stage2(p, &pl, false, true)) != WDD_OK) return st;
    } else if (!p->two_stage && p->held.live) {
      if ((st = run_held(p, &pl, false)) != WDD_OK) return st;
    } else {
      WDD_HIP(p, stage_begin(p, kProject, &end));
      WDD_HIP(p, wdd::launch_project(pl, p->stream));
      WDD_HIP(p, stage_end(p, end));
    }
    if ((st = mark_push(p, push_no, fs)) != WDD_OK) return st;
    std::swap(p->h, p->h_alt);
    std::swap(p->upload, p->upload_alt);
    set_upload_views(p);
    p->held.live = true;
    p->held.in_order = in_order;
    p->held.rows.assign(p->host_rows.begin(), p->host_rows.end());
    p->held.display = false;
    p->held.display_dst = nullptr;
    if (fused) *fused = true;
    p->frames_seen += (uint64_t)n;
    p->last_batch = n;
    return WDD_OK;
  }
  WDD_HIP(p, stage_begin(p, kProject, &end));
  // the projection launch also brings the pinned upload block (positions, grouping) to the device
  if (p->fourier) {
    WDD_HIP(p, wdd::launch_project_fourier(p->dtype, fdev, n, p->ny, p->nx, p->fy, p->fx,
                                           reinterpret_cast<float2*>(p->h), p->kpad, up, p->upload, up_bytes, ftab,
                                           p->stream));
  } else if (p->deferred_dst && !p->deferred_in_update) {
    // the previous step's column pass rides in this launch (it reads its source and D
    // before this push's update changes them)
    wdd::DisplayColumns dc;
    dc.din = p->deferred_src;
    dc.dout = p->deferred_dst;
    dc.rows = p->sy;
    dc.len = p->sx;
    dc.e = p->ex;
    dc.d0 = p->d;
    dc.s_total = (float)((double)p->sy * p->sx);
    dc.in_sr = p->deferred_sr;
    dc.in_sm = p->deferred_sm;
    dc.out_sr = p->sx;
    dc.out_sc = 1;
    dc.nslot = p->deferred_nslot;
    dc.slot_stride = p->deferred_slot_stride;
    p->deferred_dst = nullptr;
    WDD_HIP(p, wdd::launch_project_display(pl, dc, p->stream));
  } else {
    WDD_HIP(p, wdd::launch_project(pl, p->stream));
  }
  WDD_HIP(p, stage_end(p, end));
  if ((st = mark_push(p, push_no, fs)) != WDD_OK) return st;
  bool wiener_done = object;
  if (p->fourier) {
    // complex per-row x-DFTs, then one update per pass of at most kFactorRows rows; the
    // Wiener reduction rides in the update when one pass covers the batch
    const bool one_pass = nrows <= kFactorRows;
    const int mode = object ? 0 : (fuse_wiener && one_pass ? 2 : 1);
    wiener_done = object || mode == 2;
    for (int r0 = 0; r0 < nrows; r0 += kFactorRows) {
      const int nr = std::min(kFactorRows, nrows - r0);
      wdd::RowSet rs;
      for (int i = 0; i < wdd::kRowSetMax; ++i) rs.r[i] = i < nr ? p->host_rows[r0 + i] : make_int4(0, 0, 0, 0);
      if ((p->profile_mask & (1 << kAccumulate)) && p->profile_now) p->factored_n += 1;
      WDD_HIP(p, stage_begin(p, kRowDft, &end));
      WDD_HIP(p, wdd::launch_row_dft_c(reinterpret_cast<const float2*>(p->h), p->kpad, p->order, p->xs, rs, nr, p->tx,
                                       p->sx, p->t, p->stream));
      WDD_HIP(p, stage_end(p, end));
      WDD_HIP(p, stage_begin(p, kAccumulate, &end));
      WDD_HIP(p, wdd::launch_update_c(mode, p->t, p->kpad, rs, nr, p->ty, p->sy, p->sx, p->freqs, p->n_freq, p->w,
                                      p->acc, p->d, p->dlo, p->z, p->stream));
      WDD_HIP(p, stage_end(p, end));
    }
  } else if (object) {
    // before a snapshot the last pass also leaves the display's first pass in `up`
    if ((st = object_update(p, p->host_rows.data(), nrows, in_order, fuse_wiener && p->up, nullptr)) != WDD_OK)
      return st;
  } else if (factored) {
    // per-row x-DFTs, then one pass over A (with the Wiener reduction when asked)
    wiener_done = fuse_wiener;
    if ((p->profile_mask & (1 << kAccumulate)) && p->profile_now) p->factored_n += 1;
    WDD_HIP(p, stage_begin(p, kRowDft, &end));
    WDD_HIP(p, wdd::launch_row_dft(p->h, p->kpad, p->xs, p->order, p->rows, nrows, p->tx, p->sx, p->t, p->stream));
    WDD_HIP(p, stage_end(p, end));
    WDD_HIP(p, stage_begin(p, kAccumulate, &end));
    WDD_HIP(p, wdd::launch_row_update(p->acc, p->kpad, p->n_freq_pad, p->freqs, p->n_freq, p->t, p->sx, p->rows, nrows,
                                      p->ty, p->sy, p->w, p->d, p->z, fuse_wiener, p->stream));
    WDD_HIP(p, stage_end(p, end));
  } else {
    WDD_HIP(p, stage_begin(p, kAccumulate, &end));
    WDD_HIP(p, wdd::launch_accumulate(p->acc, p->kpad, p->n_freq_pad, p->freqs, p->h, p->pos, n, p->ty, p->sy, p->tx,
                                      p->sx, p->stream));
    WDD_HIP(p, stage_end(p, end));
  }
  if (fused) *fused = wiener_done;
  p->frames_seen += (uint64_t)n;
  p->last_batch = n;
  return WDD_OK;
}

// Queues the display step (optionally after the Wiener reduction) writing to `out`.
wdd_status snapshot_enqueue_impl(wdd_plan_s* p, float* out, int32_t out_on_device, bool reduce) {
  hipEvent_t end;
  wdd_status st;
  if (p->held.live) {
    if (out_on_device == WDD_OUT_DEVICE_DEFERRED && !p->held.display_dst) {
      // pipelined: the held update will leave the partial rows, the launch after it the image
      p->held.display = true;
      p->held.display_dst = reinterpret_cast<float2*>(out);
      return WDD_OK;
    }
    if ((st = flush_held(p, true)) != WDD_OK) return st;  // the partial rows for this display
  }
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  if (reduce && p->order_mode == WDD_ORDER_SPECTRUM) {  // object order keeps D current
    WDD_HIP(p, stage_begin(p, kWiener, &end));
    WDD_HIP(p, wdd::launch_wiener(p->acc, p->w, p->kpad, p->freqs, p->n_freq, p->d, p->z, p->sy, p->stream));
    WDD_HIP(p, stage_end(p, end));
  }
  // the second pass writes the displayed object straight to its destination: the caller's
  // device buffer, or the plan's pinned host buffer (copied to `out` unless it is that buffer)
  float2* dst = out_on_device ? reinterpret_cast<float2*>(out) : p->pin_out;
  WDD_HIP(p, stage_begin(p, kDisplay, &end));
  // z is conj(D) stored [vx][vy]: transform its rows along vy (u = [vx][y], written in row
  // order), then the columns of u along vx, each workgroup writing one whole output row.
  // When the object-order update has left the first pass as partial rows (up, [y][vx][slot]),
  // the column pass sums each vx's partials as it reads them.
  // With a deferred output the column pass is left to the next push's first launch.
  if (!p->up_valid)
    WDD_HIP(p, wdd::launch_dft_rows(p->z, p->u, p->sx, p->sy, p->ey, p->d, 1.f, 0, p->sy, 1, p->sy, 1, 1, 0,
                                    p->stream));
  const float2* src;
  int32_t sr, sm, nslot, slot_stride;
  column_source(p, &src, &sr, &sm, &nslot, &slot_stride);
  // (pipelined pushes have no projection launch to carry it: only the update's)
  if (out_on_device == WDD_OUT_DEVICE_DEFERRED &&
      (p->pipeline ? can_defer_to_update(p) : can_defer(p) || can_defer_to_update(p))) {
    p->deferred_dst = dst;
    p->deferred_src = src, p->deferred_sr = sr, p->deferred_sm = sm, p->deferred_nslot = nslot;
    p->deferred_slot_stride = slot_stride;
    p->deferred_in_update = p->pipeline || !can_defer(p);
    p->deferred_d0 = p->deferred_in_update ? p->d0w : p->d;
  } else if ((st = column_pass(p, src, sr, sm, nslot, slot_stride, dst)) != WDD_OK) {
    return st;
  }
  WDD_HIP(p, stage_end(p, end));
  return WDD_OK;
}

// Waits for the queued snapshot and copies it out of the pinned buffer if needed.
wdd_status snapshot_finish_impl(wdd_plan_s* p, float* out, int32_t out_on_device, uint64_t* frames_seen) {
  const size_t grid = (size_t)p->sy * p->sx;
  if (out_on_device == WDD_OUT_DEVICE_ASYNC || out_on_device == WDD_OUT_DEVICE_DEFERRED) {
    if (frames_seen) *frames_seen = p->frames_seen;
    return WDD_OK;
  }
  WDD_HIP(p, hipStreamSynchronize(p->stream));
  p->drained = p->pushes - 1;
  if (!out_on_device && reinterpret_cast<float2*>(out) != p->pin_out) std::memcpy(out, p->pin_out, grid * sizeof(float2));
  WDD_HIP(p, harvest(p));
  if (frames_seen) *frames_seen = p->frames_seen;
  return WDD_OK;
}

// Display step and the copy to `out`; blocking.
wdd_status snapshot_impl(wdd_plan_s* p, float* out, int32_t out_on_device, uint64_t* frames_seen, bool reduce) {
  wdd_status st = snapshot_enqueue_impl(p, out, out_on_device, reduce);
  if (st != WDD_OK) return st;
  return snapshot_finish_impl(p, out, out_on_device, frames_seen);
}

}  // namespace

namespace wdd {

wdd_status push_table(wdd_plan_t p, const uint64_t* frame_addrs, const int32_t* pos_yx, int32_t n, bool fuse_wiener,
                      bool* fused) {
  return push_impl(p, nullptr, pos_yx, n, 1, fuse_wiener, fused, frame_addrs);
}

wdd_status snapshot_enqueue(wdd_plan_t p, bool reduce) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  return snapshot_enqueue_impl(p, reinterpret_cast<float*>(p->pin_out), 0, reduce);
}

wdd_status plan_scan_shape(wdd_plan_t p, int32_t* sy, int32_t* sx) {
  if (!p || !sy || !sx) return wdd::fail(WDD_EINVAL, "null argument");
  *sy = p->sy;
  *sx = p->sx;
  return WDD_OK;
}

wdd_status plan_set_stream(wdd_plan_t p, void* stream) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  WDD_HIP(p, hipStreamSynchronize(p->stream));
  p->drained = p->pushes - 1;
  WDD_HIP(p, harvest(p));
  if (p->own_stream && p->stream) WDD_HIP(p, hipStreamDestroy(p->stream));
  p->stream = static_cast<hipStream_t>(stream);
  p->own_stream = false;
  return WDD_OK;
}

void plan_drop_stream(wdd_plan_t p) {
  if (p && !p->own_stream) p->stream = nullptr;
}

wdd_status snapshot_finish(wdd_plan_t p, uint64_t* frames_seen) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  return snapshot_finish_impl(p, reinterpret_cast<float*>(p->pin_out), 0, frames_seen);
}

}  // namespace wdd

extern "C" {

wdd_status wdd_push(wdd_plan_t p, const void* frames, const int32_t* pos_yx, int32_t n, int32_t frames_on_device) {
  return push_impl(p, frames, pos_yx, n, frames_on_device, false, nullptr);
}

static wdd_status check_out(const float* out, int32_t out_on_device) {
  if (!out) return wdd::fail(WDD_EINVAL, "null output");
  if (out_on_device != WDD_OUT_HOST && out_on_device != WDD_OUT_DEVICE && out_on_device != WDD_OUT_DEVICE_ASYNC &&
      out_on_device != WDD_OUT_DEVICE_DEFERRED)
    return wdd::fail(WDD_EINVAL, "out_on_device must be a wdd_out_kind");
  if (out_on_device && (reinterpret_cast<uintptr_t>(out) % 8) != 0)
    return wdd::fail(WDD_EINVAL, "device output must be 8-byte aligned");
  return WDD_OK;
}

wdd_status wdd_snapshot(wdd_plan_t p, float* out, int32_t out_on_device, uint64_t* frames_seen) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = check_out(out, out_on_device)) != WDD_OK) return st;
  return snapshot_impl(p, out, out_on_device, frames_seen, true);
}

wdd_status wdd_push_snapshot(wdd_plan_t p, const void* frames, const int32_t* pos_yx, int32_t n,
                             int32_t frames_on_device, float* out, int32_t out_on_device, uint64_t* frames_seen) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = check_out(out, out_on_device)) != WDD_OK) return st;
  bool fused = false;
  st = push_impl(p, frames, pos_yx, n, frames_on_device, n > 0, &fused);
  if (st != WDD_OK) return st;
  return snapshot_impl(p, out, out_on_device, frames_seen, !fused);
}

static wdd_status copy_rows(wdd_plan_s* p, void* dst, const void* src, size_t rows, size_t row_bytes,
                            size_t src_pitch, int32_t on_device) {
  WDD_HIP(p, hipMemcpy2DAsync(dst, row_bytes, src, src_pitch, row_bytes, rows,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, p->stream));
  WDD_HIP(p, hipStreamSynchronize(p->stream));
  return WDD_OK;
}

wdd_status wdd_snapshot_buffer(wdd_plan_t p, float** host_out) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if (!host_out) return wdd::fail(WDD_EINVAL, "null argument");
  *host_out = reinterpret_cast<float*>(p->pin_out);
  return WDD_OK;
}

wdd_status wdd_spectrum(wdd_plan_t p, float* d_out, int32_t on_device) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  if (!d_out) return wdd::fail(WDD_EINVAL, "null output");
  return copy_rows(p, d_out, p->d, 1, (size_t)p->n_freq * sizeof(float2), (size_t)p->n_freq * sizeof(float2),
                   on_device);
}

wdd_status wdd_get_wiener(wdd_plan_t p, float* w_out, int32_t on_device) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  if (!w_out) return wdd::fail(WDD_EINVAL, "null output");
  return copy_rows(p, w_out, p->w, (size_t)p->n_freq, (size_t)p->k * sizeof(float2),
                   (size_t)p->kpad * sizeof(float2), on_device);
}

wdd_status wdd_plan_export(wdd_plan_t p, double* phi, double* w, int32_t* freqs) {
  if (!p) return wdd::fail(WDD_EINVAL, "null plan");
  const wdd_tables_s& t = *p->tables;
  if (freqs) std::copy(t.freqs.begin(), t.freqs.end(), freqs);
  if (w) std::copy(t.w.begin(), t.w.end(), w);
  if (phi) {
    const int64_t K = t.k;
    if (t.basis == WDD_BASIS_FOURIER) {  // Phi[q][k] = exp(+2 pi i (q_y k_y / ny + q_x k_x / nx)) / (ny nx)
      const double norm = 1.0 / ((double)t.ny * t.nx);
      for (int64_t qy = 0; qy < t.ny; ++qy)
        for (int64_t qx = 0; qx < t.nx; ++qx)
          for (int64_t k = 0; k < K; ++k) {
            const int64_t ky = k / t.nx, kx = k % t.nx;
            const int64_t m = ((qy * ky) % t.ny) * t.nx + ((qx * kx) % t.nx) * t.ny;  // angle in units of 1/(ny nx)
            const double a = 2.0 * M_PI * (double)(m % ((int64_t)t.ny * t.nx)) / ((double)t.ny * t.nx);
            double* o = phi + 2 * ((qy * t.nx + qx) * K + k);
            o[0] = std::cos(a) * norm;
            o[1] = std::sin(a) * norm;
          }
    } else {
      for (int64_t qy = 0; qy < t.ny; ++qy)
        for (int64_t qx = 0; qx < t.nx; ++qx)
          for (int64_t k = 0; k < K; ++k)
            phi[(qy * t.nx + qx) * K + k] =
                t.psi_y[(size_t)qy * t.l + t.pairs[2 * k]] * t.psi_x[(size_t)qx * t.l + t.pairs[2 * k + 1]];
    }
  }
  return WDD_OK;
}

wdd_status wdd_get_accumulator(wdd_plan_t p, float* a_out, int32_t on_device) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  if (!a_out) return wdd::fail(WDD_EINVAL, "null output");
  if (!p->acc) return wdd::fail(WDD_ESTATE, "the object-order plan keeps no spectrum A");
  return copy_rows(p, a_out, p->acc, (size_t)p->n_freq, (size_t)p->k * sizeof(float2),
                   (size_t)p->kpad * sizeof(float2), on_device);
}

wdd_status wdd_get_projection(wdd_plan_t p, float* h_out, int32_t on_device) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  if (!h_out) return wdd::fail(WDD_EINVAL, "null output");
  if (p->last_batch == 0) return WDD_OK;
  const size_t esz = p->fourier ? sizeof(float2) : sizeof(float);
  return copy_rows(p, h_out, p->h, (size_t)p->last_batch, (size_t)p->k * esz, (size_t)p->kpad * esz,
                   on_device);
}

wdd_status wdd_plan_get_info(wdd_plan_t p, wdd_plan_info* info) {
  if (!p || !info) return wdd::fail(WDD_EINVAL, "null argument");
  info->n_freq = p->n_freq;
  info->k = p->k;
  info->l = p->l;
  info->sigma_px = p->sigma;
  info->eps_abs = p->eps_abs;
  info->frames_seen = p->frames_seen;
  info->device_bytes = p->device_bytes;
  info->update_chunks = p->nchunks;
  info->display_slots = p->up ? p->nslot : 0;
  info->pipelined = p->two_stage ? 2 : p->pipeline ? 1 : 0;
  info->kept_columns = p->ncols;
  return WDD_OK;
}

wdd_status wdd_profile_enable(wdd_plan_t p, int32_t stages) {
  const int32_t on = stages;
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  WDD_HIP(p, hipStreamSynchronize(p->stream));
  WDD_HIP(p, harvest(p));
  p->factored_n = 0;
  for (int i = 0; i < 5; ++i) {
    p->stage_ms[i] = 0;
    p->stage_n[i] = 0;
  }
  p->profile_mask = on & 0x1f;
  p->profile_tick = 0;
  p->profile_now = true;
  return WDD_OK;
}

wdd_status wdd_profile_period(wdd_plan_t p, int32_t period) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if (period < 1) return wdd::fail(WDD_EINVAL, "profile period must be >= 1");
  WDD_HIP(p, hipStreamSynchronize(p->stream));
  WDD_HIP(p, harvest(p));
  for (int i = 0; i < 5; ++i) {
    p->stage_ms[i] = 0;
    p->stage_n[i] = 0;
  }
  p->factored_n = 0;
  p->profile_period = period;
  p->profile_tick = 0;
  p->profile_now = true;
  return WDD_OK;
}

wdd_status wdd_profile_read(wdd_plan_t p, wdd_profile* out) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  if (!out) return wdd::fail(WDD_EINVAL, "null output");
  WDD_HIP(p, hipStreamSynchronize(p->stream));
  WDD_HIP(p, harvest(p));
  out->project_ms = p->stage_ms[kProject];
  out->factored_launches = p->factored_n;
  out->rowdft_ms = p->stage_ms[kRowDft];
  out->rowdft_launches = p->stage_n[kRowDft];
  out->accumulate_ms = p->stage_ms[kAccumulate];
  out->wiener_ms = p->stage_ms[kWiener];
  out->display_ms = p->stage_ms[kDisplay];
  out->project_launches = p->stage_n[kProject];
  out->accumulate_launches = p->stage_n[kAccumulate];
  out->wiener_launches = p->stage_n[kWiener];
  out->display_launches = p->stage_n[kDisplay];
  return WDD_OK;
}

// Uploads the FP64 Wiener filter of `t` as FP32 into the plan's padded layout.
static wdd_status upload_wiener(wdd_plan_s* p, const wdd_tables_s& t) {
  const size_t nfk = (size_t)p->n_freq_pad * p->kpad;
  std::vector<float2> w(nfk, make_float2(0.f, 0.f));
  for (int64_t j = 0; j < p->n_freq; ++j)
    for (int32_t k = 0; k < t.k; ++k) {
      const double* v = &t.w[((size_t)j * t.k + k) * 2];
      w[(size_t)j * p->kpad + k] = make_float2((float)v[0], (float)v[1]);
    }
  WDD_HIP(p, hipMemcpyAsync(p->w, w.data(), nfk * sizeof(float2), hipMemcpyHostToDevice, p->stream));
  WDD_HIP(p, hipStreamSynchronize(p->stream));
  return WDD_OK;
}

wdd_status wdd_update_probe(wdd_plan_t p, const wdd_probe* probe, double eps_rel) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  if (!probe) return wdd::fail(WDD_EINVAL, "null probe");
  if (p->order_mode == WDD_ORDER_OBJECT)
    return wdd::fail(WDD_ESTATE, "object order applies the Wiener filter per frame; no spectrum to re-deconvolve");
  if (probe->radius_px != p->probe.radius_px || probe->center_y != p->probe.center_y ||
      probe->center_x != p->probe.center_x)
    return wdd::fail(WDD_EINVAL, "the aperture radius and centre fix the kept frequencies and cannot change");
  wdd_options o = p->opts;
  o.eps_rel = eps_rel;
  o.sigma_px = p->sigma;
  std::shared_ptr<wdd_tables_s> t;
  try {
    t = std::make_shared<wdd_tables_s>();
    if ((st = wdd::build_tables(probe, &p->scan, &p->det, p->k, &o, t.get())) != WDD_OK) return st;
    if (t->n_freq() != p->n_freq) return wdd::fail(WDD_EINVAL, "kept frequency set changed");
    if ((st = upload_wiener(p, *t)) != WDD_OK) return st;
  } catch (const std::bad_alloc&) {
    return wdd::fail(WDD_ENOMEM, "out of host memory");
  }
  p->probe = *probe;
  p->opts.eps_rel = eps_rel;
  p->eps_abs = t->eps_abs;
  p->tables = t;
  return WDD_OK;
}

namespace {
struct CheckpointHeader {
  char magic[8];
  int32_t version, sy, sx, ny, nx, k, dtype, precision, order;
  int64_t n_freq;
  uint64_t frames_seen;
  double radius, step, sigma;
};
constexpr char kMagic[8] = {'W', 'D', 'D', 'A', 'C', 'C', '0', '1'};
}  // namespace

wdd_status wdd_checkpoint_size(wdd_plan_t p, size_t* bytes) {
  if (!p || !bytes) return wdd::fail(WDD_EINVAL, "null argument");
  const size_t per = p->order_mode == WDD_ORDER_OBJECT ? 1 : (size_t)p->k;
  *bytes = sizeof(CheckpointHeader) + (size_t)p->n_freq * per * sizeof(float2);
  return WDD_OK;
}

wdd_status wdd_checkpoint_save(wdd_plan_t p, void* host_buf, size_t bytes) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  size_t need = 0;
  wdd_checkpoint_size(p, &need);
  if (!host_buf || bytes < need) return wdd::fail(WDD_EINVAL, "checkpoint buffer needs %zu bytes", need);
  CheckpointHeader hd = {};
  std::memcpy(hd.magic, kMagic, 8);
  hd.version = 1; hd.sy = p->sy; hd.sx = p->sx; hd.ny = p->ny; hd.nx = p->nx; hd.k = p->k;
  hd.dtype = p->dtype; hd.precision = p->precision; hd.n_freq = p->n_freq; hd.frames_seen = p->frames_seen;
  hd.order = p->order_mode;
  hd.radius = p->probe.radius_px; hd.step = p->scan.step_px; hd.sigma = p->sigma;
  std::memcpy(host_buf, &hd, sizeof(hd));
  char* dst = static_cast<char*>(host_buf) + sizeof(hd);
  if (p->acc)
    WDD_HIP(p, hipMemcpy2DAsync(dst, (size_t)p->k * sizeof(float2), p->acc, (size_t)p->kpad * sizeof(float2),
                                (size_t)p->k * sizeof(float2), (size_t)p->n_freq, hipMemcpyDeviceToHost, p->stream));
  else
    WDD_HIP(p, hipMemcpyAsync(dst, p->d, (size_t)p->n_freq * sizeof(float2), hipMemcpyDeviceToHost, p->stream));
  WDD_HIP(p, hipStreamSynchronize(p->stream));
  return WDD_OK;
}

wdd_status wdd_checkpoint_load(wdd_plan_t p, const void* host_buf, size_t bytes) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  size_t need = 0;
  wdd_checkpoint_size(p, &need);
  if (!host_buf || bytes < need) return wdd::fail(WDD_EINVAL, "checkpoint image needs %zu bytes", need);
  CheckpointHeader hd;
  std::memcpy(&hd, host_buf, sizeof(hd));
  if (std::memcmp(hd.magic, kMagic, 8) != 0 || hd.version != 1)
    return wdd::fail(WDD_EINVAL, "not a checkpoint image of this library");
  if (hd.sy != p->sy || hd.sx != p->sx || hd.ny != p->ny || hd.nx != p->nx || hd.k != p->k ||
      hd.n_freq != p->n_freq || hd.radius != p->probe.radius_px || hd.step != p->scan.step_px || hd.sigma != p->sigma ||
      hd.order != p->order_mode)
    return wdd::fail(WDD_EINVAL, "checkpoint geometry or basis differs from the plan's");
  const char* src = static_cast<const char*>(host_buf) + sizeof(hd);
  if (p->acc) {
    WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->acc), (size_t)p->n_freq_pad * p->kpad * 2, p->stream));
    WDD_HIP(p, hipMemcpy2DAsync(p->acc, (size_t)p->kpad * sizeof(float2), src, (size_t)p->k * sizeof(float2),
                                (size_t)p->k * sizeof(float2), (size_t)p->n_freq, hipMemcpyHostToDevice, p->stream));
  } else {  // D itself (d is the FP32 value nearest the compensated sum; the remainder restarts at zero)
    WDD_HIP(p, hipMemcpyAsync(p->d, src, (size_t)p->n_freq * sizeof(float2), hipMemcpyHostToDevice, p->stream));
    if (p->dlo)
      WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->dlo), (size_t)p->n_freq_pad * 2, p->stream));
    WDD_HIP(p, wdd::launch_scatter_conj(p->d, p->freqs, p->n_freq, p->z, p->sy, p->stream));
  }
  p->up_valid = false;
  WDD_HIP(p, hipStreamSynchronize(p->stream));
  p->frames_seen = hd.frames_seen;
  p->last_batch = 0;
  return WDD_OK;
}

wdd_status wdd_reset(wdd_plan_t p) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  if (p->acc)
    WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->acc), (size_t)p->n_freq_pad * p->kpad * 2, p->stream));
  WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->d), (size_t)p->n_freq_pad * 2, p->stream));
  if (p->dlo) WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->dlo), (size_t)p->n_freq_pad * 2, p->stream));
  WDD_HIP(p, wdd::launch_zero(reinterpret_cast<float*>(p->z), (size_t)p->sy * p->sx * 2, p->stream));
  p->up_valid = false;
  p->frames_seen = 0;
  p->last_batch = 0;
  return WDD_OK;
}

}  // extern "C"

namespace wdd {

wdd_status check_display_args(const float* spectrum, int32_t sy, int32_t sx, const float* out) {
  if (!spectrum || !out) return fail(WDD_EINVAL, "null spectrum or output");
  if (sy < 1 || sx < 1 || sy > kDisplayMaxSide || sx > kDisplayMaxSide)
    return fail(WDD_EINVAL, "grid %d x %d outside [1, %d]", sy, sx, kDisplayMaxSide);
  if ((reinterpret_cast<uintptr_t>(spectrum) % 8) != 0 || (reinterpret_cast<uintptr_t>(out) % 8) != 0)
    return fail(WDD_EINVAL, "spectrum and output must be 8-byte aligned device memory");
  return WDD_OK;
}

// The display of a spectrum grid through the scratch `scr` (display_scratch_floats(sy, sx)
// floats): z = conj(d) transposed, rows of z along v_y into u, then the columns of u along v_x
// written as whole output rows, scaled by 1 / sqrt(sy sx |d[0]|) (eq. extract).  Nothing in
// the scratch needs to start at zero: every value is written before it is read.
wdd_status display_grid(const float* spectrum, int32_t sy, int32_t sx, float* out, float* scratch, void* stream) {
  const hipStream_t st = (hipStream_t)stream;
  const float2* d = reinterpret_cast<const float2*>(spectrum);
  const size_t cells = (size_t)sy * sx;
  float2* z = reinterpret_cast<float2*>(scratch);
  float2* u = z + cells;
  float2* ey = u + cells;
  float2* ex = ey + sy;
  hipError_t e = launch_display_prep(d, sy, sx, z, ey, ex, st);
  if (e == hipSuccess) e = launch_dft_rows(z, u, sx, sy, ey, d, 1.f, 0, sy, 1, sy, 1, 1, 0, st);
  if (e == hipSuccess)
    e = launch_dft_rows(u, reinterpret_cast<float2*>(out), sy, sx, ex, d, (float)((double)sy * sx), 1, 1, sy, sx, 1, 1,
                        0, st);
  if (e != hipSuccess) return fail(WDD_EDEVICE, "display launch: %s", hipGetErrorString(e));
  return WDD_OK;
}

}  // namespace wdd

extern "C" {

wdd_status wdd_display(const float* spectrum, int32_t sy, int32_t sx, float* out, void* hip_stream) {
  wdd_status st = wdd::check_display_args(spectrum, sy, sx, out);
  if (st != WDD_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t bytes = wdd::display_scratch_floats(sy, sx) * sizeof(float);
  float* scr = nullptr;
  hipError_t e = hipMallocAsync((void**)&scr, bytes, s);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    return wdd::fail(WDD_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  if (e != hipSuccess) return wdd::fail(WDD_EDEVICE, "hipMallocAsync: %s", hipGetErrorString(e));
  st = wdd::display_grid(spectrum, sy, sx, out, scr, hip_stream);
  const hipError_t ef = hipFreeAsync(scr, s);
  if (st != WDD_OK) return st;
  if (ef != hipSuccess) return wdd::fail(WDD_EDEVICE, "hipFreeAsync: %s", hipGetErrorString(ef));
  return WDD_OK;
}

wdd_status wdd_set_allocator(wdd_alloc_fn alloc, wdd_release_fn release, void* ctx) {
  if (alloc && !release) return wdd::fail(WDD_EINVAL, "an allocator needs its release function");
  std::lock_guard<std::mutex> lock(wdd::g_alloc_mu);
  wdd::g_alloc = alloc;
  wdd::g_release = alloc ? release : nullptr;
  wdd::g_alloc_ctx = alloc ? ctx : nullptr;
  return WDD_OK;
}

wdd_status wdd_sync(wdd_plan_t p) {
  wdd_status st = check_usable(p);
  if (st != WDD_OK) return st;
  if ((st = flush_deferred(p)) != WDD_OK) return st;
  WDD_HIP(p, hipStreamSynchronize(p->stream));
  p->drained = p->pushes - 1;
  return WDD_OK;
}

wdd_status wdd_destroy(wdd_plan_t p) {
  if (p && !p->failed) (void)flush_deferred(p);  // a display left to a next push that will not come
  release(p);
  return WDD_OK;
}

}  // extern "C"
