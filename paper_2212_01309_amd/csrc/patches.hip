// Field-of-view patches (Section 10, Discussion: a large field of view subdivided into
// patches reconstructed independently and merged), as one object on the GPU.
//
// All patches have one geometry (a Py x Px raster with the acquisition's probe, detector and
// K), so they share one set of tables: the kept frequencies, the basis and the Wiener filter
// of a plan built for the patch raster ("master" plan, object order).  Each patch keeps its
// own object spectrum D (compensated, as in the plan) and display grids.  A push projects
// the batch once, then one grouped launch updates every patch the batch touches: work items
// (row pass of a patch, chunk of kept frequencies), a frame entering every patch that
// contains its position at its local position.  A snapshot transforms all patch spectra in
// two stacked row-DFT launches and merges the patch images with the trapezoid windows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "plan.h"

namespace {

constexpr int kBlockSlots = 4;  // pinned push blocks in flight

struct Entry {
  int32_t ly, lx, frame;
};

}  // namespace

struct wdd_patches_s {
  wdd_plan_t master = nullptr;
  int32_t sy = 0, sx = 0, py = 0, px = 0, oy_ov = 0, ox_ov = 0;
  std::vector<int32_t> oy, ox;
  int32_t npatch = 0;
  int64_t nfp = 0;  // D stride per patch (the master's padded frequency count)
  float2 *d = nullptr, *dlo = nullptr, *z = nullptr, *u = nullptr, *img = nullptr;
  int32_t* origins = nullptr;  // device: oy then ox
  char* blk_dev = nullptr;
  size_t blk_cap = 0;
  char* blk_pin[kBlockSlots] = {};
  size_t pin_cap[kBlockSlots] = {};
  hipEvent_t blk_ev[kBlockSlots] = {};
  bool blk_live[kBlockSlots] = {};
  int slot = 0;
  float2* pin_out = nullptr;
  std::vector<void*> allocs;
  int64_t device_bytes = 0;
  uint64_t frames_seen = 0;
  std::vector<std::vector<Entry>> per_patch;
  std::vector<int32_t> touched;
  std::vector<char> host_blk;
};

namespace {

wdd_status hip_fail(hipError_t e, const char* what) {
  return wdd::fail(WDD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define PATCH_HIP(call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #call);    \
  } while (0)

template <typename T>
wdd_status dev_alloc(wdd_patches_s* s, T** p, size_t count) {
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    return wdd::fail(WDD_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  s->allocs.push_back(*p);
  s->device_bytes += (int64_t)bytes;
  return WDD_OK;
}

void release(wdd_patches_s* s) {
  if (!s) return;
  if (s->master) (void)hipStreamSynchronize(s->master->stream);
  for (void* a : s->allocs) (void)hipFree(a);
  if (s->blk_dev) (void)hipFree(s->blk_dev);
  for (int i = 0; i < kBlockSlots; ++i) {
    if (s->blk_pin[i]) (void)hipHostFree(s->blk_pin[i]);
    if (s->blk_ev[i]) (void)hipEventDestroy(s->blk_ev[i]);
  }
  if (s->pin_out) (void)hipHostFree(s->pin_out);
  if (s->master) wdd_destroy(s->master);
  delete s;
}

size_t align16(size_t x) { return (x + 15) / 16 * 16; }

}  // namespace

extern "C" {

wdd_status wdd_patches_create(const wdd_probe* probe, const wdd_scan* scan, const wdd_detector* det, int32_t K,
                              const wdd_patch_geometry* geo, const wdd_options* opts_in, void* hip_stream,
                              wdd_patches_t* out) {
  if (!out) return wdd::fail(WDD_EINVAL, "null output handle");
  *out = nullptr;
  if (!probe || !scan || !det || !geo) return wdd::fail(WDD_EINVAL, "null argument");
  if (scan->sy < 1 || scan->sx < 1) return wdd::fail(WDD_EINVAL, "empty raster");
  if (geo->py < 1 || geo->px < 1 || geo->py > scan->sy || geo->px > scan->sx || geo->overlap_y < 0 ||
      geo->overlap_x < 0 || geo->overlap_y >= geo->py || geo->overlap_x >= geo->px)
    return wdd::fail(WDD_EINVAL, "patches %d x %d with overlap %d, %d do not fit the %d x %d raster", geo->py, geo->px,
                     geo->overlap_y, geo->overlap_x, scan->sy, scan->sx);
  wdd_options opts;
  wdd_default_options(&opts);
  if (opts_in) opts = *opts_in;
  if (opts.basis != WDD_BASIS_HERMITE_GAUSS)
    return wdd::fail(WDD_EINVAL, "field-of-view patches use the Hermite-Gauss basis");
  opts.order = WDD_ORDER_OBJECT;  // the grouped update accumulates each patch's D
  opts.pipeline = 0;              // the patch set orders its own launches
  wdd_status st = wdd::check_plan_options(det, opts);
  if (st != WDD_OK) return st;
  wdd_patches_s* s = new (std::nothrow) wdd_patches_s();
  if (!s) return wdd::fail(WDD_ENOMEM, "out of host memory");
  try {
    s->sy = scan->sy; s->sx = scan->sx; s->py = geo->py; s->px = geo->px;
    s->oy_ov = geo->overlap_y; s->ox_ov = geo->overlap_x;
    auto origins = [](int32_t n, int32_t p, int32_t ov) {
      std::vector<int32_t> o;
      for (int32_t a = 0; a + p <= n; a += p - ov) o.push_back(a);
      if (o.back() != n - p) o.push_back(n - p);
      return o;
    };
    s->oy = origins(s->sy, s->py, s->oy_ov);
    s->ox = origins(s->sx, s->px, s->ox_ov);
    s->npatch = (int32_t)(s->oy.size() * s->ox.size());
    const wdd_scan patch_scan = {s->py, s->px, scan->step_px};
    std::shared_ptr<wdd_tables_s> t = std::make_shared<wdd_tables_s>();
    if ((st = wdd::build_tables(probe, &patch_scan, det, K, &opts, t.get())) != WDD_OK) {
      release(s);
      return st;
    }
    if ((st = wdd::plan_create_from_tables(t, probe, &patch_scan, det, opts, hip_stream, &s->master)) != WDD_OK) {
      release(s);
      return st;
    }
    s->per_patch.resize(s->npatch);
  } catch (const std::bad_alloc&) {
    release(s);
    return wdd::fail(WDD_ENOMEM, "out of host memory");
  }
  wdd_plan_s* m = s->master;
  s->nfp = m->n_freq_pad;
  const size_t cells = (size_t)s->py * s->px;
#define PALLOC(ptr, n)                                                  \
  if ((st = dev_alloc(s, &(ptr), (n))) != WDD_OK) { release(s); return st; }
  PALLOC(s->d, (size_t)s->npatch * s->nfp);
  PALLOC(s->dlo, (size_t)s->npatch * s->nfp);
  PALLOC(s->z, (size_t)s->npatch * cells);
  PALLOC(s->u, (size_t)s->npatch * cells);
  PALLOC(s->img, (size_t)s->npatch * cells);
  PALLOC(s->origins, s->oy.size() + s->ox.size());
#undef PALLOC
  hipError_t e = hipSuccess;
  std::vector<int32_t> org(s->oy);
  org.insert(org.end(), s->ox.begin(), s->ox.end());
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->origins, org.data(), org.size() * sizeof(int32_t), hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess) e = wdd::launch_zero(reinterpret_cast<float*>(s->d), (size_t)s->npatch * s->nfp * 2, m->stream);
  if (e == hipSuccess) e = wdd::launch_zero(reinterpret_cast<float*>(s->dlo), (size_t)s->npatch * s->nfp * 2, m->stream);
  if (e == hipSuccess) e = wdd::launch_zero(reinterpret_cast<float*>(s->z), (size_t)s->npatch * cells * 2, m->stream);
  for (int i = 0; i < kBlockSlots && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&s->blk_ev[i], hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->pin_out, (size_t)s->sy * s->sx * sizeof(float2), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) {
    release(s);
    return hip_fail(e, "patch set creation");
  }
  *out = s;
  return WDD_OK;
}

wdd_status wdd_patches_push(wdd_patches_t s, const void* frames, const int32_t* pos_yx, int32_t n) {
  if (!s) return wdd::fail(WDD_EINVAL, "null patch set");
  wdd_plan_s* m = s->master;
  if (m->failed) return wdd::fail(WDD_ESTATE, "patch set is unusable after an earlier device error");
  if (n < 0 || n > m->max_batch) return wdd::fail(WDD_EINVAL, "n = %d outside [0, %d]", n, m->max_batch);
  if (n == 0) return WDD_OK;
  if (!frames || !pos_yx) return wdd::fail(WDD_EINVAL, "null frames or positions");
  if (reinterpret_cast<uintptr_t>(frames) % 16 != 0) return wdd::fail(WDD_EINVAL, "device frames must be 16-byte aligned");
  for (int32_t i = 0; i < n; ++i) {
    const int32_t y = pos_yx[2 * i], x = pos_yx[2 * i + 1];
    if (y < 0 || y >= s->sy || x < 0 || x >= s->sx)
      return wdd::fail(WDD_ERANGE, "position %d = (%d, %d) outside the %d x %d raster", i, y, x, s->sy, s->sx);
  }
  // frames into every patch containing them, at local positions
  for (int32_t p : s->touched) s->per_patch[p].clear();
  s->touched.clear();
  const int32_t npx = (int32_t)s->ox.size();
  try {
    for (int32_t i = 0; i < n; ++i) {
      const int32_t y = pos_yx[2 * i], x = pos_yx[2 * i + 1];
      for (int32_t a = 0; a < (int32_t)s->oy.size(); ++a) {
        const int32_t ly = y - s->oy[a];
        if (ly < 0 || ly >= s->py) continue;
        for (int32_t b = 0; b < npx; ++b) {
          const int32_t lx = x - s->ox[b];
          if (lx < 0 || lx >= s->px) continue;
          std::vector<Entry>& v = s->per_patch[a * npx + b];
          if (v.empty()) s->touched.push_back(a * npx + b);
          v.push_back({ly, lx, i});
        }
      }
    }
    std::sort(s->touched.begin(), s->touched.end());
    // row passes (at most kRowSetMax rows each) of every touched patch.  Passes of one patch
    // add to the same D, so they go to separate launches: launch k takes the k-th pass of
    // every patch that has one (passes sorted by k, then patch).
    struct Pass {
      int32_t patch, row0, nrows, k;
    };
    std::vector<Pass> passes;
    std::vector<int4> rows;
    size_t nent = 0;
    for (int32_t p : s->touched) {
      std::vector<Entry>& v = s->per_patch[p];
      std::stable_sort(v.begin(), v.end(), [](const Entry& a, const Entry& b) { return a.ly < b.ly; });
      const int32_t r0 = (int32_t)rows.size();
      for (size_t i = 0; i < v.size(); ++i) {
        if (rows.size() == (size_t)r0 || rows.back().x != v[i].ly)
          rows.push_back(make_int4(v[i].ly, (int32_t)(nent + i), 0, 0));
        rows.back().z += 1;
      }
      for (int32_t r = r0, k = 0; r < (int32_t)rows.size(); r += wdd::kRowSetMax, ++k)
        passes.push_back({p, r, std::min<int32_t>(wdd::kRowSetMax, (int32_t)rows.size() - r), k});
      nent += v.size();
    }
    std::stable_sort(passes.begin(), passes.end(), [](const Pass& a, const Pass& b) { return a.k < b.k; });
    const size_t nchunk = m->host_chunks.size();
    const size_t nitems = passes.size() * nchunk;
    const size_t off_items = align16(passes.size() * sizeof(wdd::ObjPass));
    const size_t off_rows = off_items + align16(nitems * sizeof(int4));
    const size_t off_order = off_rows + align16(rows.size() * sizeof(int4));
    const size_t off_xs = off_order + align16(nent * sizeof(int32_t));
    const size_t bytes = off_xs + align16(nent * sizeof(int32_t));
    // device block: grown (after the stream has drained) when a push needs more
    if (bytes > s->blk_cap) {
      PATCH_HIP(hipStreamSynchronize(m->stream));
      if (s->blk_dev) PATCH_HIP(hipFree(s->blk_dev));
      s->blk_dev = nullptr;
      const size_t cap = std::max(bytes * 2, (size_t)1 << 16);
      hipError_t e = hipMalloc((void**)&s->blk_dev, cap);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        s->blk_cap = 0;
        return wdd::fail(WDD_ENOMEM, "device allocation of %zu bytes failed", cap);
      }
      s->blk_cap = cap;
    }
    const int slot = s->slot;
    s->slot = (s->slot + 1) % kBlockSlots;
    if (s->blk_live[slot]) PATCH_HIP(hipEventSynchronize(s->blk_ev[slot]));
    if (bytes > s->pin_cap[slot]) {
      if (s->blk_pin[slot]) PATCH_HIP(hipHostFree(s->blk_pin[slot]));
      s->blk_pin[slot] = nullptr;
      s->pin_cap[slot] = 0;
      const size_t cap = std::max(bytes * 2, (size_t)1 << 16);
      PATCH_HIP(hipHostMalloc((void**)&s->blk_pin[slot], cap, hipHostMallocDefault));
      s->pin_cap[slot] = cap;
    }
    char* hb = s->blk_pin[slot];
    char* db = s->blk_dev;
    int32_t* order = reinterpret_cast<int32_t*>(hb + off_order);
    int32_t* xs = reinterpret_cast<int32_t*>(hb + off_xs);
    {
      size_t k = 0;
      for (int32_t p : s->touched)
        for (const Entry& en : s->per_patch[p]) {
          order[k] = en.frame;
          xs[k] = en.lx;
          ++k;
        }
    }
    std::memcpy(hb + off_rows, rows.data(), rows.size() * sizeof(int4));
    wdd::ObjPass* op = reinterpret_cast<wdd::ObjPass*>(hb);
    int4* items = reinterpret_cast<int4*>(hb + off_items);
    int max_rows = 1;
    for (size_t i = 0; i < passes.size(); ++i) {
      const Pass& ps = passes[i];
      wdd::ObjPass o;
      std::memset(&o, 0, sizeof(o));
      o.h = m->h;
      o.order = reinterpret_cast<const int*>(db + off_order);
      o.xs = reinterpret_cast<const int*>(db + off_xs);
      o.jv = m->jv;
      o.w = m->w;
      o.d = s->d + (size_t)ps.patch * s->nfp;
      o.dlo = s->dlo + (size_t)ps.patch * s->nfp;
      o.z = s->z + (size_t)ps.patch * s->py * s->px;
      o.up = nullptr;
      o.rows = reinterpret_cast<const int4*>(db + off_rows) + ps.row0;
      o.kpad = m->kpad;
      o.nrows = ps.nrows;
      o.sx = s->px;
      o.sy = s->py;
      o.max_chunk = m->max_chunk;
      o.nslot = 1;
      o.log2sy = 0;
      o.in_order = 0;
      o.tscale = m->tscale;
      op[i] = o;
      max_rows = std::max(max_rows, ps.nrows);
      for (size_t c = 0; c < nchunk; ++c) {
        const int4 ch = m->host_chunks[c];
        items[i * nchunk + c] = make_int4((int32_t)i, ch.x, ch.y, ch.z | (ch.w << 16));
      }
    }
    // the projection of the batch, whose extra workgroup brings the block to the device
    wdd::ProjectLaunch pl;
    pl.dtype = m->dtype;
    pl.precision = m->precision;
    pl.frames = frames;
    pl.n = n;
    pl.ny = m->ny;
    pl.nx = m->nx;
    pl.psi = m->psi;
    pl.psix_lp = m->psix_lp;
    pl.psi_unscale = m->psi_unscale;
    pl.kmap = m->kmap;
    pl.kpad = m->kpad;
    pl.h = m->h;
    pl.up_src = hb;
    pl.up_dst = db;
    pl.up_bytes = bytes;
    pl.fptr = nullptr;
    PATCH_HIP(wdd::launch_project(pl, m->stream));
    PATCH_HIP(hipEventRecord(s->blk_ev[slot], m->stream));
    s->blk_live[slot] = true;
    const size_t lds = wdd::row_fused_lds_bytes(m->kpad, max_rows, m->max_chunk);
    for (size_t i0 = 0; i0 < passes.size();) {  // one launch per pass index k
      size_t i1 = i0;
      while (i1 < passes.size() && passes[i1].k == passes[i0].k) ++i1;
      PATCH_HIP(wdd::launch_row_fused_obj_group(reinterpret_cast<const wdd::ObjPass*>(db),
                                                reinterpret_cast<const int4*>(db + off_items) + i0 * nchunk,
                                                (int)((i1 - i0) * nchunk), lds, m->stream));
      i0 = i1;
    }
  } catch (const std::bad_alloc&) {
    return wdd::fail(WDD_ENOMEM, "out of host memory");
  }
  s->frames_seen += (uint64_t)n;
  return WDD_OK;
}

wdd_status wdd_patches_snapshot(wdd_patches_t s, float* out, int32_t out_on_device, uint64_t* frames_seen) {
  if (!s) return wdd::fail(WDD_EINVAL, "null patch set");
  if (!out) return wdd::fail(WDD_EINVAL, "null output");
  if (out_on_device != WDD_OUT_HOST && out_on_device != WDD_OUT_DEVICE && out_on_device != WDD_OUT_DEVICE_ASYNC)
    return wdd::fail(WDD_EINVAL, "out_on_device must be WDD_OUT_HOST, WDD_OUT_DEVICE or WDD_OUT_DEVICE_ASYNC");
  if (out_on_device && (reinterpret_cast<uintptr_t>(out) % 8) != 0)
    return wdd::fail(WDD_EINVAL, "device output must be 8-byte aligned");
  wdd_plan_s* m = s->master;
  const int64_t cells = (int64_t)s->py * s->px;
  // each patch's image: rows of conj D along v_y (all patches stacked), then its columns
  // along v_x with the patch's own normalisation 1 / sqrt(Py Px |D_p[0]|) (eq. extract)
  PATCH_HIP(wdd::launch_dft_rows_blocks(s->z, s->u, 1, s->npatch * s->px, s->py, m->ey, s->d, 1.f, 0, s->py, 1, s->py,
                                        1, 0, 0, 0, m->stream));
  PATCH_HIP(wdd::launch_dft_rows_blocks(s->u, s->img, s->npatch, s->py, s->px, m->ex, s->d, (float)cells, 1, 1, s->py,
                                        s->px, 1, cells, cells, s->nfp, m->stream));
  float2* dst = out_on_device ? reinterpret_cast<float2*>(out) : s->pin_out;
  PATCH_HIP(wdd::launch_patch_merge(s->img, s->origins, (int)s->oy.size(), s->origins + s->oy.size(),
                                    (int)s->ox.size(), s->py, s->px, s->oy_ov, s->ox_ov, dst, s->sy, s->sx,
                                    m->stream));
  if (frames_seen) *frames_seen = s->frames_seen;
  if (out_on_device == WDD_OUT_DEVICE_ASYNC) return WDD_OK;
  PATCH_HIP(hipStreamSynchronize(m->stream));
  if (!out_on_device) std::memcpy(out, s->pin_out, (size_t)s->sy * s->sx * sizeof(float2));
  return WDD_OK;
}

wdd_status wdd_patches_info(wdd_patches_t s, int32_t* npatch_y, int32_t* npatch_x, int64_t* n_freq,
                            int64_t* device_bytes) {
  if (!s) return wdd::fail(WDD_EINVAL, "null patch set");
  if (npatch_y) *npatch_y = (int32_t)s->oy.size();
  if (npatch_x) *npatch_x = (int32_t)s->ox.size();
  if (n_freq) *n_freq = s->master->n_freq;
  if (device_bytes) *device_bytes = s->device_bytes + s->master->device_bytes + (int64_t)s->blk_cap;
  return WDD_OK;
}

wdd_status wdd_patches_sync(wdd_patches_t s) {
  if (!s) return wdd::fail(WDD_EINVAL, "null patch set");
  PATCH_HIP(hipStreamSynchronize(s->master->stream));
  return WDD_OK;
}

wdd_status wdd_patches_destroy(wdd_patches_t s) {
  release(s);
  return WDD_OK;
}

}  // extern "C"
