// Internal declarations shared by the host table builder, the C ABI and the kernels.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "wdd.h"

struct wdd_tables_s {
  int32_t sy = 0, sx = 0, ny = 0, nx = 0, k = 0, l = 0;
  double step = 1.0, radius = 0.0, amplitude = 1.0, defocus = 0.0;
  double cy = 0.0, cx = 0.0;  // aperture centre in detector pixels
  double eps_rel = 0.01, sigma = 0.0, eps_abs = 0.0;
  int32_t basis = WDD_BASIS_HERMITE_GAUSS;
  std::vector<int32_t> freqs;  // [n_freq][2]  (v_y, v_x)
  std::vector<double> psi_y;   // [ny][l]
  std::vector<double> psi_x;   // [nx][l]
  std::vector<int32_t> pairs;  // [k][2]  (n_y, n_x)
  std::vector<double> w;       // [n_freq][k][2]
  int64_t n_freq() const { return (int64_t)freqs.size() / 2; }
};

namespace wdd {

// Thread-local error message handling.
wdd_status fail(wdd_status code, const char* fmt, ...);

// Host FP64 table construction (validated arguments).  kept_only: stop after the kept
// frequencies (no basis, no W: enough for plan_device_bytes, in a small part of the time).
wdd_status build_tables(const wdd_probe* probe, const wdd_scan* scan, const wdd_detector* det,
                        int32_t K, const wdd_options* opts, wdd_tables_s* t, bool kept_only = false);

// Plan operations used by the serving runtime (api.hip).
wdd_status check_plan_options(const wdd_detector* det, const wdd_options& opts);
// Device bytes a plan of these tables allocates.
int64_t plan_device_bytes(const wdd_tables_s& t, const wdd_options& opts, int32_t dtype);
// The plan keeps `t` (shared, read-only) as the tables it exports.
wdd_status plan_create_from_tables(std::shared_ptr<const wdd_tables_s> t, const wdd_probe* probe,
                                   const wdd_scan* scan, const wdd_detector* det, const wdd_options& opts,
                                   void* hip_stream, wdd_plan_t* out);
// Queues a batch whose frames sit at the given device addresses (16-byte aligned).
wdd_status push_table(wdd_plan_t p, const uint64_t* frame_addrs, const int32_t* pos_yx, int32_t n, bool fuse_wiener,
                      bool* fused);
// Queues a snapshot into the plan's pinned host buffer (with the Wiener reduction unless it
// was fused into the last push); snapshot_finish waits for it.
wdd_status snapshot_enqueue(wdd_plan_t p, bool reduce);
wdd_status snapshot_finish(wdd_plan_t p, uint64_t* frames_seen);
wdd_status plan_scan_shape(wdd_plan_t p, int32_t* sy, int32_t* sx);
// Waits for the plan's work, then moves it to `stream` (the plan's own stream, if it had
// one, is destroyed).
wdd_status plan_set_stream(wdd_plan_t p, void* stream);
// Forgets a plan's borrowed stream without waiting on it (no work of the plan may be queued
// there: the caller has synchronised it, or the plan never ran on it); the plan may then only
// be destroyed.  A plan that owns its stream keeps it.
void plan_drop_stream(wdd_plan_t p);

// The display of a spectrum grid (wdd_display): argument checks, the scratch it needs (in
// floats: two sy x sx complex grids and the twiddles of both sides) and the launches, all
// asynchronous on `stream`.
constexpr int32_t kDisplayMaxSide = 4096;
inline size_t display_scratch_floats(int32_t sy, int32_t sx) {
  return ((size_t)2 * sy * sx + (size_t)sy + (size_t)sx) * 2;
}
wdd_status check_display_args(const float* spectrum, int32_t sy, int32_t sx, const float* out);
wdd_status display_grid(const float* spectrum, int32_t sy, int32_t sx, float* out, float* scratch, void* stream);

// Largest number of columns of psi held on the device per axis (L <= 16).
constexpr int kMaxL = 16;

}  // namespace wdd
