// Launchers of the HIP kernels (kernels.hip).  All are asynchronous on `st` and
// return the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "wdd.h"

namespace wdd {

// Projection of a batch: h[b][k] = sum_q Phi[q][k] frames[b][q] for b < n.  psi: [ny][16]
// then [nx][16] FP32 (columns >= L zero); kmap[k] = 16 n_y(k) + n_x(k), or -1 for padding
// columns.  precision (a wdd_precision): WDD_FP32, or a reduced one for uint16 frames with
// psix_lp = [2][16][nx] bf16/fp16 words, the hi and lo parts of psi_x * 2^shift, and
// psi_unscale = 2^-shift.  With up_src (pinned host memory) the launch also copies up_bytes
// (a multiple of 4) from it to up_dst, in a workgroup of its own.  With fptr (pinned host
// table of n device addresses) frame b is read from fptr[b], else from frames + b ny nx.
struct ProjectLaunch {
  int dtype, precision;
  const void* frames;
  int n, ny, nx;
  const float* psi;
  const uint16_t* psix_lp;
  float psi_unscale;
  const int* kmap;
  int kpad;
  float* h;
  const void* up_src;
  void* up_dst;
  size_t up_bytes;
  const uint64_t* fptr;
};
hipError_t launch_project(const ProjectLaunch& pl, hipStream_t st);

// The projections of `count` (1..16) batches of different plans in one launch, all of one
// frame type and arithmetic and without upload blocks (up_src null); members with n = 0 are
// allowed.  Its last workgroups copy xbytes (a multiple of 4) from pinned host memory xsrc
// to device memory xdst.
constexpr int kProjectGroupMax = 16;
hipError_t launch_project_group(const ProjectLaunch* pls, int count, const void* xsrc, void* xdst, size_t xbytes,
                                hipStream_t st);
// Sets the launch attributes of the grouped kernels (done by their first launch otherwise;
// call it before capturing such launches into a graph).
hipError_t prepare_group_kernels();

// The column pass of a display from partial rows (launch_dft_rows with nslot partials and
// the final scale): `rows` output rows of power-of-two length len.
struct DisplayColumns {
  const float2* din;
  float2* dout;
  int rows, len;
  const float2* e;
  const float2* d0;
  float s_total;
  int in_sr, in_sm, out_sr, out_sc, nslot, slot_stride;
};
// launch_project and, in the same launch, that column pass: workgroups past the projections
// (and the upload copy) each write one output row.  n >= 1.
hipError_t launch_project_display(const ProjectLaunch& pl, const DisplayColumns& dc, hipStream_t st);

// Columns (in blocks of 32) per accumulation workgroup for a padded basis size.
int accumulate_col_blocks(int kpad);

// acc[j][c] += sum_{b<n} Ty[(v_y(j) s_y(b)) mod sy] Tx[(v_x(j) s_x(b)) mod sx] h[b][c].
// n_freq_pad is a multiple of 64 and kpad a multiple of 32.
hipError_t launch_accumulate(float2* acc, int kpad, int64_t n_freq_pad, const int2* freqs, const float* h,
                             const int2* pos, int n, const float2* ty, int sy, const float2* tx, int sx,
                             hipStream_t st);

// d[j] = sum_c w[j][c] acc[j][c]; z[v_x(j)][v_y(j)] = conj(d[j]) (z is [sx][sy]).
hipError_t launch_wiener(const float2* acc, const float2* w, int kpad, const int2* freqs, int64_t n_freq, float2* d,
                         float2* z, int sy, hipStream_t st);

// out[r * out_sr + c * out_sc] = scale * sum_m in[r * in_sr + m * in_sm] e[(m c) mod len] for
// r < rows, c < len (see kernels.hip).  nslot > 1 (power-of-two len): each input value is the
// sum of the nslot partials at slot_stride apart.
constexpr int kMaxSlots = 8;         // partial display rows per x-frequency
constexpr int kDisplayRowMax = 1024;  // longest row the object-order update transforms for the display
hipError_t launch_dft_rows(const float2* in, float2* out, int rows, int len, const float2* e, const float2* d0,
                           float s_total, int final_scale, int in_sr, int in_sm, int out_sr, int out_sc, int nslot,
                           int slot_stride, hipStream_t st);

// launch_dft_rows (no partials) over `blocks` grids of block_rows rows each, grid b's input,
// output and D[0] in_block, out_block and d0_block values after grid 0's.
hipError_t launch_dft_rows_blocks(const float2* in, float2* out, int blocks, int block_rows, int len, const float2* e,
                                  const float2* d0, float s_total, int final_scale, int in_sr, int in_sm, int out_sr,
                                  int out_sc, int64_t in_block, int64_t out_block, int64_t d0_block, hipStream_t st);

// Field-of-view patches: out[y][x] = sum_p w img_p[y - oy][x - ox] / sum_p w over the patches
// (row-major over the origin grid oy[npy] x ox[npx]) covering (y, x); img [npy npx][py][px];
// w = trapezoid window of the y axis times the x axis's (1 inside, linear over the overlap).
hipError_t launch_patch_merge(const float2* img, const int* oy, int npy, const int* ox, int npx, int py, int px,
                              int overlap_y, int overlap_x, float2* out, int sy, int sx, hipStream_t st);

// Row-factored accumulation (see kernels.hip): t[r][vx][c] = sum over the frames of row r of
// Tx[(vx x_b) mod sx] h[b][c] (order[i]: the batch's frame indices grouped by row, xs[i]: the
// scan x of frame order[i]); then acc[j][c] += sum_r Ty[(v_y(j) y_r) mod sy] t[r][v_x(j)][c],
// optionally followed by the Wiener reduction of launch_wiener in the same pass (z as there).
hipError_t launch_row_dft(const float* h, int kpad, const int* xs, const int* order, const int4* rows, int nrows,
                          const float2* tx, int sx, float2* t, hipStream_t st);
hipError_t launch_row_update(float2* acc, int kpad, int64_t n_freq_pad, const int2* freqs, int64_t n_freq,
                             const float2* t, int sx, const int4* rows, int nrows, const float2* ty, int sy,
                             const float2* w, float2* d, float2* z, bool fuse_wiener, hipStream_t st);

// Object-order row-factored update with the per-row x-DFT fused in (one workgroup per chunk
// of kept frequencies sharing an x-frequency; D held as the compensated pair d + dlo, d the
// FP32 value nearest the sum): d[j] += sum_r E_sy(v_y(j) y_r) sum_c w[j][c]
// T_r[v_x(j)][c] with T_r[vx][c] = sum_{frames b of row r} tscale E_sx(vx x_b) h[b][c],
// E_s(m) = exp(-2 pi i m / s); z as in launch_wiener.  rows.r[r] = (y_r, first index into
// order and xs, frame count, 0) for r < nrows <= kRowSetMax; xs[i] is the scan x of frame
// order[i].  chunks[c] = (vx, first index into jv, count <= max_chunk <= 512, slot < nslot);
// jv[i] = (j, v_y(j)).  With up set (power-of-two sy <= kDisplayRowMax, nslot <= kMaxSlots),
// up[(y sx + vx) nslot + slot] = sum_{j of chunk c} conj(d[j]) E_sy(v_y(j) y) after the update:
// the display's first pass split over the chunks; with d0out set, the launch also stores the
// updated D[0] there (the normalisation of that display, read by a later launch).  With dc,
// workgroups past the chunks write the rows of an earlier image from its partial rows (the
// column pass of launch_project_display), which must not be the `up` this launch writes.
// in_order: order[i] = i for the frames of
// the pass (row order already), which lets the kernel load their projections before the
// indices arrive.
constexpr int kRowSetMax = 16;
constexpr int kFusedThreads = 512;  // threads of a workgroup of the object-order update
struct RowSet {
  int4 r[kRowSetMax];
};
// One row pass of an object-order update, as launch_row_fused_obj takes it, for the grouped
// launch: rows[r] as RowSet, the chunk list given per work item instead.
struct ObjPass {
  const float* h;
  const int* order;
  const int* xs;
  const int2* jv;
  const float2* w;
  float2* d;
  float2* dlo;
  float2* z;
  float2* up;
  const int4* rows;  // [nrows] (y_r, first index into order and xs, frame count, 0), device memory
  int kpad, nrows, sx, sy, max_chunk, nslot, log2sy, in_order;
  float tscale;
};
// The row passes of several updates in one launch: workgroup b takes items[b] = (index into
// passes, v_x, first jv index, count | slot << 16).  lds_bytes: the largest
// row_fused_lds_bytes of the passes.  passes and items in device memory.
hipError_t launch_row_fused_obj_group(const ObjPass* passes, const int4* items, int nitems, size_t lds_bytes,
                                      hipStream_t st);
size_t row_fused_lds_bytes(int kpad, int nrows, int max_chunk);

// One spectrum-order row pass of a plan (at most kRowSetMax rows of one batch) for the
// grouped launches: the row DFT T_r = Fx_r h_r, then A += sum_r Ty T_r (with fuse, D =
// sum_k W A and z = conj D in the same pass).  All pointers are device memory.
struct SpecPass {
  const float* h;
  const int* xs;
  const int* order;
  const int4* rows;
  const float2* tx;
  const float2* ty;
  float2* t;
  float2* acc;
  const int2* freqs;
  const float2* w;
  float2* d;
  float2* z;
  int64_t n_freq;
  int nrows, sx, sy, kpad, fuse;
};
size_t row_dft_lds_bytes(int sx);
int row_dft_blocks(int sx, int kpad, int nrows);
int row_update_blocks(int64_t n_freq_pad, int kpad);
// Launch of the row DFTs (resp. updates) of npass passes; first[i] = the first workgroup of
// pass i (running sum of row_dft_blocks, resp. row_update_blocks), nblocks the total; lds
// the largest row_dft_lds_bytes.  passes and first in device memory.
hipError_t launch_row_dft_group(const SpecPass* passes, const int* first, int npass, int nblocks, size_t lds,
                                hipStream_t st);
hipError_t launch_row_update_group(const SpecPass* passes, const int* first, int npass, int nblocks, hipStream_t st);

hipError_t launch_row_fused_obj(const float* h, int kpad, const int* order, const int* xs, const RowSet& rows,
                                int nrows, float tscale, int sx, int sy, const int4* chunks, int nchunks,
                                int max_chunk, const int2* jv, const float2* w, float2* d, float2* dlo, float2* z,
                                float2* up, int nslot, bool in_order, float2* d0out, const DisplayColumns* dc,
                                hipStream_t st);

// launch_row_fused_obj with the projection `next` (a batch of the same plan, written to its own
// h and upload block) in the same launch; next.n >= 1 and row_fused_next_supported.
bool row_fused_next_supported(int dtype, int precision, int ny, int nx, int kpad);
hipError_t launch_row_fused_obj_next(const float* h, int kpad, const int* order, const int* xs, const RowSet& rows,
                                     int nrows, float tscale, int sx, int sy, const int4* chunks, int nchunks,
                                     int max_chunk, const int2* jv, const float2* w, float2* d, float2* dlo,
                                     float2* z, float2* up, int nslot, bool in_order, float2* d0out,
                                     const DisplayColumns* dc, const ProjectLaunch& next, hipStream_t st);

// Two-stage pipelined pushes: one launch with the update of a batch whose x-DFT T (per kept
// v_x: [kRowSetMax][kpad / 4][2] float4, row_fused_t_stride(kpad) apart) an earlier launch
// wrote to tin, the x-DFT of the next batch into xp.tout (one workgroup per kept v_x, xcols),
// and the projection of the batch after it (next, or null); nchunks = 0, xp.ncols = 0 leave
// their parts out.  The update's rows are urows[0 .. unrows); up, d0out, dc as in
// launch_row_fused_obj.
struct XdftPart {
  const float* h;
  const int* order;
  const int* xs;
  RowSet rows;
  int nrows;
  bool in_order;
  const int* xcols;
  int ncols;
  float4* tout;
};
int row_fused_t_stride(int kpad);
hipError_t launch_row_fused_obj_next2(int kpad, float tscale, int sx, int sy, const int4* chunks, int nchunks,
                                      int max_chunk, const int2* jv, const float2* w, float2* d, float2* dlo,
                                      float2* z, int nslot, const RowSet& urows, int unrows, const float4* tin,
                                      float2* up, float2* d0out, const XdftPart& xp, const DisplayColumns* dc,
                                      const ProjectLaunch* next, hipStream_t st);

// Full Fourier basis (K = ny nx, complex h; see kernels.hip).  Projection: h[b][k_y nx + k_x]
// = 2D DFT of frame b with exp(+2 pi i ...) / (ny nx); ny, nx powers of two, ny nx <= 4096,
// fy/fx = exp(+2 pi i m / n) for m < n / 2.  Row DFT: t[r][vx][k] = sum over the frames of
// row r of Tx[(vx x_b) mod sx] h[b][k].  Update (one workgroup per kept frequency): mode 0
// object order (d += sum_k w s), 1 spectrum order (acc += s), 2 spectrum order with the
// Wiener reduction (acc += s; d = sum_k w acc), s[k] = sum_r Ty[(v_y y_r) mod sy] t[r][v_x][k].
hipError_t launch_project_fourier(int dtype, const void* frames, int n, int ny, int nx, const float2* fy,
                                  const float2* fx, float2* h, int kpad, const void* up_src, void* up_dst,
                                  size_t up_bytes, const uint64_t* fptr, hipStream_t st);
hipError_t launch_row_dft_c(const float2* h, int kpad, const int* order, const int* xs, const RowSet& rows, int nrows,
                            const float2* tx, int sx, float2* t, hipStream_t st);
hipError_t launch_update_c(int mode, const float2* t, int kpad, const RowSet& rows, int nrows, const float2* ty, int sy,
                           int sx, const int2* freqs, int64_t n_freq, const float2* w, float2* acc, float2* d,
                           float2* dlo, float2* z, hipStream_t st);

// z[v_x(j)][v_y(j)] = conj(d[j]) for j < n_freq.
hipError_t launch_scatter_conj(const float2* d, const int2* freqs, int64_t n_freq, float2* z, int sy, hipStream_t st);

// z[vx][vy] = conj(d[vy][vx]) for the sy x sx grid d; ey, ex = exp(-2 pi i m / s) for m < s
// (FP64 arguments, FP32 values): the inputs of the two display passes (launch_dft_rows).
hipError_t launch_display_prep(const float2* d, int sy, int sx, float2* z, float2* ey, float2* ex, hipStream_t st);

hipError_t launch_zero(float* p, size_t n, hipStream_t st);

}  // namespace wdd
