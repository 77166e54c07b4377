// HIP kernels of the live WDD per-frame update for gfx950 (CDNA4, wave64).
//
//   k_project, k_project_lp   frames -> h = Phi^T vec(I)  (Section 5 reduction; FP32, or
//                             BF16/FP16 MFMA with FP32 accumulation)
//   k_row_fused_obj   object order: D[v] += sum_b F[v,b] sum_k W[v,k] h[b,k], row-factored
//                     with the scan x-DFT fused in (modified-WDD algorithm, Section 6.3)
//   k_row_dft, k_row_update   spectrum order, row-factored: A[v,k] += sum_b F[v,b] h[b,k]
//                     (Section 6.1 F = F_y (x) F_x), optionally with D = sum_k W A fused
//   k_accumulate      spectrum order, direct: the same sum on FP32 MFMA
//   k_wiener          D[v] = sum_k W[v,k] A[v,k]  (deconvolution + summation)
//   k_project_fourier, k_row_dft_c, k_update_c   the same path with the full Fourier basis
//                     (K = ny nx, complex h): conventional WDD
//   k_dft_rows        row DFTs for O~ = conj(IDFT2(D)) / sqrt(|D[0]|)   (eq. extract)
//
// Complex values are float2 (re, im).  No atomics: every output element has a
// single owner, so results are deterministic for fixed batch boundaries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include "kernels.h"

namespace {

using wdd::RowSet;
using wdd::kRowSetMax;
using wdd::kDisplayRowMax;
using wdd::kFusedThreads;
using wdd::kMaxSlots;

constexpr size_t kLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950

// Opts a kernel into the whole LDS once: a function-local static per kernel, whose
// initialisation C++ makes thread-safe (plans on several host threads may launch at once).
template <auto Kernel>
hipError_t allow_full_lds() {
  static const hipError_t e =
      hipFuncSetAttribute(reinterpret_cast<const void*>(Kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kLdsBytes);
  return e;
}


typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// Loads through global-address-space pointers.  Frames may be reached through a table of
// addresses (generic pointers); device and pinned host memory are both global memory here,
// and global loads, unlike flat ones, do not hold up waits on LDS traffic.
#define WDD_GLOBAL(T) const __attribute__((address_space(1))) T*
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ inline float gload(const float* p) { return *(WDD_GLOBAL(float))p; }
__device__ inline uint16_t gload(const uint16_t* p) { return *(WDD_GLOBAL(uint16_t))p; }
__device__ inline uint32_t gload(const uint32_t* p) { return *(WDD_GLOBAL(uint32_t))p; }
__device__ inline int gload(const int* p) { return *(WDD_GLOBAL(int))p; }
__device__ inline uint4 gload(const uint4* p) {
  const u32x4 v = *(WDD_GLOBAL(u32x4))p;
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ inline float4 gload(const float4* p) {
  const floatx4 v = *(WDD_GLOBAL(floatx4))p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline float2 gload(const float2* p) {
  const f32x2 v = *(WDD_GLOBAL(f32x2))p;
  return make_float2(v.x, v.y);
}
typedef int i32x2 __attribute__((ext_vector_type(2)));
__device__ inline int2 gload(const int2* p) {
  const i32x2 v = *(WDD_GLOBAL(i32x2))p;
  return make_int2(v.x, v.y);
}
#undef WDD_GLOBAL

// dst[i] = src[i] for i < n by `nthreads` threads, U loads in flight per thread before any
// store (a plain strided copy loop waits for each load in turn).
template <int U, typename T, typename D>
__device__ inline void stage_copy(D* dst, const T* src, int n, int tid, int nthreads) {
  for (int base = 0; base < n; base += U * nthreads) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * nthreads + tid;
      if (i < n) v[u] = gload(src + i);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * nthreads + tid;
      if (i < n) dst[i] = v[u];
    }
  }
}

// ---------------------------------------------------------------------------
// Projection.  Per frame G = psi_y^T I psi_x (L x L, L <= 16) is formed with
// v_mfma_f32_16x16x4_f32 in two stages, then h[k] = G[n_y(k)][n_x(k)].
//
// Stage 1, per 16-row tile of the frame: T[y][lx] = sum_x I[y][x] psi_x[x][lx].
// Lane l (row r16 = l % 16, group q = l / 16) reads 8 consecutive pixels
// I[y][x0 + 8q .. x0 + 8q + 7]; MFMA j of the chunk pairs k-slot q with pixel
// x0 + 8q + j on both operands, so the 8 MFMAs cover the 32 pixels of the chunk.
// Stage 2: the 16x16 tile result T (lane l holds T[4q + r][r16] in register r) is
// directly the B operand of G += psi_y^T T, MFMA r pairing k-slot q with row 4q + r.
// ---------------------------------------------------------------------------

template <typename T>
struct Chunk;
template <>
struct Chunk<uint16_t> {
  uint4 v;
  __device__ inline void load(const uint16_t* p) { v = gload(reinterpret_cast<const uint4*>(p)); }
  __device__ inline void zero() { v = make_uint4(0u, 0u, 0u, 0u); }
  // the loaded values where keep, else zero (a select on the values, after they arrive)
  __device__ inline void keep_if(bool keep) {
    v.x = keep ? v.x : 0u; v.y = keep ? v.y : 0u; v.z = keep ? v.z : 0u; v.w = keep ? v.w : 0u;
  }
  __device__ inline float get(int j) const {
    const uint32_t w = (j < 2) ? v.x : (j < 4) ? v.y : (j < 6) ? v.z : v.w;
    return (float)((j & 1) ? (w >> 16) : (w & 0xffffu));
  }
};
template <>
struct Chunk<float> {
  float4 a, b;
  __device__ inline void load(const float* p) {
    a = gload(reinterpret_cast<const float4*>(p));
    b = gload(reinterpret_cast<const float4*>(p + 4));
  }
  __device__ inline void zero() { a = b = make_float4(0.f, 0.f, 0.f, 0.f); }
  __device__ inline void keep_if(bool keep) {
    a.x = keep ? a.x : 0.f; a.y = keep ? a.y : 0.f; a.z = keep ? a.z : 0.f; a.w = keep ? a.w : 0.f;
    b.x = keep ? b.x : 0.f; b.y = keep ? b.y : 0.f; b.z = keep ? b.z : 0.f; b.w = keep ? b.w : 0.f;
  }
  __device__ inline float get(int j) const {
    switch (j) {
      case 0: return a.x; case 1: return a.y; case 2: return a.z; case 3: return a.w;
      case 4: return b.x; case 5: return b.y; case 6: return b.z; default: return b.w;
    }
  }
};

// The batch's upload block (positions, row grouping) lives in pinned host memory; one extra
// workgroup of the projection launch copies it to the device, so that no frame's workgroup
// waits for the PCIe round trip (loads complete in issue order).
__device__ inline void upload_block(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int n, int tid,
                                    int nthreads) {
  stage_copy<4>(dst, src, n, tid, nthreads);
}

// Table staging of the projection: psi ([ny][16] psi_y then [nx][16] psi_x, FP32) goes to
// LDS as psi_y [ny][16] and psi_x transposed, [16][nxp] (nxp = nx + 4: a lane's 8 basis
// values of a chunk are two 16-byte reads, and the 16 rows start in different banks), kmap to
// [kpad].  The first 8 psi values and 4 kmap values of every thread are loaded by
// table_issue before the frame loads go out and stored by table_finish after them, so the
// barrier that follows waits for the tables only, not for the frame.
struct TableRegs {
  float v[8];
  int k[4];
};
__device__ inline void table_issue(TableRegs& r, const float* __restrict__ psi, int ntab,
                                   const int* __restrict__ kmap, int kpad, int tid, int nt) {
#pragma unroll
  for (int u = 0; u < 8; ++u) r.v[u] = gload(psi + min(u * nt + tid, ntab - 1));
#pragma unroll
  for (int u = 0; u < 4; ++u) r.k[u] = gload(kmap + min(u * nt + tid, kpad - 1));
}
__device__ inline void table_store(float* __restrict__ lpsy, float* __restrict__ lpsxt, int ny, int nxp, int i,
                                   float v) {
  if (i < ny * 16) {
    lpsy[i] = v;
  } else {
    const int j = i - ny * 16;
    lpsxt[(j & 15) * nxp + (j >> 4)] = v;
  }
}
__device__ inline void table_finish(const TableRegs& r, const float* __restrict__ psi, int ntab,
                                    const int* __restrict__ kmap, int kpad, float* __restrict__ lpsy,
                                    float* __restrict__ lpsxt, int* __restrict__ lkmap, int ny, int nxp, int tid,
                                    int nt) {
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = u * nt + tid;
    if (i < ntab) table_store(lpsy, lpsxt, ny, nxp, i, r.v[u]);
  }
  for (int i = 8 * nt + tid; i < ntab; i += nt) table_store(lpsy, lpsxt, ny, nxp, i, gload(psi + i));
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = u * nt + tid;
    if (i < kpad) lkmap[i] = r.k[u];
  }
  for (int i = 4 * nt + tid; i < kpad; i += nt) lkmap[i] = gload(kmap + i);
}

// LDS floats of a projection workgroup: psi_y, transposed psi_x, per-wave G, kmap.
__host__ __device__ inline size_t project_lds_floats(int ny, int nx, int nw, int kpad) {
  return (size_t)ny * 16 + (size_t)16 * (nx + 4) + (size_t)nw * 256 + (size_t)kpad;
}

// Straight-line form of project_frame for a frame whose tiles each have a wave of their own
// (ntiles <= waves) and NCH chunks of 32 columns per row (nx <= 32 NCH), under the
// conditions of project_tile_form.  Every frame load is unconditional (indices clamped into the
// frame; lanes outside the frame get zero by a select after their load), so the wait before
// chunk c's MFMAs counts exactly the NCH - 1 - c later loads: the MFMAs of early chunks run
// while the later chunks are still arriving.  (Loads under a branch make the compiler wait
// for every load in flight before the first use of any of them.)
template <typename T, int NCH>
__device__ __forceinline__ void project_frame_tile(const T* __restrict__ frames, int ny, int nx,
                                                   const float* __restrict__ psi, const int* __restrict__ kmap,
                                                   int kpad, float* __restrict__ h, const uint64_t* __restrict__ fptr,
                                                   float* smem, int b) {
  const int nw = blockDim.x >> 6, nt = blockDim.x;
  const int nxp = nx + 4;
  float* lpsxt = smem;                   // [16][nxp]: psi_x transposed
  float* lg = lpsxt + 16 * nxp;          // [nw][256]: per-wave G
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T* f = fptr ? reinterpret_cast<const T*>(fptr[b]) : frames + (size_t)b * ny * nx;
  const int r16 = lane & 15, q = lane >> 4;
  const int ntiles = (ny + 15) >> 4;
  const int nsx = 16 * nx;
  // Only psi_x goes through LDS (every wave reads all of it).  The 4 psi_y values of a lane's
  // stage-2 rows and the kmap entries of its epilogue are loaded into registers here.
  float vx[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) vx[u] = gload(psi + (size_t)ny * 16 + min(u * nt + tid, nsx - 1));
  float av[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) av[r] = gload(psi + (size_t)min(wave * 16 + 4 * q + r, ny - 1) * 16 + r16);
  int km[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) km[u] = gload(kmap + min(u * nt + tid, kpad - 1));
  const int y = wave * 16 + r16;
  const bool row_ok = wave < ntiles && y < ny;
  const T* rowp = f + (size_t)min(y, ny - 1) * nx;
  // The table reaches LDS, and the workgroup synchronises, before any frame load is issued: a
  // barrier after the frame loads would hold every wave's MFMAs until all waves had issued
  // all their loads (issue stalls while the memory pipeline is full), so that no MFMA could
  // overlap the frame's arrival.  Every lane stores (lanes past the table write to their own
  // slot of the per-wave G area, which is written again after the MFMAs).
  float* spare = lg + tid;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = u * nt + tid;
    float* dst = i < nsx ? lpsxt + (i & 15) * nxp + (i >> 4) : spare;
    *dst = vx[u];
  }
  __syncthreads();
  Chunk<T> ch[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) ch[c].load(rowp + min(32 * c + 8 * q, nx - 8));

  const float* brow = lpsxt + r16 * nxp;
  floatx4 tacc = {0.f, 0.f, 0.f, 0.f}, tacc2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int xs = 32 * c + 8 * q;
    ch[c].keep_if(row_ok && xs < nx);
    const int xb = min(xs, nx - 8);  // a valid table column; the zeroed pixels cancel it
    const float4 b0 = *reinterpret_cast<const float4*>(brow + xb);
    const float4 b1 = *reinterpret_cast<const float4*>(brow + xb + 4);
    tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(0), b0.x, tacc, 0, 0, 0);
    tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(1), b0.y, tacc2, 0, 0, 0);
    tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(2), b0.z, tacc, 0, 0, 0);
    tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(3), b0.w, tacc2, 0, 0, 0);
    tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(4), b1.x, tacc, 0, 0, 0);
    tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(5), b1.y, tacc2, 0, 0, 0);
    tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(6), b1.z, tacc, 0, 0, 0);
    tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(7), b1.w, tacc2, 0, 0, 0);
  }
  tacc += tacc2;
  floatx4 g = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float a = (wave * 16 + 4 * q + r < ny) ? av[r] : 0.f;
    g = __builtin_amdgcn_mfma_f32_16x16x4f32(a, tacc[r], g, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) lg[wave * 256 + (4 * q + r) * 16 + r16] = g[r];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int k = u * nt + tid;
    if (k < kpad) {
      const int idx = km[u];
      float sum = 0.f;
      if (idx >= 0)
        for (int w = 0; w < nw; ++w) sum += lg[w * 256 + idx];
      h[(size_t)b * kpad + k] = sum;
    }
  }
}

// project_frame_tile for workgroups with fewer waves than tiles (k_row_fused_obj_next's 8
// waves): wave w takes the 16-row tiles w, w + nw, ..., each with all of its frame loads
// issued before its MFMAs; frames of nx <= 32 NCH columns (FULL: nx = 32 NCH, no clamps).  Every frame
// load is unconditional (indices clamped into the frame; lanes outside the frame get zero by
// a select after their load), so the wait before chunk c's MFMAs counts exactly the later
// loads of the tile: the MFMAs of early chunks run while the later chunks are still
// arriving.  (Loads under a branch make the compiler wait for every load in flight before
// the first use of any of them.)
template <typename T, int NCH, bool FULL>
__device__ __forceinline__ void project_frame_tiles(const T* __restrict__ frames, int ny, int nx,
                                                   const float* __restrict__ psi, const int* __restrict__ kmap,
                                                   int kpad, float* __restrict__ h, const uint64_t* __restrict__ fptr,
                                                   float* smem, int b) {
  const int nw = blockDim.x >> 6, nt = blockDim.x;
  const int nxp = nx + 4;
  float* lpsxt = smem;                   // [16][nxp]: psi_x transposed
  float* lg = lpsxt + 16 * nxp;          // [nw][256]: per-wave G
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T* f = fptr ? reinterpret_cast<const T*>(fptr[b]) : frames + (size_t)b * ny * nx;
  const int r16 = lane & 15, q = lane >> 4;
  const int ntiles = (ny + 15) >> 4;
  const int nsx = 16 * nx;
  // Only psi_x goes through LDS (every wave reads all of it).  The kmap entries of the
  // epilogue are loaded into registers here, the 4 psi_y values of a lane's stage-2 rows
  // after each tile's frame loads.
  float vx[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) vx[u] = gload(psi + (size_t)ny * 16 + min(u * nt + tid, nsx - 1));
  int km[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) km[u] = gload(kmap + min(u * nt + tid, kpad - 1));
  // The table reaches LDS, and the workgroup synchronises, before any frame load is issued: a
  // barrier after the frame loads would hold every wave's MFMAs until all waves had issued
  // all their loads (issue stalls while the memory pipeline is full), so that no MFMA could
  // overlap the frame's arrival.  Every lane stores (lanes past the table write to their own
  // slot of the per-wave G area, which is written again after the MFMAs).
  float* spare = lg + tid;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = u * nt + tid;
    float* dst = i < nsx ? lpsxt + (i & 15) * nxp + (i >> 4) : spare;
    *dst = vx[u];
  }
  __syncthreads();
  floatx4 g = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int t = wave; t < ntiles; t += nw) {
    // the basis row's offset passes through an empty asm statement: otherwise its LDS reads,
    // the same for every tile, are hoisted out of the loop and held in 64 registers
    int boff = r16 * nxp + (FULL ? 8 * q : 0);
    asm volatile("" : "+v"(boff));
    const float* brow = lpsxt + boff;
    const int y = t * 16 + r16;
    const bool row_ok = y < ny;
    // FULL (nx = 32 NCH): chunk c of the lane's row starts 32 c past its first pixel, no clamps
    const T* rowp = f + (size_t)min(y, ny - 1) * nx + (FULL ? 8 * q : 0);
    Chunk<T> ch[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) ch[c].load(FULL ? rowp + 32 * c : rowp + min(32 * c + 8 * q, nx - 8));
    float av[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) av[r] = gload(psi + (size_t)min(t * 16 + 4 * q + r, ny - 1) * 16 + r16);
    // all of the tile's loads go out before any MFMA: without this fence the scheduler moves
    // each chunk's load next to its first use, and every chunk waits for its own round trip
    __builtin_amdgcn_sched_barrier(0);

    floatx4 tacc = {0.f, 0.f, 0.f, 0.f}, tacc2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int xs = 32 * c + 8 * q;
      ch[c].keep_if(FULL ? row_ok : row_ok && xs < nx);
      // a valid table column; the zeroed pixels cancel it
      const int xb = FULL ? 32 * c : min(xs, nx - 8);
      const float4 b0 = *reinterpret_cast<const float4*>(brow + xb);
      const float4 b1 = *reinterpret_cast<const float4*>(brow + xb + 4);
      tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(0), b0.x, tacc, 0, 0, 0);
      tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(1), b0.y, tacc2, 0, 0, 0);
      tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(2), b0.z, tacc, 0, 0, 0);
      tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(3), b0.w, tacc2, 0, 0, 0);
      tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(4), b1.x, tacc, 0, 0, 0);
      tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(5), b1.y, tacc2, 0, 0, 0);
      tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(6), b1.z, tacc, 0, 0, 0);
      tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(7), b1.w, tacc2, 0, 0, 0);
      // one chunk's basis values at a time (left free, the scheduler reads them all first)
      __builtin_amdgcn_sched_barrier(0);
    }
    tacc += tacc2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float a = (t * 16 + 4 * q + r < ny) ? av[r] : 0.f;
      g = __builtin_amdgcn_mfma_f32_16x16x4f32(a, tacc[r], g, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) lg[wave * 256 + (4 * q + r) * 16 + r16] = g[r];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int k = u * nt + tid;
    if (k < kpad) {
      const int idx = km[u];
      float sum = 0.f;
      if (idx >= 0)
        for (int w = 0; w < nw; ++w) sum += lg[w * 256 + idx];
      h[(size_t)b * kpad + k] = sum;
    }
  }
}

// Whether project_frame_tile applies: one tile per wave, at most 256 columns, psi_x within
// 8 loads per thread, kmap within 4.
__host__ __device__ inline bool project_tile_form(int ny, int nx, int nw, int kpad) {
  const int ntiles = (ny + 15) / 16, nt = 64 * nw;
  return ntiles <= nw && nx <= 256 && nx >= 8 && nx * 16 <= 8 * nt && kpad <= 4 * nt;
}

// One workgroup per frame, one wave per 16-row tile (waves loop when the frame has
// more tiles than waves).  Once the tables are in LDS, a wave issues the loads of up to 8
// chunks of 32 pixels per row (256 columns) and runs a chunk's MFMAs as soon as that chunk
// has arrived.  Frame b of the batch; smem: project_lds_floats(ny, nx, nw, kpad).
template <typename T>
__device__ __forceinline__ void project_frame(const T* __restrict__ frames, int ny, int nx,
                                              const float* __restrict__ psi, const int* __restrict__ kmap, int kpad,
                                              float* __restrict__ h, const uint64_t* __restrict__ fptr, float* smem,
                                              int b) {
  const int nw = blockDim.x >> 6, nt = blockDim.x;
  const int nxp = nx + 4;
  float* lpsy = smem;                    // [ny][16]
  float* lpsxt = smem + ny * 16;         // [16][nxp]
  float* lg = lpsxt + 16 * nxp;          // [nw][256]
  int* lkmap = reinterpret_cast<int*>(lg + nw * 256);  // [kpad]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // frame b: contiguous after `frames`, or at the address listed in fptr[b] (pinned host table)
  const T* f = fptr ? reinterpret_cast<const T*>(fptr[b]) : frames + (size_t)b * ny * nx;
  const int r16 = lane & 15, q = lane >> 4;
  const int ntiles = (ny + 15) >> 4;
  const int ntab = (ny + nx) * 16;
  TableRegs tr;
  table_issue(tr, psi, ntab, kmap, kpad, tid, nt);
  table_finish(tr, psi, ntab, kmap, kpad, lpsy, lpsxt, lkmap, ny, nxp, tid, nt);
  __syncthreads();  // before the frame loads (see project_frame_tile)
  Chunk<T> ch[8];

  floatx4 g = {0.f, 0.f, 0.f, 0.f};
  const float* brow = lpsxt + r16 * nxp;
  for (int t = wave; t < ntiles; t += nw) {
    const int y = t * 16 + r16;
    floatx4 tacc = {0.f, 0.f, 0.f, 0.f};
    for (int xg = 0; xg < nx; xg += 256) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int xs = xg + 32 * c + 8 * q;
        if (y < ny && xs < nx) ch[c].load(f + (size_t)y * nx + xs);
        else ch[c].zero();
      }
      const int nch = min(8, (nx - xg + 31) >> 5);  // chunks of 32 columns inside the frame
      // per chunk: its 8 basis values (two 16-byte LDS reads), then 8 MFMAs alternating
      // between two accumulators, so that one MFMA chain does not serialise the loop
      floatx4 tacc2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        if (c >= nch) break;
        const int xs = xg + 32 * c + 8 * q;
        float4 b0 = make_float4(0.f, 0.f, 0.f, 0.f), b1 = b0;
        if (xs < nx) {
          b0 = *reinterpret_cast<const float4*>(brow + xs);
          b1 = *reinterpret_cast<const float4*>(brow + xs + 4);
        }
        tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(0), b0.x, tacc, 0, 0, 0);
        tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(1), b0.y, tacc2, 0, 0, 0);
        tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(2), b0.z, tacc, 0, 0, 0);
        tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(3), b0.w, tacc2, 0, 0, 0);
        tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(4), b1.x, tacc, 0, 0, 0);
        tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(5), b1.y, tacc2, 0, 0, 0);
        tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(6), b1.z, tacc, 0, 0, 0);
        tacc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ch[c].get(7), b1.w, tacc2, 0, 0, 0);
      }
      tacc += tacc2;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int yy = t * 16 + 4 * q + r;
      const float av = (yy < ny) ? lpsy[yy * 16 + r16] : 0.f;
      g = __builtin_amdgcn_mfma_f32_16x16x4f32(av, tacc[r], g, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) lg[wave * 256 + (4 * q + r) * 16 + r16] = g[r];
  __syncthreads();
  for (int k = tid; k < kpad; k += nt) {
    const int idx = lkmap[k];
    float sum = 0.f;
    if (idx >= 0)
      for (int w = 0; w < nw; ++w) sum += lg[w * 256 + idx];
    h[(size_t)b * kpad + k] = sum;
  }
}

// Reduced-precision projection of uint16 frames.  Stage 1 runs on
// v_mfma_f32_16x16x32_{bf16,f16}: the 8 consecutive pixels a lane loads are exactly
// its A operand (row r16, k-slots 8q .. 8q+7 of the 32-pixel chunk).  Counts are split
// exactly into two digits I = hi * 2^S + lo (S = 8 for bf16, 11 for fp16, both digits
// representable); the basis is given as hi (+ lo) parts; products accumulate in FP32,
// the hi-digit MFMAs are skipped for chunks where the wave has no nonzero hi digit.
// Stage 2 and the selection of h are FP32 as in k_project.  psix_lp: [2][16][nx]
// 16-bit words (hi part, lo part), pre-scaled by 2^psi_shift.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

template <bool BF>
struct LpTraits;
template <>
struct LpTraits<true> {
  typedef bf16x8 vec;
  typedef __bf16 elem;
  static constexpr int kShift = 8;
  __device__ static inline floatx4 mfma(vec a, vec b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct LpTraits<false> {
  typedef halfx8 vec;
  typedef _Float16 elem;
  static constexpr int kShift = 11;
  __device__ static inline floatx4 mfma(vec a, vec b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// LDS bytes of a reduced-precision projection workgroup: psi_y (FP32), per-wave G, kmap, and
// the 16-bit psi_x parts [2][16][nx + 8].
__host__ __device__ inline size_t project_lp_lds_bytes(int ny, int nx, int nw, int kpad) {
  return ((size_t)ny * 16 + (size_t)nw * 256 + (size_t)kpad) * 4 + (size_t)2 * 16 * (nx + 8) * 2;
}

// Frame b of a batch of uint16 frames with the reduced-precision stage 1 (see above).  The
// tables (psi_y, the 16-bit psi_x parts as 32-bit words, kmap) are loaded before the frame
// and stored after its loads have been issued, as in project_frame.
template <bool BF, bool HILO>
__device__ __forceinline__ void project_frame_lp(const uint16_t* __restrict__ frames, int ny, int nx,
                                                 const float* __restrict__ psi,
                                                 const uint16_t* __restrict__ psix_lp, float psi_unscale,
                                                 const int* __restrict__ kmap, int kpad, float* __restrict__ h,
                                                 const uint64_t* __restrict__ fptr, float* smem, int b) {
  typedef LpTraits<BF> Tr;
  typedef typename Tr::vec V;
  typedef typename Tr::elem E;
  constexpr int S = Tr::kShift;
  const int nw = blockDim.x >> 6, nt = blockDim.x;
  const int nxp = nx + 8;                                              // padded row of the 16-bit basis
  float* lpsy = smem;                                                  // [ny][16] FP32
  float* lg = lpsy + ny * 16;                                          // [nw][256]
  int* lkmap = reinterpret_cast<int*>(lg + nw * 256);                  // [kpad]
  uint16_t* lpx = reinterpret_cast<uint16_t*>(lkmap + kpad);           // [2][16][nxp]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint16_t* f = fptr ? reinterpret_cast<const uint16_t*>(fptr[b]) : frames + (size_t)b * ny * nx;
  const int r16 = lane & 15, q = lane >> 4;
  const int ntiles = (ny + 15) >> 4;
  // tables to LDS (loads with clamped indices, no branch) and the barrier before the frame
  // loads (see project_frame_tile)
  const int nsy = ny * 16, half = nx >> 1, nwords = (HILO ? 2 : 1) * 16 * half;
  const uint32_t* px32 = reinterpret_cast<const uint32_t*>(psix_lp);
  float vy[8];
  uint32_t vx[8];
  int vk[4];
#pragma unroll
  for (int u = 0; u < 8; ++u) vy[u] = gload(psi + min(u * nt + tid, nsy - 1));
#pragma unroll
  for (int u = 0; u < 8; ++u) vx[u] = gload(px32 + min(u * nt + tid, nwords - 1));
#pragma unroll
  for (int u = 0; u < 4; ++u) vk[u] = gload(kmap + min(u * nt + tid, kpad - 1));
  Chunk<uint16_t> ch[8];
  uint32_t* lpx32 = reinterpret_cast<uint32_t*>(lpx);
  const int hp = nxp >> 1;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = u * nt + tid;
    if (i < nsy) lpsy[i] = vy[u];
    if (i < nwords) lpx32[(i / half) * hp + i % half] = vx[u];
  }
  for (int i = 8 * nt + tid; i < nsy; i += nt) lpsy[i] = gload(psi + i);
  for (int i = 8 * nt + tid; i < nwords; i += nt) lpx32[(i / half) * hp + i % half] = gload(px32 + i);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = u * nt + tid;
    if (i < kpad) lkmap[i] = vk[u];
  }
  for (int i = 4 * nt + tid; i < kpad; i += nt) lkmap[i] = gload(kmap + i);
  __syncthreads();

  floatx4 g = {0.f, 0.f, 0.f, 0.f};
  const V vzero = {};
  for (int t = wave; t < ntiles; t += nw) {
    const int y = t * 16 + r16;
    floatx4 tlo = {0.f, 0.f, 0.f, 0.f}, thi = {0.f, 0.f, 0.f, 0.f};
    for (int xg = 0; xg < nx; xg += 256) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int xs = xg + 32 * c + 8 * q;
        if (y < ny && xs < nx) ch[c].load(f + (size_t)y * nx + xs);
        else ch[c].zero();
      }
      const int nch = min(8, (nx - xg + 31) >> 5);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        if (c >= nch) break;
        const int xs = xg + 32 * c + 8 * q;
        V alo, ahi;
        uint32_t any_hi = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const uint32_t v = (uint32_t)ch[c].get(j);
          const uint32_t hi = v >> S;
          any_hi |= hi;
          alo[j] = (E)(float)(v & ((1u << S) - 1u));
          ahi[j] = (E)(float)hi;
        }
        V bhi = vzero, blo = vzero;
        if (xs < nx) {
          bhi = *reinterpret_cast<const V*>(lpx + r16 * nxp + xs);
          if (HILO) blo = *reinterpret_cast<const V*>(lpx + (16 + r16) * nxp + xs);
        }
        tlo = Tr::mfma(alo, bhi, tlo);
        if (HILO) tlo = Tr::mfma(alo, blo, tlo);
        if (__any(any_hi != 0u)) {
          thi = Tr::mfma(ahi, bhi, thi);
          if (HILO) thi = Tr::mfma(ahi, blo, thi);
        }
      }
    }
    floatx4 tacc;
#pragma unroll
    for (int r = 0; r < 4; ++r) tacc[r] = (tlo[r] + thi[r] * (float)(1 << S)) * psi_unscale;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int yy = t * 16 + 4 * q + r;
      const float av = (yy < ny) ? lpsy[yy * 16 + r16] : 0.f;
      g = __builtin_amdgcn_mfma_f32_16x16x4f32(av, tacc[r], g, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) lg[wave * 256 + (4 * q + r) * 16 + r16] = g[r];
  __syncthreads();
  for (int k = tid; k < kpad; k += nt) {
    const int idx = lkmap[k];
    float sum = 0.f;
    if (idx >= 0)
      for (int w = 0; w < nw; ++w) sum += lg[w * 256 + idx];
    h[(size_t)b * kpad + k] = sum;
  }
}

// Straight-line form of project_frame_lp under the conditions of project_tile_form (see
// project_frame_tile): unconditional loads with clamped indices, lanes outside the frame
// zeroed by a select, and table stores that every lane makes (out-of-range lanes into a
// spare slot), so that chunk c's MFMAs wait only for chunk c.
template <bool BF, bool HILO, int NCH>
__device__ __forceinline__ void project_frame_lp_tile(const uint16_t* __restrict__ frames, int ny, int nx,
                                                      const float* __restrict__ psi,
                                                      const uint16_t* __restrict__ psix_lp, float psi_unscale,
                                                      const int* __restrict__ kmap, int kpad, float* __restrict__ h,
                                                      const uint64_t* __restrict__ fptr, float* smem, int b) {
  typedef LpTraits<BF> Tr;
  typedef typename Tr::vec V;
  typedef typename Tr::elem E;
  constexpr int S = Tr::kShift;
  const int nw = blockDim.x >> 6, nt = blockDim.x;
  const int nxp = nx + 8;
  float* lpsy = smem;
  float* lg = lpsy + ny * 16;
  int* lkmap = reinterpret_cast<int*>(lg + nw * 256);
  uint16_t* lpx = reinterpret_cast<uint16_t*>(lkmap + kpad);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint16_t* f = fptr ? reinterpret_cast<const uint16_t*>(fptr[b]) : frames + (size_t)b * ny * nx;
  const int r16 = lane & 15, q = lane >> 4;
  const int ntiles = (ny + 15) >> 4;
  const int nsy = ny * 16, half = nx >> 1, nwords = (HILO ? 2 : 1) * 16 * half;
  const uint32_t* px32 = reinterpret_cast<const uint32_t*>(psix_lp);
  float vy[8];
  uint32_t vx[8];
  int vk[4];
#pragma unroll
  for (int u = 0; u < 8; ++u) vy[u] = gload(psi + min(u * nt + tid, nsy - 1));
#pragma unroll
  for (int u = 0; u < 8; ++u) vx[u] = gload(px32 + min(u * nt + tid, nwords - 1));
#pragma unroll
  for (int u = 0; u < 4; ++u) vk[u] = gload(kmap + min(u * nt + tid, kpad - 1));
  const int y = wave * 16 + r16;
  const bool row_ok = wave < ntiles && y < ny;
  const uint16_t* rowp = f + (size_t)min(y, ny - 1) * nx;
  // tables to LDS and the barrier before the frame loads (see project_frame_tile)
  uint32_t* lpx32 = reinterpret_cast<uint32_t*>(lpx);
  const int hp = nxp >> 1;
  float* spare = lg + tid;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = u * nt + tid;
    float* dy = i < nsy ? lpsy + i : spare;
    *dy = vy[u];
    uint32_t* dx = i < nwords ? lpx32 + (i / half) * hp + i % half : reinterpret_cast<uint32_t*>(spare);
    *dx = vx[u];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = u * nt + tid;
    int* dk = i < kpad ? lkmap + i : reinterpret_cast<int*>(spare);
    *dk = vk[u];
  }
  __syncthreads();
  Chunk<uint16_t> ch[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) ch[c].load(rowp + min(32 * c + 8 * q, nx - 8));

  floatx4 tlo = {0.f, 0.f, 0.f, 0.f}, thi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int xs = 32 * c + 8 * q;
    ch[c].keep_if(row_ok && xs < nx);
    const int xb = min(xs, nx - 8);
    V alo, ahi;
    uint32_t any_hi = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t v = (uint32_t)ch[c].get(j);
      const uint32_t hi = v >> S;
      any_hi |= hi;
      alo[j] = (E)(float)(v & ((1u << S) - 1u));
      ahi[j] = (E)(float)hi;
    }
    const V bhi = *reinterpret_cast<const V*>(lpx + r16 * nxp + xb);
    tlo = Tr::mfma(alo, bhi, tlo);
    if (HILO) tlo = Tr::mfma(alo, *reinterpret_cast<const V*>(lpx + (16 + r16) * nxp + xb), tlo);
    if (__any(any_hi != 0u)) {
      thi = Tr::mfma(ahi, bhi, thi);
      if (HILO) thi = Tr::mfma(ahi, *reinterpret_cast<const V*>(lpx + (16 + r16) * nxp + xb), thi);
    }
  }
  floatx4 tacc;
#pragma unroll
  for (int r = 0; r < 4; ++r) tacc[r] = (tlo[r] + thi[r] * (float)(1 << S)) * psi_unscale;
  floatx4 g = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int yy = wave * 16 + 4 * q + r;
    const float av = (yy < ny) ? lpsy[min(yy, ny - 1) * 16 + r16] : 0.f;
    g = __builtin_amdgcn_mfma_f32_16x16x4f32(av, tacc[r], g, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) lg[wave * 256 + (4 * q + r) * 16 + r16] = g[r];
  __syncthreads();
  for (int k = tid; k < kpad; k += nt) {
    const int idx = lkmap[k];
    float sum = 0.f;
    if (idx >= 0)
      for (int w = 0; w < nw; ++w) sum += lg[w * 256 + idx];
    h[(size_t)b * kpad + k] = sum;
  }
}

// Whether project_frame_lp_tile applies (its 16-bit table within the first load block too).
__host__ __device__ inline bool project_lp_tile_form(int ny, int nx, int nw, int kpad) {
  const int ntiles = (ny + 15) / 16, nt = 64 * nw;
  return ntiles <= nw && nx <= 256 && ny * 16 <= 8 * nt && 2 * 16 * (nx / 2) <= 8 * nt && kpad <= 4 * nt;
}

// Arguments of a projection launch (passed by value).
struct ProjArgs {
  const void* frames;
  int n, ny, nx;
  const float* psi;
  const uint16_t* psix_lp;  // reduced precision: [2][16][nx] 16-bit parts of psi_x
  float psi_unscale;
  const int* kmap;
  int kpad;
  float* h;
  const uint32_t* up_src;  // upload block (pinned host memory) and its device copy
  uint32_t* up_dst;
  int up_words;
  const uint64_t* fptr;  // per-frame addresses (pinned host table) or null
};

// Frame b with the arithmetic PREC (a wdd_precision; reduced precisions need uint16 frames).
template <typename T, int PREC>
__device__ __forceinline__ void project_any(const ProjArgs& a, float* smem, int b) {
  if constexpr (PREC == WDD_FP32) {
    const T* fr = static_cast<const T*>(a.frames);
    if (project_tile_form(a.ny, a.nx, (int)(blockDim.x >> 6), a.kpad)) {
      switch ((a.nx + 31) >> 5) {  // chunks of 32 columns per row
        case 1: project_frame_tile<T, 1>(fr, a.ny, a.nx, a.psi, a.kmap, a.kpad, a.h, a.fptr, smem, b); return;
        case 2: project_frame_tile<T, 2>(fr, a.ny, a.nx, a.psi, a.kmap, a.kpad, a.h, a.fptr, smem, b); return;
        case 3: project_frame_tile<T, 3>(fr, a.ny, a.nx, a.psi, a.kmap, a.kpad, a.h, a.fptr, smem, b); return;
        case 4: project_frame_tile<T, 4>(fr, a.ny, a.nx, a.psi, a.kmap, a.kpad, a.h, a.fptr, smem, b); return;
        case 5: project_frame_tile<T, 5>(fr, a.ny, a.nx, a.psi, a.kmap, a.kpad, a.h, a.fptr, smem, b); return;
        case 6: project_frame_tile<T, 6>(fr, a.ny, a.nx, a.psi, a.kmap, a.kpad, a.h, a.fptr, smem, b); return;
        case 7: project_frame_tile<T, 7>(fr, a.ny, a.nx, a.psi, a.kmap, a.kpad, a.h, a.fptr, smem, b); return;
        default: project_frame_tile<T, 8>(fr, a.ny, a.nx, a.psi, a.kmap, a.kpad, a.h, a.fptr, smem, b); return;
      }
    }
    project_frame<T>(fr, a.ny, a.nx, a.psi, a.kmap, a.kpad, a.h, a.fptr, smem, b);
  } else {
    constexpr bool bf = PREC == WDD_BF16_HILO || PREC == WDD_BF16;
    constexpr bool hilo = PREC == WDD_BF16_HILO || PREC == WDD_FP16_HILO;
    const uint16_t* fr = static_cast<const uint16_t*>(a.frames);
    if (project_lp_tile_form(a.ny, a.nx, (int)(blockDim.x >> 6), a.kpad)) {
#define WDD_LP_TILE(N)                                                                                          \
  project_frame_lp_tile<bf, hilo, N>(fr, a.ny, a.nx, a.psi, a.psix_lp, a.psi_unscale, a.kmap, a.kpad, a.h, a.fptr, \
                                     smem, b);                                                                  \
  return
      switch ((a.nx + 31) >> 5) {
        case 1: WDD_LP_TILE(1);
        case 2: WDD_LP_TILE(2);
        case 3: WDD_LP_TILE(3);
        case 4: WDD_LP_TILE(4);
        case 5: WDD_LP_TILE(5);
        case 6: WDD_LP_TILE(6);
        case 7: WDD_LP_TILE(7);
        default: WDD_LP_TILE(8);
      }
#undef WDD_LP_TILE
    }
    project_frame_lp<bf, hilo>(fr, a.ny, a.nx, a.psi, a.psix_lp, a.psi_unscale, a.kmap, a.kpad, a.h, a.fptr, smem, b);
  }
}

// Workgroups b < n project frame b; with an upload block, workgroup n copies it.
template <typename T, int PREC>
__global__ __launch_bounds__(1024) void k_project(ProjArgs a) {
  extern __shared__ float4 psm[];
  if ((int)blockIdx.x == a.n) {
    upload_block(a.up_src, a.up_dst, a.up_words, (int)threadIdx.x, (int)blockDim.x);
    return;
  }
  project_any<T, PREC>(a, reinterpret_cast<float*>(psm), (int)blockIdx.x);
}

// The projections of several plans' batches in one launch (plans of one frame type and
// arithmetic): member m projects launch workgroups [first[m], first[m + 1]) as its frames
// 0, 1, ...  Workgroups past the frames bring a block of xwords words from pinned host
// memory to the device, kGroupUploadWords words each (the descriptors of the updates that
// follow).  Passed by value: the member table is read with scalar loads.
constexpr int kProjGroupMax = 16;
constexpr int kGroupUploadWords = 8192;
struct ProjGroupArgs {
  ProjArgs a[kProjGroupMax];
  int first[kProjGroupMax + 1];
  int members;
  const uint32_t* xsrc;
  uint32_t* xdst;
  int xwords;
};
static_assert(sizeof(ProjGroupArgs) <= 4096, "kernel arguments are limited to 4 KiB");

template <typename T, int PREC>
__global__ __launch_bounds__(1024) void k_project_group(ProjGroupArgs g) {
  extern __shared__ float4 gsm[];
  const int b = (int)blockIdx.x, total = g.first[g.members];
  if (b >= total) {
    const int w0 = (b - total) * kGroupUploadWords;
    upload_block(g.xsrc + w0, g.xdst + w0, min(kGroupUploadWords, g.xwords - w0), (int)threadIdx.x,
                 (int)blockDim.x);
    return;
  }
  int m = 0;
  while (m + 1 < g.members && b >= g.first[m + 1]) ++m;
  project_any<T, PREC>(g.a[m], reinterpret_cast<float*>(gsm), b - g.first[m]);
}

// ---------------------------------------------------------------------------
// Accumulation: A[j][c] += sum_b F[j][b] h[b][c] over the kept frequencies j.
// Viewed as a real GEMM with rows (j, re/im) interleaved: row 2j is Re F, row
// 2j+1 is Im F.  v_mfma_f32_32x32x2_f32; a workgroup of 4 waves owns 64
// frequencies x (NCB * 32) columns, each wave 16 frequencies (32 rows) and all
// of the workgroup's columns, held in registers for the whole batch.  The
// phase F = Ty[(v_y s_y) mod S_y] * Tx[(v_x s_x) mod S_x] is formed per lane
// from LDS tables built in FP64 on the host (Tx carries the 1/sqrt(S) factor).
// ---------------------------------------------------------------------------

// exp(-2 pi i m / s) * scale for 0 <= m < s, from the device's sincospi (no table gather).
__device__ inline float2 twiddle(int m, int s, float scale) {
  float sn, cs;
  sincospif(2.0f * (float)m / (float)s, &sn, &cs);
  return make_float2(cs * scale, -sn * scale);
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) in turn: workgroup b runs on
// XCD b mod 8.  This maps b to the row it handles so that each XCD takes a contiguous
// range of rows (a bijection of [0, n)); rows that share cache lines then share an L2.
constexpr int kXcds = 8;
__device__ inline int xcd_row(int b, int n) {
  const int per = n / kXcds;
  return b < per * kXcds ? (b % kXcds) * per + b / kXcds : b;
}

// (p mod s) for 0 <= p < 2^24 via a float reciprocal and one correction.
__device__ inline int mod_small(int p, int s, float inv) {
  int qq = (int)((float)p * inv);
  int r = p - qq * s;
  r += (r < 0) ? s : 0;
  r -= (r >= s) ? s : 0;
  return r;
}

template <int NCB>
__global__ __launch_bounds__(256) void k_accumulate(float2* __restrict__ acc, int kpad,
                                                    const int2* __restrict__ freqs,
                                                    const float* __restrict__ h, const int2* __restrict__ pos,
                                                    int n, const float2* __restrict__ ty, int sy,
                                                    const float2* __restrict__ tx, int sx) {
  constexpr int NC = NCB * 32;
  extern __shared__ float2 smem2[];
  float2* lty = smem2;                                   // [sy]
  float2* ltx = lty + sy;                                // [sx]
  int2* lpos = reinterpret_cast<int2*>(ltx + sx);        // [32]
  float* lh = reinterpret_cast<float*>(lpos + 32);       // [32][NC]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < sy; i += 256) lty[i] = ty[i];
  for (int i = tid; i < sx; i += 256) ltx[i] = tx[i];

  const int j0 = blockIdx.x * 64 + wave * 16;
  const int c0 = blockIdx.y * NC;
  const int i32 = lane & 31, half = lane >> 5;
  const int2 v = freqs[j0 + (i32 >> 1)];
  const bool im = (i32 & 1) != 0;

  floatx16 c[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      const int row = 8 * (r >> 2) + 4 * half + (r & 3);
      const float2 a = acc[(size_t)(j0 + (row >> 1)) * kpad + c0 + cb * 32 + i32];
      c[cb][r] = a.x;
      c[cb][r + 1] = a.y;
    }
  }
  const float invy = 1.0f / (float)sy, invx = 1.0f / (float)sx;

  for (int b0 = 0; b0 < n; b0 += 32) {
    __syncthreads();
    if (tid < 32) lpos[tid] = (b0 + tid < n) ? pos[b0 + tid] : make_int2(0, 0);
    for (int i = tid; i < 32 * NC; i += 256) {
      const int bb = i / NC, cc = i - bb * NC;
      lh[i] = (b0 + bb < n) ? h[(size_t)(b0 + bb) * kpad + c0 + cc] : 0.f;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      const int bl = 2 * kk + half;
      const int2 s = lpos[bl];
      const int my = mod_small(v.x * s.x, sy, invy);
      const int mx = mod_small(v.y * s.y, sx, invx);
      const float2 p = lty[my], qv = ltx[mx];
      const float a = im ? (p.x * qv.y + p.y * qv.x) : (p.x * qv.x - p.y * qv.y);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const float bv = lh[bl * NC + cb * 32 + i32];
        c[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, c[cb], 0, 0, 0);
      }
    }
  }

#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      const int row = 8 * (r >> 2) + 4 * half + (r & 3);
      acc[(size_t)(j0 + (row >> 1)) * kpad + c0 + cb * 32 + i32] = make_float2(c[cb][r], c[cb][r + 1]);
    }
  }
}

// ---------------------------------------------------------------------------
// Wiener reduction: one wave per kept frequency; D[j] = sum_k W[j][k] A[j][k].
// Also scatters conj(D[j]) into the grid z, stored transposed as [sx][sy] (zeros
// elsewhere are set once at plan creation), ready for the display DFT.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wiener(const float2* __restrict__ acc, const float2* __restrict__ w,
                                                int kpad, const int2* __restrict__ freqs, int64_t n_freq,
                                                float2* __restrict__ d, float2* __restrict__ z, int sy) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + wave;
  if (j >= n_freq) return;
  const float4* a4 = reinterpret_cast<const float4*>(acc + j * kpad);
  const float4* w4 = reinterpret_cast<const float4*>(w + j * kpad);
  float re = 0.f, im = 0.f;
  for (int i = lane; i < kpad / 2; i += 64) {
    const float4 a = a4[i], b = w4[i];
    re += a.x * b.x - a.y * b.y;
    im += a.x * b.y + a.y * b.x;
    re += a.z * b.z - a.w * b.w;
    im += a.z * b.w + a.w * b.z;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (lane == 0) {
    d[j] = make_float2(re, im);
    const int2 v = freqs[j];
    z[(size_t)v.y * sy + v.x] = make_float2(re, -im);
  }
}

// In-place radix-2 decimation-in-time FFT of buf[0 .. len) (stored in bit-reversed order)
// with the twiddles tw[m] = E[m], m < len / 2, in LDS; the nt threads of the workgroup take
// part, and every stage ends at a workgroup barrier.
__device__ inline void lds_fft(float2* buf, const float2* tw, int len, int log2len, int tid, int nt) {
  for (int s = 1; s <= log2len; ++s) {
    const int half = 1 << (s - 1);
    const int stride = len >> s;  // twiddle index step
    for (int k = tid; k < len / 2; k += nt) {
      const int grp = k >> (s - 1), p = k & (half - 1);
      const int i0 = grp * (half << 1) + p, i1 = i0 + half;
      const float2 t = tw[p * stride];
      const float2 x1 = buf[i1], x0 = buf[i0];
      const float2 tt = make_float2(t.x * x1.x - t.y * x1.y, t.x * x1.y + t.y * x1.x);
      buf[i0] = make_float2(x0.x + tt.x, x0.y + tt.y);
      buf[i1] = make_float2(x0.x - tt.x, x0.y - tt.y);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Forward DFT of each of `rows` rows of length len:
//   out[r * out_sr + c * out_sc] = scale * sum_m in[r * in_sr + m * in_sm] * E[(m c) mod len],
// E[m] = exp(-2 pi i m / len) built in FP64 on the host.  Power-of-two lengths use an
// in-LDS radix-2 decimation-in-time FFT with the twiddles staged in LDS, others a direct
// sum.  With `final_scale` set, scale = 1 / sqrt(S |D[0]|) (0 when D[0] = 0).  SLOTS
// (launched for nslot > 1, power-of-two lengths only): each input value is the sum of the
// nslot partials in[r * in_sr + m * in_sm + s * slot_stride], s < nslot <= kMaxSlots, added
// in order of s.
// ---------------------------------------------------------------------------
// One output row r of the display's column pass from partial rows: power-of-two len,
// value m the sum of in[r * in_sr + m * in_sm + s * slot_stride] over s < nslot (added in
// order of s), then the DFT along m and scale = 1 / sqrt(s_total |D[0]|) (0 when D[0] = 0):
// out[r * out_sr + c * out_sc].  The nt threads of the workgroup; lbuf: [len] data and
// [len / 2] twiddles in LDS.
__device__ __forceinline__ void display_row_partials(const float2* __restrict__ in, float2* __restrict__ out, int len,
                                                     int log2len, const float2* __restrict__ e,
                                                     const float2* __restrict__ d0, float s_total, int in_sr,
                                                     int in_sm, int out_sr, int out_sc, int nslot, int slot_stride,
                                                     int r, float2* lbuf, int tid, int nt) {
  const float2* src = in + (size_t)r * in_sr;
  float2* dst = out + (size_t)r * out_sr;
  const float2 dd = d0[0];
  const float mag = sqrtf(dd.x * dd.x + dd.y * dd.y);
  const float scale = mag > 0.f ? 1.0f / sqrtf(s_total * mag) : 0.f;
  float2* ltw = lbuf + len;
  for (int base = 0; base < len; base += 2 * nt) {  // two values of m per thread: all loads first, then the sums
    float2 v[2][kMaxSlots];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int m = base + u * nt + tid;
#pragma unroll
      for (int q = 0; q < kMaxSlots; ++q)
        if (m < len && q < nslot) v[u][q] = gload(src + (size_t)m * in_sm + (size_t)q * slot_stride);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int m = base + u * nt + tid;
      if (m >= len) continue;
      float2 a = v[u][0];
#pragma unroll
      for (int q = 1; q < kMaxSlots; ++q)
        if (q < nslot) {
          a.x += v[u][q].x;
          a.y += v[u][q].y;
        }
      lbuf[log2len ? (int)(__brev((unsigned)m) >> (32 - log2len)) : 0] = a;
    }
  }
  stage_copy<4>(ltw, e, len / 2, tid, nt);
  __syncthreads();
  lds_fft(lbuf, ltw, len, log2len, tid, nt);
  for (int c = tid; c < len; c += nt) {
    const float2 v = lbuf[c];
    dst[(size_t)c * out_sc] = make_float2(v.x * scale, v.y * scale);
  }
}

// Rows come in blocks of block_rows (several grids transformed in one launch, e.g. one per
// field-of-view patch): row r is row r % block_rows of block r / block_rows, whose input,
// output and D[0] are in_block, out_block and d0_block values further on.
template <bool SLOTS>
__global__ __launch_bounds__(256) void k_dft_rows(const float2* __restrict__ in, float2* __restrict__ out, int len,
                                                  int log2len, const float2* __restrict__ e,
                                                  const float2* __restrict__ d0, float s_total, int final_scale,
                                                  int in_sr, int in_sm, int out_sr, int out_sc, int xcd_map,
                                                  int nslot, int slot_stride, int block_rows, int64_t in_block,
                                                  int64_t out_block, int64_t d0_block) {
  extern __shared__ float2 lbuf[];  // [len] data, then [len / 2] twiddles (power-of-two lengths)
  const int rg = xcd_map ? xcd_row(blockIdx.x, gridDim.x) : (int)blockIdx.x, tid = threadIdx.x;
  if (SLOTS) {  // final_scale is set on this (the column) pass
    display_row_partials(in, out, len, log2len, e, d0, s_total, in_sr, in_sm, out_sr, out_sc, nslot, slot_stride, rg,
                         lbuf, tid, 256);
    return;
  }
  const int blk = rg / block_rows, r = rg - blk * block_rows;
  in += blk * in_block;
  out += blk * out_block;
  d0 += blk * d0_block;
  const float2* src = in + (size_t)r * in_sr;
  float2* dst = out + (size_t)r * out_sr;
  float scale = 1.0f;
  if (final_scale) {
    const float2 dd = d0[0];
    const float mag = sqrtf(dd.x * dd.x + dd.y * dd.y);
    scale = mag > 0.f ? 1.0f / sqrtf(s_total * mag) : 0.f;
  }
  if (log2len >= 0) {
    float2* ltw = lbuf + len;
    for (int base = 0; base < len; base += 8 * 256) {  // loads first, then the bit-reversed stores
      float2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int m = base + u * 256 + tid;
        if (m < len) v[u] = gload(src + (size_t)m * in_sm);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int m = base + u * 256 + tid;
        if (m < len) lbuf[log2len ? (int)(__brev((unsigned)m) >> (32 - log2len)) : 0] = v[u];
      }
    }
    stage_copy<4>(ltw, e, len / 2, tid, 256);
    __syncthreads();
    lds_fft(lbuf, ltw, len, log2len, tid, 256);
    for (int c = tid; c < len; c += 256) {
      const float2 v = lbuf[c];
      dst[(size_t)c * out_sc] = make_float2(v.x * scale, v.y * scale);
    }
  } else {
    for (int m = tid; m < len; m += 256) lbuf[m] = src[(size_t)m * in_sm];
    __syncthreads();
    for (int c = tid; c < len; c += 256) {
      float re = 0.f, im = 0.f;
      int idx = 0;
      for (int m = 0; m < len; ++m) {
        const float2 x = lbuf[m], tw = e[idx];
        re += x.x * tw.x - x.y * tw.y;
        im += x.x * tw.y + x.y * tw.x;
        idx += c;
        idx -= (idx >= len) ? len : 0;
      }
      dst[(size_t)c * out_sc] = make_float2(re * scale, im * scale);
    }
  }
}

// The column pass of a display from partial rows (display_row_partials), as launch arguments.
struct DispArgs {
  const float2* din;
  float2* dout;
  int len, log2len;
  const float2* e;
  const float2* d0;
  float s_total;
  int in_sr, in_sm, out_sr, out_sc, nslot, slot_stride;
  int rows;  // output rows (the fused update launches)
};

// Rows of the previous image's column pass in the fused update launches, two per 512-thread
// workgroup: each half takes one output row with its own LDS ([len] data, [len / 2] twiddles),
// so the display holds half as many workgroup slots as with a row per workgroup, for the same
// per-row time (a row's len / 2 butterflies per stage need no more than 256 threads).  An odd
// last row is taken by both halves, which write the same values.
static_assert(kFusedThreads == 512, "two 256-thread halves per display workgroup");
__device__ __forceinline__ void display_row_pair(const DispArgs& d, int pair, float4* fsm, int tid) {
  const int half = tid >> 8;
  const int r = min(2 * pair + half, d.rows - 1);
  float2* lbuf = reinterpret_cast<float2*>(fsm) + half * (d.len + d.len / 2);
  display_row_partials(d.din, d.dout, d.len, d.log2len, d.e, d.d0, d.s_total, d.in_sr, d.in_sm, d.out_sr, d.out_sc,
                       d.nslot, d.slot_stride, r, lbuf, tid & 255, 256);
}

// One launch for independent jobs: workgroups b < n project frame b of a batch, workgroup n
// copies the upload block (when there is one), and the rest each write one output row of
// the previous step's displayed image from its partial rows (display_row_partials).  Saves
// a kernel boundary per step when the display of a step is left to the next push.
template <typename T, int PREC>
__global__ __launch_bounds__(1024) void k_project_display(ProjArgs a, DispArgs d) {
  extern __shared__ float4 msm[];
  const int b = (int)blockIdx.x;
  if (b < a.n) {
    project_any<T, PREC>(a, reinterpret_cast<float*>(msm), b);
    return;
  }
  const int up = a.up_words > 0 ? 1 : 0;
  if (up && b == a.n) {
    upload_block(a.up_src, a.up_dst, a.up_words, (int)threadIdx.x, (int)blockDim.x);
    return;
  }
  display_row_partials(d.din, d.dout, d.len, d.log2len, d.e, d.d0, d.s_total, d.in_sr, d.in_sm, d.out_sr, d.out_sc,
                       d.nslot, d.slot_stride, b - a.n - up, reinterpret_cast<float2*>(msm), (int)threadIdx.x,
                       (int)blockDim.x);
}

// ---------------------------------------------------------------------------
// Row-factored accumulation.  The unitary scan DFT matrix is F_y (x) F_x
// (Section 6.1), so for the frames of a batch that share scan row y_r
//   T_r[vx][k] = sum_{b in row r} Tx[(vx x_b) mod Sx] h_b[k]        (k_row_dft)
//   A[v][k]   += sum_r Ty[(vy y_r) mod Sy] T_r[vx(v)][k]            (k_row_update)
// which is the direct sum over frames, regrouped.  k_row_update streams the
// accumulator once per batch and is bound by HBM bandwidth.
// rows[r] = (y_r, first index into `order`, number of frames, 0); order lists the
// batch's frame indices grouped by row.
// ---------------------------------------------------------------------------
// T_r = Fx_r h_r as a real GEMM with rows (vx, re/im) interleaved, on
// v_mfma_f32_16x16x4_f32.  A workgroup of 4 waves owns one 16 x 16 tile (8 values of
// vx x 16 columns) of row r.  Per chunk of up to 256 frames the Tx table, the frames'
// indices and x positions and the chunk's h columns are staged in LDS; wave w takes a
// quarter of the frames, and the four partial tiles are summed at the end.
constexpr int kRowChunk = 256;

__device__ __forceinline__ void row_dft_body(const float* __restrict__ h, int kpad, const int* __restrict__ xs,
                                             const int* __restrict__ order, const int4* __restrict__ rows,
                                             const float2* __restrict__ tx, int sx, float2* __restrict__ t, int bx,
                                             int by, int bz, float2* rsmem) {
  float2* ltx = rsmem;                                   // [sx]
  int* lx = reinterpret_cast<int*>(ltx + sx);            // [kRowChunk]
  int* lb = lx + kRowChunk;                              // [kRowChunk]
  float* lh = reinterpret_cast<float*>(lb + kRowChunk);  // [kRowChunk][16]; reused for the final sum
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r16 = lane & 15, q = lane >> 4;
  const int r = bz;
  const int4 row = rows[r];
  const int vx = bx * 8 + (r16 >> 1);                    // A-operand row r16 = 2 * (vx - vx0) + (re/im)
  const bool im = (r16 & 1) != 0;
  const int c0 = by * 16;
  const bool p2 = (sx & (sx - 1)) == 0;
  const float inv = 1.0f / (float)sx;
  stage_copy<4>(ltx, tx, sx, tid, 256);
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int i0 = 0; i0 < row.z; i0 += kRowChunk) {
    const int cnt = min(kRowChunk, row.z - i0);
    __syncthreads();
    if (tid < cnt) {  // the frame's index and scan x, both in row order: one round trip
      lb[tid] = order[row.y + i0 + tid];
      lx[tid] = xs[row.y + i0 + tid];
    }
    __syncthreads();
    // the chunk's h columns: all of a thread's loads first (frame index clamped into the
    // chunk, no branch around a load, so they are all in flight at once; past the chunk's
    // end they re-read its last frame), then the stores
    constexpr int kPer = kRowChunk * 16 / 256;
    float hv[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int i = tid + 256 * j;
      hv[j] = gload(h + (size_t)lb[min(i >> 4, cnt - 1)] * kpad + c0 + (i & 15));
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int i = tid + 256 * j;
      lh[i] = (i >> 4) < cnt ? hv[j] : 0.f;
    }
    __syncthreads();
    // wave w takes frames [w * per, (w + 1) * per), 4 per MFMA (k-slot q <-> frame f0 + q)
    const int per = ((cnt + 15) / 16) * 4;
    const int fbeg = wave * per, fend = min(cnt, fbeg + per);
    for (int f0 = fbeg; f0 < fend; f0 += 4) {
      const int f = f0 + q;
      float a = 0.f, bv = 0.f;
      if (f < fend) {
        if (vx < sx) {
          const int p = vx * lx[f];
          const float2 w = ltx[p2 ? (p & (sx - 1)) : mod_small(p, sx, inv)];
          a = im ? w.y : w.x;
        }
        bv = lh[f * 16 + r16];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc, 0, 0, 0);
    }
  }
  __syncthreads();
  if (wave > 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) lh[((wave - 1) * 4 + j) * 64 + lane] = acc[j];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      for (int w = 0; w < 3; ++w) acc[j] += lh[(w * 4 + j) * 64 + lane];
    // lane (q, r16) holds rows 4q .. 4q + 3 of column r16: vx = vx0 + 2q (+1), (re, im) pairs
#pragma unroll
    for (int j = 0; j < 4; j += 2) {
      const int v = bx * 8 + 2 * q + (j >> 1);
      if (v < sx) t[((size_t)r * sx + v) * kpad + c0 + r16] = make_float2(acc[j], acc[j + 1]);
    }
  }
}

__global__ __launch_bounds__(256) void k_row_dft(const float* __restrict__ h, int kpad, const int* __restrict__ xs,
                                                 const int* __restrict__ order, const int4* __restrict__ rows,
                                                 const float2* __restrict__ tx, int sx, float2* __restrict__ t) {
  extern __shared__ float2 rsmem[];
  row_dft_body(h, kpad, xs, order, rows, tx, sx, t, (int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, rsmem);
}

// One group of G = kpad / 4 consecutive lanes per kept frequency; each lane owns 4
// consecutive complex entries of A.  With FUSE the Wiener reduction of the new A (as
// k_wiener) is done in the same pass.
template <bool FUSE>
__device__ __forceinline__ void row_update_body(float2* __restrict__ acc, int kpad, const int2* __restrict__ freqs,
                                                int64_t n_freq, const float2* __restrict__ t, int sx,
                                                const int4* __restrict__ rows, int nrows,
                                                const float2* __restrict__ ty, int sy,
                                                const float2* __restrict__ w, float2* __restrict__ d,
                                                float2* __restrict__ z, int64_t block) {
  const int g = kpad >> 2;
  const int64_t gid = block * 256 + threadIdx.x;
  const int64_t j = gid / g;
  const int c = 4 * (int)(gid - j * g);
  const int2 v = freqs[j];
  const bool p2 = (sy & (sy - 1)) == 0;
  const float inv = 1.0f / (float)sy;
  float4* a4 = reinterpret_cast<float4*>(acc + j * kpad + c);
  float4 a0 = a4[0], a1 = a4[1];
  for (int r = 0; r < nrows; ++r) {
    const int p = v.x * rows[r].x;
    const float2 ph = ty[p2 ? (p & (sy - 1)) : mod_small(p, sy, inv)];
    const float4* t4 = reinterpret_cast<const float4*>(t + ((size_t)r * sx + v.y) * kpad + c);
    const float4 t0 = t4[0], t1 = t4[1];
    a0.x += ph.x * t0.x - ph.y * t0.y;
    a0.y += ph.x * t0.y + ph.y * t0.x;
    a0.z += ph.x * t0.z - ph.y * t0.w;
    a0.w += ph.x * t0.w + ph.y * t0.z;
    a1.x += ph.x * t1.x - ph.y * t1.y;
    a1.y += ph.x * t1.y + ph.y * t1.x;
    a1.z += ph.x * t1.z - ph.y * t1.w;
    a1.w += ph.x * t1.w + ph.y * t1.z;
  }
  a4[0] = a0;
  a4[1] = a1;
  if (FUSE) {
    const float4* w4 = reinterpret_cast<const float4*>(w + j * kpad + c);
    const float4 w0 = w4[0], w1 = w4[1];
    float re = (a0.x * w0.x - a0.y * w0.y) + (a0.z * w0.z - a0.w * w0.w);
    float im = (a0.x * w0.y + a0.y * w0.x) + (a0.z * w0.w + a0.w * w0.z);
    re += (a1.x * w1.x - a1.y * w1.y) + (a1.z * w1.z - a1.w * w1.w);
    im += (a1.x * w1.y + a1.y * w1.x) + (a1.z * w1.w + a1.w * w1.z);
    for (int off = g >> 1; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 64);
      im += __shfl_xor(im, off, 64);
    }
    if (c == 0 && j < n_freq) {
      d[j] = make_float2(re, im);
      z[(size_t)v.y * sy + v.x] = make_float2(re, -im);
    }
  }
}

template <bool FUSE>
__global__ __launch_bounds__(256) void k_row_update(float2* __restrict__ acc, int kpad, const int2* __restrict__ freqs,
                                                    int64_t n_freq, const float2* __restrict__ t, int sx,
                                                    const int4* __restrict__ rows, int nrows,
                                                    const float2* __restrict__ ty, int sy,
                                                    const float2* __restrict__ w, float2* __restrict__ d,
                                                    float2* __restrict__ z) {
  row_update_body<FUSE>(acc, kpad, freqs, n_freq, t, sx, rows, nrows, ty, sy, w, d, z, (int64_t)blockIdx.x);
}

// Spectrum-order row passes of several plans in one launch each (serving rounds): the
// passes' descriptors in device memory, their first workgroups in first[0 .. npass] (a
// running sum of each pass's grid); workgroup b belongs to the pass i with first[i] <= b <
// first[i + 1].
__device__ inline int group_pass(const int* __restrict__ first, int npass, int b) {
  int lo = 0, hi = npass - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_row_dft_group(const wdd::SpecPass* __restrict__ passes,
                                                       const int* __restrict__ first, int npass) {
  extern __shared__ float2 rsmem[];
  const int b = (int)blockIdx.x;
  const int i = group_pass(first, npass, b);
  const wdd::SpecPass& p = passes[i];
  const int local = b - first[i];
  const int nbx = (p.sx + 7) / 8, nby = p.kpad / 16;
  row_dft_body(p.h, p.kpad, p.xs, p.order, p.rows, p.tx, p.sx, p.t, local % nbx, (local / nbx) % nby,
               local / (nbx * nby), rsmem);
}

__global__ __launch_bounds__(256) void k_row_update_group(const wdd::SpecPass* __restrict__ passes,
                                                          const int* __restrict__ first, int npass) {
  const int b = (int)blockIdx.x;
  const int i = group_pass(first, npass, b);
  const wdd::SpecPass& p = passes[i];
  const int64_t local = b - first[i];
  if (p.fuse)
    row_update_body<true>(p.acc, p.kpad, p.freqs, p.n_freq, p.t, p.sx, p.rows, p.nrows, p.ty, p.sy, p.w, p.d, p.z,
                          local);
  else
    row_update_body<false>(p.acc, p.kpad, p.freqs, p.n_freq, p.t, p.sx, p.rows, p.nrows, p.ty, p.sy, p.w, p.d, p.z,
                           local);
}

// ---------------------------------------------------------------------------
// Row-factored update with the x-DFT fused in.  Workgroup b owns the chunk
// chunks[b] = (vx, i0, cnt): the kept frequencies jlist[i0 .. i0 + cnt), which all have
// x-frequency vx.  It first forms, for every row r of the pass,
//   T_r[k] = sum_{frames f of row r} Tx[(vx x_f) mod Sx] h_f[k]
// in LDS (the x-DFT restricted to its own vx), then streams its frequencies once:
//   D[j] += sum_r Ty[(vy y_r) mod Sy] sum_k W[j][k] T_r[k];  z = conj(D)
// (object order: the Wiener filter applied to every frame's contribution).
// Phase 1 splits the frames over G = 2048 / kpad groups of kpad / 4 threads (4
// consecutive k each, float4 loads of h) and sums the groups in LDS; phase 2 gives each
// frequency kpad / 4 consecutive lanes (4 entries each), G frequencies at a time.
// With `up` set the workgroup also takes its share of the display's first pass (the DFT
// along v_y of z = conj(D), power-of-two Sy <= 1024): the zero-padded row holding only
// its own frequencies, transformed in LDS, goes to up[y][vx][chunks[b].w] ([Sy][Sx][nslot],
// so that the display's column pass reads each output row's inputs contiguously), and that
// pass sums the nslot partials of each vx.
// ---------------------------------------------------------------------------
constexpr int kFusedFrames = 512;  // frames staged in LDS per round of phase 1
static_assert(kFusedFrames <= kFusedThreads, "phase 1 stages one frame per thread");
static_assert(kDisplayRowMax / 2 <= kFusedThreads, "one display twiddle per thread");
static_assert(kDisplayRowMax <= (1 << 24), "twiddle arguments stay exact in float");
static_assert(kDisplayRowMax * 3 / 2 <= kFusedThreads * 4, "a display row and its twiddles fit the group sums");

__device__ inline void cmac4(float4& a0, float4& a1, float2 c, const float4 h) {
  a0.x += c.x * h.x; a0.y += c.y * h.x; a0.z += c.x * h.y; a0.w += c.y * h.y;
  a1.x += c.x * h.z; a1.y += c.y * h.z; a1.z += c.x * h.w; a1.w += c.y * h.w;
}

// s = sum_r ph_r T_r over this lane's 4 entries (T_r from LDS); ph0, the twiddle of row 0,
// is given (formed once per frequency), the others are formed here
template <typename Rows>
__device__ inline void phase_sum(float4& s0, float4& s1, const float4* __restrict__ lt, int q, int kq, int nrows,
                                 const Rows& rs, int vy, int sy, bool py2, float invy, float2 ph0) {
  s0 = make_float4(0.f, 0.f, 0.f, 0.f);
  s1 = s0;
  for (int r = 0; r < nrows; ++r) {
    const int p = vy * rs.r[r].x;
    const float2 ph = r == 0 ? ph0 : twiddle(py2 ? (p & (sy - 1)) : mod_small(p, sy, invy), sy, 1.0f);
    const float4 t0 = lt[(size_t)(r * q + kq) * 2], t1 = lt[(size_t)(r * q + kq) * 2 + 1];
    s0.x += ph.x * t0.x - ph.y * t0.y; s0.y += ph.x * t0.y + ph.y * t0.x;
    s0.z += ph.x * t0.z - ph.y * t0.w; s0.w += ph.x * t0.w + ph.y * t0.z;
    s1.x += ph.x * t1.x - ph.y * t1.y; s1.y += ph.x * t1.y + ph.y * t1.x;
    s1.z += ph.x * t1.z - ph.y * t1.w; s1.w += ph.x * t1.w + ph.y * t1.z;
  }
}

__device__ inline float2 cdot4(const float4 w0, const float4 w1, const float4 v0, const float4 v1) {
  float re = (w0.x * v0.x - w0.y * v0.y) + (w0.z * v0.z - w0.w * v0.w);
  float im = (w0.x * v0.y + w0.y * v0.x) + (w0.z * v0.w + w0.w * v0.z);
  re += (w1.x * v1.x - w1.y * v1.y) + (w1.z * v1.z - w1.w * v1.w);
  im += (w1.x * v1.y + w1.y * v1.x) + (w1.z * v1.w + w1.w * v1.z);
  return make_float2(re, im);
}

// (hi, lo) += c with the rounding error kept: hi stays the FP32 value nearest the running sum
// hi + lo, lo the remainder (Knuth's two-sum, then a fast renormalisation; additions only,
// so no contraction into fused multiply-adds can change them).  Used for the object
// spectrum D, which sums one contribution per push: without it the rounding of each of the
// thousands of additions adds up to several 1e-6 of the signal beside the zero frequency.
__device__ inline void two_sum_add(float& hi, float& lo, float c) {
  const float s = hi + c;
  const float bb = s - hi;
  const float err = (hi - (s - bb)) + (c - bb);
  const float t = lo + err;
  const float h2 = s + t;
  lo = t - (h2 - s);
  hi = h2;
}
__device__ inline void two_sum_add2(float2& hi, float2& lo, float2 c) {
  two_sum_add(hi.x, lo.x, c.x);
  two_sum_add(hi.y, lo.y, c.y);
}

__device__ inline void add4(float4& a, const float4 b) {
  a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
}

// Modes of row_fused_obj_body: both phases (kFusedBoth); phase 2 from T_r given in global
// memory (kFusedGivenT: t_io holds this v_x's [nrows][q][2] float4, written by a kFusedOnlyT
// workgroup of an earlier launch from the same projections, so the results are the same bit
// for bit); phase 1 alone, T_r written to t_io (kFusedOnlyT: ch.x the v_x, the rest unused).
constexpr int kFusedBoth = 0, kFusedGivenT = 1, kFusedOnlyT = 2;

template <int MODE = kFusedBoth, typename Rows>
__device__ __forceinline__ void row_fused_obj_body(const float* __restrict__ h, int kpad, const int* __restrict__ order,
                                                   const int* __restrict__ xs, const Rows& rs, int nrows,
                                                   float tscale, int sx, int sy, const int4 ch,
                                                   const int2* __restrict__ jv, const float2* __restrict__ w,
                                                   float2* __restrict__ d, float2* __restrict__ dlo,
                                                   float2* __restrict__ z, int max_chunk, float2* __restrict__ up,
                                                   int nslot, int log2sy, int in_order, float2* __restrict__ d0out,
                                                   float4* fsm, float4* __restrict__ t_io = nullptr) {
  const int q = kpad >> 2, G = kFusedThreads / q;
  const int tid = threadIdx.x, kq = tid % q, grp = tid / q;
  float4* lt = fsm;                                           // [nrows][q][2]: T_r, 4 complex per float4 pair
  float4* lsum = lt + (size_t)nrows * q * 2;                  // [kFusedThreads][2]: group partial sums
  float2* lw = reinterpret_cast<float2*>(lsum + 2 * kFusedThreads);  // [kFusedFrames] twiddles of staged frames
  int* lb = reinterpret_cast<int*>(lw + kFusedFrames);        // [kFusedFrames] their batch indices
  int* lj = lb + kFusedFrames;                                // [max_chunk] the chunk's frequencies
  int* lvy = lj + max_chunk;                                  // [max_chunk] their y-frequencies
  float2* lph = reinterpret_cast<float2*>(lvy + max_chunk);   // [max_chunk] their row-0 twiddles
  // Every load of the prologue is unconditional, its index clamped into range (a row holds at
  // least one frame, a chunk at least one frequency): a load under a branch makes the compiler
  // wait for all loads in flight wherever a later one is used, which would serialise the
  // round trips this prologue overlaps.
  // The first staging block's frame indices and x positions, and (frames already in row
  // order, order[i] = i) the projections of this lane group's first 8 frames, depend on the
  // kernel arguments only: their loads go out before anything waits for the chunk descriptor.
  // (phase 1 only) the first staging block's frame indices and x positions, and the
  // projections of this lane group's first 8 frames
  const float4* h4 = reinterpret_cast<const float4*>(h);
  int n_first = 0, first_b = 0, first_x = 0;
  bool pre = false;
  float4 hv0[8];
  if constexpr (MODE != kFusedGivenT) {
    n_first = min(kFusedFrames, rs.r[0].z);
    const int fi = rs.r[0].y + min(tid, n_first - 1);
    first_b = gload(order + fi);
    first_x = gload(xs + fi);
    pre = in_order && grp + 7 * G < n_first;
    // (not in order: frame 0, always a valid row of h, stands in; these loads go unused)
    const int f0 = pre ? rs.r[0].y + grp : 0, fs = pre ? G : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) hv0[u] = gload(h4 + (size_t)(f0 + u * fs) * q + kq);
  }
  const int vx = ch.x, i0 = ch.y, cnt = ch.z;
  const bool px2 = (sx & (sx - 1)) == 0, py2 = (sy & (sy - 1)) == 0;
  const float invx = 1.0f / (float)sx, invy = 1.0f / (float)sy;

  // this thread's (j, v_y) of the chunk (cnt <= kFusedThreads): loaded now, stored to LDS
  // after phase 1, so that its round trip hides under phase 1's
  const int2 myjv = MODE == kFusedOnlyT ? make_int2(0, 0) : gload(jv + i0 + min(tid, cnt - 1));
  if constexpr (MODE == kFusedGivenT) {
    // T_r of this v_x, as a kFusedOnlyT workgroup left it
    for (int e = tid; e < nrows * q * 2; e += kFusedThreads) lt[e] = t_io[e];
  } else {
    // phase 1: T_r for this vx; the first block of frames is staged here, the others in the loop
    float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0;
    if (tid < n_first) {
      const int p = vx * first_x;
      lw[tid] = twiddle(px2 ? (p & (sx - 1)) : mod_small(p, sx, invx), sx, tscale);
      lb[tid] = first_b;
    }
    __syncthreads();
    if (pre) {
#pragma unroll
      for (int u = 0; u < 8; ++u) cmac4(a0, a1, lw[grp + u * G], hv0[u]);
    }
    for (int r = 0; r < nrows; ++r) {
      const int4 row = rs.r[r];
      for (int f0 = 0; f0 < row.z; f0 += kFusedFrames) {
        const int n = min(kFusedFrames, row.z - f0);
        const bool first = r == 0 && f0 == 0;
        if (!first) {
          __syncthreads();
          if (tid < n) {
            const int at = row.y + f0 + tid;
            const int b = order[at], p = vx * xs[at];
            lw[tid] = twiddle(px2 ? (p & (sx - 1)) : mod_small(p, sx, invx), sx, tscale);
            lb[tid] = b;
          }
          __syncthreads();
        }
        int i = grp + (first && pre ? 8 * G : 0);
        for (; i + 7 * G < n; i += 8 * G) {
          float4 hv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) hv[u] = h4[(size_t)lb[i + u * G] * q + kq];
#pragma unroll
          for (int u = 0; u < 8; ++u) cmac4(a0, a1, lw[i + u * G], hv[u]);
        }
        for (; i < n; i += G) cmac4(a0, a1, lw[i], h4[(size_t)lb[i] * q + kq]);
      }
      lsum[2 * tid] = a0;
      lsum[2 * tid + 1] = a1;
      __syncthreads();
      if (grp == 0) {
        for (int g = 1; g < G; ++g) {
          add4(a0, lsum[2 * (g * q + kq)]);
          add4(a1, lsum[2 * (g * q + kq) + 1]);
        }
        lt[(size_t)(r * q + kq) * 2] = a0;
        lt[(size_t)(r * q + kq) * 2 + 1] = a1;
      }
      __syncthreads();
      a0 = make_float4(0.f, 0.f, 0.f, 0.f);
      a1 = a0;
    }
    if constexpr (MODE == kFusedOnlyT) {
      for (int e = tid; e < nrows * q * 2; e += kFusedThreads) t_io[e] = lt[e];
      return;
    }
  }

  if (tid < cnt) {
    lj[tid] = myjv.x;
    lvy[tid] = myjv.y;
    const int p = myjv.y * rs.r[0].x;
    lph[tid] = twiddle(py2 ? (p & (sy - 1)) : mod_small(p, sy, invy), sy, 1.0f);
  }
  // display row (with up): the group sums are free now, so the row is cleared and its
  // twiddles formed here; phase 2 drops each conj D into its bit-reversed slot
  float2* lrow = reinterpret_cast<float2*>(lsum);  // [sy], then the twiddles [sy / 2]
  float2* ltw = lrow + sy;
  if (up) {
    for (int m = tid; m < sy; m += kFusedThreads) lrow[m] = make_float2(0.f, 0.f);
    if (tid < sy / 2) ltw[tid] = twiddle(tid, sy, 1.0f);
  }
  __syncthreads();

  // phase 2: stream the chunk's frequencies, two per lane group per round with all their
  // loads issued first
  for (int i = grp; i < cnt; i += 2 * G) {
    const bool two = i + G < cnt;
    const int ja = lj[i], jb = two ? lj[i + G] : ja;
    const float4* wa = reinterpret_cast<const float4*>(w + (size_t)ja * kpad + 4 * kq);
    const float4* wb = reinterpret_cast<const float4*>(w + (size_t)jb * kpad + 4 * kq);
    const float4 wa0 = gload(wa), wa1 = gload(wa + 1), wb0 = gload(wb), wb1 = gload(wb + 1);
    // all lanes load D: no branch around a load
    const float2 da = gload(d + ja), db = gload(d + jb), la = gload(dlo + ja), lb = gload(dlo + jb);
    const int vya = lvy[i], vyb = two ? lvy[i + G] : vya;
    float4 sa0, sa1, sb0, sb1;
    phase_sum(sa0, sa1, lt, q, kq, nrows, rs, vya, sy, py2, invy, lph[i]);
    phase_sum(sb0, sb1, lt, q, kq, nrows, rs, vyb, sy, py2, invy, lph[two ? i + G : i]);
    float2 oa = cdot4(wa0, wa1, sa0, sa1), ob = cdot4(wb0, wb1, sb0, sb1);
    for (int off = q >> 1; off > 0; off >>= 1) {
      oa.x += __shfl_xor(oa.x, off, 64);
      oa.y += __shfl_xor(oa.y, off, 64);
      ob.x += __shfl_xor(ob.x, off, 64);
      ob.y += __shfl_xor(ob.y, off, 64);
    }
    if (kq == 0) {
      float2 na = da, nla = la;
      two_sum_add2(na, nla, oa);
      d[ja] = na;
      dlo[ja] = nla;
      if (d0out && ja == 0) d0out[0] = na;  // D[0] as of this pass, for a display read later
      z[(size_t)vx * sy + vya] = make_float2(na.x, -na.y);
      if (up) lrow[log2sy ? (int)(__brev((unsigned)vya) >> (32 - log2sy)) : 0] = make_float2(na.x, -na.y);
      if (two) {
        float2 nb = db, nlb = lb;
        two_sum_add2(nb, nlb, ob);
        d[jb] = nb;
        dlo[jb] = nlb;
        if (d0out && jb == 0) d0out[0] = nb;
        z[(size_t)vx * sy + vyb] = make_float2(nb.x, -nb.y);
        if (up) lrow[log2sy ? (int)(__brev((unsigned)vyb) >> (32 - log2sy)) : 0] = make_float2(nb.x, -nb.y);
      }
    }
  }

  if (up) {  // the chunk's partial row of the display's first pass
    __syncthreads();
    lds_fft(lrow, ltw, sy, log2sy, tid, kFusedThreads);
    const size_t ustride = (size_t)sx * nslot;
    float2* dst = up + (size_t)vx * nslot + ch.w;
    for (int m = tid; m < sy; m += kFusedThreads) dst[m * ustride] = lrow[m];
  }
}

__global__ __launch_bounds__(kFusedThreads) void k_row_fused_obj(const float* __restrict__ h, int kpad,
                                                                 const int* __restrict__ order,
                                                                 const int* __restrict__ xs, RowSet rs, int nrows,
                                                                 float tscale, int sx, int sy,
                                                                 const int4* __restrict__ chunks,
                                                                 const int2* __restrict__ jv,
                                                                 const float2* __restrict__ w,
                                                                 float2* __restrict__ d, float2* __restrict__ dlo,
                                                                 float2* __restrict__ z,
                                                                 int max_chunk, float2* __restrict__ up, int nslot,
                                                                 int log2sy, int in_order, float2* __restrict__ d0out,
                                                                 int nchunks, DispArgs disp) {
  extern __shared__ float4 fsm[];
  const int b = (int)blockIdx.x;
  if (b >= nchunks) {  // two rows of the previous step's image, left to this launch (see launch_row_fused_obj)
    display_row_pair(disp, b - nchunks, fsm, (int)threadIdx.x);
    return;
  }
  // consecutive chunks (the same or neighbouring v_x, whose z entries and display partials
  // share cache lines) run on one XCD, so partly written lines meet in one L2
  const int4 ch = chunks[xcd_row(b, nchunks)];
  row_fused_obj_body(h, kpad, order, xs, rs, nrows, tscale, sx, sy, ch, jv, w, d, dlo, z, max_chunk, up, nslot, log2sy,
                     in_order, d0out, fsm);
}

// The object-order update of one batch with the projection of the next batch in the same
// launch.  The two are independent (the update reads its own batch's projections and upload
// block, the projection writes the next batch's into other buffers), so the projection's
// frame stream from HBM overlaps the update's phases that leave HBM idle (the first, which
// reads the projections from L2, and the partial display rows), and the launch boundary
// between them goes away.  Grid: projections 0 .. pfront - 1, the update's nchunks chunks,
// the other projections (512 threads: up to two 16-row tiles per wave; projection pa.n, when
// there is an upload block, copies it), then the display rows of k_row_fused_obj.
// How many of k_row_fused_obj_next's projection workgroups come before the update's chunks in
// its grid (the others follow the chunks): a few at the front start their frame stream while
// the chunks' first phase reads from L2; all of them there (or all after the display rows)
// delay chunks or leave the tail to the projections.  Measured per pipelined step, 0 / 16 /
// 32 / 64 / 96 in front: 512^2 scan, 256^2 frames 36.2 / 35.8 / 35.7 / 35.7 / 37.0 us;
// 256^2 scan, 128^2 frames 13.7 / 13.7 / 13.5 / 14.6 / 14.6 us; 128^2 scan, 64^2 frames
// 12.3 / 12.2 / 12.2 / 11.9 / 12.1 us (all in front: 37.5, 15.2, 12.2 us; all after the
// display rows: 44.2, 14.6, 12.3 us).
constexpr int kNextProjFront = 32;

// The projection of k_row_fused_obj_next (uint16 frames of nx = 32 NCH columns, 1 <= NCH <= 8,
// checked by its launcher): FP32 with up to two 16-row tiles per wave (at most 256 rows), or a
// reduced precision with one tile per wave (at most 128 rows).
template <int PREC>
__device__ __forceinline__ void project_next(const ProjArgs& a, float* smem, int b) {
  const uint16_t* fr = static_cast<const uint16_t*>(a.frames);
  if constexpr (PREC == WDD_FP32) {
#define WDD_NEXT(N) \
  project_frame_tiles<uint16_t, N, true>(fr, a.ny, a.nx, a.psi, a.kmap, a.kpad, a.h, a.fptr, smem, b); return
    switch (a.nx >> 5) {
      case 1: WDD_NEXT(1);
      case 2: WDD_NEXT(2);
      case 3: WDD_NEXT(3);
      case 4: WDD_NEXT(4);
      case 5: WDD_NEXT(5);
      case 6: WDD_NEXT(6);
      case 7: WDD_NEXT(7);
      default: WDD_NEXT(8);
    }
#undef WDD_NEXT
  } else {
    constexpr bool bf = PREC == WDD_BF16_HILO || PREC == WDD_BF16;
    constexpr bool hilo = PREC == WDD_BF16_HILO || PREC == WDD_FP16_HILO;
#define WDD_NEXT(N)                                                                                               \
  project_frame_lp_tile<bf, hilo, N>(fr, a.ny, a.nx, a.psi, a.psix_lp, a.psi_unscale, a.kmap, a.kpad, a.h, a.fptr, \
                                     smem, b);                                                                    \
  return
    switch (a.nx >> 5) {
      case 1: WDD_NEXT(1);
      case 2: WDD_NEXT(2);
      case 3: WDD_NEXT(3);
      case 4: WDD_NEXT(4);
      case 5: WDD_NEXT(5);
      case 6: WDD_NEXT(6);
      case 7: WDD_NEXT(7);
      default: WDD_NEXT(8);
    }
#undef WDD_NEXT
  }
}

template <int PREC>
__global__ __launch_bounds__(kFusedThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_row_fused_obj_next(
    const float* __restrict__ h, int kpad, const int* __restrict__ order, const int* __restrict__ xs, RowSet rs,
    int nrows, float tscale, int sx, int sy, const int4* __restrict__ chunks, const int2* __restrict__ jv,
    const float2* __restrict__ w, float2* __restrict__ d, float2* __restrict__ dlo, float2* __restrict__ z,
    int max_chunk, float2* __restrict__ up, int nslot, int log2sy, int in_order, float2* __restrict__ d0out,
    int nchunks, DispArgs disp, ProjArgs pa, int pfront) {
  extern __shared__ float4 fsm[];
  const int b = (int)blockIdx.x;
  const int nproj = pa.n + (pa.up_words > 0 ? 1 : 0);
  const int pi = b < pfront ? b : (b >= pfront + nchunks && b < nproj + nchunks) ? b - nchunks : -1;
  if (pi >= 0) {
    if (pi == pa.n)
      upload_block(pa.up_src, pa.up_dst, pa.up_words, (int)threadIdx.x, kFusedThreads);
    else
      project_next<PREC>(pa, reinterpret_cast<float*>(fsm), pi);
    return;
  }
  if (b >= nproj + nchunks) {
    display_row_pair(disp, b - nproj - nchunks, fsm, (int)threadIdx.x);
    return;
  }
  // (pfront is a multiple of 8: the chunks keep the XCDs of k_row_fused_obj's mapping)
  const int4 ch = chunks[xcd_row(b - pfront, nchunks)];
  row_fused_obj_body(h, kpad, order, xs, rs, nrows, tscale, sx, sy, ch, jv, w, d, dlo, z, max_chunk, up, nslot, log2sy,
                     in_order, d0out, fsm);
}

// Two-stage pipelined pushes: one launch holds the update of batch i - 2, whose x-DFT T_r
// (one row of kFusedOnlyT output per kept v_x) an earlier launch left in tin; the x-DFT of
// batch i - 1 into tout, one workgroup per kept v_x (xcols[0 .. ncols)), from the projections
// the launch before wrote; and the projection of batch i.  None reads what another writes.
// The chunks skip phase 1 (kFusedGivenT), so W streaming starts at once, and the x-DFT is
// formed once per v_x instead of once per chunk.  Grid: five segments (projections
// 0 .. pfront - 1, the x-DFT workgroups, the update's chunks, the other projections, the display
// rows) in the order the launcher picks.  Any part may be empty.  T per v_x:
// [kRowSetMax][kpad / 4][2] float4 at t + v_x * tstride.
struct NextArgs {
  const float* h;      // x-DFT part: the projections of batch i - 1 and their upload block
  const int* order;
  const int* xs;
  RowSet rows;
  int nrows, in_order, ncols;
  const int* xcols;
  float4* tout;
};
// Order of k_row_fused_obj_next2's grid segments, as octal digits, first segment lowest: 0 front
// projections, 1 x-DFT columns, 2 the update's chunks, 3 the other projections, 4 display rows.
// Measured per two-stage step with 32 projections in front, orders 02314 / 02341 / 02134 /
// 01234: 512^2 scan, 256^2 frames, K = 128 35.4 / 34.9 / 42.0 / 35.4 us; 256^2 scan, 128^2
// frames, K = 64 13.2 / 13.3 / 13.0 / 14.0 us; 128^2 scan, 64^2 frames, K = 256 11.1 / 11.4 /
// 11.2 / 11.6 us; order 02314 with no projection in front 35.7 / 13.1 / 10.8 us, with 64
// 35.3 / 13.1 / 11.2 us.  Frames of more than 128 rows (two tiles per wave: long projection
// workgroups) take 32 in front and the x-DFT columns last, smaller ones none in front and the
// x-DFT columns before the display rows.
constexpr int stage2_order(int s0, int s1, int s2, int s3, int s4) {
  return s0 | s1 << 3 | s2 << 6 | s3 << 9 | s4 << 12;
}
constexpr int kStage2LongProj = stage2_order(0, 2, 3, 4, 1), kStage2ShortProj = stage2_order(0, 2, 3, 1, 4);
constexpr int kStage2FrontLong = 32;

template <int PREC, bool LONG_PROJ>
__global__ __launch_bounds__(kFusedThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_row_fused_obj_next2(
    int kpad, RowSet rs, int nrows, float tscale, int sx, int sy, const int4* __restrict__ chunks,
    const int2* __restrict__ jv, const float2* __restrict__ w, float2* __restrict__ d, float2* __restrict__ dlo,
    float2* __restrict__ z, int max_chunk, float2* __restrict__ up, int nslot, int log2sy,
    float2* __restrict__ d0out, int nchunks, const float4* __restrict__ tin, int tstride, NextArgs xa,
    DispArgs disp, ProjArgs pa, int pfront) {
  extern __shared__ float4 fsm[];
  const int b = (int)blockIdx.x;
  const int nproj = pa.n > 0 ? pa.n + (pa.up_words > 0 ? 1 : 0) : 0;
  // the grid's segments, in the order for LONG_PROJ (a compile-time order: measured 0.2-0.5 us
  // per launch faster than the same order read from an argument): front projections, x-DFT
  // columns, chunks, the other projections, display rows
  constexpr int sorder = LONG_PROJ ? kStage2LongProj : kStage2ShortProj;
  const int len[5] = {pfront, xa.ncols, nchunks, nproj - pfront, (int)gridDim.x - xa.ncols - nchunks - nproj};
  int seg = 0, off = b;
  for (int k = 0; k < 5; ++k) {
    seg = (sorder >> (3 * k)) & 7;
    if (off < len[seg]) break;
    off -= len[seg];
  }
  if (seg == 0 || seg == 3) {  // a projection
    const int pi = seg == 0 ? off : pfront + off;
    if (pi == pa.n)
      upload_block(pa.up_src, pa.up_dst, pa.up_words, (int)threadIdx.x, kFusedThreads);
    else
      project_next<PREC>(pa, reinterpret_cast<float*>(fsm), pi);
    return;
  }
  if (seg == 4) {
    display_row_pair(disp, off, fsm, (int)threadIdx.x);
    return;
  }
  if (seg == 1) {  // the x-DFT of one kept v_x of batch i - 1
    const int vx = xa.xcols[off];
    row_fused_obj_body<kFusedOnlyT>(xa.h, kpad, xa.order, xa.xs, xa.rows, xa.nrows, tscale, sx, sy,
                                    make_int4(vx, 0, 1, 0), jv, w, d, dlo, z, max_chunk, nullptr, nslot, log2sy,
                                    xa.in_order, nullptr, fsm, xa.tout + (size_t)vx * tstride);
    return;
  }
  // (the chunks' first workgroup need not sit at a multiple of 8: their XCDs rotate, each XCD
  // still taking a contiguous range of neighbouring v_x)
  const int4 ch = chunks[xcd_row(off, nchunks)];
  row_fused_obj_body<kFusedGivenT>(nullptr, kpad, nullptr, nullptr, rs, nrows, tscale, sx, sy, ch, jv, w, d, dlo, z,
                                   max_chunk, up, nslot, log2sy, 1, d0out, fsm,
                                   const_cast<float4*>(tin) + (size_t)ch.x * tstride);
}

// Row passes of several object-order updates in one launch: workgroup b takes work item
// items[b] = (pass, v_x, first jv index, count | slot << 16) of the pass descriptors
// (each a row pass of one plan's frames: its own D, tables, rows and frame lists).
struct GlobalRows {
  const int4* r;
};
__global__ __launch_bounds__(kFusedThreads) void k_row_fused_obj_group(const wdd::ObjPass* __restrict__ passes,
                                                                       const int4* __restrict__ items) {
  extern __shared__ float4 fsm[];
  const int4 it = items[blockIdx.x];
  const wdd::ObjPass& p = passes[it.x];
  const int4 ch = make_int4(it.y, it.z, it.w & 0xffff, it.w >> 16);
  row_fused_obj_body(p.h, p.kpad, p.order, p.xs, GlobalRows{p.rows}, p.nrows, p.tscale, p.sx, p.sy, ch, p.jv, p.w,
                     p.d, p.dlo, p.z, p.max_chunk, p.up, p.nslot, p.log2sy, p.in_order, nullptr, fsm);
}


// ---------------------------------------------------------------------------
// Full Fourier basis (K = ny nx).  Projection: h_b[k_y nx + k_x] = sum_q I_b[q]
// exp(+2 pi i (q_y k_y / ny + q_x k_x / nx)) / (ny nx), a 2D FFT of the frame in LDS (radix-2
// decimation in time along x with the columns loaded in bit-reversed order, rows
// bit-reverse permuted, then along y).  fy, fx: exp(+2 pi i m / n) for m < n / 2.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_project_fourier(const T* __restrict__ frames, int ny, int nx, int lny,
                                                         int lnx, const float2* __restrict__ fy,
                                                         const float2* __restrict__ fx, float2* __restrict__ h,
                                                         int kpad, const uint32_t* __restrict__ up_src,
                                                         uint32_t* __restrict__ up_dst, int up_words,
                                                         const uint64_t* __restrict__ fptr) {
  extern __shared__ float2 fbuf[];  // [ny][nx], then fy [ny / 2], fx [nx / 2]
  float2* lfy = fbuf + ny * nx;
  float2* lfx = lfy + ny / 2;
  const int tid = threadIdx.x, cells = ny * nx;
  const T* f = fptr ? reinterpret_cast<const T*>(fptr[blockIdx.x]) : frames + (size_t)blockIdx.x * cells;
  for (int base = 0; base < cells; base += 16 * 256) {  // up to 16 loads in flight per thread
    T v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = base + u * 256 + tid;
      if (e < cells) v[u] = gload(f + e);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = base + u * 256 + tid;
      if (e < cells) {
        const int y = e >> lnx, x = e & (nx - 1);
        const int rx = (int)(__brev((unsigned)x) >> (32 - lnx));
        fbuf[y * nx + rx] = make_float2((float)v[u], 0.f);
      }
    }
  }
  if (blockIdx.x == 0) stage_copy<4>(up_dst, up_src, up_words, tid, 256);
  stage_copy<1>(lfy, fy, ny / 2, tid, 256);
  stage_copy<1>(lfx, fx, nx / 2, tid, 256);
  __syncthreads();
  for (int s = 1; s <= lnx; ++s) {
    const int half = 1 << (s - 1), stride = nx >> s;
    for (int k = tid; k < cells / 2; k += 256) {
      const int row = k >> (lnx - 1), bk = k & ((nx >> 1) - 1);
      const int i0 = row * nx + (bk >> (s - 1)) * (half << 1) + (bk & (half - 1));
      const float2 tw = lfx[(bk & (half - 1)) * stride];
      const float2 x0 = fbuf[i0], x1 = fbuf[i0 + half];
      const float2 tt = make_float2(tw.x * x1.x - tw.y * x1.y, tw.x * x1.y + tw.y * x1.x);
      fbuf[i0] = make_float2(x0.x + tt.x, x0.y + tt.y);
      fbuf[i0 + half] = make_float2(x0.x - tt.x, x0.y - tt.y);
    }
    __syncthreads();
  }
  for (int e = tid; e < cells; e += 256) {
    const int y = e >> lnx, x = e & (nx - 1);
    const int ry = (int)(__brev((unsigned)y) >> (32 - lny));
    if (y < ry) {
      const float2 a = fbuf[y * nx + x];
      fbuf[y * nx + x] = fbuf[ry * nx + x];
      fbuf[ry * nx + x] = a;
    }
  }
  __syncthreads();
  for (int s = 1; s <= lny; ++s) {
    const int half = 1 << (s - 1), stride = ny >> s;
    for (int k = tid; k < cells / 2; k += 256) {
      const int col = k & (nx - 1), bk = k >> lnx;
      const int i0 = ((bk >> (s - 1)) * (half << 1) + (bk & (half - 1))) * nx + col;
      const float2 tw = lfy[(bk & (half - 1)) * stride];
      const float2 x0 = fbuf[i0], x1 = fbuf[i0 + half * nx];
      const float2 tt = make_float2(tw.x * x1.x - tw.y * x1.y, tw.x * x1.y + tw.y * x1.x);
      fbuf[i0] = make_float2(x0.x + tt.x, x0.y + tt.y);
      fbuf[i0 + half * nx] = make_float2(x0.x - tt.x, x0.y - tt.y);
    }
    __syncthreads();
  }
  const float norm = 1.0f / (float)cells;
  float2* hb = h + (size_t)blockIdx.x * kpad;
  for (int e = tid; e < cells; e += 256) {
    const float2 v = fbuf[e];
    hb[e] = make_float2(v.x * norm, v.y * norm);
  }
}

// Complex per-row x-DFT: t[r][vx][k] = sum_{frames b of row r} Tx[(vx x_b) mod sx] h_b[k].
// Workgroup (k-block, vx, r); the row's frames are staged (index, twiddle) in LDS.
__global__ __launch_bounds__(256) void k_row_dft_c(const float2* __restrict__ h, int kpad,
                                                   const int* __restrict__ order, const int* __restrict__ xs,
                                                   RowSet rs, const float2* __restrict__ tx, int sx,
                                                   float2* __restrict__ t) {
  __shared__ float2 lw[256];
  __shared__ int lb[256];
  const int tid = threadIdx.x, k = blockIdx.x * 256 + tid, vx = blockIdx.y, r = blockIdx.z;
  const int4 row = rs.r[r];
  const bool px2 = (sx & (sx - 1)) == 0;
  const float invx = 1.0f / (float)sx;
  float re = 0.f, im = 0.f;
  for (int f0 = 0; f0 < row.z; f0 += 256) {
    const int n = min(256, row.z - f0);
    __syncthreads();
    if (tid < n) {
      const int at = row.y + f0 + tid;
      const int p = vx * xs[at];
      lw[tid] = tx[px2 ? (p & (sx - 1)) : mod_small(p, sx, invx)];
      lb[tid] = order[at];
    }
    __syncthreads();
    if (k < kpad)
      for (int i = 0; i < n; ++i) {
        const float2 c = lw[i], v = h[(size_t)lb[i] * kpad + k];
        re += c.x * v.x - c.y * v.y;
        im += c.x * v.y + c.y * v.x;
      }
  }
  if (k < kpad) t[((size_t)r * sx + vx) * kpad + k] = make_float2(re, im);
}

// Complex update, one workgroup per kept frequency j (each thread a stride of k):
//   s[k] = sum_r Ty[(vy y_r) mod sy] t[r][vx][k]
//   MODE 0 (object order):   D[j] += sum_k W[j][k] s[k]
//   MODE 1 (spectrum order): A[j][k] += s[k]
//   MODE 2 (spectrum order, Wiener reduction fused): A[j][k] += s[k]; D[j] = sum_k W[j][k] A[j][k]
// and z = conj(D) for modes 0 and 2.
template <int MODE>
__global__ __launch_bounds__(256) void k_update_c(const float2* __restrict__ t, int kpad, RowSet rs, int nrows,
                                                  const float2* __restrict__ ty, int sy, int sx,
                                                  const int2* __restrict__ freqs, const float2* __restrict__ w,
                                                  float2* __restrict__ acc, float2* __restrict__ d, float2* __restrict__ dlo,
                                                  float2* __restrict__ z) {
  __shared__ float2 lph[kRowSetMax];
  __shared__ float lre[4], lim[4];
  const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int2 v = freqs[j];
  const bool py2 = (sy & (sy - 1)) == 0;
  if (tid < nrows) {
    const int p = v.x * rs.r[tid].x;
    lph[tid] = ty[py2 ? (p & (sy - 1)) : mod_small(p, sy, 1.0f / (float)sy)];
  }
  __syncthreads();
  float re = 0.f, im = 0.f;
  for (int k = tid; k < kpad; k += 256) {
    float sr = 0.f, si = 0.f;
    for (int r = 0; r < nrows; ++r) {
      const float2 ph = lph[r], x = t[((size_t)r * sx + v.y) * kpad + k];
      sr += ph.x * x.x - ph.y * x.y;
      si += ph.x * x.y + ph.y * x.x;
    }
    if (MODE != 0) {
      float2 a = acc[(size_t)j * kpad + k];
      a.x += sr;
      a.y += si;
      acc[(size_t)j * kpad + k] = a;
      sr = a.x;
      si = a.y;
    }
    if (MODE != 1) {
      const float2 c = w[(size_t)j * kpad + k];
      re += c.x * sr - c.y * si;
      im += c.x * si + c.y * sr;
    }
  }
  if (MODE == 1) return;
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (lane == 0) {
    lre[wave] = re;
    lim[wave] = im;
  }
  __syncthreads();
  if (tid == 0) {
    re = (lre[0] + lre[1]) + (lre[2] + lre[3]);
    im = (lim[0] + lim[1]) + (lim[2] + lim[3]);
    float2 nd = make_float2(re, im);
    if (MODE == 0) {  // compensated: the object spectrum sums one contribution per push
      float2 lo = dlo[j];
      nd = d[j];
      two_sum_add2(nd, lo, make_float2(re, im));
      dlo[j] = lo;
    }
    d[j] = nd;
    z[(size_t)v.y * sy + v.x] = make_float2(nd.x, -nd.y);
  }
}

// z[v_x(j)][v_y(j)] = conj(d[j]) for every kept frequency (display grid from D).
__global__ void k_scatter_conj(const float2* __restrict__ d, const int2* __restrict__ freqs, int64_t n_freq,
                               float2* __restrict__ z, int sy) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n_freq) return;
  const int2 v = freqs[j];
  const float2 x = d[j];
  z[(size_t)v.y * sy + v.x] = make_float2(x.x, -x.y);
}

// Standalone display from a caller's spectrum grid d [sy][sx] (row-major, complex): the
// display's input z[vx][vy] = conj(d[vy][vx]) (transposed, as the update leaves it), and the
// forward twiddles ey[m] = exp(-2 pi i m / sy), ex[m] = exp(-2 pi i m / sx) evaluated in FP64
// (the argument 2 m / s is reduced exactly there) and rounded to FP32.
__global__ void k_display_prep(const float2* __restrict__ d, int sy, int sx, float2* __restrict__ z,
                               float2* __restrict__ ey, float2* __restrict__ ex) {
  const int64_t cells = (int64_t)sy * sx;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cells) {
    const int vy = (int)(i / sx), vx = (int)(i - (int64_t)vy * sx);
    const float2 v = d[i];
    z[(int64_t)vx * sy + vy] = make_float2(v.x, -v.y);
  }
  if (i < sy) {
    double sn, cs;
    sincospi(2.0 * (double)i / (double)sy, &sn, &cs);
    ey[i] = make_float2((float)cs, (float)-sn);
  }
  if (i < sx) {
    double sn, cs;
    sincospi(2.0 * (double)i / (double)sx, &sn, &cs);
    ex[i] = make_float2((float)cs, (float)-sn);
  }
}

__global__ void k_zero(float* __restrict__ p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t st = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += st) p[i] = 0.f;
}

template <int NCB>
hipError_t launch_acc_t(float2* acc, int kpad, int64_t n_freq_pad, const int2* freqs, const float* h,
                        const int2* pos, int n, const float2* ty, int sy, const float2* tx, int sx, hipStream_t st) {
  const size_t lds = (size_t)(sy + sx) * sizeof(float2) + 32 * sizeof(int2) + 32 * NCB * 32 * sizeof(float);
  {
    const hipError_t e = allow_full_lds<k_accumulate<NCB>>();
    if (e != hipSuccess) return e;
  }
  dim3 grid((unsigned)(n_freq_pad / 64), (unsigned)(kpad / (NCB * 32)));
  hipLaunchKernelGGL(k_accumulate<NCB>, grid, dim3(256), lds, st, acc, kpad, freqs, h, pos, n, ty, sy, tx, sx);
  return hipGetLastError();
}

}  // namespace

namespace wdd {

namespace {

ProjArgs proj_args(const ProjectLaunch& pl) {
  ProjArgs a;
  a.frames = pl.frames;
  a.n = pl.n;
  a.ny = pl.ny;
  a.nx = pl.nx;
  a.psi = pl.psi;
  a.psix_lp = pl.psix_lp;
  a.psi_unscale = pl.psi_unscale;
  a.kmap = pl.kmap;
  a.kpad = pl.kpad;
  a.h = pl.h;
  a.up_src = static_cast<const uint32_t*>(pl.up_src);
  a.up_dst = static_cast<uint32_t*>(pl.up_dst);
  a.up_words = pl.up_src ? (int)(pl.up_bytes / 4) : 0;
  a.fptr = pl.fptr;
  return a;
}

// LDS bytes of a projection workgroup of nw waves.
size_t project_lds(const ProjectLaunch& pl, int nw) {
  return pl.precision == WDD_FP32 ? project_lds_floats(pl.ny, pl.nx, nw, pl.kpad) * sizeof(float)
                                  : project_lp_lds_bytes(pl.ny, pl.nx, nw, pl.kpad);
}

template <typename T, int PREC>
hipError_t launch_project_tp(const ProjectLaunch& pl, const DisplayColumns* dc, hipStream_t st) {
  const int ntiles = (pl.ny + 15) / 16;
  const int nw_proj = std::min(ntiles, 16);
  const ProjArgs a = proj_args(pl);
  const int up = a.up_words > 0 ? 1 : 0;
  if (!dc) {
    const size_t lds = project_lds(pl, nw_proj);
    if (lds > kLdsBytes) return hipErrorInvalidValue;
    hipError_t e = allow_full_lds<k_project<T, PREC>>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_project<T, PREC>), dim3(pl.n + up), dim3(64 * nw_proj), lds, st, a);
    return hipGetLastError();
  }
  int lg = 0;
  while ((1 << lg) < dc->len) ++lg;
  if (dc->rows < 1 || (1 << lg) != dc->len || dc->nslot < 1 || dc->nslot > kMaxSlots) return hipErrorInvalidValue;
  const int threads = std::max(64 * nw_proj, 256);
  const size_t lds = std::max(project_lds(pl, threads / 64), (size_t)dc->len * sizeof(float2) * 3 / 2);
  if (lds > kLdsBytes) return hipErrorInvalidValue;
  hipError_t e = allow_full_lds<k_project_display<T, PREC>>();
  if (e != hipSuccess) return e;
  DispArgs d;
  d.din = dc->din;
  d.dout = dc->dout;
  d.len = dc->len;
  d.log2len = lg;
  d.e = dc->e;
  d.d0 = dc->d0;
  d.s_total = dc->s_total;
  d.in_sr = dc->in_sr;
  d.in_sm = dc->in_sm;
  d.out_sr = dc->out_sr;
  d.out_sc = dc->out_sc;
  d.nslot = dc->nslot;
  d.slot_stride = dc->slot_stride;
  hipLaunchKernelGGL((k_project_display<T, PREC>), dim3(pl.n + up + dc->rows), dim3(threads), lds, st, a, d);
  return hipGetLastError();
}

template <typename T, int PREC>
hipError_t launch_project_group_tp(const ProjectLaunch* pls, int count, const void* xsrc, void* xdst, size_t xbytes,
                                   hipStream_t st) {
  ProjGroupArgs g;
  std::memset(&g, 0, sizeof(g));
  int nw = 1;
  for (int m = 0; m < count; ++m) nw = std::max(nw, std::min((pls[m].ny + 15) / 16, 16));
  size_t lds = 0;
  g.first[0] = 0;
  for (int m = 0; m < count; ++m) {
    g.a[m] = proj_args(pls[m]);
    g.first[m + 1] = g.first[m] + pls[m].n;
    lds = std::max(lds, project_lds(pls[m], nw));
  }
  g.members = count;
  g.xsrc = static_cast<const uint32_t*>(xsrc);
  g.xdst = static_cast<uint32_t*>(xdst);
  g.xwords = (int)(xbytes / 4);
  if (lds > kLdsBytes) return hipErrorInvalidValue;
  const hipError_t e = allow_full_lds<k_project_group<T, PREC>>();
  if (e != hipSuccess) return e;
  const int xgroups = (g.xwords + kGroupUploadWords - 1) / kGroupUploadWords;
  hipLaunchKernelGGL((k_project_group<T, PREC>), dim3(g.first[count] + xgroups), dim3(64 * nw), lds, st, g);
  return hipGetLastError();
}

hipError_t launch_project_any(const ProjectLaunch& pl, const DisplayColumns* dc, hipStream_t st) {
  if (pl.n <= 0) return hipSuccess;
  if (pl.dtype == WDD_F32) {
    if (pl.precision != WDD_FP32) return hipErrorInvalidValue;
    return launch_project_tp<float, WDD_FP32>(pl, dc, st);
  }
  switch (pl.precision) {
    case WDD_FP32: return launch_project_tp<uint16_t, WDD_FP32>(pl, dc, st);
    case WDD_BF16_HILO: return launch_project_tp<uint16_t, WDD_BF16_HILO>(pl, dc, st);
    case WDD_FP16_HILO: return launch_project_tp<uint16_t, WDD_FP16_HILO>(pl, dc, st);
    case WDD_BF16: return launch_project_tp<uint16_t, WDD_BF16>(pl, dc, st);
    case WDD_FP16: return launch_project_tp<uint16_t, WDD_FP16>(pl, dc, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t prepare_group_kernels() {
  const hipError_t es[] = {allow_full_lds<k_project_group<float, WDD_FP32>>(),
                           allow_full_lds<k_project_group<uint16_t, WDD_FP32>>(),
                           allow_full_lds<k_project_group<uint16_t, WDD_BF16_HILO>>(),
                           allow_full_lds<k_project_group<uint16_t, WDD_FP16_HILO>>(),
                           allow_full_lds<k_project_group<uint16_t, WDD_BF16>>(),
                           allow_full_lds<k_project_group<uint16_t, WDD_FP16>>(),
                           allow_full_lds<k_row_fused_obj_group>(), allow_full_lds<k_row_dft_group>()};
  for (hipError_t e : es)
    if (e != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_project_group(const ProjectLaunch* pls, int count, const void* xsrc, void* xdst, size_t xbytes,
                                hipStream_t st) {
  if (count < 1 || count > kProjGroupMax || xbytes % 4 != 0 || (xbytes && (!xsrc || !xdst)) ||
      xbytes / 4 > (size_t)INT32_MAX)
    return hipErrorInvalidValue;
  for (int m = 0; m < count; ++m)
    if (pls[m].dtype != pls[0].dtype || pls[m].precision != pls[0].precision || pls[m].n < 0 || pls[m].up_src)
      return hipErrorInvalidValue;
  if (pls[0].dtype == WDD_F32) {
    if (pls[0].precision != WDD_FP32) return hipErrorInvalidValue;
    return launch_project_group_tp<float, WDD_FP32>(pls, count, xsrc, xdst, xbytes, st);
  }
  switch (pls[0].precision) {
    case WDD_FP32: return launch_project_group_tp<uint16_t, WDD_FP32>(pls, count, xsrc, xdst, xbytes, st);
    case WDD_BF16_HILO: return launch_project_group_tp<uint16_t, WDD_BF16_HILO>(pls, count, xsrc, xdst, xbytes, st);
    case WDD_FP16_HILO: return launch_project_group_tp<uint16_t, WDD_FP16_HILO>(pls, count, xsrc, xdst, xbytes, st);
    case WDD_BF16: return launch_project_group_tp<uint16_t, WDD_BF16>(pls, count, xsrc, xdst, xbytes, st);
    case WDD_FP16: return launch_project_group_tp<uint16_t, WDD_FP16>(pls, count, xsrc, xdst, xbytes, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_project(const ProjectLaunch& pl, hipStream_t st) { return launch_project_any(pl, nullptr, st); }

hipError_t launch_project_display(const ProjectLaunch& pl, const DisplayColumns& dc, hipStream_t st) {
  if (pl.n <= 0) return hipErrorInvalidValue;
  return launch_project_any(pl, &dc, st);
}

int accumulate_col_blocks(int kpad) {
  // columns per workgroup: as many as possible up to 4 blocks of 32 (keeps
  // 64 accumulator registers per lane and >= 2 waves per SIMD)
  if (kpad % 128 == 0) return 4;
  if (kpad % 64 == 0) return 2;
  return 1;
}

hipError_t launch_accumulate(float2* acc, int kpad, int64_t n_freq_pad, const int2* freqs, const float* h,
                             const int2* pos, int n, const float2* ty, int sy, const float2* tx, int sx,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  switch (accumulate_col_blocks(kpad)) {
    case 4: return launch_acc_t<4>(acc, kpad, n_freq_pad, freqs, h, pos, n, ty, sy, tx, sx, st);
    case 2: return launch_acc_t<2>(acc, kpad, n_freq_pad, freqs, h, pos, n, ty, sy, tx, sx, st);
    default: return launch_acc_t<1>(acc, kpad, n_freq_pad, freqs, h, pos, n, ty, sy, tx, sx, st);
  }
}

hipError_t launch_wiener(const float2* acc, const float2* w, int kpad, const int2* freqs, int64_t n_freq, float2* d,
                         float2* z, int sy, hipStream_t st) {
  const unsigned blocks = (unsigned)((n_freq + 3) / 4);
  hipLaunchKernelGGL(k_wiener, dim3(blocks), dim3(256), 0, st, acc, w, kpad, freqs, n_freq, d, z, sy);
  return hipGetLastError();
}

hipError_t launch_dft_rows(const float2* in, float2* out, int rows, int len, const float2* e, const float2* d0,
                           float s_total, int final_scale, int in_sr, int in_sm, int out_sr, int out_sc,
                           int nslot, int slot_stride, hipStream_t st) {
  int lg = -1;
  if ((len & (len - 1)) == 0) {
    lg = 0;
    while ((1 << lg) < len) ++lg;
  }
  if (nslot < 1 || nslot > kMaxSlots || (nslot > 1 && (lg < 0 || !final_scale))) return hipErrorInvalidValue;
  const size_t lds = (size_t)len * sizeof(float2) + (lg >= 0 ? (size_t)(len / 2) * sizeof(float2) : 0);
  // grids of 64 Ki cells and more: rows per XCD in contiguous ranges (a column gather would
  // otherwise bring every cache line into all 8 L2s); smaller grids gain nothing from it
  const int xcd_map = (int64_t)rows * len >= 65536;
  if (nslot > 1)
    hipLaunchKernelGGL(k_dft_rows<true>, dim3(rows), dim3(256), lds, st, in, out, len, lg, e, d0, s_total, final_scale,
                       in_sr, in_sm, out_sr, out_sc, xcd_map, nslot, slot_stride, rows, (int64_t)0, (int64_t)0,
                       (int64_t)0);
  else
    hipLaunchKernelGGL(k_dft_rows<false>, dim3(rows), dim3(256), lds, st, in, out, len, lg, e, d0, s_total, final_scale,
                       in_sr, in_sm, out_sr, out_sc, xcd_map, 1, 0, rows, (int64_t)0, (int64_t)0, (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_dft_rows_blocks(const float2* in, float2* out, int blocks, int block_rows, int len, const float2* e,
                                  const float2* d0, float s_total, int final_scale, int in_sr, int in_sm, int out_sr,
                                  int out_sc, int64_t in_block, int64_t out_block, int64_t d0_block, hipStream_t st) {
  int lg = -1;
  if ((len & (len - 1)) == 0) {
    lg = 0;
    while ((1 << lg) < len) ++lg;
  }
  if (blocks < 1 || block_rows < 1) return hipErrorInvalidValue;
  const size_t lds = (size_t)len * sizeof(float2) + (lg >= 0 ? (size_t)(len / 2) * sizeof(float2) : 0);
  hipLaunchKernelGGL(k_dft_rows<false>, dim3((unsigned)(blocks * block_rows)), dim3(256), lds, st, in, out, len, lg, e,
                     d0, s_total, final_scale, in_sr, in_sm, out_sr, out_sc, 0, 1, 0, block_rows, in_block, out_block,
                     d0_block);
  return hipGetLastError();
}

// The field-of-view patch merge: out[y][x] = sum_p w_p img_p[y - oy_p][x - ox_p] / sum_p w_p over
// the patches covering (y, x), w_p the product of the trapezoid windows of the two axes, patches
// taken in origin order (deterministic).
__device__ inline float patch_weight(int i, int p, int overlap) {
  const float o1 = (float)(overlap + 1);
  return fminf(1.0f, fminf((float)(i + 1) / o1, (float)(p - i) / o1));
}
__global__ __launch_bounds__(256) void k_patch_merge(const float2* __restrict__ img, const int* __restrict__ oy,
                                                     int npy, const int* __restrict__ ox, int npx, int py, int px,
                                                     int overlap_y, int overlap_x, float2* __restrict__ out, int sy,
                                                     int sx) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)sy * sx) return;
  const int y = (int)(i / sx), x = (int)(i - (int64_t)y * sx);
  float re = 0.f, im = 0.f, den = 0.f;
  for (int a = 0; a < npy; ++a) {
    const int ly = y - oy[a];
    if (ly < 0 || ly >= py) continue;
    const float wy = patch_weight(ly, py, overlap_y);
    for (int b = 0; b < npx; ++b) {
      const int lx = x - ox[b];
      if (lx < 0 || lx >= px) continue;
      const float w = wy * patch_weight(lx, px, overlap_x);
      const float2 v = img[((size_t)(a * npx + b) * py + ly) * px + lx];
      re += w * v.x;
      im += w * v.y;
      den += w;
    }
  }
  out[i] = den > 0.f ? make_float2(re / den, im / den) : make_float2(0.f, 0.f);
}

hipError_t launch_patch_merge(const float2* img, const int* oy, int npy, const int* ox, int npx, int py, int px,
                              int overlap_y, int overlap_x, float2* out, int sy, int sx, hipStream_t st) {
  const int64_t n = (int64_t)sy * sx;
  if (n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_patch_merge, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, img, oy, npy, ox, npx, py, px,
                     overlap_y, overlap_x, out, sy, sx);
  return hipGetLastError();
}

hipError_t launch_row_dft(const float* h, int kpad, const int* xs, const int* order, const int4* rows, int nrows,
                          const float2* tx, int sx, float2* t, hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  {
    const hipError_t e = allow_full_lds<k_row_dft>();
    if (e != hipSuccess) return e;
  }
  const size_t lds = (size_t)sx * sizeof(float2) + 2 * kRowChunk * sizeof(int) + kRowChunk * 16 * sizeof(float);
  dim3 grid((unsigned)((sx + 7) / 8), (unsigned)(kpad / 16), (unsigned)nrows);
  hipLaunchKernelGGL(k_row_dft, grid, dim3(256), lds, st, h, kpad, xs, order, rows, tx, sx, t);
  return hipGetLastError();
}

size_t row_dft_lds_bytes(int sx) {
  return (size_t)sx * sizeof(float2) + 2 * kRowChunk * sizeof(int) + kRowChunk * 16 * sizeof(float);
}
int row_dft_blocks(int sx, int kpad, int nrows) { return ((sx + 7) / 8) * (kpad / 16) * nrows; }
int row_update_blocks(int64_t n_freq_pad, int kpad) { return (int)((n_freq_pad * (kpad / 4) + 255) / 256); }

hipError_t launch_row_dft_group(const SpecPass* passes, const int* first, int npass, int nblocks, size_t lds,
                                hipStream_t st) {
  if (npass < 1 || nblocks < 1) return hipSuccess;
  if (lds > kLdsBytes) return hipErrorInvalidValue;
  const hipError_t e = allow_full_lds<k_row_dft_group>();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_row_dft_group, dim3((unsigned)nblocks), dim3(256), lds, st, passes, first, npass);
  return hipGetLastError();
}

hipError_t launch_row_update_group(const SpecPass* passes, const int* first, int npass, int nblocks, hipStream_t st) {
  if (npass < 1 || nblocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k_row_update_group, dim3((unsigned)nblocks), dim3(256), 0, st, passes, first, npass);
  return hipGetLastError();
}

hipError_t launch_row_update(float2* acc, int kpad, int64_t n_freq_pad, const int2* freqs, int64_t n_freq,
                             const float2* t, int sx, const int4* rows, int nrows, const float2* ty, int sy,
                             const float2* w, float2* d, float2* z, bool fuse_wiener, hipStream_t st) {
  const int64_t threads = n_freq_pad * (kpad / 4);
  const unsigned blocks = (unsigned)((threads + 255) / 256);
  if (fuse_wiener)
    hipLaunchKernelGGL(k_row_update<true>, dim3(blocks), dim3(256), 0, st, acc, kpad, freqs, n_freq, t, sx, rows,
                       nrows, ty, sy, w, d, z);
  else
    hipLaunchKernelGGL(k_row_update<false>, dim3(blocks), dim3(256), 0, st, acc, kpad, freqs, n_freq, t, sx, rows,
                       nrows, ty, sy, w, d, z);
  return hipGetLastError();
}

size_t row_fused_lds_bytes(int kpad, int nrows, int max_chunk) {
  return (size_t)nrows * (kpad / 4) * 32 + (size_t)kFusedThreads * 32 + (size_t)kFusedFrames * 12 +
         (size_t)max_chunk * 16;
}

namespace {

// Shared checks and set-up of the object-order update launches: the dynamic LDS, the display
// rows' arguments (dc null: none) and log2 Sy for the partial rows.
struct FusedSetup {
  size_t lds;
  DispArgs da;
  int rows_disp;
  int log2sy;
};
hipError_t fused_setup(int kpad, int nrows, int sy, int nchunks, int max_chunk, const float2* up, int nslot,
                       const DisplayColumns* dc, FusedSetup* fs) {
  if (nrows < 1 || nrows > kRowSetMax || nchunks < 1 || max_chunk < 1 || max_chunk > kFusedThreads)
    return hipErrorInvalidValue;
  fs->log2sy = 0;
  if (up) {  // the partial rows need a power-of-two Sy whose row and twiddles fit the group-sum buffer
    while ((1 << fs->log2sy) < sy) ++fs->log2sy;
    if ((1 << fs->log2sy) != sy || sy > kDisplayRowMax || nslot < 1 || nslot > kMaxSlots)
      return hipErrorInvalidValue;
  }
  fs->lds = row_fused_lds_bytes(kpad, nrows, max_chunk);
  std::memset(&fs->da, 0, sizeof(fs->da));
  fs->rows_disp = 0;
  if (dc) {
    int lg = 0;
    while ((1 << lg) < dc->len) ++lg;
    if (dc->rows < 1 || (1 << lg) != dc->len || dc->nslot < 1 || dc->nslot > kMaxSlots) return hipErrorInvalidValue;
    DispArgs& da = fs->da;
    da.din = dc->din;
    da.dout = dc->dout;
    da.len = dc->len;
    da.log2len = lg;
    da.e = dc->e;
    da.d0 = dc->d0;
    da.s_total = dc->s_total;
    da.in_sr = dc->in_sr;
    da.in_sm = dc->in_sm;
    da.out_sr = dc->out_sr;
    da.out_sc = dc->out_sc;
    da.nslot = dc->nslot;
    da.slot_stride = dc->slot_stride;
    da.rows = dc->rows;
    fs->rows_disp = (dc->rows + 1) / 2;  // two rows per workgroup (display_row_pair)
    fs->lds = std::max(fs->lds, (size_t)dc->len * sizeof(float2) * 3);
  }
  if (fs->lds > kLdsBytes) return hipErrorInvalidValue;
  return hipSuccess;
}

}  // namespace

hipError_t launch_row_fused_obj(const float* h, int kpad, const int* order, const int* xs, const RowSet& rows,
                                int nrows, float tscale, int sx, int sy, const int4* chunks, int nchunks,
                                int max_chunk, const int2* jv, const float2* w, float2* d, float2* dlo, float2* z,
                                float2* up, int nslot, bool in_order, float2* d0out, const DisplayColumns* dc,
                                hipStream_t st) {
  FusedSetup fs;
  hipError_t e = fused_setup(kpad, nrows, sy, nchunks, max_chunk, up, nslot, dc, &fs);
  if (e != hipSuccess) return e;
  if ((e = allow_full_lds<k_row_fused_obj>()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_row_fused_obj, dim3(nchunks + fs.rows_disp), dim3(kFusedThreads), fs.lds, st, h, kpad, order,
                     xs, rows, nrows, tscale, sx, sy, chunks, jv, w, d, dlo, z, max_chunk, up, nslot, fs.log2sy,
                     in_order ? 1 : 0, d0out, nchunks, fs.da);
  return hipGetLastError();
}

namespace {
constexpr int kNextWaves = kFusedThreads / 64;

size_t next_project_lds(int precision, int ny, int nx, int kpad) {
  return precision == WDD_FP32 ? project_lds_floats(ny, nx, kNextWaves, kpad) * sizeof(float)
                               : project_lp_lds_bytes(ny, nx, kNextWaves, kpad);
}
}  // namespace

bool row_fused_next_supported(int dtype, int precision, int ny, int nx, int kpad) {
  if (dtype != WDD_U16 || nx % 32 != 0 || nx < 32 || nx > 256 || ny < 1 || kpad > 4 * kFusedThreads) return false;
  if (precision == WDD_FP32) {
    if (ny > 2 * 16 * kNextWaves) return false;
  } else if (precision == WDD_BF16_HILO || precision == WDD_FP16_HILO || precision == WDD_BF16 ||
             precision == WDD_FP16) {
    if (!project_lp_tile_form(ny, nx, kNextWaves, kpad)) return false;
  } else {
    return false;
  }
  return next_project_lds(precision, ny, nx, kpad) <= kLdsBytes;
}

hipError_t launch_row_fused_obj_next(const float* h, int kpad, const int* order, const int* xs, const RowSet& rows,
                                     int nrows, float tscale, int sx, int sy, const int4* chunks, int nchunks,
                                     int max_chunk, const int2* jv, const float2* w, float2* d, float2* dlo,
                                     float2* z, float2* up, int nslot, bool in_order, float2* d0out,
                                     const DisplayColumns* dc, const ProjectLaunch& next, hipStream_t st) {
  if (next.n < 1 || next.kpad != kpad || !row_fused_next_supported(next.dtype, next.precision, next.ny, next.nx, kpad))
    return hipErrorInvalidValue;
  FusedSetup fs;
  hipError_t e = fused_setup(kpad, nrows, sy, nchunks, max_chunk, up, nslot, dc, &fs);
  if (e != hipSuccess) return e;
  const size_t lds = std::max(fs.lds, next_project_lds(next.precision, next.ny, next.nx, kpad));
  const ProjArgs pa = proj_args(next);
  const int nproj = next.n + (pa.up_words > 0 ? 1 : 0);
  const int pfront = std::min(kNextProjFront, nproj) / 8 * 8;
  static_assert(kNextProjFront % 8 == 0, "whole rounds of the 8 XCDs in front of the chunks");
  const dim3 grid(nchunks + fs.rows_disp + nproj), block(kFusedThreads);
#define WDD_LAUNCH(P)                                                                                               \
  if ((e = allow_full_lds<k_row_fused_obj_next<P>>()) != hipSuccess) return e;                                      \
  hipLaunchKernelGGL(k_row_fused_obj_next<P>, grid, block, lds, st, h, kpad, order, xs, rows, nrows, tscale, sx, sy, \
                     chunks, jv, w, d, dlo, z, max_chunk, up, nslot, fs.log2sy, in_order ? 1 : 0, d0out, nchunks,  \
                     fs.da, pa, pfront);                                                                            \
  break
  switch (next.precision) {
    case WDD_FP32: WDD_LAUNCH(WDD_FP32);
    case WDD_BF16_HILO: WDD_LAUNCH(WDD_BF16_HILO);
    case WDD_FP16_HILO: WDD_LAUNCH(WDD_FP16_HILO);
    case WDD_BF16: WDD_LAUNCH(WDD_BF16);
    case WDD_FP16: WDD_LAUNCH(WDD_FP16);
    default: return hipErrorInvalidValue;
  }
#undef WDD_LAUNCH
  return hipGetLastError();
}

int row_fused_t_stride(int kpad) { return kRowSetMax * (kpad / 4) * 2; }

hipError_t launch_row_fused_obj_next2(int kpad, float tscale, int sx, int sy, const int4* chunks, int nchunks,
                                      int max_chunk, const int2* jv, const float2* w, float2* d, float2* dlo,
                                      float2* z, int nslot, const RowSet& urows, int unrows, const float4* tin,
                                      float2* up, float2* d0out, const XdftPart& xp, const DisplayColumns* dc,
                                      const ProjectLaunch* next, hipStream_t st) {
  if (nchunks < 0 || max_chunk < 1 || max_chunk > kFusedThreads || xp.ncols < 0) return hipErrorInvalidValue;
  if (nchunks > 0 && (unrows < 1 || unrows > kRowSetMax || !tin)) return hipErrorInvalidValue;
  if (xp.ncols > 0 && (xp.nrows < 1 || xp.nrows > kRowSetMax || !xp.h || !xp.order || !xp.xs || !xp.xcols ||
                       !xp.tout))
    return hipErrorInvalidValue;
  const int nproj_frames = next ? next->n : 0;
  if (next && (next->n < 1 || next->kpad != kpad ||
               !row_fused_next_supported(next->dtype, next->precision, next->ny, next->nx, kpad)))
    return hipErrorInvalidValue;
  int log2sy = 0;
  if (up) {
    while ((1 << log2sy) < sy) ++log2sy;
    if ((1 << log2sy) != sy || sy > kDisplayRowMax || nslot < 1 || nslot > kMaxSlots) return hipErrorInvalidValue;
  }
  size_t lds = row_fused_lds_bytes(kpad, kRowSetMax, max_chunk);
  DispArgs da;
  std::memset(&da, 0, sizeof(da));
  int rows_disp = 0;
  if (dc) {
    int lg = 0;
    while ((1 << lg) < dc->len) ++lg;
    if (dc->rows < 1 || (1 << lg) != dc->len || dc->nslot < 1 || dc->nslot > kMaxSlots) return hipErrorInvalidValue;
    da.din = dc->din;
    da.dout = dc->dout;
    da.len = dc->len;
    da.log2len = lg;
    da.e = dc->e;
    da.d0 = dc->d0;
    da.s_total = dc->s_total;
    da.in_sr = dc->in_sr;
    da.in_sm = dc->in_sm;
    da.out_sr = dc->out_sr;
    da.out_sc = dc->out_sc;
    da.nslot = dc->nslot;
    da.slot_stride = dc->slot_stride;
    da.rows = dc->rows;
    rows_disp = (dc->rows + 1) / 2;  // two rows per workgroup (display_row_pair)
    lds = std::max(lds, (size_t)dc->len * sizeof(float2) * 3);
  }
  ProjArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  int precision = WDD_FP32;
  if (next) {
    pa = proj_args(*next);
    precision = next->precision;
    lds = std::max(lds, next_project_lds(next->precision, next->ny, next->nx, kpad));
  }
  if (lds > kLdsBytes) return hipErrorInvalidValue;
  const int nproj = nproj_frames > 0 ? nproj_frames + (pa.up_words > 0 ? 1 : 0) : 0;
  const bool long_proj = next && next->ny > 16 * kNextWaves;
  const int pfront = long_proj ? std::min(kStage2FrontLong, nproj) / 8 * 8 : 0;
  const int total = nproj + xp.ncols + nchunks + rows_disp;
  if (total < 1) return hipSuccess;
  NextArgs xa;
  std::memset(&xa, 0, sizeof(xa));
  xa.h = xp.h;
  xa.order = xp.order;
  xa.xs = xp.xs;
  xa.rows = xp.rows;
  xa.nrows = xp.nrows;
  xa.in_order = xp.in_order ? 1 : 0;
  xa.ncols = xp.ncols;
  xa.xcols = xp.xcols;
  xa.tout = xp.tout;
  hipError_t e;
  const dim3 grid(total), block(kFusedThreads);
#define WDD_LAUNCH2(P, O)                                                                                       \
  if ((e = allow_full_lds<k_row_fused_obj_next2<P, O>>()) != hipSuccess) return e;                              \
  hipLaunchKernelGGL((k_row_fused_obj_next2<P, O>), grid, block, lds, st, kpad, urows, unrows, tscale, sx, sy,   \
                     chunks, jv, w, d, dlo, z, max_chunk, up, nslot, log2sy, d0out, nchunks, tin,              \
                     row_fused_t_stride(kpad), xa, da, pa, pfront)
#define WDD_LAUNCH(P)                                                                                           \
  if (long_proj) {                                                                                              \
    WDD_LAUNCH2(P, true);                                                                                       \
  } else {                                                                                                      \
    WDD_LAUNCH2(P, false);                                                                                      \
  }                                                                                                             \
  break
  switch (precision) {
    case WDD_FP32: WDD_LAUNCH(WDD_FP32);
    case WDD_BF16_HILO: WDD_LAUNCH(WDD_BF16_HILO);
    case WDD_FP16_HILO: WDD_LAUNCH(WDD_FP16_HILO);
    case WDD_BF16: WDD_LAUNCH(WDD_BF16);
    case WDD_FP16: WDD_LAUNCH(WDD_FP16);
    default: return hipErrorInvalidValue;
  }
#undef WDD_LAUNCH2
#undef WDD_LAUNCH
  return hipGetLastError();
}

hipError_t launch_row_fused_obj_group(const ObjPass* passes, const int4* items, int nitems, size_t lds_bytes,
                                      hipStream_t st) {
  if (nitems < 1) return hipSuccess;
  if (lds_bytes > kLdsBytes) return hipErrorInvalidValue;
  const hipError_t e = allow_full_lds<k_row_fused_obj_group>();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_row_fused_obj_group, dim3((unsigned)nitems), dim3(kFusedThreads), lds_bytes, st, passes, items);
  return hipGetLastError();
}

hipError_t launch_project_fourier(int dtype, const void* frames, int n, int ny, int nx, const float2* fy,
                                  const float2* fx, float2* h, int kpad, const void* up_src, void* up_dst,
                                  size_t up_bytes, const uint64_t* fptr, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int lny = 0, lnx = 0;
  while ((1 << lny) < ny) ++lny;
  while ((1 << lnx) < nx) ++lnx;
  if ((1 << lny) != ny || (1 << lnx) != nx || ny < 2 || nx < 2 || ny * nx > kpad || ny * nx > 4096)
    return hipErrorInvalidValue;
  const size_t lds = ((size_t)ny * nx + ny / 2 + nx / 2) * sizeof(float2);
  if (dtype == WDD_U16)
    hipLaunchKernelGGL(k_project_fourier<uint16_t>, dim3(n), dim3(256), lds, st,
                       static_cast<const uint16_t*>(frames), ny, nx, lny, lnx, fy, fx, h, kpad,
                       static_cast<const uint32_t*>(up_src), static_cast<uint32_t*>(up_dst), (int)(up_bytes / 4),
                       fptr);
  else
    hipLaunchKernelGGL(k_project_fourier<float>, dim3(n), dim3(256), lds, st, static_cast<const float*>(frames), ny,
                       nx, lny, lnx, fy, fx, h, kpad, static_cast<const uint32_t*>(up_src),
                       static_cast<uint32_t*>(up_dst), (int)(up_bytes / 4), fptr);
  return hipGetLastError();
}

hipError_t launch_row_dft_c(const float2* h, int kpad, const int* order, const int* xs, const RowSet& rows, int nrows,
                            const float2* tx, int sx, float2* t, hipStream_t st) {
  if (nrows < 1 || nrows > kRowSetMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_row_dft_c, dim3((unsigned)((kpad + 255) / 256), (unsigned)sx, (unsigned)nrows), dim3(256), 0,
                     st, h, kpad, order, xs, rows, tx, sx, t);
  return hipGetLastError();
}

hipError_t launch_update_c(int mode, const float2* t, int kpad, const RowSet& rows, int nrows, const float2* ty, int sy,
                           int sx, const int2* freqs, int64_t n_freq, const float2* w, float2* acc, float2* d,
                           float2* dlo, float2* z, hipStream_t st) {
  if (nrows < 1 || nrows > kRowSetMax || n_freq < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_freq);
  if (mode == 0)
    hipLaunchKernelGGL(k_update_c<0>, grid, dim3(256), 0, st, t, kpad, rows, nrows, ty, sy, sx, freqs, w, acc, d, dlo, z);
  else if (mode == 1)
    hipLaunchKernelGGL(k_update_c<1>, grid, dim3(256), 0, st, t, kpad, rows, nrows, ty, sy, sx, freqs, w, acc, d, dlo, z);
  else if (mode == 2)
    hipLaunchKernelGGL(k_update_c<2>, grid, dim3(256), 0, st, t, kpad, rows, nrows, ty, sy, sx, freqs, w, acc, d, dlo, z);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_scatter_conj(const float2* d, const int2* freqs, int64_t n_freq, float2* z, int sy, hipStream_t st) {
  if (n_freq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_conj, dim3((unsigned)((n_freq + 255) / 256)), dim3(256), 0, st, d, freqs, n_freq, z, sy);
  return hipGetLastError();
}

hipError_t launch_display_prep(const float2* d, int sy, int sx, float2* z, float2* ey, float2* ex, hipStream_t st) {
  if (sy < 1 || sx < 1) return hipErrorInvalidValue;
  const int64_t n = std::max<int64_t>((int64_t)sy * sx, std::max(sy, sx));
  hipLaunchKernelGGL(k_display_prep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, sy, sx, z, ey, ex);
  return hipGetLastError();
}

hipError_t launch_zero(float* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace wdd
