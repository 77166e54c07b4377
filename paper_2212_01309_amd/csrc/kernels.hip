// HIP kernels of the live WDD per-frame update for gfx950 (CDNA4, wave64).
//
//   k_project      frames -> h = Phi^T vec(I)      (Section 5 reduction; FP32 MFMA)
//   k_accumulate   A[v,k] += sum_b F[v,b] h[b,k]   (Section 6.1 outer-product sum; FP32 MFMA)
//   k_wiener       D[v] = sum_k W[v,k] A[v,k]      (modified-WDD deconvolution + summation)
//   k_dft_rows     row DFTs for O~ = conj(IDFT2(D)) / sqrt(|D[0]|)   (eq. extract)
//
// Complex values are float2 (re, im).  No atomics: every output element has a
// single owner, so results are deterministic for fixed batch boundaries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

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
__device__ inline void load8(const T* __restrict__ row, float* v);

template <>
__device__ inline void load8<uint16_t>(const uint16_t* __restrict__ p, float* v) {
  const uint4 raw = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[2 * i] = (float)(w[i] & 0xffffu);
    v[2 * i + 1] = (float)(w[i] >> 16);
  }
}

template <>
__device__ inline void load8<float>(const float* __restrict__ p, float* v) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

template <typename T>
__global__ __launch_bounds__(256) void k_project(const T* __restrict__ frames, int ny, int nx,
                                                 const float* __restrict__ psi, const int* __restrict__ kmap,
                                                 int kpad, float* __restrict__ h) {
  extern __shared__ float smem[];
  float* lpsy = smem;               // [ny][16]
  float* lpsx = smem + ny * 16;     // [nx][16]
  float* lg = lpsx + nx * 16;       // [4][256]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < (ny + nx) * 16; i += 256) smem[i] = psi[i];
  __syncthreads();

  const T* f = frames + (size_t)blockIdx.x * ny * nx;
  const int r16 = lane & 15, q = lane >> 4;
  floatx4 g = {0.f, 0.f, 0.f, 0.f};
  const int ntiles = (ny + 15) >> 4;
  for (int t = wave; t < ntiles; t += 4) {
    const int y = t * 16 + r16;
    floatx4 tacc = {0.f, 0.f, 0.f, 0.f};
    for (int x0 = 0; x0 < nx; x0 += 32) {
      const int xs = x0 + 8 * q;
      float v[8];
      const bool ok = (y < ny) && (xs < nx);
      if (ok) {
        load8<T>(f + (size_t)y * nx + xs, v);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = 0.f;
      }
      const int xb = (xs < nx) ? xs : 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float bv = (xs < nx) ? lpsx[(xb + j) * 16 + r16] : 0.f;
        tacc = __builtin_amdgcn_mfma_f32_16x16x4f32(v[j], bv, tacc, 0, 0, 0);
      }
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
  for (int k = tid; k < kpad; k += 256) {
    const int idx = kmap[k];
    float s = 0.f;
    if (idx >= 0) s = (lg[idx] + lg[256 + idx]) + (lg[512 + idx] + lg[768 + idx]);
    h[(size_t)blockIdx.x * kpad + k] = s;
  }
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
// Also scatters conj(D[j]) into the sy x sx grid z (zeros elsewhere are set
// once at plan creation), ready for the forward DFT of the display step.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wiener(const float2* __restrict__ acc, const float2* __restrict__ w,
                                                int kpad, const int2* __restrict__ freqs, int64_t n_freq,
                                                float2* __restrict__ d, float2* __restrict__ z, int sx) {
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
    z[(size_t)v.x * sx + v.y] = make_float2(re, -im);
  }
}

// ---------------------------------------------------------------------------
// Forward DFT of each row of a rows x len array, written transposed:
// out[c * rows + r] = scale * sum_m in[r * len + m] * E[(m c) mod len],
// E[m] = exp(-2 pi i m / len) built in FP64 on the host.  Power-of-two
// lengths use an in-LDS radix-2 decimation-in-time FFT, others a direct sum.
// With `final_scale` set, scale = 1 / sqrt(S |D[0]|) (0 when D[0] = 0).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dft_rows(const float2* __restrict__ in, float2* __restrict__ out, int rows,
                                                  int len, int log2len, const float2* __restrict__ e,
                                                  const float2* __restrict__ d0, float s_total, int final_scale) {
  extern __shared__ float2 lbuf[];  // [len]
  const int r = blockIdx.x, tid = threadIdx.x;
  const float2* src = in + (size_t)r * len;
  float scale = 1.0f;
  if (final_scale) {
    const float2 dd = d0[0];
    const float mag = sqrtf(dd.x * dd.x + dd.y * dd.y);
    scale = mag > 0.f ? 1.0f / sqrtf(s_total * mag) : 0.f;
  }
  if (log2len >= 0) {
    for (int m = tid; m < len; m += 256) {
      const int rev = log2len ? (int)(__brev((unsigned)m) >> (32 - log2len)) : 0;
      lbuf[rev] = src[m];
    }
    __syncthreads();
    for (int s = 1; s <= log2len; ++s) {
      const int half = 1 << (s - 1);
      const int stride = len >> s;  // twiddle index step
      for (int k = tid; k < len / 2; k += 256) {
        const int grp = k >> (s - 1), p = k & (half - 1);
        const int i0 = grp * (half << 1) + p, i1 = i0 + half;
        const float2 tw = e[p * stride];
        const float2 x1 = lbuf[i1], x0 = lbuf[i0];
        const float2 tt = make_float2(tw.x * x1.x - tw.y * x1.y, tw.x * x1.y + tw.y * x1.x);
        lbuf[i0] = make_float2(x0.x + tt.x, x0.y + tt.y);
        lbuf[i1] = make_float2(x0.x - tt.x, x0.y - tt.y);
      }
      __syncthreads();
    }
    for (int cidx = tid; cidx < len; cidx += 256) {
      const float2 v = lbuf[cidx];
      out[(size_t)cidx * rows + r] = make_float2(v.x * scale, v.y * scale);
    }
  } else {
    for (int m = tid; m < len; m += 256) lbuf[m] = src[m];
    __syncthreads();
    for (int cidx = tid; cidx < len; cidx += 256) {
      float re = 0.f, im = 0.f;
      int idx = 0;
      for (int m = 0; m < len; ++m) {
        const float2 x = lbuf[m], tw = e[idx];
        re += x.x * tw.x - x.y * tw.y;
        im += x.x * tw.y + x.y * tw.x;
        idx += cidx;
        idx -= (idx >= len) ? len : 0;
      }
      out[(size_t)cidx * rows + r] = make_float2(re * scale, im * scale);
    }
  }
}

__global__ void k_zero(float* __restrict__ p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t st = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += st) p[i] = 0.f;
}

template <typename T>
hipError_t launch_project_t(const void* frames, int n, int ny, int nx, const float* psi, const int* kmap, int kpad,
                            float* h, hipStream_t st) {
  const size_t lds = (size_t)(ny + nx) * 16 * sizeof(float) + 4 * 256 * sizeof(float);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_project<T>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_project<T>, dim3(n), dim3(256), lds, st, static_cast<const T*>(frames), ny, nx, psi, kmap,
                     kpad, h);
  return hipGetLastError();
}

template <int NCB>
hipError_t launch_acc_t(float2* acc, int kpad, int64_t n_freq_pad, const int2* freqs, const float* h,
                        const int2* pos, int n, const float2* ty, int sy, const float2* tx, int sx, hipStream_t st) {
  const size_t lds = (size_t)(sy + sx) * sizeof(float2) + 32 * sizeof(int2) + 32 * NCB * 32 * sizeof(float);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_accumulate<NCB>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  dim3 grid((unsigned)(n_freq_pad / 64), (unsigned)(kpad / (NCB * 32)));
  hipLaunchKernelGGL(k_accumulate<NCB>, grid, dim3(256), lds, st, acc, kpad, freqs, h, pos, n, ty, sy, tx, sx);
  return hipGetLastError();
}

}  // namespace

namespace wdd {

hipError_t launch_project(int dtype, const void* frames, int n, int ny, int nx, const float* psi, const int* kmap,
                          int kpad, float* h, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (dtype == WDD_U16) return launch_project_t<uint16_t>(frames, n, ny, nx, psi, kmap, kpad, h, st);
  return launch_project_t<float>(frames, n, ny, nx, psi, kmap, kpad, h, st);
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
                         float2* z, int sx, hipStream_t st) {
  const unsigned blocks = (unsigned)((n_freq + 3) / 4);
  hipLaunchKernelGGL(k_wiener, dim3(blocks), dim3(256), 0, st, acc, w, kpad, freqs, n_freq, d, z, sx);
  return hipGetLastError();
}

hipError_t launch_dft_rows(const float2* in, float2* out, int rows, int len, const float2* e, const float2* d0,
                           float s_total, int final_scale, hipStream_t st) {
  int lg = -1;
  if ((len & (len - 1)) == 0) {
    lg = 0;
    while ((1 << lg) < len) ++lg;
  }
  const size_t lds = (size_t)len * sizeof(float2);
  hipLaunchKernelGGL(k_dft_rows, dim3(rows), dim3(256), lds, st, in, out, rows, len, lg, e, d0, s_total, final_scale);
  return hipGetLastError();
}

hipError_t launch_zero(float* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace wdd
