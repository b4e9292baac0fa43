// One-off setup of the split-lasso ADMM: copy H into the block store and
// build, per block (i,j), the Hermitian inverse of G_ij = rho I + H_ij H_ij^H
// in FP64 (Gram, Cholesky, triangular inverse, W^H W), stored as complex64.
// This is the paper's inversion step: the small m_i x m_i matrix of the
// inversion lemma (eq. inversion_lemma3), since (I + H H^H/rho)^{-1} = rho G^{-1};
// for a plan in the direct form the n_j x n_j matrix A_ij = rho I + H_ij^H H_ij
// itself (Sec. III-B, the remark on tall blocks after eq. inversion_lemma2).
//
// Every FP64 matrix is padded to a multiple of kTile with identity rows, so
// the tiled algorithms never see a ragged tile.  Tiles are 64 x 64 double2;
// each workgroup (256 threads) owns one output tile, whose products run on
// the FP64 matrix cores (AccM) or on vector FMAs (AccV).  All blocks of the
// split are processed by the same launch.
#include <algorithm>
#include <cmath>

#include "hstore.h"
#include "plan.h"

namespace admm {

namespace {

constexpr int T = kTile;  // 64
constexpr int KC = 32;    // K chunk staged in LDS

struct __align__(16) Smem {
  double2 A[T][KC + 1];
  double2 B[KC][T + 1];
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }

// Accumulators of one 64 x 64 complex tile product C += A B over K chunks of
// KC staged in LDS (sm.A: 64 x KC, sm.B: KC x 64).  Both kinds give
// zero(), chunk(sm) and each(fn): fn(row, col, value) once for every element
// the calling thread holds.
//
// AccV: FP64 vector FMAs, thread t holds rows t/16 + 16p, columns t%16 + 16q.
struct AccV {
  double2 v[4][4];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[p][q] = make_double2(0.0, 0.0);
  }
  __device__ __forceinline__ void chunk(const Smem& sm) {
    const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      double2 av[4], bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        av[q] = sm.A[tr + 16 * q][kk];
        bv[q] = sm.B[kk][tc + 16 * q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          v[p][q].x = fma(av[p].x, bv[q].x, v[p][q].x);
          v[p][q].x = fma(-av[p].y, bv[q].y, v[p][q].x);
          v[p][q].y = fma(av[p].x, bv[q].y, v[p][q].y);
          v[p][q].y = fma(av[p].y, bv[q].x, v[p][q].y);
        }
    }
  }
  template <class Fn>
  __device__ __forceinline__ void each(Fn fn) const {
    const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) fn(tr + 16 * p, tc + 16 * q, v[p][q]);
  }
};

// AccM: the FP64 matrix cores (v_mfma_f64_16x16x4f64: D[16x16] += A[16x4]
// B[4x16]; lane l supplies A[l%16][l/16] and B[l/16][l%16] and holds D rows
// l/16 + 4r, r = 0..3, of column l%16 -- the layout measured on gfx950).  Wave w computes the 32 x 32
// quarter at rows 32(w/2), columns 32(w%2) as 2 x 2 blocks of 16 x 16, each
// complex block as four real products: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.
typedef double v4d __attribute__((ext_vector_type(4)));
struct AccM {
  v4d re[2][2], im[2][2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) re[a][b] = im[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  __device__ __forceinline__ void chunk(const Smem& sm) {
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    const int r0 = 32 * (w / 2), c0 = 32 * (w % 2), i = l % 16, k = l / 16;
#pragma unroll 2
    for (int k4 = 0; k4 < KC; k4 += 4) {
      double2 av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = sm.A[r0 + 16 * a + i][k4 + k];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = sm.B[k4 + k][c0 + 16 * b + i];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].x, re[a][b], 0, 0, 0);
          re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[a].y, bv[b].y, re[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].y, im[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[b].x, im[a][b], 0, 0, 0);
        }
    }
  }
  template <class Fn>
  __device__ __forceinline__ void each(Fn fn) const {
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    const int r0 = 32 * (w / 2) + l / 16, c0 = 32 * (w % 2) + l % 16;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) fn(r0 + 16 * a + 4 * r, c0 + 16 * b, make_double2(re[a][b][r], im[a][b][r]));
  }
};

#if ADMM_SETUP_MFMA
using Acc = AccM;
#else
using Acc = AccV;
#endif
static_assert(kBlockThreads == 4 * kWave, "the tile accumulators assume four waves");

// acc += opA(X) opB(Y) over one 64-wide K range of FP64 tiles.
// X, Y point at tile origins in an ld-strided double2 matrix.
// conjTA: use X^H instead of X.  conjTB: use Y^H instead of Y.
template <bool conjTA, bool conjTB>
__device__ void tile_product(Smem& sm, const double2* __restrict__ X, const double2* __restrict__ Y,
                            int64_t ld, Acc& acc) {
  const int tid = threadIdx.x;
  for (int k0 = 0; k0 < T; k0 += KC) {
    __syncthreads();
    for (int e = tid; e < T * KC; e += kBlockThreads) {
      int r = e / KC, kk = e % KC;           // A[r][kk]
      sm.A[r][kk] = conjTA ? conjd(X[(int64_t)(k0 + kk) * ld + r]) : X[(int64_t)r * ld + k0 + kk];
      int kb = e / T, c = e % T;             // B[kb][c]
      sm.B[kb][c] = conjTB ? conjd(Y[(int64_t)c * ld + k0 + kb]) : Y[(int64_t)(k0 + kb) * ld + c];
    }
    __syncthreads();
    acc.chunk(sm);
  }
}

// ---------------------------------------------------------------------------
// Copy H (row-major m x n, complex64) into the block store with zero pads.
// grid = (rows, blocks); one workgroup per block row.
__global__ __launch_bounds__(kBlockThreads) void k_pack_c64(const float2* __restrict__ Hin, int64_t n,
                                                            const BlockDesc* __restrict__ blocks,
                                                            float2* __restrict__ Hout,
                                                            Control* ctl) {
  const BlockDesc d = blocks[blockIdx.y];
  const int r = blockIdx.x;
  if (r >= d.mi) return;
  const float2* src = Hin + (int64_t)(d.row0 + r) * n + d.col0;
  float2* dst = Hout + d.h_off + (int64_t)r * d.ld;
  bool bad = false;
  for (int c = threadIdx.x; c < d.ld; c += kBlockThreads) {
    float2 h = make_float2(0.f, 0.f);
    if (c < d.nj) {
      h = src[c];
      bad |= !(isfinite(h.x) && isfinite(h.y));
    }
    dst[c] = h;
  }
  if (bad) ctl->nonfinite = 1;
}

// Lower tiles of the block's Gram matrix in FP64 from the stored
// (dequantised) values: G = rho I + H H^H, m_i x m_i, for the inversion-lemma
// x-update (COLS = false), or A = rho I + H^H H, n_j x n_j, for the direct
// one (COLS = true; Sec. III-B, the original inversion of tall blocks).
// tiles[x] = {block, tile row, tile col, -} with tile row >= tile col.
template <class F, bool COLS>
__global__ __launch_bounds__(kBlockThreads) void k_gram_build(const int4* __restrict__ tiles,
                                                              const BlockDesc* __restrict__ blocks, HStore hs,
                                                              double rho, double2* __restrict__ A) {
  __shared__ Smem sm;
  const F f = MakeFmt<F>::make(hs);
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = blocks[t.x];
  const int tid = threadIdx.x;
  const int r0 = t.y * T, c0 = t.z * T;
  Acc acc;
  acc.zero();
  if constexpr (!COLS) {
    // G[r][c] = sum_k H[r][k] conj(H[c][k]): K runs along the rows
    for (int k0 = 0; k0 < d.nj; k0 += KC) {
      __syncthreads();
      for (int e = tid; e < T * KC; e += kBlockThreads) {
        int r = e / KC, kk = e % KC;
        sm.A[r][kk] = (r0 + r < d.mi) ? f.getd(d.h_off + (int64_t)(r0 + r) * d.ld + k0 + kk, d.row0 + r0 + r)
                                      : make_double2(0.0, 0.0);
        int kb = e / T, c = e % T;
        const double2 b = (c0 + c < d.mi) ? f.getd(d.h_off + (int64_t)(c0 + c) * d.ld + k0 + kb, d.row0 + c0 + c)
                                          : make_double2(0.0, 0.0);
        sm.B[kb][c] = make_double2(b.x, -b.y);
      }
      __syncthreads();
      acc.chunk(sm);
    }
  } else {
    // A[p][q] = sum_k conj(H[k][p]) H[k][q]: K runs down the columns; each
    // staged row segment is 64 consecutive elements of one stored row
    for (int k0 = 0; k0 < d.mi; k0 += KC) {
      __syncthreads();
      for (int e = tid; e < T * KC; e += kBlockThreads) {
        const int kk = e / T, q = e % T;
        const int row = k0 + kk;
        const int64_t re = d.h_off + (int64_t)row * d.ld;
        const double2 x = (row < d.mi && r0 + q < d.nj) ? f.getd(re + r0 + q, d.row0 + row) : make_double2(0.0, 0.0);
        sm.A[q][kk] = make_double2(x.x, -x.y);
        sm.B[kk][q] = (row < d.mi && c0 + q < d.nj) ? f.getd(re + c0 + q, d.row0 + row) : make_double2(0.0, 0.0);
      }
      __syncthreads();
      acc.chunk(sm);
    }
  }
  double2* Ab = A + d.f_off;
  acc.each([&](int rr, int cc, double2 val) {
    const int r = r0 + rr, c = c0 + cc;
    if (r >= d.gd || c >= d.gd) val = make_double2(r == c ? 1.0 : 0.0, 0.0);
    else if (r == c) val.x += rho;
    Ab[(int64_t)r * d.mt + c] = val;
  });
}

// ---------------------------------------------------------------------------
// Quantisers.  bfloat16: round to nearest even of the fp32 value.  fp8: OCP
// e4m3 (bias 7, max 448), round to nearest even, saturating, of x / s where
// s = (row max of |Re|, |Im|) / 448 in fp32 (1 for an all-zero row).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint8_t f32_to_e4m3_rne(float x) {
  const unsigned sign = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fabsf(x);
  if (!(a < 448.0f)) return (uint8_t)(sign | 0x7eu);
  if (a < 0.015625f) {                       // below 2^-6: multiples of 2^-9
    const float q = rintf(a * 512.0f);       // 0..8, 8 is the code of 2^-6
    return (uint8_t)(sign | (unsigned)q);
  }
  int e;
  const float fr = frexpf(a, &e);            // a = fr 2^e, fr in [0.5, 1)
  float mq = rintf((fr * 2.0f - 1.0f) * 8.0f);
  int E = e - 1;
  if (mq == 8.0f) {
    mq = 0.0f;
    E += 1;
  }
  unsigned code = ((unsigned)(E + 7) << 3) | (unsigned)mq;
  if (code > 0x7eu) code = 0x7eu;
  return (uint8_t)(sign | code);
}

// Row scales of the fp8 store: one workgroup per global row of the caller's H.
__global__ __launch_bounds__(kBlockThreads) void k_row_scale(const float2* __restrict__ Hin, int64_t n,
                                                             float* __restrict__ scale) {
  __shared__ float red[kBlockThreads / kWave];
  const int64_t row = blockIdx.x;
  float mx = 0.f;
  for (int64_t c = threadIdx.x; c < n; c += kBlockThreads) {
    const float2 h = Hin[row * n + c];
    mx = fmaxf(mx, fmaxf(fabsf(h.x), fabsf(h.y)));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = 0.f;
    for (int w = 0; w < kBlockThreads / kWave; ++w) m = fmaxf(m, red[w]);
    scale[row] = (m > 0.f) ? m / 448.0f : 1.0f;
  }
}

// Block store of the quantised planes with zero pads.  grid = (rows, blocks).
template <int STORAGE>
__global__ __launch_bounds__(kBlockThreads) void k_pack_q(const float2* __restrict__ Hin, int64_t n,
                                                          const BlockDesc* __restrict__ blocks, void* re_out,
                                                          void* im_out, const float* __restrict__ scale,
                                                          Control* ctl) {
  const BlockDesc d = blocks[blockIdx.y];
  const int r = blockIdx.x;
  if (r >= d.mi) return;
  const float2* src = Hin + (int64_t)(d.row0 + r) * n + d.col0;
  const int64_t o = d.h_off + (int64_t)r * d.ld;
  const float s = STORAGE == 2 ? scale[d.row0 + r] : 1.0f;
  bool bad = false;
  for (int c = threadIdx.x; c < d.ld; c += kBlockThreads) {
    float2 h = make_float2(0.f, 0.f);
    if (c < d.nj) {
      h = src[c];
      bad |= !(isfinite(h.x) && isfinite(h.y));
    }
    if (STORAGE == 1) {
      static_cast<uint16_t*>(re_out)[o + c] = f32_to_bf16_rne(h.x);
      static_cast<uint16_t*>(im_out)[o + c] = f32_to_bf16_rne(h.y);
    } else {
      static_cast<uint8_t*>(re_out)[o + c] = f32_to_e4m3_rne(h.x / s);
      static_cast<uint8_t*>(im_out)[o + c] = f32_to_e4m3_rne(h.y / s);
    }
  }
  if (bad) ctl->nonfinite = 1;
}

// Copy the block store back to dense m x n planes (complex64, or the raw
// bf16 / fp8 codes).  grid = (rows, blocks).
template <int STORAGE>
__global__ __launch_bounds__(kBlockThreads) void k_export_h(HStore hs, int64_t n,
                                                            const BlockDesc* __restrict__ blocks, void* re_out,
                                                            void* im_out) {
  const BlockDesc d = blocks[blockIdx.y];
  const int r = blockIdx.x;
  if (r >= d.mi) return;
  const int64_t o = d.h_off + (int64_t)r * d.ld, dst = (int64_t)(d.row0 + r) * n + d.col0;
  for (int c = threadIdx.x; c < d.nj; c += kBlockThreads) {
    if (STORAGE == 0) {
      static_cast<float2*>(re_out)[dst + c] = static_cast<const float2*>(hs.base)[o + c];
    } else if (STORAGE == 1) {
      static_cast<uint16_t*>(re_out)[dst + c] = static_cast<const uint16_t*>(hs.base)[o + c];
      static_cast<uint16_t*>(im_out)[dst + c] = static_cast<const uint16_t*>(hs.base_im)[o + c];
    } else {
      static_cast<uint8_t*>(re_out)[dst + c] = static_cast<const uint8_t*>(hs.base)[o + c];
      static_cast<uint8_t*>(im_out)[dst + c] = static_cast<const uint8_t*>(hs.base_im)[o + c];
    }
  }
}

// Cholesky of diagonal tile k (lower, in place).  One workgroup per block.
__global__ __launch_bounds__(kBlockThreads) void k_potrf_diag(int k, const BlockDesc* __restrict__ blocks,
                                                              double2* __restrict__ A, Control* ctl) {
  __shared__ double2 S[T][T + 1];
  const BlockDesc d = blocks[blockIdx.x];
  if (k * T >= d.mt) return;
  double2* Ak = A + d.f_off + (int64_t)(k * T) * d.mt + k * T;
  const int tid = threadIdx.x;
  for (int e = tid; e < T * T; e += kBlockThreads) S[e / T][e % T] = Ak[(int64_t)(e / T) * d.mt + e % T];
  __syncthreads();
  bool bad = false;
  for (int p = 0; p < T; ++p) {
    double dpp = S[p][p].x;
    if (!(dpp > 0.0) || !isfinite(dpp)) {
      bad = true;
      dpp = 1.0;
    }
    const double l = sqrt(dpp);
    __syncthreads();
    if (tid < T) {
      if (tid > p) S[tid][p] = make_double2(S[tid][p].x / l, S[tid][p].y / l);
      else if (tid == p) S[p][p] = make_double2(l, 0.0);
    }
    __syncthreads();
    for (int e = tid; e < T * T; e += kBlockThreads) {
      const int r = e / T, c = e % T;
      if (c > p && r >= c) {
        double2 x = cmul(S[r][p], conjd(S[c][p]));
        S[r][c].x -= x.x;
        S[r][c].y -= x.y;
      }
    }
    __syncthreads();
  }
  if (bad && tid == 0) ctl->notpd = 1;
  for (int e = tid; e < T * T; e += kBlockThreads) {
    const int r = e / T, c = e % T;
    Ak[(int64_t)r * d.mt + c] = (c <= r) ? S[r][c] : make_double2(0.0, 0.0);
  }
}

// Panel: A[i,k] <- A[i,k] L[k,k]^{-H} for every tile i > k.
// grid = (tile rows below k of the largest block, blocks).
__global__ __launch_bounds__(kBlockThreads) void k_trsm_panel(int k, const BlockDesc* __restrict__ blocks,
                                                              double2* __restrict__ A) {
  __shared__ double2 L[T][T + 1];
  __shared__ double2 X[T][T + 1];
  const BlockDesc d = blocks[blockIdx.y];
  const int i = k + 1 + blockIdx.x;
  if (i * T >= d.mt) return;
  const int tid = threadIdx.x;
  const double2* Lk = A + d.f_off + (int64_t)(k * T) * d.mt + k * T;
  double2* Ai = A + d.f_off + (int64_t)(i * T) * d.mt + k * T;
  for (int e = tid; e < T * T; e += kBlockThreads) {
    L[e / T][e % T] = Lk[(int64_t)(e / T) * d.mt + e % T];
    X[e / T][e % T] = Ai[(int64_t)(e / T) * d.mt + e % T];
  }
  __syncthreads();
  // Solve X L^H = A column by column: X[:,p] = (A[:,p] - sum_{q<p} X[:,q] conj(L[p][q])) / L[p][p]
  for (int p = 0; p < T; ++p) {
    if (tid < T) {
      const double l = L[p][p].x;
      X[tid][p] = make_double2(X[tid][p].x / l, X[tid][p].y / l);
    }
    __syncthreads();
    for (int e = tid; e < T * T; e += kBlockThreads) {
      const int r = e / T, q = e % T;
      if (q > p) {
        double2 x = cmul(X[r][p], conjd(L[q][p]));
        X[r][q].x -= x.x;
        X[r][q].y -= x.y;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < T * T; e += kBlockThreads) Ai[(int64_t)(e / T) * d.mt + e % T] = X[e / T][e % T];
}

__device__ __forceinline__ void tri_index(int p, int& a, int& b) {
  // p -> (a, b) with 0 <= b <= a, p = a(a+1)/2 + b
  int aa = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while ((aa + 1) * (aa + 2) / 2 <= p) ++aa;
  while (aa * (aa + 1) / 2 > p) --aa;
  a = aa;
  b = p - aa * (aa + 1) / 2;
}

// Trailing update A[i,l] -= A[i,k] A[l,k]^H for k < l <= i.
// grid = (pairs of the largest block, blocks).
__global__ __launch_bounds__(kBlockThreads) void k_herk_trail(int k, const BlockDesc* __restrict__ blocks,
                                                              double2* __restrict__ A) {
  __shared__ Smem sm;
  const BlockDesc d = blocks[blockIdx.y];
  const int nt = d.mt / T - k - 1;
  int ia, la;
  tri_index(blockIdx.x, ia, la);
  if (ia >= nt) return;
  const int i = k + 1 + ia, l = k + 1 + la;
  double2* Ab = A + d.f_off;
  Acc acc;
  acc.zero();
  tile_product<false, true>(sm, Ab + (int64_t)(i * T) * d.mt + k * T, Ab + (int64_t)(l * T) * d.mt + k * T,
                            d.mt, acc);
  double2* C = Ab + (int64_t)(i * T) * d.mt + l * T;
  acc.each([&](int r, int c, double2 v) {
    double2& o = C[(int64_t)r * d.mt + c];
    o.x -= v.x;
    o.y -= v.y;
  });
}

// W[k,k] = L[k,k]^{-1} (lower).  grid = (tiles of the largest block, blocks).
__global__ __launch_bounds__(kBlockThreads) void k_trtri_diag(const BlockDesc* __restrict__ blocks,
                                                              const double2* __restrict__ A,
                                                              double2* __restrict__ W) {
  __shared__ double2 L[T][T + 1];
  __shared__ double2 X[T][T + 1];
  const BlockDesc d = blocks[blockIdx.y];
  const int k = blockIdx.x;
  if (k * T >= d.mt) return;
  const int tid = threadIdx.x;
  const double2* Lk = A + d.f_off + (int64_t)(k * T) * d.mt + k * T;
  for (int e = tid; e < T * T; e += kBlockThreads) {
    const int r = e / T, c = e % T;
    L[r][c] = Lk[(int64_t)r * d.mt + c];
    X[r][c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // Forward substitution L X = I, row by row: X[p,:] /= L[p][p]; X[r,:] -= L[r][p] X[p,:] for r > p.
  for (int p = 0; p < T; ++p) {
    if (tid < T) {
      const double l = L[p][p].x;
      X[p][tid] = make_double2(X[p][tid].x / l, X[p][tid].y / l);
    }
    __syncthreads();
    for (int e = tid; e < T * T; e += kBlockThreads) {
      const int r = e / T, c = e % T;
      if (r > p) {
        double2 x = cmul(L[r][p], X[p][c]);
        X[r][c].x -= x.x;
        X[r][c].y -= x.y;
      }
    }
    __syncthreads();
  }
  double2* Wk = W + d.f_off + (int64_t)(k * T) * d.mt + k * T;
  for (int e = tid; e < T * T; e += kBlockThreads) {
    const int r = e / T, c = e % T;
    Wk[(int64_t)r * d.mt + c] = (c <= r) ? X[r][c] : make_double2(0.0, 0.0);
  }
}

// Off-diagonal tiles of W = L^{-1} at distance dist below the diagonal:
// W[k+dist,k] = -W[k+dist,k+dist] sum_{l=k}^{k+dist-1} L[k+dist,l] W[l,k].
// grid = (tiles of the largest block, blocks).
__global__ __launch_bounds__(kBlockThreads) void k_trtri_off(int dist, const BlockDesc* __restrict__ blocks,
                                                             const double2* __restrict__ A,
                                                             double2* __restrict__ W) {
  __shared__ Smem sm;
  __shared__ double2 Sx[T][T + 1];
  const BlockDesc d = blocks[blockIdx.y];
  const int k = blockIdx.x, i = k + dist;
  if (i * T >= d.mt) return;
  const int tid = threadIdx.x;
  const double2* Ab = A + d.f_off;
  double2* Wb = W + d.f_off;
  Acc acc;
  acc.zero();
  for (int l = k; l < i; ++l)
    tile_product<false, false>(sm, Ab + (int64_t)(i * T) * d.mt + l * T, Wb + (int64_t)(l * T) * d.mt + k * T,
                               d.mt, acc);
  acc.each([&](int r, int c, double2 v) { Sx[r][c] = v; });
  acc.zero();
  const double2* Wii = Wb + (int64_t)(i * T) * d.mt + i * T;
  for (int k0 = 0; k0 < T; k0 += KC) {
    __syncthreads();
    for (int e = tid; e < T * KC; e += kBlockThreads) {
      const int r = e / KC, kk = e % KC;
      sm.A[r][kk] = Wii[(int64_t)r * d.mt + k0 + kk];
      const int kb = e / T, c = e % T;
      sm.B[kb][c] = Sx[k0 + kb][c];
    }
    __syncthreads();
    acc.chunk(sm);
  }
  double2* C = Wb + (int64_t)(i * T) * d.mt + k * T;
  acc.each([&](int r, int c, double2 v) { C[(int64_t)r * d.mt + c] = make_double2(-v.x, -v.y); });
}

// G^{-1} = W^H W: tile (i,l), l <= i, = sum_{k>=i} W[k,i]^H W[k,l], written as
// complex64 to the block's packed lower-tile store (entries outside the
// block's mi x mi part are zero).  tiles[x] = {block, i, l, -}.
__global__ __launch_bounds__(kBlockThreads) void k_lauum(const int4* __restrict__ tiles,
                                                         const BlockDesc* __restrict__ blocks,
                                                         const double2* __restrict__ W,
                                                         float2* __restrict__ Ginv) {
  __shared__ Smem sm;
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = blocks[t.x];
  const int i = t.y, l = t.z, nt = d.mt / T;
  const double2* Wb = W + d.f_off;
  Acc acc;
  acc.zero();
  for (int k = i; k < nt; ++k)
    tile_product<true, false>(sm, Wb + (int64_t)(k * T) * d.mt + i * T, Wb + (int64_t)(k * T) * d.mt + l * T,
                              d.mt, acc);
  float2* G = Ginv + d.gi_off + (int64_t)(i * (i + 1) / 2 + l) * (T * T);
  acc.each([&](int rr, int cc, double2 v) {
    const bool in = i * T + rr < d.gd && l * T + cc < d.gd;
    G[rr * T + cc] = in ? make_float2((float)v.x, (float)v.y) : make_float2(0.f, 0.f);
  });
}

}  // namespace

hipError_t launch_pack_c64(const float2* Hin, int64_t n, const BlockDesc* blocks, int nblocks, int max_rows,
                           float2* Hout, Control* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_c64, dim3(max_rows, nblocks), dim3(kBlockThreads), 0, st, Hin, n, blocks, Hout,
                     ctl);
  return hipGetLastError();
}

hipError_t launch_gram_build(const Geometry& geo, const BlockDesc* dblocks, const int4* t_gram,
                             const HStore& hs, double rho, double2* A, hipStream_t st) {
  const dim3 grid((unsigned)geo.t_gram.size()), blk(kBlockThreads);
#define GRAM_BUILD(F)                                                                                   \
  do {                                                                                                  \
    if (geo.direct)                                                                                     \
      hipLaunchKernelGGL((k_gram_build<F, true>), grid, blk, 0, st, t_gram, dblocks, hs, rho, A);       \
    else                                                                                                \
      hipLaunchKernelGGL((k_gram_build<F, false>), grid, blk, 0, st, t_gram, dblocks, hs, rho, A);      \
  } while (0)
  switch (hs.storage) {
    case 0: GRAM_BUILD(FmtC64); break;
    case 1: GRAM_BUILD(FmtBF16); break;
    default: GRAM_BUILD(FmtFP8); break;
  }
#undef GRAM_BUILD
  return hipGetLastError();
}

hipError_t launch_pack_quant(const float2* Hin, int64_t m, int64_t n, const BlockDesc* blocks, int nblocks,
                             int max_rows, const HStore& hs, Control* ctl, hipStream_t st) {
  void* re = const_cast<void*>(hs.base);
  void* im = const_cast<void*>(hs.base_im);
  float* sc = const_cast<float*>(hs.row_scale);
  if (hs.storage == 2) {
    hipLaunchKernelGGL(k_row_scale, dim3((unsigned)m), dim3(kBlockThreads), 0, st, Hin, n, sc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pack_q<2>, dim3(max_rows, nblocks), dim3(kBlockThreads), 0, st, Hin, n, blocks, re, im,
                       sc, ctl);
  } else {
    hipLaunchKernelGGL(k_pack_q<1>, dim3(max_rows, nblocks), dim3(kBlockThreads), 0, st, Hin, n, blocks, re, im,
                       sc, ctl);
  }
  return hipGetLastError();
}

hipError_t launch_export_h(const HStore& hs, int64_t n, const BlockDesc* blocks, int nblocks, int max_rows,
                           void* re_out, void* im_out, hipStream_t st) {
  const dim3 grid(max_rows, nblocks);
  switch (hs.storage) {
    case 0: hipLaunchKernelGGL(k_export_h<0>, grid, dim3(kBlockThreads), 0, st, hs, n, blocks, re_out, im_out); break;
    case 1: hipLaunchKernelGGL(k_export_h<1>, grid, dim3(kBlockThreads), 0, st, hs, n, blocks, re_out, im_out); break;
    default: hipLaunchKernelGGL(k_export_h<2>, grid, dim3(kBlockThreads), 0, st, hs, n, blocks, re_out, im_out); break;
  }
  return hipGetLastError();
}

hipError_t launch_cholesky_inverse(const Geometry& geo, const BlockDesc* dblocks, const int4* t_gram,
                                   double2* A, double2* W, float2* Ginv, Control* ctl, hipStream_t st) {
  const int nb = (int)geo.blocks.size();
  const int NT = geo.max_mt / T;
  hipError_t e;
  for (int k = 0; k < NT; ++k) {
    hipLaunchKernelGGL(k_potrf_diag, dim3(nb), dim3(kBlockThreads), 0, st, k, dblocks, A, ctl);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int below = NT - k - 1;
    if (below > 0) {
      hipLaunchKernelGGL(k_trsm_panel, dim3(below, nb), dim3(kBlockThreads), 0, st, k, dblocks, A);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_herk_trail, dim3(below * (below + 1) / 2, nb), dim3(kBlockThreads), 0, st, k,
                         dblocks, A);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_trtri_diag, dim3(NT, nb), dim3(kBlockThreads), 0, st, dblocks, A, W);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int dist = 1; dist < NT; ++dist) {
    hipLaunchKernelGGL(k_trtri_off, dim3(NT - dist, nb), dim3(kBlockThreads), 0, st, dist, dblocks, A, W);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // the lower tile pairs are the same as those of the Gram build
  hipLaunchKernelGGL(k_lauum, dim3((unsigned)geo.t_gram.size()), dim3(kBlockThreads), 0, st, t_gram,
                     dblocks, W, Ginv);
  return hipGetLastError();
}

}  // namespace admm
