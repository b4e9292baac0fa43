// Streaming complex matrix-vector device routines shared by the forward
// iteration and its adjoint (included by k_iter.hip and k_adj.hip).
#pragma once

#include "hstore.h"
#include "plan.h"

namespace admm {

// acc += a * b  (complex)
__device__ __forceinline__ void cmac(float& ar, float& ai, float a_r, float a_i, float b_r,
                                     float b_i) {
  ar = fmaf(a_r, b_r, ar);
  ar = fmaf(-a_i, b_i, ar);
  ai = fmaf(a_r, b_i, ai);
  ai = fmaf(a_i, b_r, ai);
}
// acc += conj(a) * b
__device__ __forceinline__ void cmacc(float& ar, float& ai, float a_r, float a_i, float b_r,
                                      float b_i) {
  ar = fmaf(a_r, b_r, ar);
  ar = fmaf(a_i, b_i, ar);
  ai = fmaf(a_r, b_i, ai);
  ai = fmaf(-a_i, b_r, ai);
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}
__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// Rows in flight per wave in the adjoint (column) product.
template <class F> struct ColUnroll {
  static constexpr int U = F::CPL == 2 ? ADMM_COLS_UNROLL_C64 : ADMM_COLS_UNROLL_NARROW;
};
// H row products: rows per wave and lane loads in flight per row (8 rows
// for complex64, 4 for the narrow formats, whose wide lane loads fill more
// registers per row; measured), and how the row
// sums are closed: the reduce-scatter of rows_reduce measured faster for
// bfloat16, one wave sum per row for the complex64 and fp8 forms.
template <class F> struct HRows {
  static constexpr int R = F::CPL == 2 ? ADMM_ROWS_C64 : ADMM_ROWS_NARROW;
  static constexpr int U = F::CPL == 2 ? ADMM_UNROLL_C64 : ADMM_UNROLL_NARROW;
  static constexpr bool SCATTER = F::CPL == 8;
  // Load the operands of each row's epilogue (row scale, g, the other
  // sections' estimates) before streaming the row, so that their latency
  // overlaps the stream: this matters where a row is only a few lane loads
  // long (narrow formats).
  static constexpr bool PREFETCH = F::CPL == 2 ? ADMM_EPI_PREFETCH_C64 : ADMM_EPI_PREFETCH_NARROW;
};

// Dot products of R consecutive rows of a stored matrix with the complex
// vector x (FP32, padded, in the lane-permuted layout of cperm).  e0: element offset of the first row, ld: row
// stride in elements, nl: lane loads per row (ceil(ncols / CPL)), rows >=
// nvalid are clamped.  Lane l walks lane loads l, l+64, ... with U of them
// per row in flight.  Returns per-lane partial sums; rows_reduce closes them.
template <class F, int R, int U>
__device__ __forceinline__ void rows_dot(const F& f, int64_t e0, int64_t ld, int nvalid,
                                         const float4* __restrict__ x, int nl, float (&acc)[R][2]) {
  constexpr int CPL = F::CPL, X4 = CPL / 2;
  const int lane = threadIdx.x & (kWave - 1);
  typename F::Row rows[R];
#pragma unroll
  for (int rr = 0; rr < R; ++rr) {
    rows[rr] = f.row(e0 + (int64_t)(rr < nvalid ? rr : (nvalid - 1)) * ld);
    acc[rr][0] = 0.f;
    acc[rr][1] = 0.f;
  }
  auto consume = [&](const typename F::Raw& raw, const float4 (&xv)[X4], int rr) {
    float hr[CPL], hi[CPL];
    F::decode(raw, hr, hi);
#pragma unroll
    for (int q = 0; q < X4; ++q) {
      cmac(acc[rr][0], acc[rr][1], hr[2 * q], hi[2 * q], xv[q].x, xv[q].y);
      cmac(acc[rr][0], acc[rr][1], hr[2 * q + 1], hi[2 * q + 1], xv[q].z, xv[q].w);
    }
  };
  int c = lane;
  for (; c + (U - 1) * kWave < nl; c += U * kWave) {
    typename F::Raw raw[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int rr = 0; rr < R; ++rr) raw[u][rr] = F::load(rows[rr], (uint32_t)(c + u * kWave));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float4 xv[X4];
#pragma unroll
      for (int q = 0; q < X4; ++q) xv[q] = x[(((int64_t)((c + u * kWave) >> 6) * X4 + q) << 6) + ((c + u * kWave) & 63)];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) consume(raw[u][rr], xv, rr);
    }
  }
  for (; c < nl; c += kWave) {
    typename F::Raw raw[R];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) raw[rr] = F::load(rows[rr], (uint32_t)c);
    float4 xv[X4];
#pragma unroll
    for (int q = 0; q < X4; ++q) xv[q] = x[(((int64_t)(c >> 6) * X4 + q) << 6) + (c & 63)];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) consume(raw[rr], xv, rr);
  }
}

// Closes R row sums held by every lane of a wave (R a power of two <= 64).
// Afterwards every lane holds the total of row rows_reduce_row<R>(lane).
// Scatter: a reduce-scatter over lane bits 5, 4, ... (each step a lane keeps
// half of its rows and sends the other half across) and an all-reduce over
// the remaining low bits, 2(R - 1) + 2(6 - log2 R) shuffles; otherwise one
// butterfly wave sum per row, 12 R shuffles.  Both in a fixed order.
template <int R>
__device__ __forceinline__ int rows_reduce_row(int lane) {
  constexpr int LR = R >= 64 ? 6 : R >= 32 ? 5 : R >= 16 ? 4 : R >= 8 ? 3 : R >= 4 ? 2 : R >= 2 ? 1 : 0;
  return LR == 0 ? 0 : (lane >> (6 - LR)) & (R - 1);
}
template <int R, bool Scatter>
__device__ __forceinline__ void rows_reduce(float (&acc)[R][2], float& outr, float& outi) {
  static_assert(R >= 1 && R <= 64 && (R & (R - 1)) == 0, "R must be a power of two");
  if (!Scatter) {
    const int lane = threadIdx.x & (kWave - 1);
    const int want = rows_reduce_row<R>(lane);
    float r = 0.f, i = 0.f;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const float sr = wave_sum(acc[rr][0]), si = wave_sum(acc[rr][1]);
      if (rr == want) { r = sr; i = si; }
    }
    outr = r;
    outi = i;
    return;
  }
  constexpr int LR = R >= 64 ? 6 : R >= 32 ? 5 : R >= 16 ? 4 : R >= 8 ? 3 : R >= 4 ? 2 : R >= 2 ? 1 : 0;
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int st = 0; st < LR; ++st) {
    const int mask = 32 >> st;
    const int half = R >> (st + 1);
    const bool hi = (lane & mask) != 0;
#pragma unroll
    for (int q = 0; q < half; ++q) {
      const float kr = hi ? acc[q + half][0] : acc[q][0], ki = hi ? acc[q + half][1] : acc[q][1];
      const float sr = hi ? acc[q][0] : acc[q + half][0], si = hi ? acc[q][1] : acc[q + half][1];
      acc[q][0] = kr + __shfl_xor(sr, mask, kWave);
      acc[q][1] = ki + __shfl_xor(si, mask, kWave);
    }
  }
  float r = acc[0][0], i = acc[0][1];
#pragma unroll
  for (int mask = 32 >> LR; mask >= 1; mask >>= 1) {
    r += __shfl_xor(r, mask, kWave);
    i += __shfl_xor(i, mask, kWave);
  }
  outr = r;
  outi = i;
}

// Adjoint (column) product of one workgroup: columns c*CPL .. c*CPL+CPL-1 of
// block d (c = first lane load + lane), rows [rb, re) of chunk t.z, with
// out[col] = sum_rows conj(H[row, col]) * s_row * y[row] (s_row the row
// scale).  One lane load per lane, 64 lane loads per workgroup; the four
// waves take every fourth row and are added through LDS in a fixed order.
// y and out point at the block's segment (row / column space).
template <class F>
__device__ __forceinline__ void cols_partial(const F& f, const BlockDesc& d, const int4& t, int KH,
                                             const float2* __restrict__ y, float2* __restrict__ out,
                                             float (&red)[kBlockThreads / kWave - 1][2 * F::CPL][kWave]) {
  constexpr int CPL = F::CPL, U = ColUnroll<F>::U;
  constexpr int NW = kBlockThreads / kWave;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int c = t.y + lane;
  const int nl = (d.nj + CPL - 1) / CPL;
  const bool active = c < nl;
  const int rc = (d.mi + KH - 1) / KH;
  const int rb = min(d.mi, t.z * rc), re = min(d.mi, rb + rc);
  float accr[CPL], acci[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) accr[k] = acci[k] = 0.f;
  auto consume = [&](const typename F::Raw& raw, float2 yv) {
    float hr[CPL], hi[CPL];
    F::decode(raw, hr, hi);
#pragma unroll
    for (int k = 0; k < CPL; ++k) cmacc(accr[k], acci[k], hr[k], hi[k], yv.x, yv.y);
  };
  if (active) {
    const int64_t col_e = d.h_off + (int64_t)c * CPL;
    int r = rb + wave;
    for (; r + NW * (U - 1) < re; r += NW * U) {
      typename F::Raw raw[U];
      float2 yv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) raw[u] = f.load(col_e + (int64_t)(r + NW * u) * d.ld);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int rr = r + NW * u;
        const float sc = f.row_scale(d.row0 + rr);
        yv[u] = make_float2(sc * y[rr].x, sc * y[rr].y);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) consume(raw[u], yv[u]);
    }
    for (; r < re; r += NW) {
      const typename F::Raw raw = f.load(col_e + (int64_t)r * d.ld);
      const float sc = f.row_scale(d.row0 + r);
      consume(raw, make_float2(sc * y[r].x, sc * y[r].y));
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      red[wave - 1][2 * k][lane] = accr[k];
      red[wave - 1][2 * k + 1][lane] = acci[k];
    }
  }
  __syncthreads();
  if (wave == 0 && active) {
#pragma unroll
    for (int w = 0; w < NW - 1; ++w)
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        accr[k] += red[w][2 * k][lane];
        acci[k] += red[w][2 * k + 1][lane];
      }
    float4* o4 = reinterpret_cast<float4*>(out + (int64_t)c * CPL);
#pragma unroll
    for (int q = 0; q < CPL / 2; ++q)
      o4[q] = make_float4(accr[2 * q], acci[2 * q], accr[2 * q + 1], acci[2 * q + 1]);
  }
}

// One 64 x 64 tile G of a packed Hermitian matrix (lower tile (ta, tb),
// ta >= tb) applied both ways: out_ab = G x_b and, off the diagonal,
// out_ba = G^H x_a.  256 threads; thread (wave w, lane l) holds a 4 x 4
// sub-block: rows 16w + 4(l >> 4) + {0..3} and columns {2b, 2b+1, 32+2b,
// 33+2b} with b = l & 15, so each 16-byte load instruction of a wave reads
// four contiguous 256-byte row segments.  Row sums close over the 16 lanes
// of a row group by a reduce-scatter (xor 8, 4) and an all-reduce (xor 2, 1);
// column sums close over the wave by a reduce-scatter (xor 32, 16) and over
// the 4 waves through 2 KB of LDS, always in the same order.
// Operands of one tile in the thread layout of gram_tile_compute: the tile
// entries and the thread's pieces of x_b (columns) and x_a (rows).
struct GramOps {
  float4 h[4][2];
  float4 xb0, xb1, xa0, xa1;
};
__device__ __forceinline__ void gram_tile_load(const float2* __restrict__ G, const float2* __restrict__ xa,
                                               const float2* __restrict__ xb, GramOps& o) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, b = l & 15;
  const int r0 = 16 * w + 4 * (l >> 4);
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
#pragma unroll
    for (int hf = 0; hf < 2; ++hf)
      o.h[rr][hf] = ldnt4(reinterpret_cast<const float4*>(G + (r0 + rr) * 64 + 32 * hf + 2 * b));
  o.xb0 = *reinterpret_cast<const float4*>(xb + 2 * b);
  o.xb1 = *reinterpret_cast<const float4*>(xb + 32 + 2 * b);
  o.xa0 = *reinterpret_cast<const float4*>(xa + r0);
  o.xa1 = *reinterpret_cast<const float4*>(xa + r0 + 2);
}

// Row sums of one tile in the thread's 4 x 4 sub-block, added to (pr, pi):
// rows r0 + rr of G x_b over this thread's four columns.
__device__ __forceinline__ void gram_rows_acc(const GramOps& o, float (&pr)[4], float (&pi)[4]) {
  const float4 (&h)[4][2] = o.h;
  const float4 xb0 = o.xb0, xb1 = o.xb1;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    cmac(pr[rr], pi[rr], h[rr][0].x, h[rr][0].y, xb0.x, xb0.y);
    cmac(pr[rr], pi[rr], h[rr][0].z, h[rr][0].w, xb0.z, xb0.w);
    cmac(pr[rr], pi[rr], h[rr][1].x, h[rr][1].y, xb1.x, xb1.y);
    cmac(pr[rr], pi[rr], h[rr][1].z, h[rr][1].w, xb1.z, xb1.w);
  }
}
// Column sums of one tile in the thread's sub-block, added to (cr, ci):
// column slot k (k: 0 -> 2b, 1 -> 2b+1, 2 -> 32+2b, 3 -> 33+2b) of G^H x_a
// over this thread's four rows.
__device__ __forceinline__ void gram_cols_acc(const GramOps& o, float (&cr)[4], float (&ci)[4]) {
  const float4 (&h)[4][2] = o.h;
  const float4 xa0 = o.xa0, xa1 = o.xa1;
  const float xr[4] = {xa0.x, xa0.z, xa1.x, xa1.z}, xi[4] = {xa0.y, xa0.w, xa1.y, xa1.w};
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    cmacc(cr[0], ci[0], h[rr][0].x, h[rr][0].y, xr[rr], xi[rr]);
    cmacc(cr[1], ci[1], h[rr][0].z, h[rr][0].w, xr[rr], xi[rr]);
    cmacc(cr[2], ci[2], h[rr][1].x, h[rr][1].y, xr[rr], xi[rr]);
    cmacc(cr[3], ci[3], h[rr][1].z, h[rr][1].w, xr[rr], xi[rr]);
  }
}
// Closes the row sums over the 16 lanes of each row group (reduce-scatter
// xor 8, 4, all-reduce xor 2, 1); lanes with (l & 3) == 0 write out[row].
__device__ __forceinline__ void gram_rows_store(const float (&pr)[4], const float (&pi)[4],
                                                float2* __restrict__ out) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int r0 = 16 * w + 4 * (l >> 4);
  // xor 8: keep rows {2s, 2s+1}, s = bit 3 of the lane
  const bool s = (l & 8) != 0;
  float k0r = s ? pr[2] : pr[0], k0i = s ? pi[2] : pi[0];
  float k1r = s ? pr[3] : pr[1], k1i = s ? pi[3] : pi[1];
  const float o0r = s ? pr[0] : pr[2], o0i = s ? pi[0] : pi[2];
  const float o1r = s ? pr[1] : pr[3], o1i = s ? pi[1] : pi[3];
  k0r += __shfl_xor(o0r, 8, kWave);
  k0i += __shfl_xor(o0i, 8, kWave);
  k1r += __shfl_xor(o1r, 8, kWave);
  k1i += __shfl_xor(o1i, 8, kWave);
  // xor 4: keep row 2s + t, t = bit 2
  const bool t = (l & 4) != 0;
  float rr_ = t ? k1r : k0r, ri_ = t ? k1i : k0i;
  rr_ += __shfl_xor(t ? k0r : k1r, 4, kWave);
  ri_ += __shfl_xor(t ? k0i : k1i, 4, kWave);
  rr_ += __shfl_xor(rr_, 2, kWave);
  ri_ += __shfl_xor(ri_, 2, kWave);
  rr_ += __shfl_xor(rr_, 1, kWave);
  ri_ += __shfl_xor(ri_, 1, kWave);
  if ((l & 3) == 0) out[r0 + 2 * (int)s + (int)t] = make_float2(rr_, ri_);
}
// Closes the column sums over the wave (reduce-scatter xor 32, 16) and over
// the 4 waves through `red` in a fixed order; threads < 64 write out[col].
// Every thread of the workgroup must call it (it holds a barrier); `red` is
// read after that barrier, so a second call needs a barrier before it.
__device__ __forceinline__ void gram_cols_store(const float (&cr)[4], const float (&ci)[4],
                                                float2* __restrict__ out, float2 (&red)[4][64]) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, b = l & 15;
  // xor 32: keep slots {2u, 2u+1}, u = bit 5
  const bool u = (l & 32) != 0;
  float k0r = u ? cr[2] : cr[0], k0i = u ? ci[2] : ci[0];
  float k1r = u ? cr[3] : cr[1], k1i = u ? ci[3] : ci[1];
  const float o0r = u ? cr[0] : cr[2], o0i = u ? ci[0] : ci[2];
  const float o1r = u ? cr[1] : cr[3], o1i = u ? ci[1] : ci[3];
  k0r += __shfl_xor(o0r, 32, kWave);
  k0i += __shfl_xor(o0i, 32, kWave);
  k1r += __shfl_xor(o1r, 32, kWave);
  k1i += __shfl_xor(o1i, 32, kWave);
  // xor 16: keep slot 2u + v, v = bit 4, i.e. column 32u + 2b + v
  const bool v = (l & 16) != 0;
  float sr = v ? k1r : k0r, si = v ? k1i : k0i;
  sr += __shfl_xor(v ? k0r : k1r, 16, kWave);
  si += __shfl_xor(v ? k0i : k1i, 16, kWave);
  red[w][32 * (int)u + 2 * b + (int)v] = make_float2(sr, si);
  __syncthreads();
  if (tid < 64) {
    const float2 q0 = red[0][tid], q1 = red[1][tid], q2 = red[2][tid], q3 = red[3][tid];
    out[tid] = make_float2(((q0.x + q1.x) + q2.x) + q3.x, ((q0.y + q1.y) + q2.y) + q3.y);
  }
}

__device__ __forceinline__ void gram_tile_compute(const GramOps& o, bool diag, float2* __restrict__ out_ab,
                                                  float2* __restrict__ out_ba, float2 (&red)[4][64]) {
  float pr[4] = {0.f, 0.f, 0.f, 0.f}, pi[4] = {0.f, 0.f, 0.f, 0.f};
  gram_rows_acc(o, pr, pi);
  gram_rows_store(pr, pi, out_ab);
  if (diag) return;
  float cr[4] = {0.f, 0.f, 0.f, 0.f}, ci[4] = {0.f, 0.f, 0.f, 0.f};
  gram_cols_acc(o, cr, ci);
  gram_cols_store(cr, ci, out_ba, red);
}

// The same products with the tile stored as bfloat16 pairs (32-bit word per
// complex entry: Re in the low half, Im in the high half).  Thread (wave w,
// lane l) holds rows 16w + 4(l >> 4) + {0..3} and the four contiguous columns
// 4b .. 4b+3 (b = l & 15): one 16-byte load per row, 16 lanes covering a
// 256-byte row.  The reductions are those of gram_tile_compute with column
// slot k mapped to column 4b + k.
__device__ __forceinline__ void bf16pair(uint32_t w, float& re, float& im) {
  re = __uint_as_float(w << 16);
  im = __uint_as_float(w & 0xffff0000u);
}
__device__ __forceinline__ void gram_tile_apply_bf16(const uint32_t* __restrict__ G, const float2* __restrict__ xa,
                                                     const float2* __restrict__ xb, bool diag,
                                                     float2* __restrict__ out_ab, float2* __restrict__ out_ba,
                                                     float2 (&red)[4][64]) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, b = l & 15;
  const int r0 = 16 * w + 4 * (l >> 4);
  uint4 h[4];
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const v4u_t q = __builtin_nontemporal_load(reinterpret_cast<const v4u_t*>(G + (r0 + rr) * 64 + 4 * b));
    h[rr] = make_uint4(q.x, q.y, q.z, q.w);
  }
  const float4 xb0 = *reinterpret_cast<const float4*>(xb + 4 * b);
  const float4 xb1 = *reinterpret_cast<const float4*>(xb + 4 * b + 2);
  const float xbr[4] = {xb0.x, xb0.z, xb1.x, xb1.z}, xbi[4] = {xb0.y, xb0.w, xb1.y, xb1.w};
  float gr[4][4], gi[4][4];
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    bf16pair(h[rr].x, gr[rr][0], gi[rr][0]);
    bf16pair(h[rr].y, gr[rr][1], gi[rr][1]);
    bf16pair(h[rr].z, gr[rr][2], gi[rr][2]);
    bf16pair(h[rr].w, gr[rr][3], gi[rr][3]);
  }
  float pr[4], pi[4];
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    pr[rr] = 0.f;
    pi[rr] = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) cmac(pr[rr], pi[rr], gr[rr][k], gi[rr][k], xbr[k], xbi[k]);
  }
  {
    const bool s = (l & 8) != 0;
    float k0r = s ? pr[2] : pr[0], k0i = s ? pi[2] : pi[0];
    float k1r = s ? pr[3] : pr[1], k1i = s ? pi[3] : pi[1];
    const float o0r = s ? pr[0] : pr[2], o0i = s ? pi[0] : pi[2];
    const float o1r = s ? pr[1] : pr[3], o1i = s ? pi[1] : pi[3];
    k0r += __shfl_xor(o0r, 8, kWave);
    k0i += __shfl_xor(o0i, 8, kWave);
    k1r += __shfl_xor(o1r, 8, kWave);
    k1i += __shfl_xor(o1i, 8, kWave);
    const bool t = (l & 4) != 0;
    float rr_ = t ? k1r : k0r, ri_ = t ? k1i : k0i;
    rr_ += __shfl_xor(t ? k0r : k1r, 4, kWave);
    ri_ += __shfl_xor(t ? k0i : k1i, 4, kWave);
    rr_ += __shfl_xor(rr_, 2, kWave);
    ri_ += __shfl_xor(ri_, 2, kWave);
    rr_ += __shfl_xor(rr_, 1, kWave);
    ri_ += __shfl_xor(ri_, 1, kWave);
    if ((l & 3) == 0) out_ab[r0 + 2 * (int)s + (int)t] = make_float2(rr_, ri_);
  }
  if (diag) return;
  const float4 xa0 = *reinterpret_cast<const float4*>(xa + r0);
  const float4 xa1 = *reinterpret_cast<const float4*>(xa + r0 + 2);
  const float xr[4] = {xa0.x, xa0.z, xa1.x, xa1.z}, xi[4] = {xa0.y, xa0.w, xa1.y, xa1.w};
  float cr[4] = {0.f, 0.f, 0.f, 0.f}, ci[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
#pragma unroll
    for (int k = 0; k < 4; ++k) cmacc(cr[k], ci[k], gr[rr][k], gi[rr][k], xr[rr], xi[rr]);
  const bool u = (l & 32) != 0;
  float k0r = u ? cr[2] : cr[0], k0i = u ? ci[2] : ci[0];
  float k1r = u ? cr[3] : cr[1], k1i = u ? ci[3] : ci[1];
  const float o0r = u ? cr[0] : cr[2], o0i = u ? ci[0] : ci[2];
  const float o1r = u ? cr[1] : cr[3], o1i = u ? ci[1] : ci[3];
  k0r += __shfl_xor(o0r, 32, kWave);
  k0i += __shfl_xor(o0i, 32, kWave);
  k1r += __shfl_xor(o1r, 32, kWave);
  k1i += __shfl_xor(o1i, 32, kWave);
  const bool v = (l & 16) != 0;
  float sr = v ? k1r : k0r, si = v ? k1i : k0i;
  sr += __shfl_xor(v ? k0r : k1r, 16, kWave);
  si += __shfl_xor(v ? k0i : k1i, 16, kWave);
  red[w][4 * b + 2 * (int)u + (int)v] = make_float2(sr, si);
  __syncthreads();
  if (tid < 64) {
    const float2 q0 = red[0][tid], q1 = red[1][tid], q2 = red[2][tid], q3 = red[3][tid];
    out_ba[tid] = make_float2(((q0.x + q1.x) + q2.x) + q3.x, ((q0.y + q1.y) + q2.y) + q3.y);
  }
}

__device__ __forceinline__ void gram_tile_apply(const float2* __restrict__ G, const float2* __restrict__ xa,
                                                const float2* __restrict__ xb, bool diag,
                                                float2* __restrict__ out_ab, float2* __restrict__ out_ba,
                                                float2 (&red)[4][64]) {
  GramOps o;
  gram_tile_load(G, xa, xb, o);
  gram_tile_compute(o, diag, out_ab, out_ba, red);
}

// Sum of T strided complex partials in index order (loads issued eight at a
// time; the additions keep the sequential order).
__device__ __forceinline__ float2 ordered_sum(const float2* __restrict__ p, int T, int64_t stride) {
  float ar = 0.f, ai = 0.f;
  int k = 0;
  for (; k + 8 <= T; k += 8) {   // eight loads in flight, added in order
    float2 q[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) q[e] = p[(int64_t)(k + e) * stride];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      ar += q[e].x;
      ai += q[e].y;
    }
  }
  for (; k < T; ++k) {
    const float2 q = p[(int64_t)k * stride];
    ar += q.x; ai += q.y;
  }
  return make_float2(ar, ai);
}


// Final FP64 sums of the previous z-update's per-workgroup partials: each
// thread adds the partials b = tid, tid + 256, ... in order, then a fixed
// shuffle tree and a fixed wave order; writes the residual history entry and
// advances the iteration counter.  Run by one whole workgroup of 256 threads
// of the next kernel on the stream, so no fence or ticket is needed.
__device__ void zfinal(const IterArgs& a, double (&red)[kBlockThreads / kWave][kRedCount]) {
  if (a.ctl->zpending == 0) return;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  double tot[kRedCount] = {0, 0, 0, 0, 0};
  for (int b = tid; b < a.nz; b += kBlockThreads) {
#pragma unroll
    for (int q = 0; q < kRedCount; ++q) tot[q] += a.redpart[(int64_t)b * kRedCount + q];
  }
#pragma unroll
  for (int q = 0; q < kRedCount; ++q) tot[q] = wave_sum_d(tot[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < kRedCount; ++q) red[wave][q] = tot[q];
  }
  __syncthreads();
  if (tid == 0) {
    double r[kRedCount];
#pragma unroll
    for (int q = 0; q < kRedCount; ++q) {
      r[q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
      a.ctl->red[q] = r[q];
    }
    const int it = a.ctl->iter;
    if (a.hist) {
      a.hist[2 * (int64_t)it] = r[kRedRp2];
      a.hist[2 * (int64_t)it + 1] = r[kRedDv2] * a.rho2Q;
    }
    a.ctl->iter = it + 1;
    a.ctl->zpending = 0;
  }
}

// Operands of one row's epilogue: the row scale, g, and the other sections'
// estimated data when they fit kEpiSections registers (else read at the end).
struct RowEpi {
  float sc;
  float2 g;
  float2 e[kEpiSections];
  bool pre;
};
template <class F>
__device__ __forceinline__ void row_epi_load(const IterArgs& a, const BlockDesc& d, const F& f, int lr, RowEpi& o) {
  o.sc = f.row_scale(d.row0 + lr);
  if (a.direct) return;   // the direct form's row product only scales its sums
  o.g = a.g[d.row0 + lr];
  o.pre = a.P - 1 <= kEpiSections;
#pragma unroll
  for (int q = 0; q < kEpiSections; ++q) {
    const int sec = q < d.j ? q : q + 1;             // the other sections in order
    o.e[q] = (o.pre && sec < a.P) ? a.ghat[(int64_t)sec * a.m_pad + d.rpad0 + lr] : make_float2(0.f, 0.f);
  }
}
// r_ij = g'_ij - s (H c) for row lr of block (i, j), with (ar, ai) the row's
// product; eq. g_rows_columns: g'_ij = g_i minus the other sections'
// estimated data (compensated sums, sections in order), stored when P > 1.
// In the direct form the product is the block's estimated data instead,
// ghat_ij = H_ij u_j^i (Sec. III-C text).
__device__ __forceinline__ void row_epi_store(const IterArgs& a, const BlockDesc& d, int lr, float ar, float ai,
                                              const RowEpi& o) {
  const int64_t vi = (int64_t)d.j * a.m_pad + d.rpad0 + lr;
  if (a.direct) {
    a.ghat[vi] = make_float2(o.sc * ar, o.sc * ai);
    return;
  }
  float2 gpv = o.g;
  if (a.P > 1) {
    CSum sr, si;
    sr.add(gpv.x);
    si.add(gpv.y);
    if (o.pre) {
#pragma unroll
      for (int q = 0; q < kEpiSections; ++q) {
        if (q < a.P - 1) {
          sr.add(-o.e[q].x);
          si.add(-o.e[q].y);
        }
      }
    } else {
      for (int q = 0; q < a.P; ++q) {
        if (q == d.j) continue;
        const float2 e = a.ghat[(int64_t)q * a.m_pad + d.rpad0 + lr];
        sr.add(-e.x);
        si.add(-e.y);
      }
    }
    gpv = make_float2(sr.value(), si.value());
    a.gp[vi] = gpv;
  }
  a.r[vi] = make_float2(fmaf(-o.sc, ar, gpv.x), fmaf(-o.sc, ai, gpv.y));
}

}  // namespace admm
