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

// Loads in flight per row: the same bytes per lane for every format.
template <class F> struct RowUnroll { static constexpr int U = F::CPL == 2 ? 4 : 2; };
// H row products: rows per wave and lane loads in flight per row (narrow
// formats reuse each lane's vector loads across 8 rows).
template <class F> struct HRows {
  static constexpr int R = F::CPL == 2 ? 4 : 8;
  static constexpr int U = F::CPL == 2 ? 4 : 1;
};

// Dot products of R consecutive rows of a stored matrix with the complex
// vector x (FP32, padded, in the lane-permuted layout of cperm).  e0: element offset of the first row, ld: row
// stride in elements, nl: lane loads per row (ceil(ncols / CPL)), rows >=
// nvalid are clamped.  Lane l walks lane loads l, l+64, ... with U of them
// per row in flight.  The result (row scale not applied) is in every lane.
template <class F, int R, int U>
__device__ __forceinline__ void rows_dot(const F& f, int64_t e0, int64_t ld, int nvalid,
                                         const float4* __restrict__ x, int nl, float (&acc)[R][2]) {
  constexpr int CPL = F::CPL, X4 = CPL / 2;
  const int lane = threadIdx.x & (kWave - 1);
  int64_t rowoff[R];
#pragma unroll
  for (int rr = 0; rr < R; ++rr) {
    rowoff[rr] = e0 + (int64_t)(rr < nvalid ? rr : (nvalid - 1)) * ld;
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
      for (int rr = 0; rr < R; ++rr) raw[u][rr] = f.load(rowoff[rr] + (int64_t)(c + u * kWave) * CPL);
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
    for (int rr = 0; rr < R; ++rr) raw[rr] = f.load(rowoff[rr] + (int64_t)c * CPL);
    float4 xv[X4];
#pragma unroll
    for (int q = 0; q < X4; ++q) xv[q] = x[(((int64_t)(c >> 6) * X4 + q) << 6) + (c & 63)];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) consume(raw[rr], xv, rr);
  }
#pragma unroll
  for (int rr = 0; rr < R; ++rr) {
    acc[rr][0] = wave_sum(acc[rr][0]);
    acc[rr][1] = wave_sum(acc[rr][1]);
  }
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
  constexpr int CPL = F::CPL, U = RowUnroll<F>::U * 2;
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

}  // namespace admm
