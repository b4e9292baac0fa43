// Per-iteration kernels of the split-lasso ADMM (consensus-and-sectioning,
// arXiv 1811.05571 Sec. III-C), complex64 storage, FP32 arithmetic.
//
// The x-update of eq. x_solution_rows_columns is evaluated in push-through
// form.  With G_ij = rho I + H_ij H_ij^H the inversion lemma (eq.
// inversion_lemma3) gives (H^H H + rho I)^{-1} = (I - H^H G^{-1} H)/rho, so for
// c = v_j - s_j^i and b = H^H g' + rho c:
//     u_j^i = c + H_ij^H y_ij,   y_ij = G_ij^{-1} (g'_ij - H_ij c)
// and the estimated data needs no third product:
//     ghat_ij = H_ij u_j^i = g'_ij - rho y_ij.
// One iteration is four launches:
//   gemv_n  : r_ij = g'_ij - H_ij c_j^i  (and g'_ij from the estimated data,
//             eq. g_rows_columns, as g_i minus the other sections' ghat)
//   gram    : y_ij = G_ij^{-1} r_ij,  ghat_ij = g'_ij - rho y_ij
//   gemv_h  : row-chunk partials of H_ij^H y_ij
//   zupdate : u = c + sum of partials, v = S_kappa(mean_i(u + s)), kappa =
//             lambda/(Q rho) (eq. v_variable_rows_columns), s += u - v
//             (eq. s_variable_rows_columns), c = v - s, residual norms.
// The two H products stream H with 16-byte loads; the row-parallel products
// reduce each row across a wavefront with xor shuffles; the adjoint product
// keeps two columns per lane and splits the rows into chunks whose partials
// the z-update adds in a fixed order (no float atomics: runs are bitwise
// reproducible).
#include "plan.h"

namespace admm {

typedef float v4f __attribute__((ext_vector_type(4)));

// Streaming 16-byte load (H and the inverse are read once per iteration).
__device__ __forceinline__ float4 ldnt(const float4* p) {
  const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

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

// Dot products of R consecutive rows of a complex64 matrix with x.
// A points at the first row, lda4 is the row stride in float4 (2 complex)
// units, n4 the number of float4 per row to use, rows >= nvalid are clamped.
// Every lane walks columns lane, lane+64, ... with U independent loads per row
// in flight.  Result: full sums in every lane (xor reduction).
template <int R, int U>
__device__ __forceinline__ void rows_dot(const float4* __restrict__ A, int64_t lda4, int nvalid,
                                         const float4* __restrict__ x, int n4, float (&acc)[R][2]) {
  const int lane = threadIdx.x & (kWave - 1);
  const float4* rowp[R];
#pragma unroll
  for (int rr = 0; rr < R; ++rr) {
    int r = rr < nvalid ? rr : (nvalid - 1);
    rowp[rr] = A + (int64_t)r * lda4;
    acc[rr][0] = 0.f;
    acc[rr][1] = 0.f;
  }
  int c = lane;
  for (; c + (U - 1) * kWave < n4; c += U * kWave) {
    float4 xv[U];
    float4 hv[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      xv[u] = x[c + u * kWave];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) hv[u][rr] = ldnt(rowp[rr] + c + u * kWave);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        cmac(acc[rr][0], acc[rr][1], hv[u][rr].x, hv[u][rr].y, xv[u].x, xv[u].y);
        cmac(acc[rr][0], acc[rr][1], hv[u][rr].z, hv[u][rr].w, xv[u].z, xv[u].w);
      }
  }
  for (; c < n4; c += kWave) {
    float4 xv = x[c];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      float4 hv = ldnt(rowp[rr] + c);
      cmac(acc[rr][0], acc[rr][1], hv.x, hv.y, xv.x, xv.y);
      cmac(acc[rr][0], acc[rr][1], hv.z, hv.w, xv.z, xv.w);
    }
  }
#pragma unroll
  for (int rr = 0; rr < R; ++rr) {
    acc[rr][0] = wave_sum(acc[rr][0]);
    acc[rr][1] = wave_sum(acc[rr][1]);
  }
}

// r_ij = g'_ij - H_ij c_j^i for kRowsPerWG rows of one block per workgroup.
// tiles[x] = {block, first row, -, -}.
__global__ __launch_bounds__(kBlockThreads) void k_gemv_n(IterArgs a, const int4* __restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int row = t.y + wave * kRowsPerWave;
  if (row >= d.mi) return;
  const int nvalid = min(kRowsPerWave, d.mi - row);
  const float4* A = reinterpret_cast<const float4*>(a.H + d.h_off + (int64_t)row * d.ld);
  const float4* x = reinterpret_cast<const float4*>(a.c + (int64_t)d.i * a.n_pad + d.cpad0);
  float acc[kRowsPerWave][2];
  rows_dot<kRowsPerWave, 4>(A, d.ld / 2, nvalid, x, (d.nj + 1) / 2, acc);
  if (lane < nvalid) {
    float ar = 0.f, ai = 0.f;
#pragma unroll
    for (int rr = 0; rr < kRowsPerWave; ++rr)
      if (rr == lane) { ar = acc[rr][0]; ai = acc[rr][1]; }
    const int lr = row + lane;                       // row inside the block
    const int64_t vi = (int64_t)d.j * a.m_pad + d.rpad0 + lr;
    float2 gpv = a.g[d.row0 + lr];
    if (a.P > 1) {
      // eq. g_rows_columns: subtract the other sections' estimated data
      for (int q = 0; q < a.P; ++q) {
        if (q == d.j) continue;
        float2 e = a.ghat[(int64_t)q * a.m_pad + d.rpad0 + lr];
        gpv.x -= e.x;
        gpv.y -= e.y;
      }
      a.gp[vi] = gpv;
    }
    a.r[vi] = make_float2(gpv.x - ar, gpv.y - ai);
  }
}

// y_ij = G_ij^{-1} r_ij (row-parallel over the stored Hermitian inverse) and
// ghat_ij = g'_ij - rho y_ij.
__global__ __launch_bounds__(kBlockThreads) void k_gram(IterArgs a, const int4* __restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int row = t.y + wave * kRowsPerWave;
  if (row >= d.mi) return;
  const int nvalid = min(kRowsPerWave, d.mi - row);
  const float4* A = reinterpret_cast<const float4*>(a.Ginv + d.gi_off + (int64_t)row * d.ldr);
  const int64_t seg = (int64_t)d.j * a.m_pad + d.rpad0;
  const float4* x = reinterpret_cast<const float4*>(a.r + seg);
  float acc[kRowsPerWave][2];
  rows_dot<kRowsPerWave, 4>(A, d.ldr / 2, nvalid, x, (d.mi + 1) / 2, acc);
  if (lane < nvalid) {
    float ar = 0.f, ai = 0.f;
#pragma unroll
    for (int rr = 0; rr < kRowsPerWave; ++rr)
      if (rr == lane) { ar = acc[rr][0]; ai = acc[rr][1]; }
    const int64_t vi = seg + row + lane;
    a.y[vi] = make_float2(ar, ai);
    // With one column block g'_ij is g_i itself and was not stored.
    const float2 gpv = (a.P > 1) ? a.gp[vi] : a.g[d.row0 + row + lane];
    a.ghat[vi] = make_float2(fmaf(-a.rho, ar, gpv.x), fmaf(-a.rho, ai, gpv.y));
  }
}

// Partial adjoint products: part[chunk][i][col] = sum over the chunk's rows
// of conj(H_ij[row, col]) y_ij[row].  Two columns per lane, kColsPerWG4 lanes
// per workgroup.  tiles[x] = {block, first float4 column, chunk, -}.
template <int U>
__global__ __launch_bounds__(kBlockThreads) void k_gemv_h(IterArgs a, const int4* __restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  const int c4 = t.y + threadIdx.x;
  const int n4 = (d.nj + 1) / 2;
  if (c4 >= n4) return;
  const int rc = (d.mi + a.KH - 1) / a.KH;
  const int rb = min(d.mi, t.z * rc), re = min(d.mi, rb + rc);
  const int64_t lda4 = d.ld / 2;
  const float4* A = reinterpret_cast<const float4*>(a.H + d.h_off) + c4;
  const float2* y = a.y + (int64_t)d.j * a.m_pad + d.rpad0;
  float a0r = 0.f, a0i = 0.f, a1r = 0.f, a1i = 0.f;
  int r = rb;
  for (; r + U <= re; r += U) {
    float4 hv[U];
    float2 yv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      hv[u] = ldnt(A + (int64_t)(r + u) * lda4);
      yv[u] = y[r + u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cmacc(a0r, a0i, hv[u].x, hv[u].y, yv[u].x, yv[u].y);
      cmacc(a1r, a1i, hv[u].z, hv[u].w, yv[u].x, yv[u].y);
    }
  }
  for (; r < re; ++r) {
    float4 hv = ldnt(A + (int64_t)r * lda4);
    float2 yv = y[r];
    cmacc(a0r, a0i, hv.x, hv.y, yv.x, yv.y);
    cmacc(a1r, a1i, hv.z, hv.w, yv.x, yv.y);
  }
  float4* out = reinterpret_cast<float4*>(a.part + ((int64_t)t.z * a.Q + d.i) * a.n_pad + d.cpad0);
  out[c4] = make_float4(a0r, a0i, a1r, a1i);
}

// z-update, dual update and residual norms for kZCols columns of one column
// block.  tiles[x] = {column block, first column, -, -}.  Each workgroup
// writes its five FP64 partial sums; the last workgroup to arrive (ticket)
// adds them in workgroup order, so the result does not depend on timing.
__global__ __launch_bounds__(kBlockThreads) void k_zupdate(IterArgs a, const int4* __restrict__ tiles) {
  __shared__ double red[kBlockThreads / kWave][kRedCount];
  __shared__ int last;
  const int4 t = tiles[blockIdx.x];
  const ColDesc cd = a.cols[t.x];
  const int col = t.y + threadIdx.x;
  const bool valid = col < cd.nj;
  double acc[kRedCount] = {0, 0, 0, 0, 0};
  if (valid) {
    const int64_t p = cd.cpad0 + col;
    float ar = 0.f, ai = 0.f;
    for (int i = 0; i < a.Q; ++i) {
      float2 ci = a.c[(int64_t)i * a.n_pad + p];
      float ur = ci.x, ui = ci.y;
      for (int k = 0; k < a.KH; ++k) {
        float2 pk = a.part[((int64_t)k * a.Q + i) * a.n_pad + p];
        ur += pk.x;
        ui += pk.y;
      }
      float2 si = a.s[(int64_t)i * a.n_pad + p];
      ar += ur + si.x;
      ai += ui + si.y;
    }
    const float invQ = 1.0f / (float)a.Q;
    ar *= invQ;
    ai *= invQ;
    if (!(isfinite(ar) && isfinite(ai))) a.ctl->nonfinite = 1;
    // eq. softhresholding with sign(a) = a/|a|
    const float mag = sqrtf(ar * ar + ai * ai);
    float vr = 0.f, vi = 0.f;
    if (mag > a.kappa) {
      const float sc = 1.0f - a.kappa / mag;
      vr = ar * sc;
      vi = ai * sc;
    }
    const float2 vold = a.v[p];
    a.v[p] = make_float2(vr, vi);
    for (int i = 0; i < a.Q; ++i) {
      const int64_t ip = (int64_t)i * a.n_pad + p;
      float2 ci = a.c[ip];
      float ur = ci.x, ui = ci.y;
      for (int k = 0; k < a.KH; ++k) {
        float2 pk = a.part[((int64_t)k * a.Q + i) * a.n_pad + p];
        ur += pk.x;
        ui += pk.y;
      }
      float2 si = a.s[ip];
      const float dr = ur - vr, di = ui - vi;
      const float sr = si.x + dr, sim = si.y + di;
      a.s[ip] = make_float2(sr, sim);
      a.c[ip] = make_float2(vr - sr, vi - sim);
      acc[kRedRp2] += (double)dr * dr + (double)di * di;
      acc[kRedU2] += (double)ur * ur + (double)ui * ui;
      acc[kRedS2] += (double)sr * sr + (double)sim * sim;
    }
    const double dvr = (double)vr - vold.x, dvi = (double)vi - vold.y;
    acc[kRedDv2] = dvr * dvr + dvi * dvi;
    acc[kRedV2] = (double)vr * vr + (double)vi * vi;
  }
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int q = 0; q < kRedCount; ++q) {
    double w = wave_sum_d(acc[q]);
    if (lane == 0) red[wave][q] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < kRedCount; ++q) {
      double s = 0.0;
      for (int w = 0; w < kBlockThreads / kWave; ++w) s += red[w][q];
      a.redpart[(int64_t)blockIdx.x * kRedCount + q] = s;
    }
    __threadfence();
    const int tk = atomicAdd(&a.ctl->ticket, 1);
    last = (tk == (int)gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x < kRedCount) {
    const int q = threadIdx.x;
    double s = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b)
      s += __hip_atomic_load(a.redpart + (int64_t)b * kRedCount + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.ctl->red[q] = s;
    const int it = a.ctl->iter;
    if (a.hist) {
      if (q == kRedRp2) a.hist[2 * (int64_t)it] = s;
      if (q == kRedDv2) a.hist[2 * (int64_t)it + 1] = s * a.rho2Q;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.ctl->iter += 1;
    a.ctl->ticket = 0;
  }
}

// Copy between the padded column space and a dense n-vector (reps copies at
// the given strides).  to_padded = 0: padded -> dense.
__global__ void k_cols_copy(const ColDesc* __restrict__ cols, int P, const float2* __restrict__ src,
                            float2* __restrict__ dst, int64_t src_stride, int64_t dst_stride,
                            int to_padded) {
  const int j = blockIdx.y, rep = blockIdx.z;
  const ColDesc cd = cols[j];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < cd.nj; c += gridDim.x * blockDim.x) {
    const int64_t pi = cd.cpad0 + c, di = cd.col0 + c;
    if (to_padded)
      dst[rep * dst_stride + pi] = src[rep * src_stride + di];
    else
      dst[rep * dst_stride + di] = src[rep * src_stride + pi];
  }
}

// Copy between padded row space [P][m_pad] and dense [P][m].
__global__ void k_rows_copy(const BlockDesc* __restrict__ blocks, int64_t m, int64_t m_pad,
                            const float2* __restrict__ src, float2* __restrict__ dst, int to_padded) {
  const BlockDesc d = blocks[blockIdx.y];
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < d.mi; r += gridDim.x * blockDim.x) {
    const int64_t pi = (int64_t)d.j * m_pad + d.rpad0 + r, di = (int64_t)d.j * m + d.row0 + r;
    if (to_padded)
      dst[pi] = src[di];
    else
      dst[di] = src[pi];
  }
}

// c_j^i = v_j - s_j^i on the valid columns (after a state import).
__global__ void k_make_c(const ColDesc* __restrict__ cols, int64_t n_pad, const float2* __restrict__ v,
                         const float2* __restrict__ s, float2* __restrict__ c) {
  const int j = blockIdx.y, i = blockIdx.z;
  const ColDesc cd = cols[j];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < cd.nj; k += gridDim.x * blockDim.x) {
    const int64_t p = cd.cpad0 + k, ip = (int64_t)i * n_pad + p;
    c[ip] = make_float2(v[p].x - s[ip].x, v[p].y - s[ip].y);
  }
}

__global__ void k_fill_zero(uint4* p, size_t n16) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n16; k += (size_t)gridDim.x * blockDim.x)
    p[k] = make_uint4(0, 0, 0, 0);
}

// ---- launchers ------------------------------------------------------------
hipError_t launch_gemv_n(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_n, dim3(ntiles), dim3(kBlockThreads), 0, st, a, tiles);
  return hipGetLastError();
}
hipError_t launch_gram(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_gram, dim3(ntiles), dim3(kBlockThreads), 0, st, a, tiles);
  return hipGetLastError();
}
hipError_t launch_gemv_h(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_h<8>, dim3(ntiles), dim3(kBlockThreads), 0, st, a, tiles);
  return hipGetLastError();
}
hipError_t launch_zupdate(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_zupdate, dim3(ntiles), dim3(kBlockThreads), 0, st, a, tiles);
  return hipGetLastError();
}
hipError_t launch_unpad_cols(const ColDesc* cols, int P, int64_t n, const float2* src, float2* dst,
                             int64_t src_stride, int64_t dst_stride, int reps, int to_padded,
                             hipStream_t st) {
  int gx = (int)std::min<int64_t>(64, (n / P + 255) / 256 + 1);
  hipLaunchKernelGGL(k_cols_copy, dim3(gx, P, reps), dim3(256), 0, st, cols, P, src, dst, src_stride,
                     dst_stride, to_padded);
  return hipGetLastError();
}
hipError_t launch_unpad_rows(const BlockDesc* blocks, int nblocks, int64_t m, int64_t m_pad,
                             const float2* src, float2* dst, int to_padded, hipStream_t st) {
  hipLaunchKernelGGL(k_rows_copy, dim3(8, nblocks), dim3(256), 0, st, blocks, m, m_pad, src, dst,
                     to_padded);
  return hipGetLastError();
}
hipError_t launch_make_c(const ColDesc* cols, int P, int Q, int64_t n_pad, const float2* v, const float2* s,
                         float2* c, hipStream_t st) {
  hipLaunchKernelGGL(k_make_c, dim3(16, P, Q), dim3(256), 0, st, cols, n_pad, v, s, c);
  return hipGetLastError();
}
hipError_t launch_fill(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  size_t n16 = bytes / 16;
  int grid = (int)std::min<size_t>(4096, (n16 + 255) / 256);
  hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, st, reinterpret_cast<uint4*>(p), n16);
  return hipGetLastError();
}

}  // namespace admm
