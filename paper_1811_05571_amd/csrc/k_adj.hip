// Reverse mode of K unrolled iterations (arXiv 1811.05571 Sec. III-C scheme as
// computed by the forward kernels).  For one iteration k -> k+1 the forward is,
// per block (i,j) and column block j,
//   g'_ij = g_i - sum_{q!=j} ghat_iq,   c_ij = v_j - s_ij
//   y_ij  = G_ij^{-1} (g'_ij - H_ij c_ij),   G_ij = rho I + H_ij H_ij^H
//   ghat'_ij = g'_ij - rho y_ij,           u_ij = c_ij + H_ij^H y_ij
//   a_j   = mean_i (u_ij + s_ij),          v'_j = S_kappa(a_j), kappa = lambda/(Q rho)
//   s'_ij = s_ij + u_ij - v'_j.
// Given the adjoints of (v', s', ghat') the reverse step is
//   w    = vb' - sum_i sb'_i,   ab = J_S(a)^T w,   kb += -Re(conj(w) a)/|a| (|a| > kappa)
//   ub_i = sb'_i + ab/Q                                         (k_adj_z)
//   yb   = H ub - rho ghb'                                      (k_adj_rows)
//   rb   = G^{-1} yb,  gpb = ghb' + rb,  rhob += -Re(gpb^H y)   (k_adj_gram)
//   w_i  = H^H rb  (row-chunk partials)                         (k_adj_cols)
//   vb   = sum_i (ub_i - w_i),   sb_i = w_i                     (k_adj_v)
//   gb_i += sum_j gpb_ij,  ghb_iq = -(sum_j gpb_ij - gpb_iq)    (next k_adj_rows)
// with J_S(a)^T w = (1 - kappa/|a|) w + kappa a Re(conj(a) w)/|a|^3 for
// |a| > kappa (0 otherwise), and finally lambda_b = kb/(Q rho),
// rho_b += -lambda kb/(Q rho^2).  Gradients use the convention
// dL/dRe z + j dL/dIm z.  Vectors are FP32; the scalar sums and the gradient
// of g accumulate in FP64.
#include "gemv.h"

namespace admm {

// Adds the workgroup's FP64 sum of v (fixed shuffle tree and wave order) to
// its own slot wgpart[blockIdx.x].  Each launch of a kernel adds into the same
// slots in stream order, so the slots hold per-workgroup sums over the
// iterations; k_adj_scalars adds the slots once at the end of the sweep (no
// fences or tickets between workgroups).
__device__ __forceinline__ void slot_accumulate(double v, double* wgpart) {
  __shared__ double red[kBlockThreads / kWave];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int nw = blockDim.x / kWave;
  v = wave_sum_d(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    wgpart[blockIdx.x] += s;
  }
}

// Reverse z-update: tiles = z-update tiles (kZCols columns per workgroup).
__global__ __launch_bounds__(kZCols) void k_adj_z(AdjArgs a, const int4* __restrict__ tiles, const float2* arec) {
  const int4 t = tiles[blockIdx.x];
  const ColDesc cd = a.cols[t.x];
  const int col = t.y + threadIdx.x;
  double kb = 0.0;
  if (col < cd.nj) {
    const int64_t p = cd.cpad0 + col;
    float wr = a.vb[p].x, wi = a.vb[p].y;
    for (int i = 0; i < a.Q; ++i) {
      const float2 sb = a.sb[(int64_t)i * a.n_pad + p];
      wr -= sb.x;
      wi -= sb.y;
    }
    const float2 av = arec[p];
    const float mag = sqrtf(av.x * av.x + av.y * av.y);
    float abr = 0.f, abi = 0.f;
    if (mag > a.kappa) {
      const float inv = 1.0f / mag;
      const float proj = av.x * wr + av.y * wi;          // Re(conj(a) w)
      const float f1 = 1.0f - a.kappa * inv, f2 = a.kappa * inv * inv * inv * proj;
      abr = f1 * wr + f2 * av.x;
      abi = f1 * wi + f2 * av.y;
      kb = -(double)proj * inv;
    }
    const float invQ = 1.0f / (float)a.Q;
    const int64_t pc = cd.cpad0 + cperm(col, a.cpl);   // ub is a row-product input
    for (int i = 0; i < a.Q; ++i) {
      const float2 sb = a.sb[(int64_t)i * a.n_pad + p];
      a.ub[(int64_t)i * a.n_pad + pc] = make_float2(fmaf(abr, invQ, sb.x), fmaf(abi, invQ, sb.y));
    }
  }
  slot_accumulate(kb, a.kpart);
}

// yb_ij = H_ij ub_i - rho ghb_ij, with ghb (adjoint of the estimated data the
// next iteration read) and the g-gradient contribution formed from gpb of
// the later iteration.  tiles = row tiles.
template <class F>
__global__ __launch_bounds__(kBlockThreads) void k_adj_rows(AdjArgs a, const int4* __restrict__ tiles) {
  const F f = MakeFmt<F>::make(a.hs);
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  // wave index in a scalar register: the rows' addresses are then wave-uniform
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  constexpr int R = HRows<F>::R;
  const int row = t.y + wave * R;
  if (row >= d.mi) return;
  const int nvalid = min(R, d.mi - row);
  const float4* x = reinterpret_cast<const float4*>(a.ub + (int64_t)d.i * a.n_pad + d.cpad0);
  float acc[R][2];
  rows_dot<F, R, HRows<F>::U>(f, d.h_off + (int64_t)row * d.ld, d.ld, nvalid, x, (d.nj + F::CPL - 1) / F::CPL,
                              acc);
  float ar, ai;
  rows_reduce<R, HRows<F>::SCATTER>(acc, ar, ai);
  const int rw = rows_reduce_row<R>(lane);
  if ((lane & (kWave / R - 1)) == 0 && rw < nvalid) {
    const int lr = row + rw;
    const float sc = f.row_scale(d.row0 + lr);
    const int64_t vi = (int64_t)d.j * a.m_pad + d.rpad0 + lr;
    double tr = 0.0, ti = 0.0;
    for (int q = 0; q < a.P; ++q) {
      const float2 e = a.gpb[(int64_t)q * a.m_pad + d.rpad0 + lr];
      tr += e.x;
      ti += e.y;
    }
    float ghr = 0.f, ghi = 0.f;
    if (a.P > 1) {
      const float2 own = a.gpb[vi];
      ghr = -(float)(tr - own.x);
      ghi = -(float)(ti - own.y);
    }
    a.ghb[vi] = make_float2(ghr, ghi);
    if (d.j == 0) {
      double2 gb = a.gbar[d.row0 + lr];
      a.gbar[d.row0 + lr] = make_double2(gb.x + tr, gb.y + ti);
    }
    a.yb[vi] = make_float2(fmaf(sc, ar, -a.rho * ghr), fmaf(sc, ai, -a.rho * ghi));
  }
}

// rb_ij = G_ij^{-1} yb_ij over the packed tiles (pieces), then per row:
// gpb_ij = ghb_ij + rb_ij, rho_b += -Re(gpb^H y).
__global__ __launch_bounds__(kBlockThreads) void k_adj_gram_tile(AdjArgs a, const int4* __restrict__ tiles) {
  __shared__ float2 tt[4][64];
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  const int T = d.mt / kTile;
  const int64_t toff = d.gi_off + (int64_t)(t.y * (t.y + 1) / 2 + t.z) * (kTile * kTile);
  const float2* x = a.yb + (int64_t)d.j * a.m_pad + d.rpad0;
  float2* part = a.gpart + (int64_t)d.gpo * kTile;
  if (a.Ginv16)   // the forward's (rounded) inverse: the adjoint of the map actually applied
    gram_tile_apply_bf16(a.Ginv16 + toff, x + t.y * kTile, x + t.z * kTile, t.y == t.z,
                         part + (int64_t)(t.y * T + t.z) * kTile, part + (int64_t)(t.z * T + t.y) * kTile, tt);
  else
    gram_tile_apply(a.Ginv + toff, x + t.y * kTile, x + t.z * kTile, t.y == t.z,
                    part + (int64_t)(t.y * T + t.z) * kTile, part + (int64_t)(t.z * T + t.y) * kTile, tt);
}

__global__ __launch_bounds__(kTile) void k_adj_gram_reduce(AdjArgs a, const int4* __restrict__ tiles,
                                                           const float2* __restrict__ yrec) {
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  const int T = d.mt / kTile;
  const int row = t.y * kTile + threadIdx.x;
  double rhob = 0.0;
  if (row < d.mi) {
    const float2* part = a.gpart + ((int64_t)d.gpo + (int64_t)t.y * T) * kTile + threadIdx.x;
    const float2 q = ordered_sum(part, T, kTile);
    const float ar = q.x, ai = q.y;
    const int64_t vi = (int64_t)d.j * a.m_pad + d.rpad0 + row;
    a.rb[vi] = make_float2(ar, ai);
    const float2 gh = a.ghb[vi];
    const float gr = gh.x + ar, gi = gh.y + ai;
    a.gpb[vi] = make_float2(gr, gi);
    const float2 y = yrec[vi];
    rhob = -((double)gr * y.x + (double)gi * y.y);
  }
  slot_accumulate(rhob, a.rpart);
}

// w = H^H rb, row-chunk partials.  tiles = adjoint-product tiles.
template <class F>
__global__ __launch_bounds__(kBlockThreads) void k_adj_cols(AdjArgs a, const int4* __restrict__ tiles) {
  __shared__ float red[kBlockThreads / kWave - 1][2 * F::CPL][kWave];
  const F f = MakeFmt<F>::make(a.hs);
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  cols_partial<F>(f, d, t, a.KH, a.rb + (int64_t)d.j * a.m_pad + d.rpad0,
                  a.part + ((int64_t)t.z * a.Q + d.i) * a.n_pad + d.cpad0, red);
}

// vb = sum_i (ub_i - w_i), sb_i = w_i (ub in the row-product input layout).
// tiles = z-update tiles.
__global__ __launch_bounds__(kZCols) void k_adj_v(AdjArgs a, const int4* __restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const ColDesc cd = a.cols[t.x];
  const int col = t.y + threadIdx.x;
  if (col >= cd.nj) return;
  const int64_t p = cd.cpad0 + col, pc = cd.cpad0 + cperm(col, a.cpl);
  float vr = 0.f, vi = 0.f;
  for (int i = 0; i < a.Q; ++i) {
    float wr = 0.f, wi = 0.f;
    for (int k = 0; k < a.KH; ++k) {
      const float2 q = a.part[((int64_t)k * a.Q + i) * a.n_pad + p];
      wr += q.x;
      wi += q.y;
    }
    const float2 u = a.ub[(int64_t)i * a.n_pad + pc];
    vr += u.x - wr;
    vi += u.y - wi;
    a.sb[(int64_t)i * a.n_pad + p] = make_float2(wr, wi);
  }
  a.vb[p] = make_float2(vr, vi);
}

// gb_i += sum_j gpb_ij for the first iteration's local data; then the output.
__global__ void k_adj_gflush(AdjArgs a, const BlockDesc* __restrict__ blocks, int nblocks, float2* grad_g) {
  const BlockDesc d = blocks[blockIdx.y];
  if (d.j != 0) return;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < d.mi; r += gridDim.x * blockDim.x) {
    double tr = 0.0, ti = 0.0;
    for (int q = 0; q < a.P; ++q) {
      const float2 e = a.gpb[(int64_t)q * a.m_pad + d.rpad0 + r];
      tr += e.x;
      ti += e.y;
    }
    const double2 gb = a.gbar[d.row0 + r];
    grad_g[d.row0 + r] = make_float2((float)(gb.x + tr), (float)(gb.y + ti));
  }
}

hipError_t launch_adj_iteration(const AdjArgs& a, const Geometry& G, const int4* t_hrows, const int4* t_gram,
                                const int4* t_gtr, const int4* t_cols, const int4* t_z, const float2* arec,
                                const float2* yrec, hipStream_t st) {
  const int nc = (int)G.t_cols.size(), nz = (int)G.t_z.size();
  const int ng = (int)G.t_gram.size(), ngt = (int)G.t_gtr.size();
  const int nh = (int)G.t_hrows.size();
  hipLaunchKernelGGL(k_adj_z, dim3(nz), dim3(kZCols), 0, st, a, t_z, arec);
  switch (a.hs.storage) {
    case 0: hipLaunchKernelGGL(k_adj_rows<FmtC64>, dim3(nh), dim3(kRowWaves * kWave), 0, st, a, t_hrows); break;
    case 1: hipLaunchKernelGGL(k_adj_rows<FmtBF16>, dim3(nh), dim3(kRowWaves * kWave), 0, st, a, t_hrows); break;
    default: hipLaunchKernelGGL(k_adj_rows<FmtFP8>, dim3(nh), dim3(kRowWaves * kWave), 0, st, a, t_hrows); break;
  }
  hipLaunchKernelGGL(k_adj_gram_tile, dim3(ng), dim3(kBlockThreads), 0, st, a, t_gram);
  hipLaunchKernelGGL(k_adj_gram_reduce, dim3(ngt), dim3(kTile), 0, st, a, t_gtr, yrec);
  switch (a.hs.storage) {
    case 0: hipLaunchKernelGGL(k_adj_cols<FmtC64>, dim3(nc), dim3(kBlockThreads), 0, st, a, t_cols); break;
    case 1: hipLaunchKernelGGL(k_adj_cols<FmtBF16>, dim3(nc), dim3(kBlockThreads), 0, st, a, t_cols); break;
    default: hipLaunchKernelGGL(k_adj_cols<FmtFP8>, dim3(nc), dim3(kBlockThreads), 0, st, a, t_cols); break;
  }
  hipLaunchKernelGGL(k_adj_v, dim3(nz), dim3(kZCols), 0, st, a, t_z);
  return hipGetLastError();
}

// kbar = sum of the k_adj_z slots, rbar = sum of the k_adj_gram_reduce slots
// (each in slot order, then a fixed shuffle tree); one workgroup.
__global__ __launch_bounds__(kBlockThreads) void k_adj_scalars(AdjArgs a, int nk, int nr) {
  __shared__ double red[2][kBlockThreads / kWave];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  double k = 0.0, r = 0.0;
  for (int b = threadIdx.x; b < nk; b += kBlockThreads) k += a.kpart[b];
  for (int b = threadIdx.x; b < nr; b += kBlockThreads) r += a.rpart[b];
  k = wave_sum_d(k);
  r = wave_sum_d(r);
  if (lane == 0) {
    red[0][wave] = k;
    red[1][wave] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.ctl->kbar = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    a.ctl->rbar = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  }
}

hipError_t launch_adj_scalars(const AdjArgs& a, int nk, int nr, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_scalars, dim3(1), dim3(kBlockThreads), 0, st, a, nk, nr);
  return hipGetLastError();
}

hipError_t launch_adj_gflush(const AdjArgs& a, const BlockDesc* blocks, int nblocks, float2* grad_g,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_adj_gflush, dim3(8, nblocks), dim3(256), 0, st, a, blocks, nblocks, grad_g);
  return hipGetLastError();
}

}  // namespace admm
