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
// One iteration is five launches:
//   gemv_n  : r_ij = g'_ij - H_ij c_j^i  (and g'_ij from the estimated data,
//             eq. g_rows_columns, as g_i minus the other sections' ghat)
//   gram    : y_ij = G_ij^{-1} r_ij (packed Hermitian tiles, two launches),
//             ghat_ij = g'_ij - rho y_ij
//   gemv_h  : row-chunk partials of H_ij^H y_ij
//   zupdate : u = c + sum of partials, v = S_kappa(mean_i(u + s)), kappa =
//             lambda/(Q rho) (eq. v_variable_rows_columns), s += u - v
//             (eq. s_variable_rows_columns), c = v - s, per-workgroup FP64
//             partial sums of the residual norms; the first workgroup of the
//             next gemv_n (or k_zfinal at the end of a solve) adds them.
// The two H products stream H with 16-byte loads; the row-parallel products
// reduce each row across a wavefront with xor shuffles; the adjoint product
// keeps two columns per lane and splits the rows into chunks whose partials
// the z-update adds in a fixed order (no float atomics: runs are bitwise
// reproducible).
#include "gemv.h"

namespace admm {

__global__ __launch_bounds__(kBlockThreads) void k_zfinal(IterArgs a) {
  __shared__ double red[kBlockThreads / kWave][kRedCount];
  zfinal(a, red);
}

// r_ij = g'_ij - H_ij c_j^i for 4 * HRows<F>::R rows of one block per workgroup.
// tiles[x] = {block, first row, -, -}.  Workgroup 0 first completes the
// previous iteration's residual sums (zfinal).
// XS: the block's c is first copied to LDS by the whole workgroup (its
// layout unchanged), so its vector loads do not hold registers across the
// stream's loads and the workgroup reads it from L2 once instead of per wave.
template <class F, bool XS>
__global__ __launch_bounds__(kBlockThreads) void k_gemv_n(IterArgs a, const int4* __restrict__ tiles) {
  // the work descriptors first: before any store they are scalar loads
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  if (blockIdx.x == 0) {
    __shared__ double red[kBlockThreads / kWave][kRedCount];
    zfinal(a, red);
    if (a.direct && threadIdx.x == 0) *a.uref = 1;   // ghat = H y from here on
  }
  const F f = MakeFmt<F>::make(a.hs);
  // wave index in a scalar register: the rows' addresses are then wave-uniform
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  constexpr int R = HRows<F>::R;
  const int row = t.y + wave * R;
  const float4* xg = reinterpret_cast<const float4*>(a.c + (int64_t)d.i * a.n_pad + d.cpad0);
  __shared__ float4 xs[XS ? kXStage : 1];
  if (XS) {
    // whole groups of 64 lane loads: inside the block's padded segment of c
    const int n4 = (d.nj + kWave * F::CPL - 1) / (kWave * F::CPL) * kWave * (F::CPL / 2);
    for (int k = threadIdx.x; k < n4; k += kRowWaves * kWave) xs[k] = xg[k];
    __syncthreads();
  }
  if (row >= d.mi) return;
  const int nvalid = min(R, d.mi - row);
  const float4* x = XS ? xs : xg;
  // The lane that writes row rr after the reduction (one per row).
  const int rr = rows_reduce_row<R>(lane);
  const bool writer = (lane & (kWave / R - 1)) == 0 && rr < nvalid;
  const int lr = row + rr;                           // row inside the block
  constexpr bool PF = HRows<F>::PREFETCH;            // epilogue operands loaded ahead of the stream
  RowEpi epi;
  if (PF && writer) row_epi_load(a, d, f, lr, epi);
  float acc[R][2];
  rows_dot<F, R, HRows<F>::U>(f, d.h_off + (int64_t)row * d.ld, d.ld, nvalid, x, (d.nj + F::CPL - 1) / F::CPL,
                              acc);
  float ar, ai;
  rows_reduce<R, HRows<F>::SCATTER>(acc, ar, ai);
  if (writer) {
    if (!PF) row_epi_load(a, d, f, lr, epi);
    row_epi_store(a, d, lr, ar, ai, epi);
  }
}

// The same product with whole rows per workgroup (column blocks of at most
// K * 256 lane loads): N rows of one block, every thread issuing all of its
// lane loads of those rows (and the matching pieces of c) at once, so a
// workgroup reads whole contiguous rows and ends (measured faster than
// streaming interleaved rows per wave).  Row sums close over each wave and
// then over the four waves in a fixed order.  tiles[x] = {block, first row,
// -, -}.  (N, K) = WholeRows<F>: about eight 16-byte loads per thread.  Used
// for complex64 and bf16; fp8, whose rows are only 8 KB, streams faster
// through k_gemv_n.
template <class F>
struct WholeRows {
  static constexpr int N = F::CPL == 2 ? 2 : (F::CPL == 8 ? ADMM_WHOLE_N_BF16 : ADMM_WHOLE_N_FP8);
  static constexpr int K = kWholeCols / (kBlockThreads * F::CPL);
};
// WIDE: the rows are longer than one chunk of kBlockThreads * K lane loads;
// the workgroup streams them chunk by chunk, the row sums carried in registers.
template <class F, bool WIDE>
__global__ __launch_bounds__(kBlockThreads) void k_gemv_nw(IterArgs a, const int4* __restrict__ tiles) {
  constexpr int N = WholeRows<F>::N, K = WholeRows<F>::K, NW = kBlockThreads / kWave;
  constexpr int CPL = F::CPL, X4 = CPL / 2;
  __shared__ float red[NW][2 * N];
  const int4 t = tiles[blockIdx.x];   // before any store: scalar loads
  const BlockDesc d = a.blocks[t.x];
  if (blockIdx.x == 0) {
    __shared__ double zred[NW][kRedCount];
    zfinal(a, zred);
    if (a.direct && threadIdx.x == 0) *a.uref = 1;   // ghat = H y from here on
  }
  const F f = MakeFmt<F>::make(a.hs);
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int nvalid = min(N, d.mi - t.y);
  const int nl = (d.nj + CPL - 1) / CPL;
  const float4* x = reinterpret_cast<const float4*>(a.c + (int64_t)d.i * a.n_pad + d.cpad0);
  RowEpi epi;
  if constexpr (!WIDE) {
    // All loads first and without branches: lane loads past the row are
    // clamped to its last one and their contributions dropped afterwards.
    typename F::Raw h[N][K];
    float4 xv[K][X4];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const typename F::Row rp = f.row(d.h_off + (int64_t)(t.y + min(r, nvalid - 1)) * d.ld);
#pragma unroll
      for (int k = 0; k < K; ++k) h[r][k] = F::load(rp, (uint32_t)min(tid + kBlockThreads * k, nl - 1));
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int c = min(tid + kBlockThreads * k, nl - 1);   // c in the lane-permuted layout (cperm)
#pragma unroll
      for (int q = 0; q < X4; ++q) xv[k][q] = x[(((c >> 6) * X4 + q) << 6) + (c & 63)];
    }
    // epilogue operands: wave 0, lane l for row min(l, nvalid - 1) (a uniform branch)
    if (wave == 0) row_epi_load(a, d, f, t.y + min(lane, nvalid - 1), epi);
#pragma unroll
    for (int r = 0; r < N; ++r) {
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (tid + kBlockThreads * k >= nl) continue;
        float hr[CPL], hi[CPL];
        F::decode(h[r][k], hr, hi);
#pragma unroll
        for (int q = 0; q < X4; ++q) {
          cmac(sr, si, hr[2 * q], hi[2 * q], xv[k][q].x, xv[k][q].y);
          cmac(sr, si, hr[2 * q + 1], hi[2 * q + 1], xv[k][q].z, xv[k][q].w);
        }
      }
      sr = wave_sum(sr);
      si = wave_sum(si);
      if (lane == 0) {
        red[wave][2 * r] = sr;
        red[wave][2 * r + 1] = si;
      }
    }
  } else {
    // The same chunk by chunk, the epilogue operands loaded first; each
    // thread's row sums run on across the chunks in the same order.
    if (wave == 0) row_epi_load(a, d, f, t.y + min(lane, nvalid - 1), epi);
    float sr[N], si[N];
#pragma unroll
    for (int r = 0; r < N; ++r) sr[r] = si[r] = 0.f;
    for (int c0 = 0; c0 < nl; c0 += kBlockThreads * K) {
      typename F::Raw h[N][K];
      float4 xv[K][X4];
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const typename F::Row rp = f.row(d.h_off + (int64_t)(t.y + min(r, nvalid - 1)) * d.ld);
#pragma unroll
        for (int k = 0; k < K; ++k) h[r][k] = F::load(rp, (uint32_t)min(c0 + tid + kBlockThreads * k, nl - 1));
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int c = min(c0 + tid + kBlockThreads * k, nl - 1);
#pragma unroll
        for (int q = 0; q < X4; ++q) xv[k][q] = x[(((c >> 6) * X4 + q) << 6) + (c & 63)];
      }
#pragma unroll
      for (int r = 0; r < N; ++r) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (c0 + tid + kBlockThreads * k >= nl) continue;
          float hr[CPL], hi[CPL];
          F::decode(h[r][k], hr, hi);
#pragma unroll
          for (int q = 0; q < X4; ++q) {
            cmac(sr[r], si[r], hr[2 * q], hi[2 * q], xv[k][q].x, xv[k][q].y);
            cmac(sr[r], si[r], hr[2 * q + 1], hi[2 * q + 1], xv[k][q].z, xv[k][q].w);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const float wr = wave_sum(sr[r]), wi = wave_sum(si[r]);
      if (lane == 0) {
        red[wave][2 * r] = wr;
        red[wave][2 * r + 1] = wi;
      }
    }
  }
  __syncthreads();
  if (tid < nvalid) {
    float ar = red[0][2 * tid], ai = red[0][2 * tid + 1];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      ar += red[w][2 * tid];
      ai += red[w][2 * tid + 1];
    }
    row_epi_store(a, d, t.y + tid, ar, ai, epi);
  }
}

// The block's segment of the Gram-space vectors r and y: row space in the
// inversion-lemma form, column space in the direct form.
__device__ __forceinline__ int64_t gvec(const IterArgs& a, const BlockDesc& d) {
  return a.direct ? (int64_t)d.i * a.n_pad + d.cpad0 : (int64_t)d.j * a.m_pad + d.rpad0;
}

// y_ij and ghat_ij = g'_ij - rho y_ij of a block of one tile from its single
// piece, read back by the workgroup that stored it (the sum k_gram_reduce
// forms, 0 + piece, bit for bit).
__device__ __forceinline__ void gram_single_finish(const IterArgs& a, const BlockDesc& d, const float2* part) {
  __syncthreads();   // the piece's stores, by other threads of the workgroup
  const int l = threadIdx.x;
  if (l >= d.mi) return;   // d.mi <= kTile
  const float2 v = part[l];
  const float ar = 0.f + v.x, ai = 0.f + v.y;
  const int64_t vi = (int64_t)d.j * a.m_pad + d.rpad0 + l;
  a.y[vi] = make_float2(ar, ai);
  const float2 gpv = (a.P > 1) ? a.gp[vi] : a.g[d.row0 + l];
  a.ghat[vi] = make_float2(fmaf(-a.rho, ar, gpv.x), fmaf(-a.rho, ai, gpv.y));
}

// y_ij = G_ij^{-1} r_ij over the packed lower tiles of the inverse: every
// tile is read once and contributes to two 64-row pieces of y (gram_tile_apply);
// k_gram_reduce adds the pieces in tile order and forms ghat_ij = g'_ij - rho y_ij.
// The same from the bfloat16-pair copy of the inverse.
template <bool FIN>
__global__ __launch_bounds__(kBlockThreads) void k_gram_tile_bf16(IterArgs a, const int4* __restrict__ tiles) {
  __shared__ float2 tt[4][64];
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  const int T = d.mt / kTile;
  const uint32_t* G = a.Ginv16 + d.gi_off + (int64_t)(t.y * (t.y + 1) / 2 + t.z) * (kTile * kTile);
  const float2* x = a.r + gvec(a, d);
  float2* part = a.gpart + (int64_t)d.gpo * kTile;
  gram_tile_apply_bf16(G, x + t.y * kTile, x + t.z * kTile, t.y == t.z, part + (int64_t)(t.y * T + t.z) * kTile,
                       part + (int64_t)(t.z * T + t.y) * kTile, tt);
  if (FIN) gram_single_finish(a, d, part);
}

// Round to nearest even of each component to bfloat16, packed as (Re | Im << 16).
__global__ void k_to_bf16_pairs(const float2* __restrict__ src, uint32_t* __restrict__ dst, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const float2 v = src[k];
    const uint32_t re = __builtin_bit_cast(uint16_t, (__bf16)v.x), im = __builtin_bit_cast(uint16_t, (__bf16)v.y);
    dst[k] = re | (im << 16);
  }
}

// tiles[x] = {block, tile row, tile col, -} (lower pairs), one per workgroup.
// FIN (every block one tile): the tile's piece is y_ij itself, and the
// workgroup also does k_gram_reduce's part (y, ghat).
template <bool FIN>
__global__ __launch_bounds__(kBlockThreads) void k_gram_tile(IterArgs a, const int4* __restrict__ tiles) {
  __shared__ float2 tt[4][64];
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  const int T = d.mt / kTile;
  const float2* G = a.Ginv + d.gi_off + (int64_t)(t.y * (t.y + 1) / 2 + t.z) * (kTile * kTile);
  const float2* x = a.r + gvec(a, d);
  float2* part = a.gpart + (int64_t)d.gpo * kTile;
  gram_tile_apply(G, x + t.y * kTile, x + t.z * kTile, t.y == t.z, part + (int64_t)(t.y * T + t.z) * kTile,
                  part + (int64_t)(t.z * T + t.y) * kTile, tt);
  if (FIN) gram_single_finish(a, d, part);
}

// y_ij = G^{-1} r over patches of up to 4 x 4 lower tiles (complex64
// inverse).  The workgroup takes patch (R, C) = (t.y, t.z), C <= R, of block
// t.x: tile rows 4R .. 4R+3 and columns 4C .. 4C+3 that exist (only c <= a on
// the diagonal patch, whose diagonal tiles apply whole).  Each thread keeps
// its sub-block's sums (the layout of gram_tile_compute) of G x_c per patch
// row and of G^H x_a per patch column across the patch's tiles, one tile in
// flight at a time; the workgroup then stores one 64-vector per patch row
// (slot C of that row tile) and per patch column (slot R + 1): NS =
// ceil(T/4) + 1 slots per row tile instead of T single-tile pieces, which
// cuts the partial stores 4x and with them most of their cost.
__global__ __launch_bounds__(kBlockThreads) void k_gram_patch(IterArgs a, const int4* __restrict__ tiles) {
  __shared__ float2 red[4][64];
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  const int T = d.mt / kTile, NS = (T + 3) / 4 + 1;
  const int R = t.y, C = t.z, a0 = 4 * R, c0 = 4 * C;
  const int na = min(4, T - a0), nc = min(4, T - c0);
  const bool dg = R == C;
  const float2* x = a.r + gvec(a, d);
  const float2* G0 = a.Ginv + d.gi_off;
  float pr[4][4], pi[4][4], cr[4][4], ci[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int k = 0; k < 4; ++k) pr[q][k] = pi[q][k] = cr[q][k] = ci[q][k] = 0.f;
#pragma unroll
  for (int aa = 0; aa < 4; ++aa) {
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      if (aa >= na || cc >= nc || (dg && cc > aa)) continue;   // uniform over the workgroup
      const int ta = a0 + aa, tc = c0 + cc;
      GramOps o;
      gram_tile_load(G0 + (int64_t)(ta * (ta + 1) / 2 + tc) * (kTile * kTile), x + ta * kTile, x + tc * kTile, o);
      gram_rows_acc(o, pr[aa], pi[aa]);
      if (!(dg && cc == aa)) gram_cols_acc(o, cr[cc], ci[cc]);
      // the sums are materialised per tile, so the compiler cannot defer the
      // products (and keep every tile's entries in registers) to the stores
#pragma unroll
      for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(pr[aa][k]), "+v"(pi[aa][k]), "+v"(cr[cc][k]), "+v"(ci[cc][k]));
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  float2* part = a.gpart + (int64_t)d.gpo * kTile;
#pragma unroll
  for (int aa = 0; aa < 4; ++aa)
    if (aa < na) gram_rows_store(pr[aa], pi[aa], part + ((int64_t)(a0 + aa) * NS + C) * kTile);
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) {
    if (cc >= nc) continue;
    if (cc > 0) __syncthreads();   // red is read by the previous store
    gram_cols_store(cr[cc], ci[cc], part + ((int64_t)(c0 + cc) * NS + R + 1) * kTile, red);
  }
}

// PATCH: pieces laid out by k_gram_patch (NS = ceil(T/4) + 1 slots per row
// tile), else by k_gram_tile / k_gram_tile_bf16 (T slots).
static_assert(kBlockThreads / kTile == 4, "k_gram_reduce adds four interleaved sums per row");
template <bool PATCH>
__global__ __launch_bounds__(kBlockThreads) void k_gram_reduce(IterArgs a, const int4* __restrict__ tiles) {
  __shared__ float2 red[kBlockThreads / kTile][kTile];
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  const int T = d.mt / kTile;
  const int NS = PATCH ? (T + 3) / 4 + 1 : T;
  const int l = threadIdx.x & (kTile - 1), q = threadIdx.x / kTile;
  const float2* part = a.gpart + ((int64_t)d.gpo + (int64_t)t.y * NS) * kTile + l;
  float sr = 0.f, si = 0.f;
#pragma unroll 4
  for (int k = q; k < NS; k += kBlockThreads / kTile) {
    const float2 v = part[(int64_t)k * kTile];
    sr += v.x;
    si += v.y;
  }
  red[q][l] = make_float2(sr, si);
  __syncthreads();
  const int row = t.y * kTile + l;
  if (threadIdx.x >= kTile || row >= d.mi) return;
  const float2 q0 = red[0][l], q1 = red[1][l], q2 = red[2][l], q3 = red[3][l];
  const float ar = ((q0.x + q1.x) + q2.x) + q3.x, ai = ((q0.y + q1.y) + q2.y) + q3.y;
  const int64_t vi = (int64_t)d.j * a.m_pad + d.rpad0 + row;
  a.y[vi] = make_float2(ar, ai);
  // With one column block g'_ij is g_i itself and was not stored.
  const float2 gpv = (a.P > 1) ? a.gp[vi] : a.g[d.row0 + row];
  a.ghat[vi] = make_float2(fmaf(-a.rho, ar, gpv.x), fmaf(-a.rho, ai, gpv.y));
}

// Partial adjoint products: part[chunk][i][col] = sum over the chunk's rows
// of conj(H_ij[row, col]) y_ij[row] (cols_partial).
// tiles[x] = {block, first lane load, chunk, -}.
template <class F>
__global__ __launch_bounds__(kBlockThreads) void k_gemv_h(IterArgs a, const int4* __restrict__ tiles) {
  __shared__ float red[kBlockThreads / kWave - 1][2 * F::CPL][kWave];
  const F f = MakeFmt<F>::make(a.hs);
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x];
  cols_partial<F>(f, d, t, a.KH, a.y + (int64_t)d.j * a.m_pad + d.rpad0,
                  a.part + ((int64_t)t.z * a.Q + d.i) * a.n_pad + d.cpad0, red);
}

// z-update, dual update and residual norms for kZCols columns of one column
// block (one wavefront per workgroup, one column per lane).
// tiles[x] = {column block, first column, -, -}.  Replicas stay in registers
// when Q <= MAXQ (MAXQ = 0: any Q, partials are read twice).  Each workgroup
// writes its five FP64 partial sums (a fixed shuffle tree over its lanes);
// zfinal adds them in the next kernel.
// SRC: where the replicas u_j^i come from.  0: u = c + the row-chunk
// partials of H^H y (inversion-lemma form).  1, 2: direct form, u = u_ref +
// A_ij^{-1} d_ij, the sum of the Gram-apply pieces of the column's 64-tile
// (laid out by k_gram_patch, 1, or by k_gram_tile / k_gram_tile_bf16, 2)
// added to the previous u kept in y (u_ref = 0 while *uref is 0); the new u
// is stored in y in the layout of c for the next row product.
template <int MAXQ, int SRC>
__global__ __launch_bounds__(kZCols) void k_zupdate(IterArgs a, const int4* __restrict__ tiles) {
  const bool from_uref = SRC != 0 && *a.uref != 0;   // direct form: u = u_ref + the pieces
  const int4 t = tiles[blockIdx.x];
  const ColDesc cd = a.cols[t.x];
  const int col = t.y + threadIdx.x;
  const bool valid = col < cd.nj;
  double acc[kRedCount] = {0, 0, 0, 0, 0};
  if (valid) {
    const int64_t p = cd.cpad0 + col;
    const int64_t pc = cd.cpad0 + cperm(col, a.cpl);   // position of c (row-product input layout)
    const int Q = MAXQ > 0 ? MAXQ : a.Q;
    float ur[MAXQ > 0 ? MAXQ : 1], ui[MAXQ > 0 ? MAXQ : 1];
    // u = c + the row-chunk partials, and the consensus sum of u + s over the
    // replicas: compensated FP32 sums in fixed order
    auto replica = [&](int i, float& xr, float& xi) {
      CSum sr, si;
      if constexpr (SRC == 0) {
        const float2 ci = a.c[(int64_t)i * a.n_pad + pc];
        sr.add(ci.x);
        si.add(ci.y);
        const float2* pp = a.part + (int64_t)i * a.n_pad + p;
        const int64_t stride = (int64_t)a.Q * a.n_pad;
#pragma unroll 8
        for (int k = 0; k < a.KH; ++k) {
          const float2 pk = pp[k * stride];
          sr.add(pk.x);
          si.add(pk.y);
        }
      } else {
        if (from_uref) {
          const float2 u0 = a.y[(int64_t)i * a.n_pad + pc];
          sr.add(u0.x);
          si.add(u0.y);
        }
        const BlockDesc& d = a.blocks[i * a.P + t.x];
        const int T = d.mt / kTile, NS = SRC == 1 ? (T + 3) / 4 + 1 : T;
        const float2* pp = a.gpart + ((int64_t)d.gpo + (int64_t)(col / kTile) * NS) * kTile + (col % kTile);
        for (int k = 0; k < NS; ++k) {
          const float2 pk = pp[(int64_t)k * kTile];
          sr.add(pk.x);
          si.add(pk.y);
        }
      }
      xr = sr.value();
      xi = si.value();
    };
    constexpr int kUnrollQ = MAXQ > 0 ? MAXQ : 1;
    CSum mr, mi;
#pragma unroll kUnrollQ
    for (int i = 0; i < Q; ++i) {
      if (MAXQ > 0 && i >= a.Q) break;
      float xr, xi;
      replica(i, xr, xi);
      if (MAXQ > 0) {
        ur[i] = xr;
        ui[i] = xi;
      }
      const float2 si = a.s[(int64_t)i * a.n_pad + p];
      mr.add(xr);
      mr.add(si.x);
      mi.add(xi);
      mi.add(si.y);
    }
    float ar = mr.value(), ai = mi.value();
    const float invQ = 1.0f / (float)a.Q;
    ar *= invQ;
    ai *= invQ;
    if (!(isfinite(ar) && isfinite(ai))) a.ctl->nonfinite = 1;
    if (a.arec) a.arec[p] = make_float2(ar, ai);
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
#pragma unroll kUnrollQ
    for (int i = 0; i < Q; ++i) {
      if (MAXQ > 0 && i >= a.Q) break;
      const int64_t ip = (int64_t)i * a.n_pad + p;
      float xr, xi;
      if (MAXQ > 0) {
        xr = ur[i];
        xi = ui[i];
      } else {
        replica(i, xr, xi);
      }
      const float2 si = a.s[ip];
      const float dr = xr - vr, di = xi - vi;
      const float sr = si.x + dr, sim = si.y + di;
      a.s[ip] = make_float2(sr, sim);
      a.c[(int64_t)i * a.n_pad + pc] = make_float2(vr - sr, vi - sim);
      if (SRC != 0) a.y[(int64_t)i * a.n_pad + pc] = make_float2(xr, xi);
      acc[kRedRp2] += (double)dr * dr + (double)di * di;
      acc[kRedU2] += (double)xr * xr + (double)xi * xi;
      acc[kRedS2] += (double)sr * sr + (double)sim * sim;
    }
    const double dvr = (double)vr - vold.x, dvi = (double)vi - vold.y;
    acc[kRedDv2] = dvr * dvr + dvi * dvi;
    acc[kRedV2] = (double)vr * vr + (double)vi * vi;
  }
  const int lane = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kRedCount; ++q) acc[q] = wave_sum_d(acc[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < kRedCount; ++q) a.redpart[(int64_t)blockIdx.x * kRedCount + q] = acc[q];
    if (blockIdx.x == 0) a.ctl->zpending = 1;
  }
}

// Direct form.  The x-update of eq. x_solution_rows_columns,
// u = A^{-1}(H^H g' + rho c) with A = H^H H + rho I, is evaluated as a
// correction of a reference point u_ref whose product H u_ref is known:
//     u = u_ref + A^{-1} d,   d = H^H (g' - H u_ref) + rho (c - u_ref),
// the same u for any u_ref.  With u_ref the previous iteration's u (kept in
// y; its product is that block's estimate ghat_ij), g' - H u_ref is the row
// block's residual g_i - sum_q ghat_iq, the same for every j; the inverse
// then acts on a correction that vanishes at the fixed point, so its
// rounding (FP32, or the bfloat16 copy) scales with the step and not with u.
// After a reset or a state import (*uref = 0) u_ref = 0 and d = H^H g' + rho c.
//
// gp of every block of some rows: the residual g_i - sum_q ghat_iq (one
// compensated sum, sections in order), or with u_ref = 0 the local data g'_ij
// = g_i - sum_{q != j} ghat_iq (eq. g_rows_columns, that sum with the block's
// own estimate added back to a copy).  tiles[x] = {row block, first row, -,
// -}, kBlockThreads rows each.  Workgroup 0 first completes the previous
// z-update's residual sums.
__global__ __launch_bounds__(kBlockThreads) void k_dgp(IterArgs a, const int4* __restrict__ tiles) {
  const bool ur = *a.uref != 0;
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = a.blocks[t.x * a.P];
  if (blockIdx.x == 0) {
    __shared__ double red[kBlockThreads / kWave][kRedCount];
    zfinal(a, red);
  }
  const int lr = t.y + threadIdx.x;
  if (lr >= d.mi) return;
  const float2 g = a.g[d.row0 + lr];
  const float2* e = a.ghat + d.rpad0 + lr;
  CSum tr, ti;
  tr.add(g.x);
  ti.add(g.y);
#pragma unroll 8
  for (int q = 0; q < a.P; ++q) {
    const float2 eq = e[(int64_t)q * a.m_pad];
    tr.add(-eq.x);
    ti.add(-eq.y);
  }
  float2* gp = a.gp + d.rpad0 + lr;
  if (ur) {
    const float2 r = make_float2(tr.value(), ti.value());
#pragma unroll 8
    for (int j = 0; j < a.P; ++j) gp[(int64_t)j * a.m_pad] = r;
    return;
  }
#pragma unroll 8
  for (int j = 0; j < a.P; ++j) {
    const float2 ej = e[(int64_t)j * a.m_pad];
    CSum sr = tr, si = ti;
    sr.add(ej.x);
    si.add(ej.y);
    gp[(int64_t)j * a.m_pad] = make_float2(sr.value(), si.value());
  }
}

// Direct form, the right-hand side d_ij = H_ij^H gp_ij + rho (c - u_ref) from
// c and u_ref (both in the lane-permuted layout of c) and the row-chunk
// partials of the adjoint product (compensated, in chunk order), stored in r
// in the natural column layout that the Gram apply reads.  grid = (column
// tiles, Q); tiles[x] = {column block, first column, -, -} (those of the
// z-update).
__global__ __launch_bounds__(kZCols) void k_dbsum(IterArgs a, const int4* __restrict__ tiles) {
  const bool ur = *a.uref != 0;
  const int4 t = tiles[blockIdx.x];
  const ColDesc cd = a.cols[t.x];
  const int i = blockIdx.y, col = t.y + threadIdx.x;
  if (col >= cd.nj) return;
  const int64_t p = (int64_t)i * a.n_pad + cd.cpad0 + col, pc = (int64_t)i * a.n_pad + cd.cpad0 + cperm(col, a.cpl);
  float2 c = a.c[pc];
  if (ur) {
    const float2 u0 = a.y[pc];
    c = make_float2(c.x - u0.x, c.y - u0.y);
  }
  CSum sr, si;
  sr.add(a.rho * c.x);
  si.add(a.rho * c.y);
  const int64_t stride = (int64_t)a.Q * a.n_pad;
#pragma unroll 8
  for (int k = 0; k < a.KH; ++k) {
    const float2 pk = a.part[k * stride + p];
    sr.add(pk.x);
    si.add(pk.y);
  }
  a.r[p] = make_float2(sr.value(), si.value());
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

// c_j^i = v_j - s_j^i on the valid columns (after a state import), stored in
// the lane-permuted layout of the row products.
__global__ void k_make_c(const ColDesc* __restrict__ cols, int64_t n_pad, int cpl, const float2* __restrict__ v,
                         const float2* __restrict__ s, float2* __restrict__ c) {
  const int j = blockIdx.y, i = blockIdx.z;
  const ColDesc cd = cols[j];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < cd.nj; k += gridDim.x * blockDim.x) {
    const int64_t p = cd.cpad0 + k, ip = (int64_t)i * n_pad + p;
    c[(int64_t)i * n_pad + cd.cpad0 + cperm(k, cpl)] = make_float2(v[p].x - s[ip].x, v[p].y - s[ip].y);
  }
}

__global__ void k_fill_zero(uint4* p, size_t n16) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n16; k += (size_t)gridDim.x * blockDim.x)
    p[k] = make_uint4(0, 0, 0, 0);
}

// ---- launchers ------------------------------------------------------------

hipError_t launch_gemv_n(const IterArgs& a, const int4* tiles, int ntiles, const int4* wtiles, int nwtiles,
                          hipStream_t st, KTime kt) {
  if (nwtiles > 0) {
    if (a.wide) {
      switch (a.hs.storage) {
        case 0: LAUNCH_TIMED((k_gemv_nw<FmtC64, true>), dim3(nwtiles), dim3(kBlockThreads), st, kt, a, wtiles); break;
        case 1: LAUNCH_TIMED((k_gemv_nw<FmtBF16, true>), dim3(nwtiles), dim3(kBlockThreads), st, kt, a, wtiles); break;
        default: LAUNCH_TIMED((k_gemv_nw<FmtFP8, true>), dim3(nwtiles), dim3(kBlockThreads), st, kt, a, wtiles); break;
      }
    } else {
      switch (a.hs.storage) {
        case 0: LAUNCH_TIMED((k_gemv_nw<FmtC64, false>), dim3(nwtiles), dim3(kBlockThreads), st, kt, a, wtiles); break;
        case 1: LAUNCH_TIMED((k_gemv_nw<FmtBF16, false>), dim3(nwtiles), dim3(kBlockThreads), st, kt, a, wtiles); break;
        default: LAUNCH_TIMED((k_gemv_nw<FmtFP8, false>), dim3(nwtiles), dim3(kBlockThreads), st, kt, a, wtiles); break;
      }
    }
    return hipGetLastError();
  }
  switch (a.hs.storage) {
    case 0: LAUNCH_TIMED((k_gemv_n<FmtC64, false>), dim3(ntiles), dim3(kRowWaves * kWave), st, kt, a, tiles); break;
    case 1:
      if (ADMM_XLDS_NARROW && a.xstage)
        LAUNCH_TIMED((k_gemv_n<FmtBF16, true>), dim3(ntiles), dim3(kRowWaves * kWave), st, kt, a, tiles);
      else
        LAUNCH_TIMED((k_gemv_n<FmtBF16, false>), dim3(ntiles), dim3(kRowWaves * kWave), st, kt, a, tiles);
      break;
    default:
      if (ADMM_XLDS_NARROW && a.xstage)
        LAUNCH_TIMED((k_gemv_n<FmtFP8, true>), dim3(ntiles), dim3(kRowWaves * kWave), st, kt, a, tiles);
      else
        LAUNCH_TIMED((k_gemv_n<FmtFP8, false>), dim3(ntiles), dim3(kRowWaves * kWave), st, kt, a, tiles);
      break;
  }
  return hipGetLastError();
}
hipError_t launch_gram(const IterArgs& a, const int4* t_gram, int n_gram, const int4* t_gpatch, int n_gpatch,
                       const int4* t_gtr, int n_gtr, hipStream_t st, KTime kt, bool reduce) {
  const bool patch = !a.Ginv16 && n_gpatch > 0;
  // one lower tile per row tile: every block is a single tile
  const bool fin = reduce && !patch && n_gram == n_gtr;
  const KTime ka{kt.start, (reduce && !fin) ? nullptr : kt.stop};
  if (a.Ginv16) {
    if (fin)
      LAUNCH_TIMED(k_gram_tile_bf16<true>, dim3(n_gram), dim3(kBlockThreads), st, ka, a, t_gram);
    else
      LAUNCH_TIMED(k_gram_tile_bf16<false>, dim3(n_gram), dim3(kBlockThreads), st, ka, a, t_gram);
  } else if (patch) {
    LAUNCH_TIMED(k_gram_patch, dim3(n_gpatch), dim3(kBlockThreads), st, ka, a, t_gpatch);
  } else {
    if (fin)
      LAUNCH_TIMED(k_gram_tile<true>, dim3(n_gram), dim3(kBlockThreads), st, ka, a, t_gram);
    else
      LAUNCH_TIMED(k_gram_tile<false>, dim3(n_gram), dim3(kBlockThreads), st, ka, a, t_gram);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !reduce || fin) return e;
  if (patch)
    LAUNCH_TIMED(k_gram_reduce<true>, dim3(n_gtr), dim3(kBlockThreads), st, (KTime{nullptr, kt.stop}), a, t_gtr);
  else
    LAUNCH_TIMED(k_gram_reduce<false>, dim3(n_gtr), dim3(kBlockThreads), st, (KTime{nullptr, kt.stop}), a, t_gtr);
  return hipGetLastError();
}
hipError_t launch_gemv_h(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st, KTime kt) {
  switch (a.hs.storage) {
    case 0: LAUNCH_TIMED(k_gemv_h<FmtC64>, dim3(ntiles), dim3(kBlockThreads), st, kt, a, tiles); break;
    case 1: LAUNCH_TIMED(k_gemv_h<FmtBF16>, dim3(ntiles), dim3(kBlockThreads), st, kt, a, tiles); break;
    default: LAUNCH_TIMED(k_gemv_h<FmtFP8>, dim3(ntiles), dim3(kBlockThreads), st, kt, a, tiles); break;
  }
  return hipGetLastError();
}
template <int SRC>
void zupdate_go(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st, KTime kt) {
  if (a.Q <= 4)
    LAUNCH_TIMED((k_zupdate<4, SRC>), dim3(ntiles), dim3(kZCols), st, kt, a, tiles);
  else if (a.Q <= 8)
    LAUNCH_TIMED((k_zupdate<8, SRC>), dim3(ntiles), dim3(kZCols), st, kt, a, tiles);
  else if (a.Q <= 32)
    LAUNCH_TIMED((k_zupdate<32, SRC>), dim3(ntiles), dim3(kZCols), st, kt, a, tiles);
  else
    LAUNCH_TIMED((k_zupdate<0, SRC>), dim3(ntiles), dim3(kZCols), st, kt, a, tiles);
}
hipError_t launch_zupdate(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st, KTime kt, int src) {
  switch (src) {
    case 0: zupdate_go<0>(a, tiles, ntiles, st, kt); break;
    case 1: zupdate_go<1>(a, tiles, ntiles, st, kt); break;
    default: zupdate_go<2>(a, tiles, ntiles, st, kt); break;
  }
  return hipGetLastError();
}
hipError_t launch_direct_gp(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st, KTime kt) {
  LAUNCH_TIMED(k_dgp, dim3(ntiles), dim3(kBlockThreads), st, kt, a, tiles);
  return hipGetLastError();
}
hipError_t launch_direct_rhs(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st, KTime kt) {
  LAUNCH_TIMED(k_dbsum, dim3(ntiles, a.Q), dim3(kZCols), st, kt, a, tiles);
  return hipGetLastError();
}
hipError_t launch_to_bf16_pairs(const float2* src, uint32_t* dst, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_to_bf16_pairs, dim3(grid), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_zfinal(const IterArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_zfinal, dim3(1), dim3(kBlockThreads), 0, st, a);
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
hipError_t launch_make_c(const ColDesc* cols, int P, int Q, int64_t n_pad, int cpl, const float2* v,
                         const float2* s, float2* c, hipStream_t st) {
  hipLaunchKernelGGL(k_make_c, dim3(16, P, Q), dim3(256), 0, st, cols, n_pad, cpl, v, s, c);
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
