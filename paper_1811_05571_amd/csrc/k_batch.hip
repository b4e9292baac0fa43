// Kernels of the batched multi-scene form (see batch.h).
//
// Forward product, per (H0 frequency tile f, column block j):
//     R = H0[f, C_j] X,   X = [c_{s,i(s,f),j}] over the scenes that measure f,
// then r_s = g'_s - phase_s o R[:, s] for every scene-tile.  Adjoint product:
//     U = H0[f, C_j]^H Y', Y' = [conj(phase_s) o y_s] over the same scenes,
// written as one partial per (scene-tile, column) and added per row block
// by the z-update.  Both are complex GEMMs done as real MFMA GEMMs
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation): H0 is stored in bfloat16,
// the FP32 vector operand is split exactly enough into three bfloat16 terms
// (x = x1 + x2 + x3 + O(2^-27 |x|)) so that the products keep FP32 accuracy.
#include "batch.h"

namespace admm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u32x4 ld16(const uint16_t* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
}

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Eight complex FP32 values -> three bfloat16 terms each of Re and Im.
struct Split {
  bf16x8 r1, r2, r3, i1, i2, i3;
};
__device__ __forceinline__ void split8(const float (&re)[8], const float (&im)[8], Split& s) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    __bf16 a = (__bf16)re[e];
    float rr = re[e] - (float)a;
    __bf16 b = (__bf16)rr;
    rr -= (float)b;
    s.r1[e] = a;
    s.r2[e] = b;
    s.r3[e] = (__bf16)rr;
    a = (__bf16)im[e];
    rr = im[e] - (float)a;
    b = (__bf16)rr;
    rr -= (float)b;
    s.i1[e] = a;
    s.i2[e] = b;
    s.i3[e] = (__bf16)rr;
  }
}

// acc += A X for complex A = (Ar, Ai), X split:  Cr += Ar Xr - Ai Xi, Ci += Ar Xi + Ai Xr.
__device__ __forceinline__ void cmfma(const bf16x8& Ar, const bf16x8& Ai, const bf16x8& nAi, const Split& x,
                                      f32x4& cr, f32x4& ci) {
  cr = mfma(Ar, x.r1, cr);
  cr = mfma(Ar, x.r2, cr);
  cr = mfma(Ar, x.r3, cr);
  cr = mfma(nAi, x.i1, cr);
  cr = mfma(nAi, x.i2, cr);
  cr = mfma(nAi, x.i3, cr);
  ci = mfma(Ar, x.i1, ci);
  ci = mfma(Ar, x.i2, ci);
  ci = mfma(Ar, x.i3, ci);
  ci = mfma(Ai, x.r1, ci);
  ci = mfma(Ai, x.r2, ci);
  ci = mfma(Ai, x.r3, ci);
}

__device__ __forceinline__ bf16x8 as_bf16(const u32x4& v) { return __builtin_bit_cast(bf16x8, v); }

// Forward product.  One workgroup = 4 waves x 16 rows of tile f (64 rows) x
// up to 16*NT scene-tiles.  MFMA operand layout (16x16x32): lane l holds row
// (A) / column (B) l%16 and k = 8(l/16) .. 8(l/16)+7; the result holds
// column l%16, rows 4(l/16) .. 4(l/16)+3.
template <int NT>
__global__ __launch_bounds__(kBlockThreads) void k_bgemm_n(BatchArgs a, const GemmItem* __restrict__ items) {
  const GemmItem it = items[blockIdx.x];
  const BlockDesc pj = a.pseudo[it.j];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int kq = 8 * (lane >> 4);
  const int64_t arow = (int64_t)it.f * a.tile_rows + it.m0 + 16 * wave + (lane & 15);
  const uint16_t* are = a.h_re + pj.h_off + arow * pj.ld + kq;
  const uint16_t* aim = a.h_im + pj.h_off + arow * pj.ld + kq;
  const float4* xs[NT];
  bool xv[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int t = 16 * nt + (lane & 15);
    xv[nt] = t < it.cnt;
    const SceneTile st = a.stab[it.st0 + (xv[nt] ? t : 0)];
    xs[nt] = reinterpret_cast<const float4*>(a.c + (int64_t)st.rep * a.n_pad + pj.cpad0 + kq);
  }
  f32x4 cr[NT], ci[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) cr[nt] = ci[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const u32x4 sgn = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  for (int k0 = 0; k0 < pj.nj; k0 += 32) {
    const u32x4 ur = ld16(are + k0), ui = ld16(aim + k0);
    const bf16x8 Ar = as_bf16(ur), Ai = as_bf16(ui), nAi = as_bf16(ui ^ sgn);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      float re[8], im[8];
      if (xv[nt]) {
        const float4* xp = xs[nt] + (k0 >> 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 v = xp[q];
          re[2 * q] = v.x;
          im[2 * q] = v.y;
          re[2 * q + 1] = v.z;
          im[2 * q + 1] = v.w;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) re[e] = im[e] = 0.f;
      }
      Split x;
      split8(re, im, x);
      cmfma(Ar, Ai, nAi, x, cr[nt], ci[nt]);
    }
  }
  // epilogue: r = g' - phase * (H0 x)
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int t = 16 * nt + (lane & 15);
    if (t >= it.cnt) continue;
    const SceneTile st = a.stab[it.st0 + t];
    const RowBlockDesc rb = a.rbd[st.rep];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int rr = it.m0 + 16 * wave + 4 * (lane >> 4) + e;
      const int64_t gr = st.row0 + rr;
      const int lr = st.lr0 + rr;
      const float2 ph = a.phases[gr];
      const float hr = ph.x * cr[nt][e] - ph.y * ci[nt][e];
      const float hi = ph.x * ci[nt][e] + ph.y * cr[nt][e];
      const int64_t vi = (int64_t)it.j * a.m_pad + rb.rpad0 + lr;
      float2 gpv = a.g[gr];
      if (a.P > 1) {
        for (int q = 0; q < a.P; ++q) {
          if (q == it.j) continue;
          const float2 e2 = a.ghat[(int64_t)q * a.m_pad + rb.rpad0 + lr];
          gpv.x -= e2.x;
          gpv.y -= e2.y;
        }
        a.gp[vi] = gpv;
      }
      a.r[vi] = make_float2(gpv.x - hr, gpv.y - hi);
    }
  }
}

// Adjoint product.  One workgroup = 4 waves x 16 columns of block j (64
// columns) x up to 16*NT scene-tiles; K = the tile's rows, read from the
// transposed store so that every lane's 8 k-values are contiguous.
template <int NT>
__global__ __launch_bounds__(kBlockThreads) void k_bgemm_h(BatchArgs a, const GemmItem* __restrict__ items) {
  const GemmItem it = items[blockIdx.x];
  const BlockDesc pj = a.pseudo[it.j];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int kq = 8 * (lane >> 4);
  const int col = it.m0 + 16 * wave + (lane & 15);
  const int colc = min(col, pj.nj - 1);
  const uint16_t* are = a.t_re + pj.gi_off + (int64_t)colc * a.ldt + (int64_t)it.f * a.tile_rows + kq;
  const uint16_t* aim = a.t_im + pj.gi_off + (int64_t)colc * a.ldt + (int64_t)it.f * a.tile_rows + kq;
  const float4* ys[NT];
  const float4* ps[NT];
  bool yv[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int t = 16 * nt + (lane & 15);
    yv[nt] = t < it.cnt;
    const SceneTile st = a.stab[it.st0 + (yv[nt] ? t : 0)];
    const RowBlockDesc rb = a.rbd[st.rep];
    ys[nt] = reinterpret_cast<const float4*>(a.y + (int64_t)it.j * a.m_pad + rb.rpad0 + st.lr0 + kq);
    ps[nt] = reinterpret_cast<const float4*>(a.phases + (int64_t)st.row0 + kq);
  }
  f32x4 cr[NT], ci[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) cr[nt] = ci[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const u32x4 sgn = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  for (int k0 = 0; k0 < a.tile_rows; k0 += 32) {
    const u32x4 ur = ld16(are + k0), ui = ld16(aim + k0);
    // conj(H0)^T: real part Ar, imaginary part -Ai
    const bf16x8 Ar = as_bf16(ur), cAi = as_bf16(ui ^ sgn), Ai = as_bf16(ui);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      float re[8], im[8];
      if (yv[nt]) {
        const float4* yp = ys[nt] + (k0 >> 1);
        const float4* pp = ps[nt] + (k0 >> 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 yy = yp[q], ph = pp[q];
          // conj(phase) * y
          re[2 * q] = ph.x * yy.x + ph.y * yy.y;
          im[2 * q] = ph.x * yy.y - ph.y * yy.x;
          re[2 * q + 1] = ph.z * yy.z + ph.w * yy.w;
          im[2 * q + 1] = ph.z * yy.w - ph.w * yy.z;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) re[e] = im[e] = 0.f;
      }
      Split x;
      split8(re, im, x);
      // (Ar + i cAi)(Xr + i Xi) with cAi = -Ai
      cmfma(Ar, cAi, Ai, x, cr[nt], ci[nt]);
    }
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int t = 16 * nt + (lane & 15);
    if (t >= it.cnt) continue;
    const SceneTile st = a.stab[it.st0 + t];
    float2* out = a.part + (int64_t)st.pslot * a.n_pad + pj.cpad0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int cc = it.m0 + 16 * wave + 4 * (lane >> 4) + e;
      if (cc < pj.nj) out[cc] = make_float2(cr[nt][e], ci[nt][e]);
    }
  }
}

// Per-scene z-update: tiles {scene, column block, first column}, 64 columns per workgroup.
__global__ __launch_bounds__(kZCols) void k_bzupdate(BatchArgs a, const ColDesc* __restrict__ cols,
                                                     const int4* __restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const SceneDesc sd = a.scenes[t.x];
  const ColDesc cd = cols[t.y];
  const int col = t.z + threadIdx.x;
  if (col >= cd.nj) return;
  const int64_t p = cd.cpad0 + col;
  auto replica = [&](int i) {
    const int rep = sd.rb0 + i;
    float2 u = a.c[(int64_t)rep * a.n_pad + p];
    const int s0 = a.cuts[sd.cut0 + i], s1 = a.cuts[sd.cut0 + i + 1];
    for (int sl = s0; sl < s1; ++sl) {
      const float2 q = a.part[(int64_t)(sd.pslot0 + sl) * a.n_pad + p];
      u.x += q.x;
      u.y += q.y;
    }
    return u;
  };
  float ar = 0.f, ai = 0.f;
  for (int i = 0; i < sd.Q; ++i) {
    const float2 u = replica(i);
    const float2 sv = a.s[(int64_t)(sd.rb0 + i) * a.n_pad + p];
    ar += u.x + sv.x;
    ai += u.y + sv.y;
  }
  const float invQ = 1.0f / (float)sd.Q;
  ar *= invQ;
  ai *= invQ;
  if (!(isfinite(ar) && isfinite(ai))) a.ctl->nonfinite = 1;
  const float mag = sqrtf(ar * ar + ai * ai);
  float vr = 0.f, vi = 0.f;
  if (mag > sd.kappa) {
    const float sc = 1.0f - sd.kappa / mag;
    vr = ar * sc;
    vi = ai * sc;
  }
  a.v[(int64_t)t.x * a.n_pad + p] = make_float2(vr, vi);
  for (int i = 0; i < sd.Q; ++i) {
    const float2 u = replica(i);
    const int64_t ip = (int64_t)(sd.rb0 + i) * a.n_pad + p;
    const float2 sv = a.s[ip];
    const float sr = sv.x + u.x - vr, si = sv.y + u.y - vi;
    a.s[ip] = make_float2(sr, si);
    a.c[ip] = make_float2(vr - sr, vi - si);
  }
}

// H0^T store: [j][n_j][ldt] from the block store [j][m0][ld_j]; 64 x 64 tiles.
__global__ __launch_bounds__(kBlockThreads) void k_btranspose(BatchArgs a, int64_t m0) {
  __shared__ uint16_t tr[64][65], ti[64][65];
  const BlockDesc pj = a.pseudo[blockIdx.z];
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  if (c0 >= pj.nj) return;
  for (int e = threadIdx.x; e < 64 * 64; e += kBlockThreads) {
    const int r = e / 64, c = e % 64;
    uint16_t vr = 0, vi = 0;
    if (r0 + r < m0 && c0 + c < pj.nj) {
      const int64_t o = pj.h_off + (int64_t)(r0 + r) * pj.ld + c0 + c;
      vr = a.h_re[o];
      vi = a.h_im[o];
    }
    tr[r][c] = vr;
    ti[r][c] = vi;
  }
  __syncthreads();
  uint16_t* ore = const_cast<uint16_t*>(a.t_re);
  uint16_t* oim = const_cast<uint16_t*>(a.t_im);
  for (int e = threadIdx.x; e < 64 * 64; e += kBlockThreads) {
    const int c = e / 64, r = e % 64;
    if (c0 + c < pj.nj && r0 + r < a.ldt) {
      const int64_t o = pj.gi_off + (int64_t)(c0 + c) * a.ldt + r0 + r;
      ore[o] = tr[r][c];
      oim[o] = ti[r][c];
    }
  }
}

// Gram of a scene block from the shared per-column-block Gram G0_j of H0:
// G[r][c] = rho delta + phase_r conj(phase_c) G0_j[R(r)][R(c)], R the H0 row
// of scene-block row r.  Tiles {block, tile row, tile col} (lower); the
// diagonal tiles are written in full, pads as identity.
__global__ __launch_bounds__(kBlockThreads) void k_bgram_assemble(const int4* __restrict__ tiles,
                                                                  const BlockDesc* __restrict__ blocks,
                                                                  const int32_t* __restrict__ blk_tile0,
                                                                  const int32_t* __restrict__ tiles_flat,
                                                                  const float2* __restrict__ phases,
                                                                  const double2* __restrict__ G0,
                                                                  const BlockDesc* __restrict__ pseudo,
                                                                  int tile_rows, double rho,
                                                                  double2* __restrict__ A) {
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = blocks[t.x];
  const BlockDesc pj = pseudo[d.j];
  const int tile0 = blk_tile0[t.x];
  for (int e = threadIdx.x; e < kTile * kTile; e += kBlockThreads) {
    const int r = t.y * kTile + e / kTile, c = t.z * kTile + e % kTile;
    double2 val;
    if (r >= d.mi || c >= d.mi) {
      val = make_double2(r == c ? 1.0 : 0.0, 0.0);
    } else {
      const int hi = max(r, c), lo = min(r, c);
      const int64_t R = (int64_t)tiles_flat[tile0 + hi / tile_rows] * tile_rows + hi % tile_rows;
      const int64_t C = (int64_t)tiles_flat[tile0 + lo / tile_rows] * tile_rows + lo % tile_rows;
      const double2 g0 = G0[pj.f_off + R * pj.mt + C];
      const float2 pa = phases[d.row0 + hi], pb = phases[d.row0 + lo];
      // pa conj(pb)
      const double wr = (double)pa.x * pb.x + (double)pa.y * pb.y;
      const double wi = (double)pa.y * pb.x - (double)pa.x * pb.y;
      val = make_double2(wr * g0.x - wi * g0.y, wr * g0.y + wi * g0.x);
      if (r < c) val.y = -val.y;
      if (r == c) val.x += rho;
    }
    A[d.f_off + (int64_t)r * d.mt + c] = val;
  }
}

__global__ void k_bunpad_v(const ColDesc* __restrict__ cols, int64_t n, int64_t n_pad, const float2* __restrict__ v,
                           float2* __restrict__ out) {
  const int j = blockIdx.y, s = blockIdx.z;
  const ColDesc cd = cols[j];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < cd.nj; c += gridDim.x * blockDim.x)
    out[(int64_t)s * n + cd.col0 + c] = v[(int64_t)s * n_pad + cd.cpad0 + c];
}

}  // namespace

hipError_t launch_bgemm_n(const BatchArgs& a, const GemmItem* items, int nitems, int variant, hipStream_t st) {
  switch (variant) {
    case 1: hipLaunchKernelGGL(k_bgemm_n<1>, dim3(nitems), dim3(kBlockThreads), 0, st, a, items); break;
    case 2: hipLaunchKernelGGL(k_bgemm_n<2>, dim3(nitems), dim3(kBlockThreads), 0, st, a, items); break;
    default: hipLaunchKernelGGL(k_bgemm_n<4>, dim3(nitems), dim3(kBlockThreads), 0, st, a, items); break;
  }
  return hipGetLastError();
}

hipError_t launch_bgemm_h(const BatchArgs& a, const GemmItem* items, int nitems, int variant, hipStream_t st) {
  switch (variant) {
    case 1: hipLaunchKernelGGL(k_bgemm_h<1>, dim3(nitems), dim3(kBlockThreads), 0, st, a, items); break;
    case 2: hipLaunchKernelGGL(k_bgemm_h<2>, dim3(nitems), dim3(kBlockThreads), 0, st, a, items); break;
    default: hipLaunchKernelGGL(k_bgemm_h<4>, dim3(nitems), dim3(kBlockThreads), 0, st, a, items); break;
  }
  return hipGetLastError();
}

hipError_t launch_bzupdate(const BatchArgs& a, const ColDesc* cols, const int4* tiles, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_bzupdate, dim3(ntiles), dim3(kZCols), 0, st, a, cols, tiles);
  return hipGetLastError();
}

hipError_t launch_btranspose(const BatchArgs& a, int P, int64_t m0, int max_nj, hipStream_t st) {
  hipLaunchKernelGGL(k_btranspose, dim3((unsigned)((m0 + 63) / 64), (unsigned)((max_nj + 63) / 64), P),
                     dim3(kBlockThreads), 0, st, a, m0);
  return hipGetLastError();
}

hipError_t launch_bgram_assemble(const int4* tiles, int ntiles, const BlockDesc* blocks, const int32_t* blk_tile0,
                                 const int32_t* tiles_flat, const float2* phases, const double2* G0,
                                 const BlockDesc* pseudo, int tile_rows, double rho, double2* A, hipStream_t st) {
  hipLaunchKernelGGL(k_bgram_assemble, dim3(ntiles), dim3(kBlockThreads), 0, st, tiles, blocks, blk_tile0,
                     tiles_flat, phases, G0, pseudo, tile_rows, rho, A);
  return hipGetLastError();
}

hipError_t launch_bunpad_v(const ColDesc* cols, int P, int64_t n, int S, int64_t n_pad, const float2* v,
                           float2* out, hipStream_t st) {
  hipLaunchKernelGGL(k_bunpad_v, dim3(8, P, S), dim3(256), 0, st, cols, n, n_pad, v, out);
  return hipGetLastError();
}

}  // namespace admm
