// Kernels of the batched multi-scene form (see batch.h).
//
// Forward product, per (H0 frequency tile f, column block j):
//     R = H0[f, C_j] X,   X = [c_{s,i(s,f),j}] over the scenes that measure f,
// then r_s = g'_s - phase_s o R[:, s] for every scene-tile.  Adjoint product:
//     U = H0[f, C_j]^H Y', Y' = [conj(phase_s) o y_s] over the same scenes,
// written as one partial per (scene-tile, column) and added per row block
// by the z-update.  Both are complex GEMMs done as real MFMA GEMMs
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation): H0 is stored in bfloat16,
// the FP32 vector operand is split into three bfloat16 terms
// (x = x1 + x2 + x3 + O(2^-27 |x|)) so that the products keep FP32 accuracy.
// The split is done once per iteration by the producer of each operand (the
// z-update for c, k_bsplit_y for conj(phase) o y) into six bf16 planes that
// the GEMMs load directly.
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

// Three bfloat16 terms each of Re and Im of eight complex values.
struct Split {
  bf16x8 r1, r2, r3, i1, i2, i3;
};

// x -> bf16 terms t1 + t2 + t3 (each the round-to-nearest-even bf16 of the
// remainder), as 16-bit codes.
__device__ __forceinline__ void split3(float x, uint16_t& t1, uint16_t& t2, uint16_t& t3) {
  const __bf16 a = (__bf16)x;
  float r = x - (float)a;
  const __bf16 b = (__bf16)r;
  r -= (float)b;
  const __bf16 c = (__bf16)r;
  t1 = __builtin_bit_cast(uint16_t, a);
  t2 = __builtin_bit_cast(uint16_t, b);
  t3 = __builtin_bit_cast(uint16_t, c);
}

// Writes the six planes of one complex value at element e (plane stride ps).
__device__ __forceinline__ void store_split(uint16_t* __restrict__ base, int64_t ps, int64_t e, float re, float im) {
  uint16_t t1, t2, t3;
  split3(re, t1, t2, t3);
  base[e] = t1;
  base[ps + e] = t2;
  base[2 * ps + e] = t3;
  split3(im, t1, t2, t3);
  base[3 * ps + e] = t1;
  base[4 * ps + e] = t2;
  base[5 * ps + e] = t3;
}

// Eight consecutive elements of each of the six planes (16-byte loads).
__device__ __forceinline__ void load_split(const uint16_t* __restrict__ p, int64_t ps, Split& x) {
  x.r1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
  x.r2 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p + ps));
  x.r3 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p + 2 * ps));
  x.i1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p + 3 * ps));
  x.i2 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p + 4 * ps));
  x.i3 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p + 5 * ps));
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

// ---- MFMA GEMM tiles -------------------------------------------------------
// MFMA operand layout (16x16x32 bf16): lane l holds row (A) / column (B)
// l%16 and k = 8(l/16) .. 8(l/16)+7; the result holds column l%16, rows
// 4(l/16) .. 4(l/16)+3.  A workgroup of 4 waves computes (4 * 16 * MS rows) x
// (64 scene-tile columns); wave w owns MS row subtiles and all four column
// subtiles, so each B fragment feeds MS complex MFMA groups.  Per 32-wide
// k-step the B operand (64 columns x 32 k x six bf16 planes, 24 KB) is staged
// once in LDS (double buffer: the next step's pieces are loaded into registers
// during the current step's MFMAs); A comes straight from global memory, one
// step ahead.
constexpr int kGN = 64;   // scene-tile columns per workgroup
constexpr int kGK = 32;   // k per step
constexpr int kAT = 16 * kGK;   // elements of one k-tile of the A stores (16 rows x 32 k)

struct __attribute__((aligned(16))) BStage {
  uint16_t v[2][6][kGN][kGK];
};
static_assert(alignof(BStage) == 16, "16-byte LDS accesses");

// LDS position of the 16-byte chunk q (k = 8q .. 8q+7) of column col: the
// chunks of a column are permuted by an XOR with ((col >> 1) ^ (col >> 2)) & 3
// so that the fragment reads (16 lanes = 16 consecutive columns, one chunk)
// and the staging writes meet distinct banks in every 8- and 16-lane group;
// unpermuted, the 64-byte column stride put 4 lanes of 8 on each bank group.
__device__ __forceinline__ int bchunk(int col, int q) { return 8 * (q ^ (((col >> 1) ^ (col >> 2)) & 3)); }

// This thread's piece of a B step: column tid/4, k offset 8 (tid % 4); six
// 16-byte loads from plane stride ps.
__device__ __forceinline__ void bstage_load(const uint16_t* __restrict__ src, int64_t ps, u32x4 (&r)[6]) {
#pragma unroll
  for (int p = 0; p < 6; ++p) r[p] = *reinterpret_cast<const u32x4*>(src + p * ps);
}
__device__ __forceinline__ void bstage_store(BStage& bs, int buf, const u32x4 (&r)[6]) {
  const int col = threadIdx.x >> 2, k = bchunk(col, threadIdx.x & 3);
#pragma unroll
  for (int p = 0; p < 6; ++p) *reinterpret_cast<u32x4*>(&bs.v[buf][p][col][k]) = r[p];
}
__device__ __forceinline__ void bstage_frag(const BStage& bs, int buf, int nt, Split& x) {
  const int lane = threadIdx.x & (kWave - 1);
  const int col = 16 * nt + (lane & 15), k = bchunk(col, lane >> 4);
  x.r1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&bs.v[buf][0][col][k]));
  x.r2 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&bs.v[buf][1][col][k]));
  x.r3 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&bs.v[buf][2][col][k]));
  x.i1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&bs.v[buf][3][col][k]));
  x.i2 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&bs.v[buf][4][col][k]));
  x.i3 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&bs.v[buf][5][col][k]));
}

// Accumulates over k in [k0, k1) (multiples of kGK, at least one step):
// a_re/a_im[m] point at this lane's 16 bytes of subtile m's k-tile at k = 0
// in the k-tiled A store (step k is kAT elements on per kGK), bsrc at this
// thread's B piece at k = 0, plane stride ps.  conj_a: use conj(A).  A streams from HBM, so its loads run two steps
// ahead in three register sets used in rotation (the loop is unrolled by
// three, so no loop-carried copy makes a step wait for loads it does not
// use); B comes from the cache-resident split planes one step ahead through
// the LDS double buffer.  Loads past the last step re-read the last step.
template <int MS>
__device__ __forceinline__ void gemm_tile(const uint16_t* const (&a_re)[MS], const uint16_t* const (&a_im)[MS],
                                          const uint16_t* __restrict__ bsrc, int64_t ps, int k0, int k1, int ntv,
                                          bool conj_a, BStage& bs, f32x4 (&accr)[MS][4], f32x4 (&acci)[MS][4]) {
  const u32x4 sgn = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  const int klast = k1 - kGK;
  u32x4 br[6];
  u32x4 a0r[MS], a0i[MS], a1r[MS], a1i[MS], a2r[MS], a2i[MS];
  auto load_a = [&](int k, u32x4 (&r)[MS], u32x4 (&i)[MS]) {
#pragma unroll
    for (int m = 0; m < MS; ++m) {
      r[m] = ld16(a_re[m] + (int64_t)(k / kGK) * kAT);
      i[m] = ld16(a_im[m] + (int64_t)(k / kGK) * kAT);
    }
  };
  bstage_load(bsrc + k0, ps, br);
  load_a(k0, a0r, a0i);
  load_a(min(k0 + kGK, klast), a1r, a1i);
  bstage_store(bs, 0, br);
  __syncthreads();
  int buf = 0;
  // one k-step with A operands (cr, ci); loads step k + 2's A into (nr, ni)
  auto step = [&](int k, const u32x4 (&cr)[MS], const u32x4 (&ci)[MS], u32x4 (&nr)[MS], u32x4 (&ni)[MS]) {
    bstage_load(bsrc + min(k + kGK, klast), ps, br);
    // B before A in issue order: the counter wait before the LDS stores at
    // the end of this step then does not cover the A loads two steps ahead
    __builtin_amdgcn_sched_barrier(0);
    load_a(min(k + 2 * kGK, klast), nr, ni);
    bf16x8 A1[MS], A2[MS], A3[MS];   // (Re, Im, -Im) of A, or (Re, -Im, Im) for conj(A)
#pragma unroll
    for (int m = 0; m < MS; ++m) {
      A1[m] = as_bf16(cr[m]);
      A2[m] = as_bf16(conj_a ? (ci[m] ^ sgn) : ci[m]);
      A3[m] = as_bf16(conj_a ? ci[m] : (ci[m] ^ sgn));
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      if (nt < ntv) {
        Split x;
        bstage_frag(bs, buf, nt, x);
#pragma unroll
        for (int m = 0; m < MS; ++m) cmfma(A1[m], A2[m], A3[m], x, accr[m][nt], acci[m][nt]);
      }
    }
    bstage_store(bs, buf ^ 1, br);   // buffer buf ^ 1 was last read before the previous barrier
    __syncthreads();
    buf ^= 1;
  };
  int k = k0;
  for (; k + 3 * kGK <= k1; k += 3 * kGK) {
    step(k, a0r, a0i, a2r, a2i);
    step(k + kGK, a1r, a1i, a0r, a0i);
    step(k + 2 * kGK, a2r, a2i, a1r, a1i);
  }
  if (k < k1) step(k, a0r, a0i, a2r, a2i);
  if (k + kGK < k1) step(k + kGK, a1r, a1i, a0r, a0i);
}

// Forward product, one k-chunk: partial sums of H0[f, C_j] X over columns
// [it.m0, it.pad[0]) for rows [it.pad[2], it.pad[2] + 64 MS) of the tile and
// the up to 64 scene-tiles of the item, written to partial slot it.pad[1]
// ([slot][64 scene-tile columns][tile_rows], complex: the finisher's threads,
// one per row, then read consecutive entries).
template <int MS>
__global__ __launch_bounds__(kBlockThreads) void k_bgemm_n(BatchArgs a, const GemmItem* __restrict__ items) {
  __shared__ BStage bs;
  const GemmItem it = items[blockIdx.x];
  const BlockDesc pj = a.pseudo[it.j];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int kq = 8 * (lane >> 4);
  const uint16_t* are[MS];
  const uint16_t* aim[MS];
#pragma unroll
  for (int m = 0; m < MS; ++m) {
    // 16-row subtile of this wave's rows; lane: row lane % 16, k offset kq
    const int64_t r16 = ((int64_t)it.f * a.tile_rows + it.pad[2]) / 16 + wave * MS + m;
    const int64_t o = pj.h_off + r16 * (pj.ld / kGK) * kAT + (lane & 15) * kGK + kq;
    are[m] = a.hk_re + o;
    aim[m] = a.hk_im + o;
  }
  // B piece of this thread: the split planes of c (columns beyond cnt read a
  // valid scene-tile; their results are not stored)
  const int bcol = threadIdx.x >> 2;
  const SceneTile stb = a.stab[it.st0 + min(bcol, it.cnt - 1)];
  const uint16_t* bsrc = a.cs + (int64_t)stb.rep * a.n_pad + pj.cpad0 + 8 * (threadIdx.x & 3);
  f32x4 accr[MS][4], acci[MS][4];
#pragma unroll
  for (int m = 0; m < MS; ++m)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) accr[m][nt] = acci[m][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ntv = (it.cnt + 15) >> 4;
  if (it.m0 < it.pad[0])   // an empty chunk writes zeros
    gemm_tile<MS>(are, aim, bsrc, (int64_t)a.R * a.n_pad, it.m0, it.pad[0], ntv, false, bs, accr, acci);
  float2* out = a.pn + (int64_t)it.pad[1] * a.tile_rows * kGN;
#pragma unroll
  for (int m = 0; m < MS; ++m)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int col = 16 * nt + (lane & 15);
      if (col >= it.cnt) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = it.pad[2] + 16 * (wave * MS + m) + 4 * (lane >> 4) + e;
        out[(int64_t)col * a.tile_rows + row] = make_float2(accr[m][nt][e], acci[m][nt][e]);
      }
    }
}

// r = g' - phase o (sum of the KS k-chunk partials, in chunk order) for one
// (scene-tile, column block): blockIdx.x = scene-tile entry, blockIdx.y = j,
// one thread per tile row.
__global__ __launch_bounds__(kBlockThreads) void k_bgemm_n_fin(BatchArgs a, int KS) {
  const int p = blockIdx.x, j = blockIdx.y, rr = threadIdx.x;
  if (rr >= a.tile_rows) return;
  const SceneTile st = a.stab[p];
  const int2 gc = a.st_gc[p];
  const int64_t g = gc.x + j;
  float hr = 0.f, hi = 0.f;
  for (int kc = 0; kc < KS; ++kc) {
    const float2 q = a.pn[(((int64_t)kc * a.NG + g) * kGN + gc.y) * a.tile_rows + rr];
    hr += q.x;
    hi += q.y;
  }
  const RowBlockDesc rb = a.rbd[st.rep];
  const int64_t gr = st.row0 + rr;
  const int lr = st.lr0 + rr;
  const float2 ph = a.phases[gr];
  const float pr = ph.x * hr - ph.y * hi, pi = ph.x * hi + ph.y * hr;
  const int64_t vi = (int64_t)j * a.m_pad + rb.rpad0 + lr;
  float2 gpv = a.g[gr];
  if (a.P > 1) {
    // the other sections' estimated data, compensated sums in section order
    CSum sr, si;
    sr.add(gpv.x);
    si.add(gpv.y);
    for (int q = 0; q < a.P; ++q) {
      if (q == j) continue;
      const float2 e2 = a.ghat[(int64_t)q * a.m_pad + rb.rpad0 + lr];
      sr.add(-e2.x);
      si.add(-e2.y);
    }
    gpv = make_float2(sr.value(), si.value());
    a.gp[vi] = gpv;
  }
  a.r[vi] = make_float2(gpv.x - pr, gpv.y - pi);
}

// Adjoint product: U = H0[f, C_j]^H Y' for 4 * 16 * MS columns of block j
// (from it.m0) and the up to 64 scene-tiles of the item; K = the tile's rows,
// read from the transposed store.  Writes one partial per (scene-tile, column).
template <int MS>
__global__ __launch_bounds__(kBlockThreads) void k_bgemm_h(BatchArgs a, const GemmItem* __restrict__ items) {
  __shared__ BStage bs;
  const GemmItem it = items[blockIdx.x];
  const BlockDesc pj = a.pseudo[it.j];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int kq = 8 * (lane >> 4);
  const uint16_t* are[MS];
  const uint16_t* aim[MS];
#pragma unroll
  for (int m = 0; m < MS; ++m) {
    const int col = it.m0 + 16 * (wave * MS + m) + (lane & 15);
    const int64_t colc = min(col, pj.nj - 1);
    const int64_t o = pj.gi_off + (colc / 16) * (a.ldt / kGK) * kAT + (colc % 16) * kGK +
                      ((int64_t)it.f * a.tile_rows / kGK) * kAT + kq;
    are[m] = a.t_re + o;
    aim[m] = a.t_im + o;
  }
  const int bcol = threadIdx.x >> 2;
  const SceneTile stb = a.stab[it.st0 + min(bcol, it.cnt - 1)];
  const RowBlockDesc rbb = a.rbd[stb.rep];
  const uint16_t* bsrc = a.ys + (int64_t)it.j * a.m_pad + rbb.rpad0 + stb.lr0 + 8 * (threadIdx.x & 3);
  f32x4 accr[MS][4], acci[MS][4];
#pragma unroll
  for (int m = 0; m < MS; ++m)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) accr[m][nt] = acci[m][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ntv = (it.cnt + 15) >> 4;
  gemm_tile<MS>(are, aim, bsrc, (int64_t)a.P * a.m_pad, 0, a.tile_rows, ntv, true, bs, accr, acci);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int t = 16 * nt + (lane & 15);
    if (t >= it.cnt) continue;
    float2* out = a.part + (int64_t)a.stab[it.st0 + t].pslot * a.n_pad + pj.cpad0;
#pragma unroll
    for (int m = 0; m < MS; ++m) {
      // four consecutive columns per lane: two 16-byte stores when all exist
      const int cc = it.m0 + 16 * (wave * MS + m) + 4 * (lane >> 4);
      if (cc + 3 < pj.nj) {
        float4* o4 = reinterpret_cast<float4*>(out + cc);
        o4[0] = make_float4(accr[m][nt][0], acci[m][nt][0], accr[m][nt][1], acci[m][nt][1]);
        o4[1] = make_float4(accr[m][nt][2], acci[m][nt][2], accr[m][nt][3], acci[m][nt][3]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (cc + e < pj.nj) out[cc + e] = make_float2(accr[m][nt][e], acci[m][nt][e]);
      }
    }
  }
}

// Per-scene z-update: tiles {scene, column block, first column}, 64 columns
// per workgroup.  u_i = c_i + the adjoint partials of row block i's tiles is
// formed once and kept in registers (scenes have at most kMaxQ row blocks;
// more are recomputed in the second pass).
constexpr int kMaxQ = 8;
__global__ __launch_bounds__(kZCols) void k_bzupdate(BatchArgs a, const ColDesc* __restrict__ cols,
                                                     const int4* __restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const SceneDesc sd = a.scenes[t.x];
  const ColDesc cd = cols[t.y];
  const int col = t.z + threadIdx.x;
  if (col >= cd.nj) return;
  const int64_t p = cd.cpad0 + col;
  // compensated FP32 sums in fixed order (CSum): u = c + tile partials, and
  // the consensus sum of u + s over the replicas
  auto replica = [&](int i) {
    const int rep = sd.rb0 + i;
    const float2 c0 = a.c[(int64_t)rep * a.n_pad + p];
    CSum ur_, ui_;
    ur_.add(c0.x);
    ui_.add(c0.y);
    const int s0 = a.cuts[sd.cut0 + i], s1 = a.cuts[sd.cut0 + i + 1];
    for (int sl = s0; sl < s1; ++sl) {
      const float2 q = a.part[(int64_t)(sd.pslot0 + sl) * a.n_pad + p];
      ur_.add(q.x);
      ui_.add(q.y);
    }
    return make_float2(ur_.value(), ui_.value());
  };
  float2 ur[kMaxQ];
  CSum mr, mi;
  auto add_mean = [&](int i, const float2& u) {
    const float2 sv = a.s[(int64_t)(sd.rb0 + i) * a.n_pad + p];
    mr.add(u.x);
    mr.add(sv.x);
    mi.add(u.y);
    mi.add(sv.y);
  };
#pragma unroll
  for (int i = 0; i < kMaxQ; ++i)
    if (i < sd.Q) {
      ur[i] = replica(i);
      add_mean(i, ur[i]);
    }
  for (int i = kMaxQ; i < sd.Q; ++i) add_mean(i, replica(i));
  const float invQ = 1.0f / (float)sd.Q;
  const float ar = mr.value() * invQ, ai = mi.value() * invQ;
  if (!(isfinite(ar) && isfinite(ai))) a.ctl->nonfinite = 1;
  const float mag = sqrtf(ar * ar + ai * ai);
  float vr = 0.f, vi = 0.f;
  if (mag > sd.kappa) {
    const float sc = 1.0f - sd.kappa / mag;
    vr = ar * sc;
    vi = ai * sc;
  }
  a.v[(int64_t)t.x * a.n_pad + p] = make_float2(vr, vi);
  auto update = [&](int i, const float2& u) {
    const int64_t ip = (int64_t)(sd.rb0 + i) * a.n_pad + p;
    const float2 sv = a.s[ip];
    const float sr = sv.x + u.x - vr, si = sv.y + u.y - vi;
    a.s[ip] = make_float2(sr, si);
    a.c[ip] = make_float2(vr - sr, vi - si);
    store_split(a.cs, (int64_t)a.R * a.n_pad, ip, vr - sr, vi - si);
  };
#pragma unroll
  for (int i = 0; i < kMaxQ; ++i)
    if (i < sd.Q) update(i, ur[i]);
  for (int i = kMaxQ; i < sd.Q; ++i) update(i, replica(i));
}

// conj(phase) o y of every scene row, split into the six planes of ys.
// Grid (row chunks, row blocks); rows beyond the block are not touched.
__global__ __launch_bounds__(kBlockThreads) void k_bsplit_y(BatchArgs a) {
  const RowBlockDesc rb = a.rbd[blockIdx.y];
  const int64_t ps = (int64_t)a.P * a.m_pad;
  for (int r = blockIdx.x * kBlockThreads + threadIdx.x; r < rb.mi; r += gridDim.x * kBlockThreads) {
    const float2 ph = a.phases[(int64_t)rb.row0 + r];
    for (int j = 0; j < a.P; ++j) {
      const int64_t e = (int64_t)j * a.m_pad + rb.rpad0 + r;
      const float2 yy = a.y[e];
      store_split(a.ys, ps, e, ph.x * yy.x + ph.y * yy.y, ph.x * yy.y - ph.y * yy.x);
    }
  }
}

// H0^T store, k-tiled (rows: the block's columns, padded to 16 with zeros;
// K = ldt), from the block store [j][m0][ld_j]; 64 x 64 tiles.
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
  const int nj16 = (pj.nj + 15) / 16 * 16;
  for (int e = threadIdx.x; e < 64 * 64; e += kBlockThreads) {
    const int c = e / 64, r = e % 64;
    const int cc = c0 + c, rr = r0 + r;
    if (cc < nj16 && rr < a.ldt) {
      const int64_t o = pj.gi_off + ((int64_t)(cc / 16) * (a.ldt / kGK) + rr / kGK) * kAT + (cc % 16) * kGK + rr % kGK;
      ore[o] = tr[r][c];
      oim[o] = ti[r][c];
    }
  }
}

// The forward GEMM's k-tiled copy of block j = blockIdx.y of the block store
// (same offset and size: m0 x ld_j, both multiples of 16 and 32), one
// 16-byte unit of eight k per thread; unit u is element 8u of the tiled
// layout.
__global__ __launch_bounds__(kBlockThreads) void k_btile_h(BatchArgs a, int64_t m0) {
  const BlockDesc pj = a.pseudo[blockIdx.y];
  const int KB = pj.ld / kGK;
  const int64_t units = m0 * pj.ld / 8;
  uint16_t* dre = const_cast<uint16_t*>(a.hk_re) + pj.h_off;
  uint16_t* dim = const_cast<uint16_t*>(a.hk_im) + pj.h_off;
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x) {
    const int c8 = (int)(u & 3);
    const int64_t t = u >> 2;
    const int rr = (int)(t & 15);
    const int64_t t2 = t >> 4;
    const int kb = (int)(t2 % KB);
    const int64_t row = (t2 / KB) * 16 + rr, col = (int64_t)kb * kGK + 8 * c8;
    const int64_t src = pj.h_off + row * pj.ld + col;
    *reinterpret_cast<uint4*>(dre + 8 * u) = *reinterpret_cast<const uint4*>(a.h_re + src);
    *reinterpret_cast<uint4*>(dim + 8 * u) = *reinterpret_cast<const uint4*>(a.h_im + src);
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

hipError_t launch_bgemm_n(const BatchArgs& a, const GemmItem* items, int nitems, int ks, int ms, hipStream_t st) {
  switch (ms) {
    case 1: hipLaunchKernelGGL(k_bgemm_n<1>, dim3(nitems), dim3(kBlockThreads), 0, st, a, items); break;
    case 2: hipLaunchKernelGGL(k_bgemm_n<2>, dim3(nitems), dim3(kBlockThreads), 0, st, a, items); break;
    default: hipLaunchKernelGGL(k_bgemm_n<4>, dim3(nitems), dim3(kBlockThreads), 0, st, a, items); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bgemm_n_fin, dim3(a.NST, a.P), dim3(kBlockThreads), 0, st, a, ks);
  return hipGetLastError();
}

hipError_t launch_bgemm_h(const BatchArgs& a, const GemmItem* items, int nitems, int ms, hipStream_t st) {
  hipLaunchKernelGGL(k_bsplit_y, dim3(8, a.R), dim3(kBlockThreads), 0, st, a);
  switch (ms) {
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

hipError_t launch_btile_h(const BatchArgs& a, int P, int64_t m0, hipStream_t st) {
  hipLaunchKernelGGL(k_btile_h, dim3(1024, (unsigned)P), dim3(kBlockThreads), 0, st, a, m0);
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
