// Single-pass iteration of the split-lasso ADMM (arXiv 1811.05571, Sec. III-C)
// over a column-slab copy of H.
//
// The two-pass iteration (k_iter.hip) reads H twice per iteration: once for
// the forward products H_ij c and once for the adjoint products H_ij^H y.  The
// z-update of a column needs only that column of every replica (the mean over
// the row blocks and the element-wise threshold of eqs. v_variable_rows_columns
// and softhresholding), so a workgroup holding a slab of CPL columns over all
// rows can, in one visit of the slab:
//   1. form u_j^i = c_j^i + H_ij^H y_ij on the slab's columns for every i
//      (the x-update of eq. x_solution_rows_columns in push-through form),
//   2. apply the z-update and the dual update (eq. s_variable_rows_columns)
//      to those columns, giving the next c = v - s, and
//   3. accumulate the next iteration's forward products H_ij c_j^i from the
//      slab it still holds in registers.
// Every element of H then comes from HBM once per iteration.  A workgroup owns
// a run of slabs of one column block and keeps, for every row, its part of
// H c over its slabs; k_fz_rows adds the parts of a column block's workgroups
// in a fixed order and forms r_ij = g'_ij - H_ij c (g'_ij by eq.
// g_rows_columns).  One iteration is k_fz_rows, the Gram apply of k_iter.hip
// (y = G^{-1} r, ghat = g' - rho y) and k_fz_slab.  Sums run in a fixed order
// (no atomics), so runs are bitwise reproducible.
#include "gemv.h"

namespace admm {

// Workgroup barrier for data exchanged through LDS: the wave's own LDS
// accesses complete (lgkmcnt 0), then s_barrier; the empty asm statements
// keep the compiler from moving memory accesses across it.  Unlike
// __syncthreads it leaves global loads in flight, including the next slab's
// rows (a workgroup fence would wait for those).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt, expcnt not waited for
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// a + b = s + e exactly (Knuth's two-sum; the same s and e for (b, a)).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// r_ij = g'_ij - s_row (H_ij c) for the rows of one tile, H_ij c the sum of
// the column block's workgroup parts (s_row: fp8 row scale).
// tiles[x] = {block, first row, S, -}: kBlockThreads / S rows, S threads per
// row (S a power of two); thread s of a row adds the s-th of S consecutive
// runs of the parts in order, then the row's first thread adds the S run sums
// in run order (S = 1: one ordered sum).  Workgroup 0 first completes the
// previous iteration's residual sums.
template <class F>
__global__ __launch_bounds__(kBlockThreads) void k_fz_rows(IterArgs a, FzArgs z, const int4* __restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];   // descriptors before any store: scalar loads
  const BlockDesc d = a.blocks[t.x];
  const int2 wr = z.colwg[d.j];
  if (blockIdx.x == 0) {
    __shared__ double red[kBlockThreads / kWave][kRedCount];
    zfinal(a, red);
  }
  const F f = MakeFmt<F>::make(a.hs);
  const int S = t.z, R = kBlockThreads / S;
  const int r = threadIdx.x & (R - 1), s = threadIdx.x / R;
  const int lr = t.y + r;
  const bool live = lr < d.mi;
  const int T = wr.y - wr.x, w0 = T * s / S, w1 = T * (s + 1) / S;
  RowEpi epi;
  if (live && s == 0) row_epi_load(a, d, f, lr, epi);
  float2 hc = make_float2(0.f, 0.f);
  if (live) hc = ordered_sum(z.fpart + (int64_t)(wr.x + w0) * a.m_pad + d.rpad0 + lr, w1 - w0, a.m_pad);
  if (S > 1) {
    __shared__ float2 runs[kBlockThreads];
    runs[threadIdx.x] = hc;
    __syncthreads();
    if (s == 0) {
      float ar = 0.f, ai = 0.f;
      for (int q = 0; q < S; ++q) {
        ar += runs[q * R + r].x;
        ai += runs[q * R + r].y;
      }
      hc = make_float2(ar, ai);
    }
  }
  if (live && s == 0) row_epi_store(a, d, lr, hc.x, hc.y, epi);
}

// The slab pass.  Workgroup w takes the run of slabs [sl0, sl1) of column
// block j (work[w]); wave v holds the ngw[v] 64-row groups g0[v] .. of one row block
// wblk[v] (a row block spans whole waves), lane l row 64 g + l of group g, one
// 16-byte lane load per row: RPL lane loads of the current slab stay in
// registers.  Per slab:
//   adjoint : per-lane sums of conj(H) y over the lane's rows, closed over
//             the wave (reduce-scatter) into red[wave];
//   z-update: lane i*CPL + t of wave 0 owns replica i of column t of the
//             slab: u^i = c^i + the sums of block i's waves (compensated), the
//             mean over the replicas by a compensated butterfly, the
//             threshold, the duals and c, residual partial sums in FP64;
//   forward : every lane adds H[row, slab] c^{i(row)}[slab] to its row sums.
// The lane loads go to a second register set: the next slab's are issued as
// a slab's processing starts and stay in flight through its adjoint step,
// z-update and forward step.
// mode 1 skips the first two steps (forward products of the state's c).
// YL: y of the column block in LDS instead of RPL registers per lane.
template <class F, int NT, int RPL, bool YL>
__global__ __launch_bounds__(NT, 4) void k_fz_slab(IterArgs a, FzArgs z) {   // >= 4 waves per SIMD: <= 128 VGPRs
  constexpr int CPL = F::CPL, NW = NT / kWave;
  static_assert(NW <= kFzMaxWaves && RPL <= 32, "slab kernel shape");
  static_assert(kFzMaxQ * CPL <= kWave, "the z-update takes one lane of wave 0 per replica and column");
  __shared__ float2 ys[YL ? NT * RPL : 1];
  __shared__ float red[NW][2 * CPL];
  __shared__ float2 zc[kFzMaxQ * CPL], zs[kFzMaxQ * CPL], zv[CPL], cn[kFzMaxQ * CPL];
  __shared__ int bws[kFzMaxQ + 1];            // waves of each row block (read per lane)
  // The z-update's new s, c (replica i, column t of slab g0 + k at [k][i CPL
  // + t]) and v of a group of kGS slabs: written out as whole 128-byte lines
  // per replica once the group is done (16-byte pieces per slab, scattered
  // through the stream of H, cost 7 % of the kernel's time).
  constexpr int kGS = 8;
  __shared__ float2 ws_s[kGS][kFzMaxQ * CPL], ws_c[kGS][kFzMaxQ * CPL], ws_v[kGS][CPL];
  const int4 wk = z.work[blockIdx.x];
  const int j = wk.x, sl0 = wk.y, sl1 = wk.z, sgb = wk.w;
  const ColDesc cd = a.cols[j];
  const F f = MakeFmt<F>::make(z.hsl);
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int ngw = z.ngw[wave], blk = z.wblk[wave];
  const int rb = kWave * z.g0[wave] + lane;   // this lane's row in its first group
  const int Q = a.Q, QC = a.Q * CPL;
  const int64_t mp = a.m_pad, np = a.n_pad;
  const bool full = z.mode == 0;

  // h: the rows of the slab being processed; hn: the next slab's, loaded
  // straight into registers while this one is processed (staging them in
  // LDS instead measured 6 % slower: the loads into LDS and the loop's own
  // LDS traffic share the LDS).
  typename F::Raw h[RPL];
  float2 yv[YL ? 1 : RPL];
  float fr[RPL], fi[RPL];
  typename F::Raw hn[RPL];
  auto stage = [&](int sl) {   // slab sl's rows of this wave -> hn
    const float4* sp = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(z.hsl.base) +
                                                       ((int64_t)(sgb + sl) * mp * CPL) * 8);
#pragma unroll
    for (int k = 0; k < RPL; ++k)
      if (k < ngw) hn[k] = typename F::Raw{ldnt4(sp + rb + kWave * k)};
  };
  auto unstage = [&]() {   // after the wait for hn at a slab's start
#pragma unroll
    for (int k = 0; k < RPL; ++k) h[k] = hn[k];
  };
  {
    const float2* yj = a.y + (int64_t)j * mp;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      fr[k] = fi[k] = 0.f;
      if (!YL) yv[k] = make_float2(0.f, 0.f);
      h[k] = typename F::Raw{};
      hn[k] = typename F::Raw{};
      if (k < ngw) {
        const int rp = rb + kWave * k;
        float2 yy = yj[rp];
        if constexpr (CPL == 16) {   // fp8: (diag(s) Hq)^H y = Hq^H (s o y)
          const int lr = rp - z.rpad0[blk];
          const float sc = lr < z.mi[blk] ? f.row_scale(z.row0[blk] + lr) : 0.f;
          yy = make_float2(sc * yy.x, sc * yy.y);
        }
        if (YL)
          ys[rp] = yy;
        else
          yv[k] = yy;
      }
    }
  }
  stage(sl0);
  // c, s and the previous v of the slab's columns: thread t < Q*CPL holds
  // replica t / CPL of column t % CPL; issued one slab ahead.
  float2 pc = make_float2(0.f, 0.f), ps = pc, pv = pc;
  auto prefetch = [&](int sl) {
    if (tid < QC) {
      const int i = tid / CPL, q = tid - i * CPL;
      const int col = sl * CPL + q;
      pc = ps = pv = make_float2(0.f, 0.f);
      if (col < cd.nj) {
        pc = a.c[(int64_t)i * np + cd.cpad0 + cperm(col, a.cpl)];
        if (full) {
          ps = a.s[(int64_t)i * np + cd.cpad0 + col];
          if (tid < CPL) pv = a.v[cd.cpad0 + col];
        }
      }
    }
  };
  prefetch(sl0);
  // residual partial sums of the z-update lanes (wave 0), in LDS: the
  // registers go to the next slab's rows
  __shared__ double racc[kRedCount][kWave];
  if (wave == 0)
#pragma unroll
    for (int q = 0; q < kRedCount; ++q) racc[q][lane] = 0.0;
  // butterfly levels of the replica sum: lanes i*CPL + t, i < Q, span the
  // lowest log2(CPL) + ceil(log2 Q) lane bits (the lanes above hold zeros)
  int qspan = CPL;
  while (qspan < QC) qspan <<= 1;
  if (tid <= Q) bws[tid] = z.bw[tid];
  lds_barrier();   // ys and bws complete

  // slabs [g0, g1) of the group buffers -> s, c, v (wave 0; issued after a
  // slab's wait, so the next slab's wait gives the writes a slab's time)
  auto flush = [&](int g0, int g1) {
    if (wave == 0) {
      const int ncol = (g1 - g0) * CPL;
      for (int e = lane; e < Q * kGS * CPL; e += kWave) {
        const int i = e / (kGS * CPL), k = e - i * (kGS * CPL), col = g0 * CPL + k;
        if (k < ncol && col < cd.nj) {
          const int slot = k / CPL, t = k - slot * CPL;
          // 32-bit element offsets from the (uniform) array bases
          const uint32_t p = (uint32_t)(cd.cpad0 + col), r = (uint32_t)i * (uint32_t)np;
          a.s[r + p] = ws_s[slot][i * CPL + t];
          a.c[r + (uint32_t)(cd.cpad0 + cperm(col, a.cpl))] = ws_c[slot][i * CPL + t];
          if (i == 0) a.v[p] = ws_v[slot][t];
        }
      }
    }
  };
  for (int sl = sl0; sl < sl1; ++sl) {
    const bool more = sl + 1 < sl1;
    const int g0 = max(sl0, sl - sl % kGS);   // this slab's group
    // this slab's rows in hn (loaded a slab ago), the prefetched c, s, v and
    // the group stores of the previous slab's start: all complete
    __builtin_amdgcn_s_waitcnt(0);
    unstage();
    if (full && sl > sl0 && sl % kGS == 0) flush(max(sl0, sl - kGS), sl);   // the previous group
    if (tid < QC) {   // read after this slab's first barrier
      zc[tid] = pc;
      zs[tid] = ps;
      if (tid < CPL) zv[tid] = pv;
    }
    if (more) {
      stage(sl + 1);
    }
    if (full) {
      float ar[CPL][2];
#pragma unroll
      for (int q = 0; q < CPL; ++q) ar[q][0] = ar[q][1] = 0.f;
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        if (k < ngw) {
          float hr[CPL], hi[CPL];
          F::decode(h[k], hr, hi);
          const float2 yk = YL ? ys[rb + kWave * k] : yv[k];
#pragma unroll
          for (int q = 0; q < CPL; ++q) cmacc(ar[q][0], ar[q][1], hr[q], hi[q], yk.x, yk.y);
        }
      }
      if (ngw > 0) {
        float outr, outi;
        rows_reduce<CPL, true>(ar, outr, outi);
        if ((lane & (kWave / CPL - 1)) == 0) {
          const int q = rows_reduce_row<CPL>(lane);
          red[wave][2 * q] = outr;
          red[wave][2 * q + 1] = outi;
        }
      }
      lds_barrier();
      if (wave == 0) {
        // lane i*CPL + t: replica i of the slab's column t
        const int i = lane / CPL, t = lane - i * CPL, col = sl * CPL + t;
        const bool act = i < Q, valid = act && col < cd.nj;
        float xr = 0.f, xi = 0.f, sr0 = 0.f, si0 = 0.f;
        if (valid) {
          // u^i = c^i + H_ij^H y_ij: block i's wave sums, compensated, in order
          const float2 ci = zc[lane];
          CSum ur, ui;
          ur.add(ci.x);
          ui.add(ci.y);
#pragma unroll 1
          for (int w = bws[i]; w < bws[i + 1]; ++w) {
            ur.add(red[w][2 * t]);
            ui.add(red[w][2 * t + 1]);
          }
          xr = ur.value();
          xi = ui.value();
          const float2 sv = zs[lane];
          sr0 = sv.x;
          si0 = sv.y;
        }
        // consensus sum of u^i + s^i over the replicas (lanes t, t + CPL, ...):
        // a compensated butterfly over the replica lanes, so every lane of the
        // column ends with the same total
        float mr, er, mi, ei;
        two_sum(xr, sr0, mr, er);
        two_sum(xi, si0, mi, ei);
        for (int msk = CPL; msk < qspan; msk <<= 1) {
          const float omr = __shfl_xor(mr, msk, kWave), oer = __shfl_xor(er, msk, kWave);
          const float omi = __shfl_xor(mi, msk, kWave), oei = __shfl_xor(ei, msk, kWave);
          float e1, e2;
          two_sum(mr, omr, mr, e1);
          two_sum(mi, omi, mi, e2);
          er = (er + oer) + e1;
          ei = (ei + oei) + e2;
        }
        if (valid) {
          const float invQ = 1.0f / (float)Q;
          const float mar = (mr + er) * invQ, mai = (mi + ei) * invQ;
          if (!(isfinite(mar) && isfinite(mai))) a.ctl->nonfinite = 1;
          // eq. softhresholding with sign(a) = a/|a|
          const float mag = sqrtf(mar * mar + mai * mai);
          float vr = 0.f, vi = 0.f;
          if (mag > a.kappa) {
            const float sc = 1.0f - a.kappa / mag;
            vr = mar * sc;
            vi = mai * sc;
          }
          const float dr = xr - vr, di = xi - vi;
          const float sr = sr0 + dr, sim = si0 + di;
          const float2 cnew = make_float2(vr - sr, vi - sim);
          ws_s[sl - g0][lane] = make_float2(sr, sim);
          ws_c[sl - g0][lane] = cnew;
          cn[lane] = cnew;
          racc[kRedRp2][lane] += (double)dr * dr + (double)di * di;
          racc[kRedU2][lane] += (double)xr * xr + (double)xi * xi;
          racc[kRedS2][lane] += (double)sr * sr + (double)sim * sim;
          if (i == 0) {
            ws_v[sl - g0][t] = make_float2(vr, vi);
            const float2 vo = zv[t];
            const double dvr = (double)vr - vo.x, dvi = (double)vi - vo.y;
            racc[kRedDv2][lane] += dvr * dvr + dvi * dvi;
            racc[kRedV2][lane] += (double)vr * vr + (double)vi * vi;
          }
        } else if (act) {
          cn[lane] = make_float2(0.f, 0.f);
        }
      }
      lds_barrier();
    } else {
      lds_barrier();   // the previous slab's forward step has read cn
      if (tid < QC) cn[tid] = zc[tid];
      lds_barrier();
    }
    if (more) prefetch(sl + 1);   // into LDS at the next slab's start
    float2 cb[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) cb[q] = cn[blk * CPL + q];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      if (k < ngw) {
        float hr[CPL], hi[CPL];
        F::decode(h[k], hr, hi);
#pragma unroll
        for (int q = 0; q < CPL; ++q) cmac(fr[k], fi[k], hr[q], hi[q], cb[q].x, cb[q].y);
      }
    }
  }
  if (full && sl1 > sl0) flush(max(sl0, (sl1 - 1) - (sl1 - 1) % kGS), sl1);   // the last group
  float2* fp = z.fpart + (int64_t)blockIdx.x * mp;
#pragma unroll
  for (int k = 0; k < RPL; ++k)
    if (k < ngw) fp[rb + kWave * k] = make_float2(fr[k], fi[k]);
  if (full && wave == 0) {
    double acc[kRedCount];
#pragma unroll
    for (int q = 0; q < kRedCount; ++q) acc[q] = wave_sum_d(racc[q][lane]);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < kRedCount; ++q) a.redpart[(int64_t)blockIdx.x * kRedCount + q] = acc[q];
      if (blockIdx.x == 0) a.ctl->zpending = 1;
    }
  }
}

// Slab store from the H store (setup): row rp of slab sl of column block j
// holds lane load sl of row rp - rpad0_i of block (i, j); pad rows stay zero.
// grid = (ceil(m_pad / 256), P).
template <class F>
__global__ __launch_bounds__(kBlockThreads) void k_pack_slabs(HStore src, HStore dst,
                                                              const BlockDesc* __restrict__ blocks, int Q, int P,
                                                              int64_t m_pad, FzArgs z) {
  constexpr int CPL = F::CPL;
  constexpr int ES = CPL == 2 ? 8 : (CPL == 8 ? 2 : 1);   // bytes per element of a plane
  constexpr int NPL = CPL == 2 ? 1 : 2;                    // planes
  const int j = blockIdx.y;
  const int64_t rp = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x;
  if (rp >= m_pad) return;
  int i = 0;
  while (i + 1 < Q && rp >= z.rpad0[i + 1]) ++i;
  const int lr = (int)(rp - z.rpad0[i]);
  if (lr >= z.mi[i]) return;
  const BlockDesc d = blocks[i * P + j];
  const int ns = (d.nj + CPL - 1) / CPL;
  const int64_t sgb = z.work[z.colwg[j].x].w;
  const char* sp[2] = {static_cast<const char*>(src.base), static_cast<const char*>(src.base_im)};
  char* dp[2] = {static_cast<char*>(const_cast<void*>(dst.base)), static_cast<char*>(const_cast<void*>(dst.base_im))};
  for (int sl = 0; sl < ns; ++sl) {
    const int64_t se = (d.h_off + (int64_t)lr * d.ld + (int64_t)sl * CPL) * ES;
    const int64_t de = ((sgb + sl) * m_pad + rp) * CPL * ES;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl)
      *reinterpret_cast<uint4*>(dp[pl] + de) = *reinterpret_cast<const uint4*>(sp[pl] + se);
  }
}

// ---- launchers ------------------------------------------------------------
hipError_t launch_fz_rows(const IterArgs& a, const FzArgs& z, const int4* tiles, int ntiles, hipStream_t st,
                          KTime kt) {
  switch (a.hs.storage) {
    case 0: LAUNCH_TIMED(k_fz_rows<FmtC64>, dim3(ntiles), dim3(kBlockThreads), st, kt, a, z, tiles); break;
    case 1: LAUNCH_TIMED(k_fz_rows<FmtBF16>, dim3(ntiles), dim3(kBlockThreads), st, kt, a, z, tiles); break;
    default: LAUNCH_TIMED(k_fz_rows<FmtFP8>, dim3(ntiles), dim3(kBlockThreads), st, kt, a, z, tiles); break;
  }
  return hipGetLastError();
}

namespace {
template <class F, int NT, int RPL, bool YL>
hipError_t fz_go(const IterArgs& a, const FzArgs& z, hipStream_t st, KTime kt) {
  LAUNCH_TIMED((k_fz_slab<F, NT, RPL, YL>), dim3(z.nwg), dim3(NT), st, kt, a, z);
  return hipGetLastError();
}
}  // namespace

// Shapes built (complex64 storage): 512 threads (8 waves of rows, two
// workgroups per CU) and 1024 threads (16 waves, one workgroup per CU), each
// with RPL 1..6 groups of 64 rows per wave and y in LDS.  bf16 / fp8 lane loads decode into four times the registers per row
// and take the two-pass kernels.
hipError_t launch_fz_slab(const IterArgs& a, const FzArgs& z, int nt, int rpl, hipStream_t st, KTime kt) {
  if (a.hs.storage != 0) return hipErrorInvalidValue;
  if (nt == 512) {
    switch (rpl) {
      case 1: return fz_go<FmtC64, 512, 1, true>(a, z, st, kt);
      case 2: return fz_go<FmtC64, 512, 2, true>(a, z, st, kt);
      case 3: return fz_go<FmtC64, 512, 3, true>(a, z, st, kt);
      case 4: return fz_go<FmtC64, 512, 4, true>(a, z, st, kt);
      case 6: return fz_go<FmtC64, 512, 6, true>(a, z, st, kt);
      default: return hipErrorInvalidValue;
    }
  }
  if (nt == 1024) {
    switch (rpl) {
      case 1: return fz_go<FmtC64, 1024, 1, true>(a, z, st, kt);
      case 2: return fz_go<FmtC64, 1024, 2, true>(a, z, st, kt);
      case 3: return fz_go<FmtC64, 1024, 3, true>(a, z, st, kt);
      case 4: return fz_go<FmtC64, 1024, 4, true>(a, z, st, kt);
      case 6: return fz_go<FmtC64, 1024, 6, true>(a, z, st, kt);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pack_slabs(const HStore& src, const HStore& dst, const BlockDesc* blocks, int Q, int P,
                             int64_t m_pad, const FzArgs& z, hipStream_t st) {
  const dim3 grid((unsigned)((m_pad + kBlockThreads - 1) / kBlockThreads), (unsigned)P);
  if (src.storage != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack_slabs<FmtC64>, grid, dim3(kBlockThreads), 0, st, src, dst, blocks, Q, P, m_pad, z);
  return hipGetLastError();
}

}  // namespace admm
