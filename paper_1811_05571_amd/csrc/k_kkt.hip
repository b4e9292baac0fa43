// FP64 lasso optimality check of an image v over the stored H.
//
// At a fixed point of any of the splittings the duals satisfy
// H^H (g - H v) in lambda * subdifferential(|v|_1) (the x-update optimality
// summed over replicas, with the v-update of eq. v_variable_rows_columns).
// This check computes z = H^H (g - H v) accumulated in double and the largest
// distance of z_n to lambda * d|v_n|: |z_n - lambda v_n/|v_n|| on the support,
// max(0, |z_n| - lambda) off it.
#include "hstore.h"
#include "plan.h"

namespace admm {

namespace {

__device__ __forceinline__ double wsum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}
__device__ __forceinline__ double wmax(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, kWave));
  return x;
}

// e[row] = g[row] - sum_j H_ij[row,:] v_j for every global row; one wave per
// row, looping over the P blocks of the row.  grid = ceil(m / 4) workgroups.
template <class F>
__global__ __launch_bounds__(kBlockThreads) void k_kkt_resid(const BlockDesc* __restrict__ blocks, int Q, int P,
                                                             const int64_t* __restrict__ row_block,
                                                             int64_t m, HStore hs,
                                                             const float2* __restrict__ g,
                                                             const float2* __restrict__ vpad,
                                                             double2* __restrict__ e) {
  const F f = MakeFmt<F>::make(hs);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int64_t row = (int64_t)blockIdx.x * (kBlockThreads / kWave) + wave;
  if (row >= m) return;
  const int i = (int)row_block[row];
  double ar = 0.0, ai = 0.0;
  for (int j = 0; j < P; ++j) {
    const BlockDesc d = blocks[i * P + j];
    const int64_t ro = d.h_off + (row - d.row0) * d.ld;
    const float2* vj = vpad + d.cpad0;
    for (int c = lane; c < d.nj; c += kWave) {
      const double2 h = f.getd(ro + c, (int)row);
      const float2 v = vj[c];
      ar += h.x * v.x - h.y * v.y;
      ai += h.x * v.y + h.y * v.x;
    }
  }
  ar = wsum(ar);
  ai = wsum(ai);
  if (lane == 0) e[row] = make_double2((double)g[row].x - ar, (double)g[row].y - ai);
}

// part[(chunk*Q + i)*n_pad + col] = sum over the chunk's rows of block (i,j)
// of conj(H[row,col]) e[row], in double; one column per thread.
// tiles[x] = {block, first column, chunk, -}.
template <class F>
__global__ __launch_bounds__(kBlockThreads) void k_kkt_adj(const int4* __restrict__ tiles,
                                                           const BlockDesc* __restrict__ blocks, int Q, int KH,
                                                           int64_t n_pad, HStore hs,
                                                           const double2* __restrict__ e,
                                                           double2* __restrict__ part) {
  const F f = MakeFmt<F>::make(hs);
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = blocks[t.x];
  const int col = t.y + threadIdx.x;
  if (col >= d.nj) return;
  const int rc = (d.mi + KH - 1) / KH;
  const int rb = min(d.mi, t.z * rc), re = min(d.mi, rb + rc);
  double ar = 0, ai = 0;
  for (int r = rb; r < re; ++r) {
    const double2 h = f.getd(d.h_off + (int64_t)r * d.ld + col, d.row0 + r);
    const double2 y = e[d.row0 + r];
    ar += h.x * y.x + h.y * y.y;
    ai += h.x * y.y - h.y * y.x;
  }
  part[((int64_t)t.z * Q + d.i) * n_pad + d.cpad0 + col] = make_double2(ar, ai);
}

// z = sum of the partials over chunks and row blocks; violation per column;
// maximum over all columns (per-workgroup maxima, then the last workgroup).
// tiles = z-update tiles {column block, first column}.
__global__ __launch_bounds__(kBlockThreads) void k_kkt_final(const int4* __restrict__ tiles,
                                                             const ColDesc* __restrict__ cols, int Q, int KH,
                                                             int64_t n_pad, const double2* __restrict__ part,
                                                             const float2* __restrict__ vpad, double lam,
                                                             double* __restrict__ wgmax, Control* ctl) {
  __shared__ double red[kBlockThreads / kWave];
  __shared__ int last;
  const int4 t = tiles[blockIdx.x];
  const ColDesc cd = cols[t.x];
  const int col = t.y + threadIdx.x;
  const int nw = blockDim.x / kWave;
  double viol = 0.0;
  if (col < cd.nj) {
    const int64_t p = cd.cpad0 + col;
    double zr = 0.0, zi = 0.0;
    for (int i = 0; i < Q; ++i)
      for (int k = 0; k < KH; ++k) {
        const double2 q = part[((int64_t)k * Q + i) * n_pad + p];
        zr += q.x;
        zi += q.y;
      }
    const double vr = vpad[p].x, vi = vpad[p].y;
    const double mag = sqrt(vr * vr + vi * vi);
    if (mag > 0.0) {
      const double dr = zr - lam * vr / mag, di = zi - lam * vi / mag;
      viol = sqrt(dr * dr + di * di);
    } else {
      viol = fmax(0.0, sqrt(zr * zr + zi * zi) - lam);
    }
    if (!isfinite(viol)) viol = INFINITY;
  }
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const double w = wmax(viol);
  if (lane == 0) red[wave] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int q = 0; q < nw; ++q) mx = fmax(mx, red[q]);
    wgmax[blockIdx.x] = mx;
    __threadfence();
    last = (atomicAdd(&ctl->kkt_ticket, 1) == (int)gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b)
      mx = fmax(mx, __hip_atomic_load(wgmax + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    ctl->kkt = mx;
    ctl->kkt_ticket = 0;
  }
}

}  // namespace

hipError_t launch_kkt_all(const BlockDesc* dblocks, const ColDesc* dcols, const int64_t* drow_block,
                          const int4* t_kadj, int n_tkadj, const int4* t_z, int n_tz, int64_t m, int64_t n_pad,
                          int Q, int P, int KH, const HStore& hs, const float2* g, const float2* vpad,
                          double lam, double2* e, double2* part, double* wgmax, Control* ctl, hipStream_t st) {
  const dim3 gr((unsigned)((m + 3) / 4)), ga(n_tkadj), blk(kBlockThreads);
  switch (hs.storage) {
    case 0:
      hipLaunchKernelGGL(k_kkt_resid<FmtC64>, gr, blk, 0, st, dblocks, Q, P, drow_block, m, hs, g, vpad, e);
      hipLaunchKernelGGL(k_kkt_adj<FmtC64>, ga, blk, 0, st, t_kadj, dblocks, Q, KH, n_pad, hs, e, part);
      break;
    case 1:
      hipLaunchKernelGGL(k_kkt_resid<FmtBF16>, gr, blk, 0, st, dblocks, Q, P, drow_block, m, hs, g, vpad, e);
      hipLaunchKernelGGL(k_kkt_adj<FmtBF16>, ga, blk, 0, st, t_kadj, dblocks, Q, KH, n_pad, hs, e, part);
      break;
    default:
      hipLaunchKernelGGL(k_kkt_resid<FmtFP8>, gr, blk, 0, st, dblocks, Q, P, drow_block, m, hs, g, vpad, e);
      hipLaunchKernelGGL(k_kkt_adj<FmtFP8>, ga, blk, 0, st, t_kadj, dblocks, Q, KH, n_pad, hs, e, part);
      break;
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  // one z-update tile (kZCols columns) per workgroup
  hipLaunchKernelGGL(k_kkt_final, dim3(n_tz), dim3(kZCols), 0, st, t_z, dcols, Q, KH, n_pad, part, vpad, lam, wgmax,
                     ctl);
  return hipGetLastError();
}

}  // namespace admm
