// FP64 lasso optimality check of an image v over the stored H.
//
// At a fixed point of any of the splittings the duals satisfy
// H^H (g - H v) in lambda * subdifferential(|v|_1) (the x-update optimality
// summed over replicas, with the v-update of eq. v_variable_rows_columns).
// This check computes z = H^H (g - H v) accumulated in double and the largest
// distance of z_n to lambda * d|v_n|: |z_n - lambda v_n/|v_n|| on the support,
// max(0, |z_n| - lambda) off it.
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
__global__ __launch_bounds__(kBlockThreads) void k_kkt_resid(const BlockDesc* __restrict__ blocks, int Q, int P,
                                                             const int64_t* __restrict__ row_block,
                                                             int64_t m, const float2* __restrict__ H,
                                                             const float2* __restrict__ g,
                                                             const float2* __restrict__ vpad,
                                                             double2* __restrict__ e) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int64_t row = (int64_t)blockIdx.x * (kBlockThreads / kWave) + wave;
  if (row >= m) return;
  const int i = (int)row_block[row];
  double ar = 0.0, ai = 0.0;
  for (int j = 0; j < P; ++j) {
    const BlockDesc d = blocks[i * P + j];
    const float2* Hr = H + d.h_off + (row - d.row0) * d.ld;
    const float2* vj = vpad + d.cpad0;
    for (int c = lane; c < d.nj; c += kWave) {
      const float2 h = Hr[c], v = vj[c];
      ar += (double)h.x * v.x - (double)h.y * v.y;
      ai += (double)h.x * v.y + (double)h.y * v.x;
    }
  }
  ar = wsum(ar);
  ai = wsum(ai);
  if (lane == 0) e[row] = make_double2((double)g[row].x - ar, (double)g[row].y - ai);
}

// part[(chunk*Q + i)*n_pad + col] = sum over the chunk's rows of block (i,j)
// of conj(H[row,col]) e[row], in double.  tiles = the adjoint-product tiles
// {block, first float4 column, chunk}: two columns per thread.
__global__ __launch_bounds__(kBlockThreads) void k_kkt_adj(const int4* __restrict__ tiles,
                                                           const BlockDesc* __restrict__ blocks, int Q, int KH,
                                                           int64_t n_pad, const float2* __restrict__ H,
                                                           const double2* __restrict__ e,
                                                           double2* __restrict__ part) {
  const int4 t = tiles[blockIdx.x];
  const BlockDesc d = blocks[t.x];
  const int c4 = t.y + threadIdx.x;
  if (c4 >= (d.nj + 1) / 2) return;
  const int rc = (d.mi + KH - 1) / KH;
  const int rb = min(d.mi, t.z * rc), re = min(d.mi, rb + rc);
  const float4* A = reinterpret_cast<const float4*>(H + d.h_off) + c4;
  const int64_t lda4 = d.ld / 2;
  double a0r = 0, a0i = 0, a1r = 0, a1i = 0;
  for (int r = rb; r < re; ++r) {
    const float4 h = A[(int64_t)r * lda4];
    const double2 y = e[d.row0 + r];
    a0r += (double)h.x * y.x + (double)h.y * y.y;
    a0i += (double)h.x * y.y - (double)h.y * y.x;
    a1r += (double)h.z * y.x + (double)h.w * y.y;
    a1i += (double)h.z * y.y - (double)h.w * y.x;
  }
  double2* out = part + ((int64_t)t.z * Q + d.i) * n_pad + d.cpad0 + 2 * (int64_t)c4;
  out[0] = make_double2(a0r, a0i);
  out[1] = make_double2(a1r, a1i);
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
    for (int q = 0; q < kBlockThreads / kWave; ++q) mx = fmax(mx, red[q]);
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
                          const int4* t_cols, int n_tcols, const int4* t_z, int n_tz, int64_t m, int64_t n_pad,
                          int Q, int P, int KH, const float2* H, const float2* g, const float2* vpad,
                          double lam, double2* e, double2* part, double* wgmax, Control* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_kkt_resid, dim3((unsigned)((m + 3) / 4)), dim3(kBlockThreads), 0, st, dblocks, Q, P,
                     drow_block, m, H, g, vpad, e);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_kkt_adj, dim3(n_tcols), dim3(kBlockThreads), 0, st, t_cols, dblocks, Q, KH, n_pad, H, e,
                     part);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(k_kkt_final, dim3(n_tz), dim3(kBlockThreads), 0, st, t_z, dcols, Q, KH, n_pad, part, vpad,
                     lam, wgmax, ctl);
  return hipGetLastError();
}

}  // namespace admm
