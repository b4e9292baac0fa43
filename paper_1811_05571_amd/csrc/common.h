// Shared definitions of the HIP ADMM library: block descriptors, layout
// constants and complex helpers.  Included by every translation unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace admm {

// Column (pixel) and row (measurement) vectors are stored padded per block so
// that every block segment starts on a 512-byte boundary and every row of the
// stored H starts 16-byte aligned.  Pads hold zeros and are never written by
// the iteration.  Column blocks are padded to whole groups of 64 lane loads
// (64 * CPL columns, see cperm).
constexpr int kColPad = 64;    // complex elements (minimum)
constexpr int kRowPad = 64;    // complex elements
constexpr int kTile = 64;      // FP64 setup tile edge (Cholesky / inverse)

constexpr int kWave = 64;      // CDNA wavefront
constexpr int kBlockThreads = 256;

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Position of column `col` (inside its block) in the lane-permuted layout of
// the row products' input vector.  Lane l of a wave reads columns
// l*CPL .. l*CPL+CPL-1 of each group of 64*CPL columns; storing pair q of
// lane l at pair index q*64 + l makes the q-th load of all 64 lanes one
// contiguous 1 KB access.  The identity for CPL = 2.
__host__ __device__ __forceinline__ int cperm(int col, int cpl) {
  const int grp = 64 * cpl;
  const int g = col / grp, rem = col - g * grp;
  const int l = rem / cpl, k = rem - l * cpl;
  return g * grp + (((k >> 1) * 64 + l) << 1) + (k & 1);
}

// One (i, j) block of the split.  All offsets are in elements of the
// region they index.
struct BlockDesc {
  int64_t h_off;    // H store: first element (complex) of the block
  int64_t gi_off;   // inverse store (complex64): first element of the block's
                    // packed lower 64 x 64 tiles, tile (a, b), a >= b, at
                    // gi_off + (a(a+1)/2 + b) * 4096, row-major, pads zero
  int64_t f_off;    // FP64 setup scratch (double2): first element
  int32_t i, j;     // row block, column block
  int32_t mi, nj;   // rows, columns
  int32_t ld;       // H row stride (complex elements) = padded nj
  int32_t ldr;      // padded mi
  int32_t gd;       // edge of the block's Gram matrix: mi (inversion-lemma
                    // x-update, G = rho I + H H^H) or nj (direct x-update,
                    // A = H^H H + rho I)
  int32_t mt;       // gd rounded up to kTile (setup matrices are mt x mt)
  int32_t row0;     // first global row
  int32_t col0;     // first global column
  int32_t rpad0;    // offset of row block i in padded row space
  int32_t cpad0;    // offset of column block j in padded column space
  int32_t gpo;      // Gram-apply partials: first of the block's (mt/64)^2 64-vectors
};

// Compensated (Neumaier) FP32 sum: s + c carries the exact running sum to
// about twice FP32 precision; terms are added in call order.
struct CSum {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float x) {
    const float t = s + x;
    c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  __device__ __forceinline__ float value() const { return s + c; }
};

// Scalars of the per-iteration reduction (FP64).
enum : int {
  kRedRp2 = 0,   // sum_ij |u_j^i - v_j|^2
  kRedDv2 = 1,   // sum_j |v_j - v_j^prev|^2
  kRedU2 = 2,    // sum_ij |u_j^i|^2
  kRedV2 = 3,    // sum_j |v_j|^2
  kRedS2 = 4,    // sum_ij |s_j^i|^2
  kRedCount = 5
};

// Device-side control words kept in the workspace.
struct Control {
  int32_t iter;          // iterations done in the current solve (device counter)
  int32_t zpending;      // the z-update's partial sums await their final addition
  int32_t nonfinite;     // sticky NaN/Inf flag
  int32_t notpd;         // Cholesky pivot failure flag
  int32_t kkt_ticket;    // arrival counter of the KKT reduction
  int32_t unused0;
  int32_t unused1;
  int32_t pad;
  double red[kRedCount]; // last iteration's reduction scalars
  double kkt;            // last KKT violation (unscaled)
  double kbar;           // adjoint: d L / d kappa summed over iterations (k_adj_scalars)
  double rbar;           // adjoint: d L / d rho through G^{-1} and ghat (k_adj_scalars)
};
static_assert(sizeof(Control) % 16 == 0, "Control size");

// Storage-independent view of an H block row for the device kernels.
struct HStore {
  const void* base;      // C64: float2*, BF16: two planes of uint16, FP8: two planes of uint8
  const void* base_im;   // imaginary plane (BF16/FP8), unused for C64
  const float* row_scale;// FP8 per-row scales (indexed by global row), else null
  int storage;
};

}  // namespace admm
