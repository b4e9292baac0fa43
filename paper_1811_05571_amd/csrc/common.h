// Shared definitions of the HIP ADMM library: block descriptors, layout
// constants and complex helpers.  Included by every translation unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace admm {

// Column (pixel) and row (measurement) vectors are stored padded per block so
// that every block segment starts on a 512-byte boundary and every row of the
// stored H starts 16-byte aligned.  Pads hold zeros and are never written by
// the iteration.
constexpr int kColPad = 64;    // complex elements
constexpr int kRowPad = 64;    // complex elements
constexpr int kTile = 64;      // FP64 setup tile edge (Cholesky / inverse)

constexpr int kWave = 64;      // CDNA wavefront
constexpr int kBlockThreads = 256;

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// One (i, j) block of the split.  All offsets are in elements of the
// region they index.
struct BlockDesc {
  int64_t h_off;    // H store: first element (complex) of the block
  int64_t gi_off;   // inverse store (complex64): first element
  int64_t f_off;    // FP64 setup scratch (double2): first element
  int32_t i, j;     // row block, column block
  int32_t mi, nj;   // rows, columns
  int32_t ld;       // H row stride (complex elements) = padded nj
  int32_t ldr;      // inverse row stride = padded mi
  int32_t mt;       // mi rounded up to kTile (setup matrices are mt x mt)
  int32_t row0;     // first global row
  int32_t col0;     // first global column
  int32_t rpad0;    // offset of row block i in padded row space
  int32_t cpad0;    // offset of column block j in padded column space
  int32_t pad_;
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
  int32_t ticket;        // arrival counter of the z-update reduction
  int32_t nonfinite;     // sticky NaN/Inf flag
  int32_t notpd;         // Cholesky pivot failure flag
  int32_t kkt_ticket;    // arrival counter of the KKT reduction
  int32_t pad[3];
  double red[kRedCount]; // last iteration's reduction scalars
  double kkt;            // last KKT violation (unscaled)
  double pad2[2];
};

// Storage-independent view of an H block row for the device kernels.
struct HStore {
  const void* base;      // C64: float2*, BF16: two planes of uint16, FP8: two planes of uint8
  const void* base_im;   // imaginary plane (BF16/FP8), unused for C64
  const float* row_scale;// FP8 per-row scales (indexed by global row), else null
  int storage;
};

}  // namespace admm
