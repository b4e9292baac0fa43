// Batched multi-scene form: S scenes that share one instrument matrix H0.
// Scene s measures the rows of its frequency tiles (tile_rows consecutive
// rows of H0 each), every row multiplied by a unit phase:
//     H_s = diag(phase_s) H0[rows_s, :].
// Each scene has its own row split (cuts at tile boundaries) and lambda; all
// scenes share the column split and rho.  The products of all scenes with
// the shared H0 are dense multi-right-hand-side GEMMs per (frequency tile,
// column block), run on MFMA with H0 in bfloat16.
#pragma once

#include "plan.h"

namespace admm {

// One (scene, tile slot) pair: a 256-row slice of a scene.
struct SceneTile {
  int32_t s;       // scene
  int32_t rep;     // global row block (replica) of the slice
  int32_t lr0;     // first row of the slice inside its row block
  int32_t row0;    // first row of the slice in the packed scene-row space
  int32_t pslot;   // partial slot of the adjoint product (global scene-tile index)
  int32_t f;       // tile of H0
  int32_t pad[2];
};

struct SceneDesc {
  int32_t rb0;     // first global row block of the scene
  int32_t Q;       // row blocks
  int32_t pslot0;  // first partial slot
  int32_t cut0;    // offset of the scene's Q+1 cuts (tile units) in the cuts array
  float kappa;     // lambda_s / (Q_s rho)
  int32_t pad[3];
};

struct RowBlockDesc {
  int32_t rpad0;   // offset in padded row space
  int32_t mi;
  int32_t row0;    // first packed scene row
  int32_t tile0;   // index of its first tile in the flattened scene-tiles array
};

// Work item of the GEMM kernels.
struct GemmItem {
  int32_t f, j;    // H0 tile, column block
  int32_t m0;      // first row (forward) / first column (adjoint) of the item
  int32_t st0;     // first scene-tile of the tile's group
  int32_t cnt;     // scene-tiles in the item (<= 64)
  int32_t pad[3];  // forward: end k, partial slot, first row
};

struct BatchArgs {
  const uint16_t *h_re, *h_im;     // H0 bf16 planes, block store [j][m0][ld_j]
  // The GEMMs' operand stores, k-tiled: a matrix of rows x K is kept as
  // tiles of 16 rows x 32 k, [row / 16][k / 32][row % 16][k % 32], so one
  // k-step of a wave's 16-row subtile is one contiguous kilobyte and its
  // k-steps follow each other in memory.
  const uint16_t *hk_re, *hk_im;   // H0 per column block: rows m0, K = ld_j (offset h_off)
  const uint16_t *t_re, *t_im;     // H0^T per column block: rows round_up(n_j, 16), K = ldt (offset gi_off)
  const BlockDesc* pseudo;         // per column block j: h_off/ld (H0 store), gi_off (H0^T store),
                                   // f_off/mt (FP64 Gram G0_j), nj, cpad0
  const SceneTile* stab;
  const SceneDesc* scenes;
  const RowBlockDesc* rbd;
  const int32_t* cuts;
  const float2* phases;            // packed per scene row
  const float2* g;                 // packed per scene row
  float2 *c, *s, *v, *part, *gp, *ghat, *r, *y;
  // bfloat16 three-term splits of the GEMM vector operands, plane p in
  // {Re t1, Re t2, Re t3, Im t1, Im t2, Im t3}:
  //   cs: of c, [p][R][n_pad];  ys: of conj(phase) o y, [p][P][m_pad]
  uint16_t *cs, *ys;
  // forward GEMM k-chunk partials [chunk][group][64][tile_rows] and, per
  // scene-tile entry, {first group index (add j), column in the group}
  float2* pn;
  const int2* st_gc;
  Control* ctl;
  int64_t m_pad, n_pad;
  int P, tile_rows, ldt, R, NG, NST;
};

// Work items: forward {f, j, first k, first scene-tile, count, end k, partial
// slot, first row}; adjoint {f, j, first column, first scene-tile, count}.
// The forward GEMM (64 * ms rows per workgroup) over ks k-chunks, then the sum
// of the chunks and r = g' - phase o (H0 x).
hipError_t launch_bgemm_n(const BatchArgs& a, const GemmItem* items, int nitems, int ks, int ms, hipStream_t st);
// The adjoint GEMM (64 * ms columns per workgroup), preceded by the split of
// conj(phase) o y (k_bsplit_y).
hipError_t launch_bgemm_h(const BatchArgs& a, const GemmItem* items, int nitems, int ms, hipStream_t st);
hipError_t launch_bzupdate(const BatchArgs& a, const ColDesc* cols, const int4* tiles, int ntiles, hipStream_t st);
hipError_t launch_btranspose(const BatchArgs& a, int P, int64_t m0, int max_nj, hipStream_t st);
// The k-tiled copy hk of the block store (after it is written).
hipError_t launch_btile_h(const BatchArgs& a, int P, int64_t m0, hipStream_t st);
hipError_t launch_bgram_assemble(const int4* tiles, int ntiles, const BlockDesc* blocks, const int32_t* blk_tile0,
                                 const int32_t* tiles_flat, const float2* phases, const double2* G0,
                                 const BlockDesc* pseudo, int tile_rows, double rho, double2* A, hipStream_t st);
hipError_t launch_bunpad_v(const ColDesc* cols, int P, int64_t n, int S, int64_t n_pad, const float2* v,
                           float2* out, hipStream_t st);

}  // namespace admm
