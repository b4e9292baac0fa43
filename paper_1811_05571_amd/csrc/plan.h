// Host-side plan of the ADMM library and the launchers each kernel file
// exports to the C ABI layer.
#pragma once

#include <algorithm>

#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "common.h"

namespace admm {

struct ColDesc {       // one column block j
  int32_t nj, cpad0, col0, ld;
};

// Single-pass iteration over a column-slab copy of H (k_fused.hip).  A slab
// is CPL consecutive columns of one column block over every row of the
// padded row space; in the slab store it is m_pad x CPL elements, row-major,
// so one 16-byte lane load per plane reads one row of it.  A workgroup owns a
// strided set of slabs of one column block; each of its waves owns up to RPL
// consecutive 64-row groups of one row block (a row block spans whole waves).
constexpr int kFzMaxWaves = 16;     // waves per workgroup
constexpr int kFzMaxQ = 16;         // row blocks (each needs at least one wave)
struct FzArgs {
  HStore hsl;                       // slab store (same formats as the H store; row scales by global row)
  float2* fpart;                    // [workgroup][m_pad]: that workgroup's part of H c for every row
  const int4* work;                 // per workgroup {column block, first slab, end slab, slab base of the block}
  const int2* colwg;                // per column block {first workgroup, end workgroup}
  int nwg, mode;                    // mode 0: full iteration step, 1: forward products only (c of the state)
  int ngw[kFzMaxWaves];             // 64-row groups of each wave
  int g0[kFzMaxWaves];              // first group of each wave (padded row 64 g0)
  int wblk[kFzMaxWaves];            // row block of each wave
  int bw[kFzMaxQ + 1];              // waves of row block i: [bw[i], bw[i+1])
  int rpad0[kFzMaxQ], mi[kFzMaxQ], row0[kFzMaxQ];   // row blocks (row scales of fp8)
};
#ifndef ADMM_FZR_LOADS
#define ADMM_FZR_LOADS 16               // most workgroup parts of H c one thread of the row kernel adds
#endif
constexpr int kFzRpl[] = {1, 2, 3, 4, 6};   // row groups per wave built (512 and 1024 threads)
#ifndef ADMM_FZ_WGS
#define ADMM_FZ_WGS 512                 // about this many slab-pass workgroups (two per CU)
#endif

struct Layout {
  size_t H = 0, H_im = 0, H_scale = 0, Ginv = 0, Ginv16 = 0, F64a = 0, F64b = 0;
  size_t c = 0, s = 0, v = 0, part = 0, gp = 0, ghat = 0, r = 0, y = 0;
  size_t blocks = 0, cols = 0, t_rows = 0, t_cols = 0, t_z = 0, t_gram = 0, t_kadj = 0, t_hrows = 0, t_gtr = 0;
  size_t t_wrows = 0, t_gpatch = 0;
  size_t gpart = 0;
  size_t Hs = 0, Hs_im = 0, fpart = 0, t_fz = 0, fz_colwg = 0, t_fzr = 0, hs_bytes = 0;
  size_t t_dgp = 0, dflag = 0;
  size_t ctl = 0, redpart = 0, row_block = 0, kkt_e = 0, kkt_v = 0, kkt_part = 0, kkt_max = 0;
  size_t vb = 0, sb = 0, ub = 0, ghb = 0, gpb = 0, yb = 0, rb = 0, gbar = 0, kpart = 0, rpart = 0;
  size_t total = 0;
  size_t h_bytes = 0, ginv_bytes = 0;
};

struct Geometry {
  int64_t m = 0, n = 0;
  int Q = 0, P = 0, storage = 0;   // storage: H format (ADMM_STORAGE_*)
  bool inv16 = false;              // a bfloat16-pair copy of the inverses is kept and applied
  bool force_patches = false;      // ADMM_GRAM_PATCHES
  bool direct = false;             // every block takes the direct x-update (Gram space = column space)
  std::vector<int64_t> ro, co;
  std::vector<BlockDesc> blocks;   // Q*P, index b = i*P + j
  std::vector<ColDesc> cols;       // P
  int64_t m_pad = 0, n_pad = 0;    // padded row / column space lengths
  int KH = 1;                      // row chunks of the adjoint product
  int max_mt = 0;                  // largest tile-padded block edge
  std::vector<int4> t_rows, t_cols, t_z, t_gram, t_kadj, t_hrows, t_gtr;
  std::vector<int4> t_wrows;       // whole-row tiles of the row product (empty: not used)
  std::vector<int4> t_gpatch;      // 4 x 4 tile patches of the Gram apply (empty: single tiles)
  // single-pass iteration (empty t_fz: the two-pass kernels run)
  bool fz = false;
  int fz_nt = 0, fz_rpl = 0;       // threads per workgroup, 64-row groups per wave
  int64_t fz_slabs = 0;            // slabs in the slab store
  std::vector<int4> t_fz;          // per workgroup {j, first slab, end slab, slab base of block j}
  std::vector<int2> fz_colwg;      // per column block {first, end workgroup}
  std::vector<int4> t_fzr;         // row kernel: {block, first row, S, -}, 256 / S rows each
  FzArgs fzt{};                    // the host part of the single-pass arguments (tables)
  std::vector<int4> t_dgp;         // direct form: {row block, first row, -, -}, kBlockThreads rows each
  Layout lay;
};

// Launch shapes of the H products.  Build-time constants; the defaults are the
// measured best on MI355X at 6144 x 32000 (-D overrides serve tuning sweeps).
#ifndef ADMM_ROW_WAVES
#define ADMM_ROW_WAVES 4        // waves per workgroup of the H row products
#endif
#ifndef ADMM_ROWS_C64
#define ADMM_ROWS_C64 8         // rows per wave of the complex64 row product
#endif
#ifndef ADMM_UNROLL_C64
#define ADMM_UNROLL_C64 4       // lane loads in flight per row (complex64)
#endif
#ifndef ADMM_ROWS_NARROW
#define ADMM_ROWS_NARROW 4      // rows per wave of the bf16 / fp8 row product
#endif
#ifndef ADMM_EPI_PREFETCH_C64
#define ADMM_EPI_PREFETCH_C64 1 // complex64 row product: load the row epilogue's operands before the stream
#endif
#ifndef ADMM_EPI_PREFETCH_NARROW
#define ADMM_EPI_PREFETCH_NARROW 1  // the same for bf16 / fp8
#endif
#ifndef ADMM_UNROLL_NARROW
#define ADMM_UNROLL_NARROW 1    // lane loads in flight per row (bf16 / fp8)
#endif
#ifndef ADMM_COLS_UNROLL_C64
#define ADMM_COLS_UNROLL_C64 8  // rows in flight per wave of the adjoint product (complex64)
#endif
#ifndef ADMM_COLS_UNROLL_NARROW
#define ADMM_COLS_UNROLL_NARROW 4  // the same for bf16 / fp8
#endif
#ifndef ADMM_COLS_WG_TARGET
#define ADMM_COLS_WG_TARGET 1024  // about this many workgroups of the adjoint product (bf16, fp8)
#endif
#ifndef ADMM_COLS_WG_TARGET_C64
#define ADMM_COLS_WG_TARGET_C64 4096  // the same for complex64 storage
#endif
constexpr int kRowWaves = ADMM_ROW_WAVES;
#ifndef ADMM_XLDS_NARROW
#define ADMM_XLDS_NARROW 1      // bf16 / fp8 row product: stage each block's c in LDS (when it fits)
#endif
constexpr int kXStage = 2048;    // float4 of c staged per workgroup (32 KB: column blocks up to 4096)
constexpr int kEpiSections = 7;  // other sections whose estimates the row epilogue prefetches (P <= 8)
#ifndef ADMM_WHOLE_ROWS
#define ADMM_WHOLE_ROWS 1       // complex64 row product with whole rows per workgroup where blocks allow
#endif
#ifndef ADMM_WHOLE_ROWS_BF16
#define ADMM_WHOLE_ROWS_BF16 1  // the same for bf16
#endif
#ifndef ADMM_WHOLE_ROWS_FP8
#define ADMM_WHOLE_ROWS_FP8 0   // the same for fp8 (measured slower: 74 vs 71 us at 6144 x 32000)
#endif
#ifndef ADMM_WHOLE_WIDE
#define ADMM_WHOLE_WIDE 1       // whole-row product also for column blocks wider than kWholeCols (in chunks)
#endif
#ifndef ADMM_WHOLE_N_BF16
#define ADMM_WHOLE_N_BF16 4     // rows per workgroup of the whole-row product, bf16
#endif
#ifndef ADMM_WHOLE_N_FP8
#define ADMM_WHOLE_N_FP8 8      // the same for fp8
#endif
#ifndef ADMM_SETUP_MFMA
#define ADMM_SETUP_MFMA 1       // FP64 setup tile products on the matrix cores (0: vector FMAs)
#endif
#ifndef ADMM_GRAM_PATCH
#define ADMM_GRAM_PATCH 1       // complex64 inverses applied in 4 x 4 tile patches
#endif
// Gram-apply pieces per block (64-vectors): single tiles use T per row tile,
// 4 x 4 patches ceil(T/4) + 1; the region holds either layout.
inline int64_t gram_part_vecs(int64_t T) { return std::max(T * T, T * ((T + 3) / 4 + 1)); }
constexpr size_t kGramPatchMin = 4096;   // patches used by default from this many on
constexpr int kWholeCols = 4096; // columns per chunk of the whole-row product
// rows per workgroup of the whole-row product (its tiles follow it)
inline int whole_rows(int storage) { return storage == 0 ? 2 : (storage == 1 ? ADMM_WHOLE_N_BF16 : ADMM_WHOLE_N_FP8); }

static_assert(kRowWaves >= 1 && kRowWaves <= kBlockThreads / kWave, "row waves");

// Rows handled by one workgroup of the row-parallel products.
constexpr int kRowsPerWave = 4;
constexpr int kRowsPerWG = kRowsPerWave * (kBlockThreads / kWave);
// Lane loads (CPL complex columns each) handled by one workgroup of the
// adjoint product: its four waves share the columns and split the rows.
constexpr int kColsPerWGLoads = kWave;
// Complex columns per lane load for a storage format.
inline int cols_per_load(int storage) { return storage == 0 ? 2 : (storage == 1 ? 8 : 16); }
// Rows per wave of the H row products (the tiles of k_gemv_n follow it).
inline int rows_per_wave(int storage) { return storage == 0 ? ADMM_ROWS_C64 : ADMM_ROWS_NARROW; }
// Bytes per stored complex element.
inline int elem_bytes(int storage) { return storage == 0 ? 8 : (storage == 1 ? 4 : 2); }
constexpr int kZCols = kWave;   // columns (lanes) per z-update workgroup

int build_geometry(Geometry& geo, int64_t m, int64_t n, int Q, const int64_t* row_off, int P,
                   const int64_t* col_off, int storage, std::string& err);

// ---- kernel launchers (return hipError_t) --------------------------------
struct IterArgs {
  const BlockDesc* blocks;
  const ColDesc* cols;
  HStore hs;
  const float2* Ginv;
  const uint32_t* Ginv16;  // bfloat16-pair copy of Ginv (same element offsets), or null: use Ginv
  const float2* g;      // caller's measurements
  // c, s, v, part: column space [Q][n_pad]; gp, ghat: row space [P][m_pad];
  // r, y: the Gram space, row space in the inversion-lemma form (r_ij, y_ij),
  // column space in the direct form (b_ij, and u_j^i in the layout of c)
  float2 *c, *s, *v, *part, *gp, *ghat, *r, *y;
  float2* gpart;        // Gram-apply pieces (BlockDesc::gpo)
  Control* ctl;
  double* redpart;
  double* hist;         // device, 2 per iteration, or null
  float2* arec;         // device, pre-threshold mean of this iteration (column space), or null
  int64_t m_pad, n_pad;
  int Q, P, KH;
  int nz;               // z-update workgroups (partial sums in redpart)
  float rho, kappa;
  double rho2Q;         // rho^2 Q for the dual residual
  int cpl;              // columns per lane load of the storage (layout of c, see cperm)
  int xstage;           // 1: every column block's c fits kXStage float4 of LDS (row product stages it)
  int wide;             // 1: some column block is wider than kWholeCols (the whole-row product loops over chunks)
  int direct;           // 1: direct x-update (the row products write ghat = H u instead of r and g')
  int* uref;            // direct form, device word: 1 when y holds the last iteration's u and ghat_ij =
                        // H_ij y_ij (the x-update then corrects that u), 0 after a reset or a state import
};

// Adjoint (reverse-mode) sweep of one iteration.
struct AdjArgs {
  const BlockDesc* blocks;
  const ColDesc* cols;
  HStore hs;
  const float2* Ginv;
  const uint32_t* Ginv16;  // as IterArgs::Ginv16
  float2 *vb, *sb, *ub, *ghb, *gpb, *yb, *rb, *part, *gpart;
  double2* gbar;
  double *kpart, *rpart;
  Control* ctl;
  int64_t m_pad, n_pad;
  int Q, P, KH;
  float rho, kappa;
  int cpl;              // layout of ub (see cperm)
};
hipError_t launch_adj_iteration(const AdjArgs& a, const Geometry& G, const int4* t_hrows, const int4* t_gram,
                                const int4* t_gtr, const int4* t_cols, const int4* t_z, const float2* arec,
                                const float2* yrec, hipStream_t st);
// Final kbar / rbar from the per-workgroup slots of nk z-workgroups and nr
// Gram-reduce workgroups.
hipError_t launch_adj_scalars(const AdjArgs& a, int nk, int nr, hipStream_t st);
hipError_t launch_adj_gflush(const AdjArgs& a, const BlockDesc* blocks, int nblocks, float2* grad_g,
                             hipStream_t st);

// Optional start / stop events carried by the dispatch packets themselves
// (hipExtLaunchKernelGGL), so timing adds no packets between kernels.
struct KTime {
  hipEvent_t start = nullptr, stop = nullptr;
};
// Plain launch unless timing events are given (then on the dispatch packet).
#define LAUNCH_TIMED(kern, grid, block, st, kt, ...)                                               \
  do {                                                                                               \
    const KTime kt_ = kt;                                                                            \
    if (kt_.start || kt_.stop)                                                                       \
      hipExtLaunchKernelGGL(kern, grid, block, 0, st, kt_.start, kt_.stop, 0, __VA_ARGS__);           \
    else                                                                                             \
      hipLaunchKernelGGL(kern, grid, block, 0, st, __VA_ARGS__);                                     \
  } while (0)
hipError_t launch_gemv_n(const IterArgs& a, const int4* tiles, int ntiles, const int4* wtiles, int nwtiles,
                          hipStream_t st, KTime kt = {});
// reduce = false: the apply kernel only (the direct form's z-update adds the pieces).
hipError_t launch_gram(const IterArgs& a, const int4* t_gram, int n_gram, const int4* t_gpatch, int n_gpatch,
                       const int4* t_gtr, int n_gtr, hipStream_t st, KTime kt = {}, bool reduce = true);
hipError_t launch_gemv_h(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st, KTime kt = {});
// src: 0 inversion-lemma form; direct form with the Gram pieces of
// k_gram_patch (1) or of the single-tile kernels (2).
hipError_t launch_zupdate(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st, KTime kt = {},
                          int src = 0);
// Direct x-update: g' of every block (t_dgp), b = H^H g' + rho c (t_z tiles).
hipError_t launch_direct_gp(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st, KTime kt = {});
hipError_t launch_direct_rhs(const IterArgs& a, const int4* tiles, int ntiles, hipStream_t st, KTime kt = {});
// Single-pass iteration (k_fused.hip).
hipError_t launch_fz_rows(const IterArgs& a, const FzArgs& z, const int4* tiles, int ntiles, hipStream_t st,
                          KTime kt = {});
hipError_t launch_fz_slab(const IterArgs& a, const FzArgs& z, int nt, int rpl, hipStream_t st, KTime kt = {});
hipError_t launch_pack_slabs(const HStore& src, const HStore& dst, const BlockDesc* blocks, int Q, int P,
                             int64_t m_pad, const FzArgs& z, hipStream_t st);
// Final addition of a pending z-update's partial sums (one workgroup).
hipError_t launch_zfinal(const IterArgs& a, hipStream_t st);
// Round n complex64 values to bfloat16 pairs (Re low half, Im high half).
hipError_t launch_to_bf16_pairs(const float2* src, uint32_t* dst, size_t n, hipStream_t st);
hipError_t launch_unpad_cols(const ColDesc* cols, int P, int64_t n, const float2* src, float2* dst,
                             int64_t src_stride, int64_t dst_stride, int reps, int to_padded,
                             hipStream_t st);
hipError_t launch_unpad_rows(const BlockDesc* blocks, int nblocks, int64_t m, int64_t m_pad,
                             const float2* src, float2* dst, int to_padded, hipStream_t st);
hipError_t launch_fill(void* p, size_t bytes, hipStream_t st);

// setup
hipError_t launch_pack_c64(const float2* Hin, int64_t n, const BlockDesc* blocks, int nblocks,
                           int max_rows, float2* Hout, Control* ctl, hipStream_t st);
hipError_t launch_gram_build(const Geometry& geo, const BlockDesc* dblocks, const int4* t_gram,
                             const HStore& hs, double rho, double2* A, hipStream_t st);
hipError_t launch_pack_quant(const float2* Hin, int64_t m, int64_t n, const BlockDesc* blocks, int nblocks,
                             int max_rows, const HStore& hs, Control* ctl, hipStream_t st);
hipError_t launch_export_h(const HStore& hs, int64_t n, const BlockDesc* blocks, int nblocks, int max_rows,
                           void* re_out, void* im_out, hipStream_t st);
hipError_t launch_cholesky_inverse(const Geometry& geo, const BlockDesc* dblocks, const int4* t_gram,
                                   double2* A, double2* W, float2* Ginv, Control* ctl, hipStream_t st);

// KKT check (FP64)
hipError_t launch_kkt_all(const BlockDesc* dblocks, const ColDesc* dcols, const int64_t* drow_block,
                          const int4* t_kadj, int n_tkadj, const int4* t_z, int n_tz, int64_t m, int64_t n_pad,
                          int Q, int P, int KH, const HStore& hs, const float2* g, const float2* vpad,
                          double lam, double2* e, double2* part, double* wgmax, Control* ctl, hipStream_t st);
hipError_t launch_make_c(const ColDesc* cols, int P, int Q, int64_t n_pad, int cpl, const float2* v,
                         const float2* s, float2* c, hipStream_t st);

}  // namespace admm
