// C ABI of the batched multi-scene form: plan construction (shared
// instrument store, its transpose, shared per-column-block Gram, per-scene
// block inverses in bounded FP64 groups), the MFMA tile autotuner, hipGraph
// replay of the iteration and profiling.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/admm.h"
#include "batch.h"

using namespace admm;

namespace admm {
int admm_fail(int code, const char* fmt, ...);  // defined in api.hip (sets admm_last_error)
}

namespace {

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

#define BHIP(expr)                                                                                \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return admm_fail(ADMM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Autotuned variants: forward (rows per workgroup / 64, k-chunks per column
// block); adjoint columns per workgroup / 64.
#ifndef ADMM_FWD_MS
#define ADMM_FWD_MS {2, 2, 1}
#endif
#ifndef ADMM_FWD_KS
#define ADMM_FWD_KS {1, 2, 2}
#endif
constexpr int kFwdMS[3] = ADMM_FWD_MS;
constexpr int kSplitVariants[3] = ADMM_FWD_KS;
constexpr int kAdjMS[3] = {1, 2, 4};
constexpr int max3(const int (&v)[3]) { return v[0] > v[1] ? (v[0] > v[2] ? v[0] : v[2]) : (v[1] > v[2] ? v[1] : v[2]); }
// rows per forward workgroup / 64 of variant v for a tile height
inline int fwd_ms(int v, int tile_rows) { return std::min(kFwdMS[v], tile_rows / 64); }
constexpr int kGroupW = 64;   // scene-tile columns of one GEMM item

struct BatchGeo {
  int64_t m0 = 0, n = 0;
  int tile_rows = 0, F = 0, S = 0, P = 0;
  std::vector<int64_t> co;
  std::vector<std::vector<int32_t>> tiles, cuts;
  std::vector<int64_t> soff;          // first packed row of each scene
  int64_t rows_total = 0;             // sum of m_s
  std::vector<BlockDesc> pseudo;      // per column block
  std::vector<ColDesc> cols;
  std::vector<BlockDesc> blocks;      // (rep, j)
  std::vector<RowBlockDesc> rbd;
  std::vector<SceneDesc> scenes;
  std::vector<SceneTile> stab;        // grouped by tile f
  std::vector<int32_t> st_off;        // F+1
  std::vector<int32_t> cuts_flat, tiles_flat;
  std::vector<int4> t_gram, t_gtr, t_z, t_gpatch;
  int64_t gpart_vecs = 0;
  std::vector<GemmItem> items_n[3], items_h[3];
  int64_t m_pad = 0, n_pad = 0, ldt = 0, mt0 = 0;
  int R = 0, NST = 0, max_nj = 0;
  // workspace
  size_t o_hre = 0, o_him = 0, o_hkre = 0, o_hkim = 0, o_tre = 0, o_tim = 0, o_ginv = 0, o_ginv16 = 0, o_G0 = 0, o_A = 0, o_W = 0, group_bytes = 0;
  bool inv16 = false;              // a bfloat16-pair copy of the inverses is kept and applied
  int64_t ginv_elems = 0;
  size_t o_c = 0, o_s = 0, o_v = 0, o_part = 0, o_gp = 0, o_ghat = 0, o_r = 0, o_y = 0, o_cs = 0, o_ys = 0, o_phase = 0;
  size_t o_pseudo = 0, o_cols = 0, o_blocks = 0, o_rbd = 0, o_scenes = 0, o_stab = 0, o_cuts = 0, o_tiles = 0;
  int NG = 0;                      // forward GEMM groups (f, scene-tile group, j)
  std::vector<int2> st_gc;         // per scene-tile entry: first group, column in group
  size_t o_pn = 0, o_stgc = 0;
  size_t o_tgpatch = 0;
  size_t o_tgram = 0, o_tgtr = 0, o_gpart = 0, o_tz = 0, o_items_n[3] = {0, 0, 0}, o_items_h[3] = {0, 0, 0}, o_ctl = 0;
  size_t o_gblocks = 0, o_ggram = 0, o_gtile0 = 0, g_max_blocks = 0, g_max_gram = 0, o_t0gram = 0;
  std::vector<int4> t0_gram;          // lower tiles of the pseudo blocks (G0)
  size_t total = 0;
};

int build_batch(BatchGeo& G, int64_t m0, int64_t n, int tile_rows, int S, const int32_t* tiles,
                const int64_t* tiles_off, const int32_t* cuts, const int64_t* cuts_off, int P,
                const int64_t* col_off, int flags, std::string& err) {
  if (flags & ~(ADMM_INVERSE_BF16 | ADMM_GRAM_PATCHES)) {
    err = "unknown flags";
    return ADMM_EINVAL;
  }
  G.inv16 = (flags & ADMM_INVERSE_BF16) != 0;
  const bool force_patches = (flags & ADMM_GRAM_PATCHES) != 0;
  char buf[256];
  if (m0 < 1 || n < 1 || (tile_rows != 64 && tile_rows != 128 && tile_rows != 256) || m0 % tile_rows || S < 1 || P < 1 || P > n ||
      !tiles || !tiles_off || !cuts || !cuts_off) {
    err = "need m0, n >= 1, tile_rows in {64, 128, 256} dividing m0, S >= 1, 1 <= P <= n and non-NULL scene tables";
    return ADMM_EINVAL;
  }
  G.m0 = m0;
  G.n = n;
  G.tile_rows = tile_rows;
  G.F = (int)(m0 / tile_rows);
  G.S = S;
  G.P = P;
  // column split
  G.co.assign(P + 1, 0);
  if (col_off) {
    for (int j = 0; j <= P; ++j) G.co[j] = col_off[j];
    bool ok = G.co[0] == 0 && G.co[P] == n;
    for (int j = 0; j < P && ok; ++j) ok = G.co[j + 1] > G.co[j];
    if (!ok) {
      err = "column offsets must increase strictly from 0 to n";
      return ADMM_EINVAL;
    }
  } else {
    for (int j = 0; j < P; ++j) G.co[j + 1] = G.co[j] + n / P + (j < n % P ? 1 : 0);
  }
  // scenes
  G.tiles.assign(S, {});
  G.cuts.assign(S, {});
  G.soff.assign(S + 1, 0);
  for (int s = 0; s < S; ++s) {
    const int64_t t0 = tiles_off[s], t1 = tiles_off[s + 1], c0 = cuts_off[s], c1 = cuts_off[s + 1];
    if (t1 <= t0 || c1 - c0 < 2) {
      err = "every scene needs at least one tile and one row block";
      return ADMM_EINVAL;
    }
    const int T = (int)(t1 - t0);
    for (int64_t k = t0; k < t1; ++k) {
      const int f = tiles[k];
      if (f < 0 || f >= G.F || (k > t0 && f <= tiles[k - 1])) {
        snprintf(buf, sizeof buf, "scene %d: tile indices must increase strictly inside [0, %d)", s, G.F);
        err = buf;
        return ADMM_EINVAL;
      }
      G.tiles[s].push_back(f);
    }
    for (int64_t k = c0; k < c1; ++k) G.cuts[s].push_back(cuts[k]);
    bool ok = G.cuts[s].front() == 0 && G.cuts[s].back() == T;
    for (size_t k = 1; k < G.cuts[s].size() && ok; ++k) ok = G.cuts[s][k] > G.cuts[s][k - 1];
    if (!ok) {
      snprintf(buf, sizeof buf, "scene %d: cuts must increase strictly from 0 to its tile count", s);
      err = buf;
      return ADMM_EINVAL;
    }
    G.soff[s + 1] = G.soff[s] + (int64_t)T * tile_rows;
  }
  G.rows_total = G.soff[S];
  // column space
  G.cols.resize(P);
  G.pseudo.assign(P, BlockDesc{});
  G.mt0 = round_up(m0, kTile);
  G.ldt = round_up(m0, kColPad);
  if ((G.ldt * 2) % 4096 == 0) G.ldt += kColPad;
  int64_t acc = 0, hoff = 0, toff = 0, foff = 0;
  G.max_nj = 0;
  for (int j = 0; j < P; ++j) {
    const int nj = (int)(G.co[j + 1] - G.co[j]);
    const int64_t ldc = round_up(nj, 128);
    G.cols[j] = ColDesc{nj, (int32_t)acc, (int32_t)G.co[j], (int32_t)ldc};
    BlockDesc& d = G.pseudo[j];
    d.i = 0;
    d.j = j;
    d.mi = (int32_t)m0;
    d.nj = nj;
    int64_t ldh = round_up(nj, kColPad);
    if ((ldh * 2) % 4096 == 0) ldh += kColPad;
    d.ld = (int32_t)ldh;
    d.ldr = 0;
    d.gd = d.mi;
    d.mt = (int32_t)G.mt0;
    d.row0 = 0;
    d.col0 = (int32_t)G.co[j];
    d.cpad0 = (int32_t)acc;
    d.h_off = hoff;
    d.gi_off = toff;
    d.f_off = foff;
    hoff += m0 * ldh;
    toff += (int64_t)((nj + 15) / 16 * 16) * G.ldt;   // k-tiled, rows padded to 16
    foff += G.mt0 * G.mt0;
    acc += ldc;
    G.max_nj = std::max(G.max_nj, nj);
  }
  G.n_pad = acc;
  // row blocks, blocks, scene tables
  G.rbd.clear();
  G.blocks.clear();
  G.scenes.clear();
  G.cuts_flat.clear();
  G.tiles_flat.clear();
  int64_t rpad = 0, gioff = 0, gpo = 0;
  int pslot = 0;
  std::vector<std::vector<SceneTile>> by_f(G.F);
  for (int s = 0; s < S; ++s) {
    SceneDesc sd{};
    sd.rb0 = (int32_t)G.rbd.size();
    sd.Q = (int32_t)G.cuts[s].size() - 1;
    sd.pslot0 = pslot;
    sd.cut0 = (int32_t)G.cuts_flat.size();
    const int tflat0 = (int)G.tiles_flat.size();
    for (int c : G.cuts[s]) G.cuts_flat.push_back(c);
    for (int f : G.tiles[s]) G.tiles_flat.push_back(f);
    for (int i = 0; i < sd.Q; ++i) {
      const int ca = G.cuts[s][i], cb = G.cuts[s][i + 1];
      RowBlockDesc rb{};
      rb.mi = (cb - ca) * tile_rows;
      rb.rpad0 = (int32_t)rpad;
      rb.row0 = (int32_t)(G.soff[s] + (int64_t)ca * tile_rows);
      rb.tile0 = tflat0 + ca;
      const int rep = (int)G.rbd.size();
      for (int j = 0; j < P; ++j) {
        BlockDesc d{};
        d.i = rep;
        d.j = j;
        d.mi = rb.mi;
        d.nj = G.cols[j].nj;
        // the batch applies the inversion-lemma x-update only; blocks this tall,
        // where it would stream more than the direct form, are rejected
        if ((int64_t)d.mi * d.mi >= 2 * (int64_t)d.mi * d.nj + (int64_t)d.nj * d.nj) {
          snprintf(buf, sizeof buf, "scene %d block (%d,%d) is %d x %d: at least (1 + sqrt 2) times taller than wide",
                   s, i, j, d.mi, d.nj);
          err = buf;
          return ADMM_EUNSUPPORTED;
        }
        d.ldr = (int32_t)round_up(d.mi, kRowPad);
        d.gd = d.mi;
        d.mt = (int32_t)round_up(d.mi, kTile);
        d.row0 = rb.row0;
        d.col0 = G.cols[j].col0;
        d.rpad0 = rb.rpad0;
        d.cpad0 = G.cols[j].cpad0;
        d.gi_off = gioff;
        d.gpo = (int32_t)gpo;
        d.ld = 0;
        d.h_off = 0;
        d.f_off = 0;  // set per setup group
        const int64_t T = d.mt / kTile;
        gioff += T * (T + 1) / 2 * kTile * kTile;
        gpo += gram_part_vecs(T);
        G.blocks.push_back(d);
      }
      for (int sl = ca; sl < cb; ++sl) {
        SceneTile st{};
        st.s = s;
        st.rep = rep;
        st.lr0 = (sl - ca) * tile_rows;
        st.row0 = (int32_t)(G.soff[s] + (int64_t)sl * tile_rows);
        st.pslot = pslot + sl;
        st.f = G.tiles[s][sl];
        by_f[st.f].push_back(st);
      }
      rpad += round_up(rb.mi, kRowPad);
      G.rbd.push_back(rb);
    }
    pslot += (int)G.tiles[s].size();
    G.scenes.push_back(sd);
  }
  G.R = (int)G.rbd.size();
  G.NST = pslot;
  G.m_pad = rpad;
  G.stab.clear();
  G.st_off.assign(G.F + 1, 0);
  for (int f = 0; f < G.F; ++f) {
    G.st_off[f] = (int32_t)G.stab.size();
    for (auto& st : by_f[f]) G.stab.push_back(st);
  }
  G.st_off[G.F] = (int32_t)G.stab.size();
  // work tables
  G.t_gram.clear();
  G.t_gtr.clear();
  G.t_gpatch.clear();
  for (size_t b = 0; b < G.blocks.size(); ++b) {
    const int T = G.blocks[b].mt / kTile;
    for (int a2 = 0; a2 < T; ++a2) {
      for (int c2 = 0; c2 <= a2; ++c2) G.t_gram.push_back(make_int4((int)b, a2, c2, 0));
      G.t_gtr.push_back(make_int4((int)b, a2, 0, 0));
    }
    if (ADMM_GRAM_PATCH)
      for (int a2 = 0; a2 < (T + 3) / 4; ++a2)
        for (int c2 = 0; c2 <= a2; ++c2) G.t_gpatch.push_back(make_int4((int)b, a2, c2, 0));
  }
  // patches for the complex64 inverses when asked or when they fill the GPU
  if (G.inv16 || !(force_patches || G.t_gpatch.size() >= kGramPatchMin)) G.t_gpatch.clear();
  G.gpart_vecs = gpo;
  G.t_z.clear();
  for (int s = 0; s < S; ++s)
    for (int j = 0; j < P; ++j)
      for (int c = 0; c < G.cols[j].nj; c += kZCols) G.t_z.push_back(make_int4(s, j, c, 0));
  // GEMM work items.  The items of one (tile, column block, scene group) read
  // the same vector operand; workgroups are dealt to the 8 XCDs round-robin by
  // index, so such items are placed at indices congruent mod 8 (windows of 8
  // groups, item s of group g at window base + 8 s + g) to share one L2.
  auto xcd_order = [](const std::vector<std::vector<GemmItem>>& groups, std::vector<GemmItem>& out) {
    out.clear();
    for (size_t w0 = 0; w0 < groups.size(); w0 += 8) {
      const size_t w1 = std::min(groups.size(), w0 + 8);
      size_t most = 0;
      for (size_t g = w0; g < w1; ++g) most = std::max(most, groups[g].size());
      for (size_t sub = 0; sub < most; ++sub)
        for (size_t g = w0; g < w1; ++g)
          if (sub < groups[g].size()) out.push_back(groups[g][sub]);
    }
  };
  // GEMM groups (f, scene-tile group of kGroupW, j) and the scene-tile -> group table
  G.NG = 0;
  G.st_gc.assign(G.stab.size(), make_int2(0, 0));
  std::vector<std::array<int, 5>> groups;   // f, j, st0, cnt, g
  for (int f = 0; f < G.F; ++f) {
    const int a0 = G.st_off[f], cntf = G.st_off[f + 1] - a0;
    for (int k = 0; k < cntf; k += kGroupW) {
      for (int q = k; q < std::min(cntf, k + kGroupW); ++q) G.st_gc[a0 + q] = make_int2(G.NG, q - k);
      for (int j = 0; j < P; ++j) groups.push_back({f, j, a0 + k, std::min(kGroupW, cntf - k), G.NG + j});
      G.NG += P;
    }
  }
  for (int v = 0; v < 3; ++v) {
    std::vector<std::vector<GemmItem>> gn, gh;
    for (const auto& g : groups) {
      const int f = g[0], j = g[1], st0 = g[2], cnt = g[3], gi = g[4];
      const int nk = (int)round_up(G.cols[j].nj, 32);
      const int ks = kSplitVariants[v];
      const int chunk = (int)round_up((nk + ks - 1) / ks, 32);
      const int rows = 64 * fwd_ms(v, tile_rows);
      gn.emplace_back();
      for (int kc = 0; kc < ks; ++kc) {
        const int k0 = std::min(nk, kc * chunk), k1 = std::min(nk, (kc + 1) * chunk);
        for (int r0 = 0; r0 < tile_rows; r0 += rows)
          gn.back().push_back(GemmItem{f, j, k0, st0, cnt, {k1, kc * G.NG + gi, r0}});
      }
      gh.emplace_back();
      for (int c = 0; c < G.cols[j].nj; c += 64 * kAdjMS[v])
        gh.back().push_back(GemmItem{f, j, c, st0, cnt, {0, 0, 0}});
    }
    xcd_order(gn, G.items_n[v]);
    xcd_order(gh, G.items_h[v]);
  }
  G.t0_gram.clear();
  for (int j = 0; j < P; ++j)
    for (int a = 0; a < G.mt0 / kTile; ++a)
      for (int c = 0; c <= a; ++c) G.t0_gram.push_back(make_int4(j, a, c, 0));
  // FP64 setup groups: largest block sets the minimum group size
  size_t max_blk = 0, all_blk = 0;
  for (auto& d : G.blocks) {
    max_blk = std::max(max_blk, (size_t)d.mt * d.mt * 16);
    all_blk += (size_t)d.mt * d.mt * 16;
  }
  // up to 16 GB of FP64 per group matrix (two of them), never more than all
  // blocks need: fewer, wider setup launches
  G.group_bytes = std::max<size_t>(max_blk, std::min<size_t>(all_blk, (size_t)16 << 30));
  {
    size_t cur = 0, nb = 0, ng = 0;
    G.g_max_blocks = G.g_max_gram = 0;
    for (auto& d : G.blocks) {
      const size_t sz = (size_t)d.mt * d.mt * 16;
      if (cur + sz > G.group_bytes) {
        G.g_max_blocks = std::max(G.g_max_blocks, nb);
        G.g_max_gram = std::max(G.g_max_gram, ng);
        cur = nb = ng = 0;
      }
      cur += sz;
      nb += 1;
      ng += (size_t)(d.mt / kTile) * (d.mt / kTile + 1) / 2;
    }
    G.g_max_blocks = std::max(G.g_max_blocks, nb);
    G.g_max_gram = std::max(G.g_max_gram, ng);
  }
  // layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = a256(off + bytes);
    return o;
  };
  G.o_hre = take((size_t)hoff * 2);
  G.o_him = take((size_t)hoff * 2);
  G.o_hkre = take((size_t)hoff * 2);
  G.o_hkim = take((size_t)hoff * 2);
  G.o_tre = take((size_t)toff * 2);
  G.o_tim = take((size_t)toff * 2);
  G.o_ginv = take((size_t)gioff * 8);
  G.ginv_elems = gioff;
  if (G.inv16) G.o_ginv16 = take((size_t)gioff * 4);
  G.o_G0 = take((size_t)foff * 16);
  G.o_A = take(G.group_bytes);
  G.o_W = take(G.group_bytes);
  const size_t colv = (size_t)G.n_pad * 8, rowv = (size_t)G.m_pad * 8;
  G.o_c = take(colv * G.R);
  G.o_s = take(colv * G.R);
  G.o_v = take(colv * S);
  G.o_part = take(colv * G.NST);
  G.o_gp = take(rowv * P);
  G.o_ghat = take(rowv * P);
  G.o_r = take(rowv * P);
  G.o_y = take(rowv * P);
  G.o_cs = take((size_t)G.n_pad * G.R * 12);   // six bf16 planes (state: cleared with it)
  G.o_ys = take((size_t)G.m_pad * P * 12);
  G.o_phase = take(8 * (size_t)G.rows_total);   // from here on: not cleared per solve
  G.o_pn = take((size_t)max3(kSplitVariants) * G.NG * G.tile_rows * kGroupW * 8);
  G.o_stgc = take(8 * G.st_gc.size());
  G.o_pseudo = take(sizeof(BlockDesc) * P);
  G.o_cols = take(sizeof(ColDesc) * P);
  G.o_blocks = take(sizeof(BlockDesc) * G.blocks.size());
  G.o_rbd = take(sizeof(RowBlockDesc) * G.rbd.size());
  G.o_scenes = take(sizeof(SceneDesc) * S);
  G.o_stab = take(sizeof(SceneTile) * G.stab.size());
  G.o_cuts = take(4 * G.cuts_flat.size());
  G.o_tiles = take(4 * G.tiles_flat.size());
  G.o_tgram = take(16 * G.t_gram.size());
  G.o_tgpatch = take(16 * std::max<size_t>(G.t_gpatch.size(), 1));
  G.o_tgtr = take(16 * G.t_gtr.size());
  G.o_gpart = take((size_t)G.gpart_vecs * kTile * 8);
  G.o_tz = take(16 * G.t_z.size());
  for (int v = 0; v < 3; ++v) {
    G.o_items_n[v] = take(sizeof(GemmItem) * G.items_n[v].size());
    G.o_items_h[v] = take(sizeof(GemmItem) * G.items_h[v].size());
  }
  G.o_t0gram = take(16 * G.t0_gram.size());
  G.o_gblocks = take(sizeof(BlockDesc) * G.g_max_blocks);
  G.o_ggram = take(16 * G.g_max_gram);
  G.o_gtile0 = take(4 * G.g_max_blocks);
  G.o_ctl = take(sizeof(Control));
  G.total = off;
  return ADMM_OK;
}

}  // namespace

struct admm_batch {
  BatchGeo geo;
  double rho = 1.0;
  std::vector<double> lam;
  char* ws = nullptr;
  int var_n = 2, var_h = 2;
  hipStream_t gstream = nullptr;      // capture / replay stream (default priority)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t graph = nullptr;
  const void* graph_g = nullptr;
  bool use_graph = true;
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[4];
  double prof_ms[4] = {0, 0, 0, 0};
  int64_t prof_n[4] = {0, 0, 0, 0};
  double tune_ms[2][3] = {{0, 0, 0}, {0, 0, 0}};
};

namespace {

template <class T>
T* at(admm_batch* b, size_t off) {
  return reinterpret_cast<T*>(b->ws + off);
}

BatchArgs batch_args(admm_batch* b, const float2* g) {
  const BatchGeo& G = b->geo;
  BatchArgs a{};
  a.h_re = at<uint16_t>(b, G.o_hre);
  a.h_im = at<uint16_t>(b, G.o_him);
  a.hk_re = at<uint16_t>(b, G.o_hkre);
  a.hk_im = at<uint16_t>(b, G.o_hkim);
  a.t_re = at<uint16_t>(b, G.o_tre);
  a.t_im = at<uint16_t>(b, G.o_tim);
  a.pseudo = at<BlockDesc>(b, G.o_pseudo);
  a.stab = at<SceneTile>(b, G.o_stab);
  a.scenes = at<SceneDesc>(b, G.o_scenes);
  a.rbd = at<RowBlockDesc>(b, G.o_rbd);
  a.cuts = at<int32_t>(b, G.o_cuts);
  a.phases = at<float2>(b, G.o_phase);
  a.g = g;
  a.c = at<float2>(b, G.o_c);
  a.s = at<float2>(b, G.o_s);
  a.v = at<float2>(b, G.o_v);
  a.part = at<float2>(b, G.o_part);
  a.gp = at<float2>(b, G.o_gp);
  a.ghat = at<float2>(b, G.o_ghat);
  a.r = at<float2>(b, G.o_r);
  a.y = at<float2>(b, G.o_y);
  a.cs = at<uint16_t>(b, G.o_cs);
  a.ys = at<uint16_t>(b, G.o_ys);
  a.pn = at<float2>(b, G.o_pn);
  a.st_gc = at<int2>(b, G.o_stgc);
  a.NG = G.NG;
  a.NST = G.NST;
  a.ctl = at<Control>(b, G.o_ctl);
  a.m_pad = G.m_pad;
  a.n_pad = G.n_pad;
  a.P = G.P;
  a.tile_rows = G.tile_rows;
  a.ldt = (int)G.ldt;
  a.R = G.R;
  return a;
}

IterArgs gram_args(admm_batch* b, const float2* g) {
  const BatchGeo& G = b->geo;
  IterArgs a{};
  a.blocks = at<BlockDesc>(b, G.o_blocks);
  a.cols = at<ColDesc>(b, G.o_cols);
  a.Ginv = at<float2>(b, G.o_ginv);
  a.Ginv16 = G.inv16 ? at<uint32_t>(b, G.o_ginv16) : nullptr;
  a.g = g;
  a.gp = at<float2>(b, G.o_gp);
  a.ghat = at<float2>(b, G.o_ghat);
  a.r = at<float2>(b, G.o_r);
  a.y = at<float2>(b, G.o_y);
  a.gpart = at<float2>(b, G.o_gpart);
  a.ctl = at<Control>(b, G.o_ctl);
  a.m_pad = G.m_pad;
  a.n_pad = G.n_pad;
  a.P = G.P;
  a.rho = (float)b->rho;
  a.cpl = 2;
  return a;
}

// One iteration: forward GEMM, Gram apply, adjoint GEMM, z-update.
hipError_t launch_iteration(admm_batch* b, const float2* g, hipStream_t st, bool timed_events) {
  const BatchGeo& G = b->geo;
  const BatchArgs a = batch_args(b, g);
  const IterArgs ga = gram_args(b, g);
  auto run = [&](int k, auto&& f) -> hipError_t {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed_events) {
      hipError_t e = hipEventCreate(&e0);
      if (e == hipSuccess) e = hipEventCreate(&e1);
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      if (e != hipSuccess) return e;
    }
    hipError_t e = f();
    if (e != hipSuccess) return e;
    if (timed_events) {
      if ((e = hipEventRecord(e1, st)) != hipSuccess) return e;
      b->ev[k].emplace_back(e0, e1);
    }
    return hipSuccess;
  };
  hipError_t e;
  if ((e = run(0, [&] {
         return launch_bgemm_n(a, at<GemmItem>(b, G.o_items_n[b->var_n]), (int)G.items_n[b->var_n].size(),
                               kSplitVariants[b->var_n], fwd_ms(b->var_n, G.tile_rows), st);
       })) != hipSuccess)
    return e;
  if ((e = run(1, [&] {
         return launch_gram(ga, at<int4>(b, G.o_tgram), (int)G.t_gram.size(), at<int4>(b, G.o_tgpatch),
                            (int)G.t_gpatch.size(), at<int4>(b, G.o_tgtr), (int)G.t_gtr.size(), st);
       })) != hipSuccess)
    return e;
  if ((e = run(2, [&] {
         return launch_bgemm_h(a, at<GemmItem>(b, G.o_items_h[b->var_h]), (int)G.items_h[b->var_h].size(),
                               kAdjMS[b->var_h], st);
       })) != hipSuccess)
    return e;
  return run(3, [&] { return launch_bzupdate(a, at<ColDesc>(b, G.o_cols), at<int4>(b, G.o_tz), (int)G.t_z.size(), st); });
}

int drain(admm_batch* b) {
  for (int k = 0; k < 4; ++k) {
    for (auto& pr : b->ev[k]) {
      BHIP(hipEventSynchronize(pr.second));
      float ms = 0.f;
      BHIP(hipEventElapsedTime(&ms, pr.first, pr.second));
      b->prof_ms[k] += ms;
      b->prof_n[k] += 1;
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    b->ev[k].clear();
  }
  return ADMM_OK;
}

// Time each variant of both GEMMs (3 launches, best) and keep the fastest.
int autotune(admm_batch* b, hipStream_t st) {
  static std::mutex mu;
  static std::map<std::tuple<int64_t, int64_t, int, int, int, int>, std::pair<int, int>> cache;
  const BatchGeo& G = b->geo;
  const auto key = std::make_tuple(G.m0, G.n, G.P, G.S, G.NST, G.tile_rows);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      b->var_n = it->second.first;
      b->var_h = it->second.second;
      return ADMM_OK;
    }
  }
  const BatchArgs a = batch_args(b, at<float2>(b, G.o_r));  // any valid row vector as g: values are not used
  hipEvent_t e0, e1;
  BHIP(hipEventCreate(&e0));
  BHIP(hipEventCreate(&e1));
  for (int which = 0; which < 2; ++which) {
    float best = 1e30f;
    for (int v = 0; v < 3; ++v) {
      float vbest = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        BHIP(hipEventRecord(e0, st));
        if (which == 0)
          BHIP(launch_bgemm_n(a, at<GemmItem>(b, G.o_items_n[v]), (int)G.items_n[v].size(), kSplitVariants[v],
                              fwd_ms(v, G.tile_rows), st));
        else
          BHIP(launch_bgemm_h(a, at<GemmItem>(b, G.o_items_h[v]), (int)G.items_h[v].size(), kAdjMS[v], st));
        BHIP(hipEventRecord(e1, st));
        BHIP(hipEventSynchronize(e1));
        float ms = 0.f;
        BHIP(hipEventElapsedTime(&ms, e0, e1));
        vbest = std::min(vbest, ms);
      }
      b->tune_ms[which][v] = vbest;
      if (vbest < best) {
        best = vbest;
        (which == 0 ? b->var_n : b->var_h) = v;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = {b->var_n, b->var_h};
  return ADMM_OK;
}

}  // namespace

extern "C" {

int admm_batch_workspace_bytes(int64_t m0, int64_t n, int tile_rows, int S, const int32_t* tiles,
                               const int64_t* tiles_off, const int32_t* cuts, const int64_t* cuts_off, int P,
                               const int64_t* col_off, int flags, size_t* out_bytes) {
  if (!out_bytes) return admm_fail(ADMM_EINVAL, "out_bytes is NULL");
  BatchGeo G;
  std::string err;
  int rc = build_batch(G, m0, n, tile_rows, S, tiles, tiles_off, cuts, cuts_off, P, col_off, flags, err);
  if (rc) return admm_fail(rc, "%s", err.c_str());
  *out_bytes = G.total;
  return ADMM_OK;
}

int admm_batch_setup(admm_batch** out, const void* H0, int64_t m0, int64_t n, int tile_rows, int S,
                     const int32_t* tiles, const int64_t* tiles_off, const int32_t* cuts, const int64_t* cuts_off,
                     const void* phases, int P, const int64_t* col_off, int flags, double rho, const double* lambdas,
                     void* workspace, size_t workspace_bytes, void* stream) {
  if (!out) return admm_fail(ADMM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!H0 || !phases || !lambdas) return admm_fail(ADMM_EINVAL, "H0, phases and lambdas must not be NULL");
  if (!(rho > 0.0) || !std::isfinite(rho)) return admm_fail(ADMM_EINVAL, "rho must be finite and > 0");
  for (int s = 0; s < S; ++s)
    if (!(lambdas[s] >= 0.0) || !std::isfinite(lambdas[s]))
      return admm_fail(ADMM_EINVAL, "lambda of scene %d must be finite and >= 0", s);
  admm_batch* b = new admm_batch;
  std::string err;
  int rc = build_batch(b->geo, m0, n, tile_rows, S, tiles, tiles_off, cuts, cuts_off, P, col_off, flags, err);
  if (rc) {
    delete b;
    return admm_fail(rc, "%s", err.c_str());
  }
  BatchGeo& G = b->geo;
  if (!workspace || workspace_bytes < G.total || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
    delete b;
    return admm_fail(ADMM_EWORKSPACE, "workspace needs %zu bytes at 256-byte alignment", G.total);
  }
  b->ws = static_cast<char*>(workspace);
  b->rho = rho;
  b->lam.assign(lambdas, lambdas + S);
  for (int s = 0; s < S; ++s) G.scenes[s].kappa = (float)(lambdas[s] / (G.scenes[s].Q * rho));
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto bail = [&](int code) {
    delete b;
    return code;
  };
#define STRY(expr)                                                                                          \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) return bail(admm_fail(ADMM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_))); \
  } while (0)
  STRY(launch_fill(b->ws, G.o_ginv, st));                 // H0 planes and transpose (with pads)
  STRY(launch_fill(b->ws + G.o_c, G.total - G.o_c, st));  // state, tables, control
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(b->ws + off, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  STRY(up(G.o_pseudo, G.pseudo.data(), sizeof(BlockDesc) * G.pseudo.size()));
  STRY(up(G.o_cols, G.cols.data(), sizeof(ColDesc) * G.cols.size()));
  STRY(up(G.o_blocks, G.blocks.data(), sizeof(BlockDesc) * G.blocks.size()));
  STRY(up(G.o_rbd, G.rbd.data(), sizeof(RowBlockDesc) * G.rbd.size()));
  STRY(up(G.o_scenes, G.scenes.data(), sizeof(SceneDesc) * G.scenes.size()));
  STRY(up(G.o_stab, G.stab.data(), sizeof(SceneTile) * G.stab.size()));
  STRY(up(G.o_cuts, G.cuts_flat.data(), 4 * G.cuts_flat.size()));
  STRY(up(G.o_tiles, G.tiles_flat.data(), 4 * G.tiles_flat.size()));
  STRY(up(G.o_tgram, G.t_gram.data(), 16 * G.t_gram.size()));
  if (!G.t_gpatch.empty()) STRY(up(G.o_tgpatch, G.t_gpatch.data(), 16 * G.t_gpatch.size()));
  STRY(up(G.o_tgtr, G.t_gtr.data(), 16 * G.t_gtr.size()));
  STRY(up(G.o_tz, G.t_z.data(), 16 * G.t_z.size()));
  STRY(up(G.o_stgc, G.st_gc.data(), 8 * G.st_gc.size()));
  for (int v = 0; v < 3; ++v) {
    STRY(up(G.o_items_n[v], G.items_n[v].data(), sizeof(GemmItem) * G.items_n[v].size()));
    STRY(up(G.o_items_h[v], G.items_h[v].data(), sizeof(GemmItem) * G.items_h[v].size()));
  }
  STRY(up(G.o_t0gram, G.t0_gram.data(), 16 * G.t0_gram.size()));
  STRY(hipMemcpyAsync(b->ws + G.o_phase, phases, 8 * (size_t)G.rows_total, hipMemcpyDeviceToDevice, st));
  Control* ctl = at<Control>(b, G.o_ctl);
  // instrument: bf16 planes, its transpose, and the shared Gram G0_j = H0_j H0_j^H (FP64)
  HStore hs{};
  hs.base = b->ws + G.o_hre;
  hs.base_im = b->ws + G.o_him;
  hs.row_scale = nullptr;
  hs.storage = ADMM_STORAGE_BF16;
  const BlockDesc* dpseudo = at<BlockDesc>(b, G.o_pseudo);
  STRY(launch_pack_quant(static_cast<const float2*>(H0), m0, n, dpseudo, P, (int)m0, hs, ctl, st));
  STRY(launch_btranspose(batch_args(b, nullptr), P, m0, G.max_nj, st));
  STRY(launch_btile_h(batch_args(b, nullptr), P, m0, st));
  {
    Geometry g0;
    g0.t_gram = G.t0_gram;
    STRY(launch_gram_build(g0, dpseudo, at<int4>(b, G.o_t0gram), hs, 0.0, at<double2>(b, G.o_G0), st));
  }
  // per-scene block inverses, in groups of bounded FP64 scratch
  {
    size_t i0 = 0;
    while (i0 < G.blocks.size()) {
      Geometry gg;
      std::vector<int32_t> tile0;
      size_t cur = 0;
      int64_t foff = 0;
      size_t i1 = i0;
      while (i1 < G.blocks.size()) {
        BlockDesc d = G.blocks[i1];
        const size_t sz = (size_t)d.mt * d.mt * 16;
        if (i1 > i0 && cur + sz > G.group_bytes) break;
        d.f_off = foff;
        foff += (int64_t)d.mt * d.mt;
        cur += sz;
        const int b_local = (int)gg.blocks.size();
        gg.blocks.push_back(d);
        gg.max_mt = std::max(gg.max_mt, d.mt);
        tile0.push_back(G.rbd[d.i].tile0);
        for (int a2 = 0; a2 < d.mt / kTile; ++a2)
          for (int c2 = 0; c2 <= a2; ++c2) gg.t_gram.push_back(make_int4(b_local, a2, c2, 0));
        ++i1;
      }
      BlockDesc* dgb = at<BlockDesc>(b, G.o_gblocks);
      int4* dgg = at<int4>(b, G.o_ggram);
      int32_t* dgt = at<int32_t>(b, G.o_gtile0);
      STRY(up(G.o_gblocks, gg.blocks.data(), sizeof(BlockDesc) * gg.blocks.size()));
      STRY(up(G.o_ggram, gg.t_gram.data(), 16 * gg.t_gram.size()));
      STRY(up(G.o_gtile0, tile0.data(), 4 * tile0.size()));
      STRY(launch_bgram_assemble(dgg, (int)gg.t_gram.size(), dgb, dgt, at<int32_t>(b, G.o_tiles),
                                 at<float2>(b, G.o_phase), at<double2>(b, G.o_G0), dpseudo, G.tile_rows, rho,
                                 at<double2>(b, G.o_A), st));
      STRY(launch_cholesky_inverse(gg, dgb, dgg, at<double2>(b, G.o_A), at<double2>(b, G.o_W),
                                   at<float2>(b, G.o_ginv), ctl, st));
      // the host vectors of this group must outlive the asynchronous uploads
      STRY(hipStreamSynchronize(st));
      i0 = i1;
    }
  }
  if (G.inv16)
    STRY(launch_to_bf16_pairs(at<float2>(b, G.o_ginv), at<uint32_t>(b, G.o_ginv16), (size_t)G.ginv_elems, st));
  Control hc;
  STRY(hipMemcpyAsync(&hc, ctl, sizeof hc, hipMemcpyDeviceToHost, st));
  STRY(hipStreamSynchronize(st));
  if (hc.nonfinite) return bail(admm_fail(ADMM_ENONFINITE, "H0 holds NaN or Inf"));
  if (hc.notpd) return bail(admm_fail(ADMM_ENOTPD, "a Gram matrix pivot was not positive"));
  if ((rc = autotune(b, st))) return bail(rc);
  STRY(hipStreamCreate(&b->gstream));
  STRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
  STRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
#undef STRY
  *out = b;
  return ADMM_OK;
}

int admm_batch_solve(admm_batch* b, const void* g, int iters, void* v_out, int use_graph, void* stream) {
  if (!b) return admm_fail(ADMM_EINVAL, "batch plan is NULL");
  if (!g || !v_out) return admm_fail(ADMM_EINVAL, "g and v_out must not be NULL");
  if (iters < 0) return admm_fail(ADMM_EINVAL, "iters must be >= 0");
  const BatchGeo& G = b->geo;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // zero the state: c, s, v, partials and the row vectors are contiguous
  BHIP(launch_fill(b->ws + G.o_c, G.o_phase - G.o_c, st));
  BHIP(launch_fill(at<Control>(b, G.o_ctl), 16, st));
  const float2* gp = static_cast<const float2*>(g);
  const bool graph = use_graph && !b->prof;
  if (graph && iters > 0) {
    if (!b->graph || b->graph_g != g) {
      if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
      }
      hipGraph_t gr = nullptr;
      BHIP(hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal));
      hipError_t e = launch_iteration(b, gp, b->gstream, false);
      hipError_t e2 = hipStreamEndCapture(b->gstream, &gr);
      if (e != hipSuccess) return admm_fail(ADMM_EHIP, "capture failed: %s", hipGetErrorString(e));
      if (e2 != hipSuccess) return admm_fail(ADMM_EHIP, "end capture failed: %s", hipGetErrorString(e2));
      BHIP(hipGraphInstantiate(&b->graph, gr, nullptr, nullptr, 0));
      (void)hipGraphDestroy(gr);
      b->graph_g = g;
    }
    BHIP(hipEventRecord(b->ev_in, st));
    BHIP(hipStreamWaitEvent(b->gstream, b->ev_in, 0));
    for (int k = 0; k < iters; ++k) BHIP(hipGraphLaunch(b->graph, b->gstream));
    BHIP(hipEventRecord(b->ev_out, b->gstream));
    BHIP(hipStreamWaitEvent(st, b->ev_out, 0));
  } else {
    for (int k = 0; k < iters; ++k) BHIP(launch_iteration(b, gp, st, b->prof));
  }
  BHIP(launch_bunpad_v(at<ColDesc>(b, G.o_cols), G.P, G.n, G.S, G.n_pad, at<float2>(b, G.o_v),
                       static_cast<float2*>(v_out), st));
  Control hc;
  BHIP(hipMemcpyAsync(&hc, at<Control>(b, G.o_ctl), sizeof hc, hipMemcpyDeviceToHost, st));
  BHIP(hipStreamSynchronize(st));
  if (hc.nonfinite) return admm_fail(ADMM_ENONFINITE, "a NaN or Inf reached the iterates");
  return ADMM_OK;
}

int admm_batch_profile(admm_batch* b, int enable) {
  if (!b) return admm_fail(ADMM_EINVAL, "batch plan is NULL");
  int rc = drain(b);
  if (rc) return rc;
  for (int k = 0; k < 4; ++k) {
    b->prof_ms[k] = 0;
    b->prof_n[k] = 0;
  }
  b->prof = enable != 0;
  return ADMM_OK;
}

int admm_batch_profile_read(admm_batch* b, int kernel, double* total_ms, int64_t* launches) {
  if (!b) return admm_fail(ADMM_EINVAL, "batch plan is NULL");
  if (kernel < 0 || kernel > 3) return admm_fail(ADMM_EINVAL, "unknown kernel id %d", kernel);
  int rc = drain(b);
  if (rc) return rc;
  if (total_ms) *total_ms = b->prof_ms[kernel];
  if (launches) *launches = b->prof_n[kernel];
  return ADMM_OK;
}

int admm_batch_info(const admm_batch* b, int64_t* info) {
  if (!b || !info) return admm_fail(ADMM_EINVAL, "batch plan and info must not be NULL");
  const BatchGeo& G = b->geo;
  int64_t v[16] = {G.m0, G.n, G.S, G.P, G.R, G.NST, (int64_t)G.total, G.ginv_elems * 8,
                   kSplitVariants[b->var_n], 64 * kAdjMS[b->var_h], (int64_t)G.items_n[b->var_n].size(),
                   (int64_t)G.items_h[b->var_h].size(), G.rows_total, 64 * fwd_ms(b->var_n, G.tile_rows), (int64_t)G.t_gpatch.size(), 0};
  std::memcpy(info, v, sizeof v);
  return ADMM_OK;
}

int admm_batch_tuning(const admm_batch* b, double* ms6) {
  if (!b || !ms6) return admm_fail(ADMM_EINVAL, "batch plan and output must not be NULL");
  for (int w = 0; w < 2; ++w)
    for (int v = 0; v < 3; ++v) ms6[3 * w + v] = b->tune_ms[w][v];
  return ADMM_OK;
}

void admm_batch_destroy(admm_batch* b) {
  if (!b) return;
  drain(b);
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->gstream) (void)hipStreamDestroy(b->gstream);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  delete b;
}

}  // extern "C"
