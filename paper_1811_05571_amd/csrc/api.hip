// C ABI of the split-lasso ADMM library: argument checks, workspace layout,
// plan lifetime and the host side of setup / solve / KKT check.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/admm.h"
#include "plan.h"

using namespace admm;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(ADMM_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                   \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace admm {
// Error helper shared with the batched form (sets admm_last_error).
int admm_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}
}  // namespace admm

namespace admm {

int build_geometry(Geometry& geo, int64_t m, int64_t n, int Q, const int64_t* row_off, int P,
                   const int64_t* col_off, int storage, std::string& err) {
  char buf[256];
  if (m < 1 || n < 1) {
    err = "m and n must be >= 1";
    return ADMM_EINVAL;
  }
  if (m > (int64_t)1 << 30 || n > (int64_t)1 << 30) {
    err = "m and n must be < 2^30";
    return ADMM_EINVAL;
  }
  if (Q < 1 || Q > m || P < 1 || P > n) {
    snprintf(buf, sizeof buf, "need 1 <= Q <= m and 1 <= P <= n (Q=%d P=%d m=%lld n=%lld)", Q, P,
             (long long)m, (long long)n);
    err = buf;
    return ADMM_EINVAL;
  }
  const bool inv16 = (storage & ADMM_INVERSE_BF16) != 0;
  const bool force_patches = (storage & ADMM_GRAM_PATCHES) != 0;
  const bool two_pass = (storage & ADMM_TWO_PASS) != 0;
  const bool want_lemma = (storage & ADMM_XUPDATE_LEMMA) != 0, want_direct = (storage & ADMM_XUPDATE_DIRECT) != 0;
  storage &= ~(ADMM_INVERSE_BF16 | ADMM_GRAM_PATCHES | ADMM_TWO_PASS | ADMM_XUPDATE_LEMMA | ADMM_XUPDATE_DIRECT);
  if (storage != ADMM_STORAGE_C64 && storage != ADMM_STORAGE_BF16 && storage != ADMM_STORAGE_FP8) {
    err = "unknown storage";
    return ADMM_EINVAL;
  }
  if (want_lemma && want_direct) {
    err = "ADMM_XUPDATE_LEMMA and ADMM_XUPDATE_DIRECT exclude each other";
    return ADMM_EINVAL;
  }
  geo.inv16 = inv16;
  geo.force_patches = force_patches;
  auto offsets = [&](int64_t total, int parts, const int64_t* given, std::vector<int64_t>& o) -> bool {
    o.assign(parts + 1, 0);
    if (given) {
      for (int k = 0; k <= parts; ++k) o[k] = given[k];
      if (o[0] != 0 || o[parts] != total) return false;
      for (int k = 0; k < parts; ++k)
        if (o[k + 1] <= o[k]) return false;
      return true;
    }
    const int64_t base = total / parts, extra = total % parts;
    for (int k = 0; k < parts; ++k) o[k + 1] = o[k] + base + (k < extra ? 1 : 0);
    return true;
  };
  if (!offsets(m, Q, row_off, geo.ro)) {
    err = "row offsets must increase strictly from 0 to m";
    return ADMM_EINVAL;
  }
  if (!offsets(n, P, col_off, geo.co)) {
    err = "column offsets must increase strictly from 0 to n";
    return ADMM_EINVAL;
  }
  geo.m = m;
  geo.n = n;
  geo.Q = Q;
  geo.P = P;
  geo.storage = storage;
  // padded spaces
  std::vector<int64_t> ldc(P), cpad0(P), ldr(Q), rpad0(Q);
  int64_t acc = 0;
  const int colpad = std::max(kColPad, 64 * cols_per_load(storage));
  for (int j = 0; j < P; ++j) {
    ldc[j] = round_up(geo.co[j + 1] - geo.co[j], colpad);
    cpad0[j] = acc;
    acc += ldc[j];
  }
  geo.n_pad = acc;
  acc = 0;
  for (int i = 0; i < Q; ++i) {
    ldr[i] = round_up(geo.ro[i + 1] - geo.ro[i], kRowPad);
    rpad0[i] = acc;
    acc += ldr[i];
  }
  geo.m_pad = acc;
  if (geo.n_pad > INT32_MAX || geo.m_pad > INT32_MAX) {
    err = "problem too large";
    return ADMM_EINVAL;
  }
  // H store row stride: whole 64-element groups (every lane load stays in
  // the row), moved off multiples of 4 KB so consecutive rows do not all
  // start on the same HBM channel.
  auto row_stride = [&](int64_t nj) {
    int64_t ldh = round_up(nj, kColPad);
    if ((ldh * elem_bytes(storage)) % 4096 == 0) ldh += kColPad;
    return ldh;
  };
  // Shape of the single-pass iteration (k_fused.hip) if the plan takes it:
  // complex64 storage, at most kFzMaxQ row blocks, each row block on a whole
  // number of waves: 512-thread workgroups (8 waves, two per CU) with RPL
  // from kFzRpl, else 1024 threads (16 waves, one per CU) with RPL <= 6.
  // Otherwise, with ADMM_TWO_PASS or in the direct form, the two-pass kernels.
  std::vector<int> gi(Q);   // 64-row groups of each row block
  for (int i = 0; i < Q; ++i) gi[i] = (int)(ldr[i] / kWave);
  int fz_nt = 0, fz_rpl = 0;
  if (!two_pass && storage == ADMM_STORAGE_C64 && Q <= kFzMaxQ) {
    auto waves = [&](int rpl) {
      int w = 0;
      for (int i = 0; i < Q; ++i) w += (gi[i] + rpl - 1) / rpl;
      return w;
    };
    const char* ent = getenv("ADMM_FZ_NT");
    const int want_nt = ent ? atoi(ent) : 0;
    if (want_nt != 1024)
      for (int r : kFzRpl)
        if (waves(r) <= 8) {
          fz_nt = 512;
          fz_rpl = r;
          break;
        }
    if (!fz_nt)
      for (int r : {1, 2, 3, 4, 6})
        if (waves(r) <= 16) {
          fz_nt = 1024;
          fz_rpl = r;
          break;
        }
  }
  // Form of the x-update (Sec. III-B, the remark after eq. inversion_lemma2;
  // Sec. III-C before eq. inversion_lemma3): unless a flag fixes it, the one
  // whose iteration streams fewer bytes, H once (single pass) or twice plus
  // the packed m_i x m_i inverses, or H twice plus the packed n_j x n_j ones.
  {
    auto packed = [](int64_t e) {
      const double T = (double)((e + kTile - 1) / kTile);
      return T * (T + 1) / 2 * kTile * kTile;
    };
    double hb = 0.0, lem = 0.0, dir = 0.0;
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j < P; ++j) {
        const int64_t mi = geo.ro[i + 1] - geo.ro[i], nj = geo.co[j + 1] - geo.co[j];
        hb += (double)mi * (double)row_stride(nj) * elem_bytes(storage);
        lem += packed(mi);
        dir += packed(nj);
      }
    const double esz = inv16 ? 4.0 : 8.0;
    const double lemma_bytes = (fz_nt ? 1.0 : 2.0) * hb + esz * lem, direct_bytes = 2.0 * hb + esz * dir;
    geo.direct = want_direct || (!want_lemma && direct_bytes < lemma_bytes);
  }
  geo.blocks.clear();
  int64_t hoff = 0, gioff = 0, foff = 0, gpo = 0;
  int max_mi = 0;
  geo.max_mt = 0;
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < P; ++j) {
      BlockDesc d{};
      d.i = i;
      d.j = j;
      d.mi = (int32_t)(geo.ro[i + 1] - geo.ro[i]);
      d.nj = (int32_t)(geo.co[j + 1] - geo.co[j]);
      d.ld = (int32_t)row_stride(d.nj);
      d.ldr = (int32_t)ldr[i];
      d.gd = geo.direct ? d.nj : d.mi;
      d.mt = (int32_t)round_up(d.gd, kTile);
      d.row0 = (int32_t)geo.ro[i];
      d.col0 = (int32_t)geo.co[j];
      d.rpad0 = (int32_t)rpad0[i];
      d.cpad0 = (int32_t)cpad0[j];
      d.h_off = hoff;
      d.gi_off = gioff;
      d.f_off = foff;
      d.gpo = (int32_t)gpo;
      hoff += (int64_t)d.mi * d.ld;
      const int64_t T = d.mt / kTile;
      gioff += T * (T + 1) / 2 * kTile * kTile;
      gpo += gram_part_vecs(T);
      foff += (int64_t)d.mt * d.mt;
      max_mi = std::max(max_mi, d.mi);
      geo.max_mt = std::max(geo.max_mt, d.mt);
      geo.blocks.push_back(d);
    }
  geo.cols.resize(P);
  for (int j = 0; j < P; ++j)
    geo.cols[j] = ColDesc{(int32_t)(geo.co[j + 1] - geo.co[j]), (int32_t)cpad0[j], (int32_t)geo.co[j],
                          (int32_t)ldc[j]};
  // workgroup tables
  geo.t_rows.clear();
  geo.t_cols.clear();
  geo.t_z.clear();
  geo.t_gram.clear();
  geo.t_kadj.clear();
  geo.t_hrows.clear();
  geo.t_gtr.clear();
  geo.t_wrows.clear();
  geo.t_gpatch.clear();
  const int cpl = cols_per_load(storage);
  int wg_per_chunk = 0;
  for (size_t b = 0; b < geo.blocks.size(); ++b) {
    const BlockDesc& d = geo.blocks[b];
    for (int r = 0; r < d.mi; r += kRowsPerWG) geo.t_rows.push_back(make_int4((int)b, r, 0, 0));
    const int hrows = rows_per_wave(storage) * kRowWaves;
    for (int r = 0; r < d.mi; r += hrows) geo.t_hrows.push_back(make_int4((int)b, r, 0, 0));
    for (int r = 0; r < d.mi; r += whole_rows(storage)) geo.t_wrows.push_back(make_int4((int)b, r, 0, 0));
    const int nl = (d.nj + cpl - 1) / cpl;
    wg_per_chunk += (nl + kColsPerWGLoads - 1) / kColsPerWGLoads;
    const int nt = d.mt / kTile;
    for (int a = 0; a < nt; ++a) {
      for (int c = 0; c <= a; ++c) geo.t_gram.push_back(make_int4((int)b, a, c, 0));
      geo.t_gtr.push_back(make_int4((int)b, a, 0, 0));
    }
    if (ADMM_GRAM_PATCH)
      for (int a = 0; a < (nt + 3) / 4; ++a)
        for (int c = 0; c <= a; ++c) geo.t_gpatch.push_back(make_int4((int)b, a, c, 0));
  }
  // 4 x 4 tile patches of the Gram apply: complex64 inverses only, when asked
  // or when there are enough of them to fill the GPU.
  if (!ADMM_GRAM_PATCH || geo.inv16 || !(geo.force_patches || geo.t_gpatch.size() >= kGramPatchMin))
    geo.t_gpatch.clear();
  // The whole-row product reads rows of up to kWholeCols columns in one
  // chunk, longer ones chunk by chunk (ADMM_WHOLE_WIDE).  Rows shorter than
  // half a chunk leave most of its lane loads idle: the streaming row
  // product serves those blocks (measured 236 against 385 us at 6144 x 1000
  // blocks, 60 against 125 us at 2160 x 703).
  {
    bool whole = storage == ADMM_STORAGE_C64 ? ADMM_WHOLE_ROWS
                 : (storage == ADMM_STORAGE_BF16 ? ADMM_WHOLE_ROWS_BF16 : ADMM_WHOLE_ROWS_FP8);
    for (const BlockDesc& d : geo.blocks)
      whole = whole && (d.nj <= kWholeCols || ADMM_WHOLE_WIDE) && d.nj >= kWholeCols / 2;
    if (!whole) geo.t_wrows.clear();
  }
  // Row chunks of the adjoint product: about ADMM_COLS_WG_TARGET(_C64)
  // workgroups in total, at least 32 rows (8 per wave) per chunk.
  {
    const int target = storage == 0 ? ADMM_COLS_WG_TARGET_C64 : ADMM_COLS_WG_TARGET;
    const int want = std::max(1, (target + wg_per_chunk - 1) / wg_per_chunk);
    const int cap = std::max(1, max_mi / 32);
    geo.KH = std::min(std::min(want, cap), 32);
  }
  for (int k = 0; k < geo.KH; ++k)
    for (size_t b = 0; b < geo.blocks.size(); ++b) {
      const BlockDesc& d = geo.blocks[b];
      const int nl = (d.nj + cpl - 1) / cpl;
      for (int c = 0; c < nl; c += kColsPerWGLoads) geo.t_cols.push_back(make_int4((int)b, c, k, 0));
      for (int c = 0; c < d.nj; c += kBlockThreads) geo.t_kadj.push_back(make_int4((int)b, c, k, 0));
    }
  for (int j = 0; j < P; ++j)
    for (int c = 0; c < geo.cols[j].nj; c += kZCols) geo.t_z.push_back(make_int4(j, c, 0, 0));

  // direct form: rows of the local-data kernel
  geo.t_dgp.clear();
  if (geo.direct)
    for (int i = 0; i < Q; ++i)
      for (int64_t r = 0; r < geo.ro[i + 1] - geo.ro[i]; r += kBlockThreads)
        geo.t_dgp.push_back(make_int4(i, (int)r, 0, 0));

  // Single-pass iteration tables (shape chosen above)
  geo.fz = false;
  geo.t_fz.clear();
  geo.fz_colwg.clear();
  geo.t_fzr.clear();
  geo.fzt = FzArgs{};
  if (fz_nt && !geo.direct) {
    const int nt = fz_nt, rpl = fz_rpl;
    {
      FzArgs& z = geo.fzt;
      int w = 0;
      for (int i = 0; i < Q; ++i) {
        z.bw[i] = w;
        for (int g = 0; g < gi[i]; g += rpl, ++w) {
          z.ngw[w] = std::min(rpl, gi[i] - g);
          z.g0[w] = (int)(rpad0[i] / kWave) + g;
          z.wblk[w] = i;
        }
        z.rpad0[i] = (int)rpad0[i];
        z.mi[i] = (int)(geo.ro[i + 1] - geo.ro[i]);
        z.row0[i] = (int)geo.ro[i];
      }
      z.bw[Q] = w;
      // slabs of CPL columns per column block, spread over at most
      // ADMM_FZ_WGS workgroups (those resident at once: two of 512 threads or
      // one of 1024 per CU) in proportion to the block widths, by largest
      // remainders, at least one per block; one workgroup more than fit
      // would run alone after the others and double the kernel's time.
      // Workgroup q of a block of ns slabs with N workgroups takes the run of
      // slabs [q ns / N, (q + 1) ns / N): its new s, c and v then fill whole
      // cache lines (eight slabs at a time) instead of 16-byte pieces.
      const int cplz = cols_per_load(storage);
      std::vector<int64_t> ns(P);
      int64_t tot = 0;
      for (int j = 0; j < P; ++j) tot += (ns[j] = (geo.cols[j].nj + cplz - 1) / cplz);
      int target = nt == 512 ? ADMM_FZ_WGS : ADMM_FZ_WGS / 2;
      if (const char* e = getenv("ADMM_FZ_WGS")) target = std::max(1, atoi(e));
      std::vector<int64_t> nw(P);
      std::vector<std::pair<double, int>> rem(P);
      int64_t given = 0;
      for (int j = 0; j < P; ++j) {
        const double share = (double)target * (double)ns[j] / (double)tot;
        nw[j] = std::max<int64_t>(1, std::min<int64_t>(ns[j], (int64_t)share));
        rem[j] = {share - std::floor(share), j};
        given += nw[j];
      }
      std::stable_sort(rem.begin(), rem.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
        return a.first > b.first;
      });
      for (int k = 0; k < P && given < target; ++k) {
        const int j = rem[k].second;
        if (nw[j] < ns[j]) {
          ++nw[j];
          ++given;
        }
      }
      int64_t sgb = 0;
      for (int j = 0; j < P; ++j) {
        const int nwj = (int)nw[j];
        const int w0 = (int)geo.t_fz.size();
        for (int q = 0; q < nwj; ++q)
          geo.t_fz.push_back(make_int4(j, (int)(ns[j] * q / nwj), (int)(ns[j] * (q + 1) / nwj), (int)sgb));
        geo.fz_colwg.push_back(make_int2(w0, (int)geo.t_fz.size()));
        sgb += ns[j];
      }
      geo.fz_slabs = sgb;
      // row kernel: S threads per row share a column block's parts, S the
      // smallest power of two that leaves each at most ADMM_FZR_LOADS of them
      // (a row's parts are dependent loads: a long run is a chain of latencies)
      int64_t tmax = 1;
      for (int j = 0; j < P; ++j) tmax = std::max(tmax, nw[j]);
      int loads = ADMM_FZR_LOADS;
      if (const char* e = getenv("ADMM_FZR_LOADS")) loads = std::max(1, atoi(e));
      int S = 1;
      while (S < kWave && tmax > (int64_t)S * loads) S *= 2;
      const int R = kBlockThreads / S;
      for (size_t b = 0; b < geo.blocks.size(); ++b)
        for (int r = 0; r < geo.blocks[b].mi; r += R) geo.t_fzr.push_back(make_int4((int)b, r, S, 0));
      z.nwg = (int)geo.t_fz.size();
      geo.fz = true;
      geo.fz_nt = nt;
      geo.fz_rpl = rpl;
    }
  }

  // workspace layout
  Layout& L = geo.lay;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t plane = (size_t)hoff * (storage == ADMM_STORAGE_C64 ? 8 : (storage == ADMM_STORAGE_BF16 ? 2 : 1));
  L.H = take(plane);
  L.h_bytes = plane;
  if (storage != ADMM_STORAGE_C64) {
    L.H_im = take(plane);
    L.h_bytes += plane;
  }
  if (storage == ADMM_STORAGE_FP8) {
    L.H_scale = take(4 * (size_t)m);
    L.h_bytes += 4 * (size_t)m;
  }
  // column-slab copy of H for the single-pass iteration (zeroed with H at setup)
  L.hs_bytes = geo.fz ? (size_t)geo.fz_slabs * (size_t)geo.m_pad * (size_t)cols_per_load(storage) * 8 : 0;
  L.Hs = take(L.hs_bytes);
  L.ginv_bytes = (size_t)gioff * 8;
  L.Ginv = take(L.ginv_bytes);
  if (geo.inv16) L.Ginv16 = take((size_t)gioff * 4);
  L.F64a = take((size_t)foff * 16);
  L.F64b = take((size_t)foff * 16);
  const size_t colv = (size_t)geo.n_pad * 8, rowv = (size_t)geo.m_pad * 8;
  L.c = take(colv * Q);
  L.s = take(colv * Q);
  L.v = take(colv);
  L.part = take(colv * Q * geo.KH);
  L.gp = take(rowv * P);
  L.ghat = take(rowv * P);
  // the Gram-space vectors: row space, or column space in the direct form
  const size_t gspace = geo.direct ? colv * Q : rowv * P;
  L.r = take(gspace);
  L.y = take(gspace);
  L.fpart = take((size_t)geo.t_fz.size() * rowv);   // in the state region: zeroed with it
  L.dflag = take(16);                                  // direct form: the u_ref word (zeroed with the state)
  L.blocks = take(sizeof(BlockDesc) * geo.blocks.size());
  L.cols = take(sizeof(ColDesc) * P);
  L.t_rows = take(16 * geo.t_rows.size());
  L.t_cols = take(16 * geo.t_cols.size());
  L.t_z = take(16 * geo.t_z.size());
  L.t_gram = take(16 * geo.t_gram.size());
  L.t_kadj = take(16 * geo.t_kadj.size());
  L.t_hrows = take(16 * geo.t_hrows.size());
  L.t_wrows = take(16 * std::max<size_t>(geo.t_wrows.size(), 1));
  L.t_gpatch = take(16 * std::max<size_t>(geo.t_gpatch.size(), 1));
  L.t_gtr = take(16 * geo.t_gtr.size());
  L.t_fz = take(16 * std::max<size_t>(geo.t_fz.size(), 1));
  L.fz_colwg = take(8 * std::max<size_t>(geo.fz_colwg.size(), 1));
  L.t_fzr = take(16 * std::max<size_t>(geo.t_fzr.size(), 1));
  L.t_dgp = take(16 * std::max<size_t>(geo.t_dgp.size(), 1));
  L.gpart = take((size_t)gpo * kTile * 8);
  L.ctl = take(sizeof(Control));
  L.redpart = take(8 * kRedCount * std::max(geo.t_z.size(), geo.t_fz.size()));
  L.row_block = take(8 * (size_t)m);
  L.kkt_e = take(16 * (size_t)m);
  L.kkt_v = take(colv);
  L.kkt_part = take(2 * colv * Q * geo.KH);
  L.kkt_max = take(8 * geo.t_z.size());
  // adjoint sweep
  L.vb = take(colv);
  L.sb = take(colv * Q);
  L.ub = take(colv * Q);
  L.ghb = take(rowv * P);
  L.gpb = take(rowv * P);
  L.yb = take(rowv * P);
  L.rb = take(rowv * P);
  L.gbar = take(16 * (size_t)m);
  L.kpart = take(8 * geo.t_z.size());
  L.rpart = take(8 * geo.t_rows.size());
  L.total = off;
  return ADMM_OK;
}

}  // namespace admm

// Device scratch of admm_kkt_noalloc: one array per GPU, held until the
// process ends.  In host code `scratch` only names the symbol; its device
// address on the current GPU comes from hipGetSymbolAddress (static_scratch).
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kScratchDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call per device and kept.
int static_scratch(char** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices)
    return fail(ADMM_EUNSUPPORTED, "device %d is beyond the %d devices of the static scratch table", dev,
                kScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(ADMM_EHIP, "hipGetSymbolAddress returned no address for the static scratch");
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return ADMM_OK;
}
}  // namespace

struct admm_plan {
  Geometry geo;
  double rho = 1.0, lam = 0.0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  float2 *H = nullptr, *Ginv = nullptr, *c = nullptr, *s = nullptr, *v = nullptr, *part = nullptr;
  uint32_t* Ginv16 = nullptr;
  float2 *gp = nullptr, *ghat = nullptr, *r = nullptr, *y = nullptr, *kkt_v = nullptr;
  double2 *F64a = nullptr, *F64b = nullptr, *kkt_e = nullptr, *kkt_part = nullptr;
  BlockDesc* d_blocks = nullptr;
  ColDesc* d_cols = nullptr;
  int4 *t_rows = nullptr, *t_cols = nullptr, *t_z = nullptr, *t_gram = nullptr, *t_kadj = nullptr, *t_hrows = nullptr;
  int4* t_wrows = nullptr;
  int4* t_gpatch = nullptr;
  int4* t_gtr = nullptr;
  float2* gpart = nullptr;
  HStore hs{};
  Control* ctl = nullptr;
  double *redpart = nullptr, *kkt_max = nullptr;
  int64_t* row_block = nullptr;
  std::vector<int64_t> h_row_block;
  int k_done = 0;
  uint64_t serial = 0;
  float2 *vb = nullptr, *sb = nullptr, *ub = nullptr, *ghb = nullptr, *gpb = nullptr, *yb = nullptr, *rb = nullptr;
  double2* gbar = nullptr;
  double *kpart = nullptr, *rpart = nullptr;
  // single-pass iteration: tables, arguments, and whether the workgroup parts
  // of H c in the workspace belong to the current c (else a forward-only slab
  // pass recomputes them before the first iteration)
  int4 *t_fz = nullptr, *t_fzr = nullptr;
  int2* fz_colwg = nullptr;
  int4* t_dgp = nullptr;   // direct form: rows of the local-data kernel
  int* dflag = nullptr;    // direct form: 1 when y holds the last u and ghat = H y
  FzArgs fz{};
  bool fz_valid = true;
  // graph replay of fixed-length runs of iterations (admm_solve): captured on
  // an internal stream, keyed by what the captured launches depend on
  bool graphs = false;   // plain launches: faster than graph replay on MI355X (admm_set_graphs)
  hipStream_t gs = nullptr;
  hipEvent_t gin = nullptr, gout = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void* gkey_g = nullptr;
  const void* gkey_hist = nullptr;
  float gkey_kappa = 0.f;
  int gkey_chunk = 0;
  // profiling
  bool prof = false;
  int prof_every = 1;    // time the kernels of every prof_every-th iteration
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[ADMM_K_COUNT];
  std::vector<hipEvent_t> pool;
  double prof_ms[ADMM_K_COUNT] = {};
  int64_t prof_n[ADMM_K_COUNT] = {};
};

namespace {

template <class T>
T* at(admm_plan* p, size_t off) {
  return reinterpret_cast<T*>(p->ws + off);
}

hipError_t ev_get(admm_plan* p, hipEvent_t* e) {
  if (!p->pool.empty()) {
    *e = p->pool.back();
    p->pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Launch through the profiler when it is on.
// The events ride on the kernels' own dispatch packets (KTime), so a profiled
// solve has the same kernel-to-kernel spacing as an unprofiled one.
template <class F>
int timed(admm_plan* p, int kind, int iter, hipStream_t st, F&& launch) {
  KTime kt;
  const bool on = p->prof && iter % p->prof_every == 0;
  if (on) {
    HIP_TRY(ev_get(p, &kt.start));
    HIP_TRY(ev_get(p, &kt.stop));
  }
  hipError_t e = launch(kt);
  if (e != hipSuccess) return fail(ADMM_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  if (on) p->ev[kind].emplace_back(kt.start, kt.stop);
  return ADMM_OK;
}

int drain_profile(admm_plan* p) {
  for (int k = 0; k < ADMM_K_COUNT; ++k) {
    for (auto& pr : p->ev[k]) {
      HIP_TRY(hipEventSynchronize(pr.second));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
      p->prof_ms[k] += ms;
      p->prof_n[k] += 1;
      p->pool.push_back(pr.first);
      p->pool.push_back(pr.second);
    }
    p->ev[k].clear();
  }
  return ADMM_OK;
}

IterArgs iter_args(admm_plan* p, const float2* g, double* hist) {
  IterArgs a{};
  a.blocks = p->d_blocks;
  a.cols = p->d_cols;
  a.hs = p->hs;
  a.Ginv = p->Ginv;
  a.Ginv16 = p->Ginv16;
  a.g = g;
  a.c = p->c;
  a.s = p->s;
  a.v = p->v;
  a.part = p->part;
  a.gp = p->gp;
  a.ghat = p->ghat;
  a.r = p->r;
  a.y = p->y;
  a.gpart = p->gpart;
  a.ctl = p->ctl;
  a.redpart = p->redpart;
  a.nz = (int)p->geo.t_z.size();
  a.hist = hist;
  a.arec = nullptr;
  a.m_pad = p->geo.m_pad;
  a.n_pad = p->geo.n_pad;
  a.Q = p->geo.Q;
  a.P = p->geo.P;
  a.KH = p->geo.KH;
  a.rho = (float)p->rho;
  a.kappa = (float)(p->lam / (p->geo.Q * p->rho));
  a.rho2Q = p->rho * p->rho * p->geo.Q;
  a.cpl = cols_per_load(p->geo.storage);
  int64_t x4 = 0;   // float4 of c per column block in the row product's layout
  for (const ColDesc& cd : p->geo.cols)
    x4 = std::max<int64_t>(x4, (int64_t)(cd.nj + kWave * a.cpl - 1) / (kWave * a.cpl) * kWave * (a.cpl / 2));
  a.xstage = x4 <= kXStage ? 1 : 0;
  a.wide = 0;
  for (const ColDesc& cd : p->geo.cols) a.wide |= cd.nj > kWholeCols ? 1 : 0;
  a.direct = p->geo.direct ? 1 : 0;
  a.uref = p->dflag;
  return a;
}

int reset_state(admm_plan* p, hipStream_t st) {
  const Layout& L = p->geo.lay;
  // c, s, v, part, gp, ghat, r, y are contiguous in the layout
  const size_t bytes = L.blocks - L.c;
  HIP_TRY(launch_fill(p->ws + L.c, bytes, st));
  p->k_done = 0;
  p->fz_valid = true;   // zero parts of H c for c = 0
  return ADMM_OK;
}

}  // namespace


namespace {

constexpr uint32_t kTapeMagic = 0x45504154u;  // "TAPE"

struct TapeHeader {
  uint32_t magic, version;
  int32_t iters, interval, nseg, Q, P, pad;
  int64_t m_pad, n_pad;
  double lam, rho;
  uint64_t serial;
  uint64_t pad2[23];
};
static_assert(sizeof(TapeHeader) == 256, "tape header");

struct TapeLayout {
  size_t ckpt = 0, ckpt_stride = 0, v = 0, s = 0, ghat = 0, yrec = 0, arec = 0, total = 0;
};

TapeLayout tape_layout(const Geometry& G, int iters, int interval) {
  TapeLayout t;
  const size_t colv = (size_t)G.n_pad * 8, rowv = (size_t)G.m_pad * 8;
  t.v = 0;
  t.s = align256(colv);
  t.ghat = t.s + align256(colv * G.Q);
  t.ckpt_stride = t.ghat + align256(rowv * G.P);
  const int nseg = (iters + interval - 1) / interval;
  t.ckpt = 256;
  t.yrec = t.ckpt + t.ckpt_stride * nseg;
  t.arec = t.yrec + align256(rowv * G.P) * interval;
  t.total = t.arec + align256(colv) * interval;
  return t;
}

}  // namespace

extern "C" {

int admm_version(void) { return 100; }

const char* admm_strerror(int status) {
  switch (status) {
    case ADMM_OK: return "ADMM_OK";
    case ADMM_EINVAL: return "ADMM_EINVAL: invalid argument";
    case ADMM_EWORKSPACE: return "ADMM_EWORKSPACE: workspace missing, too small or misaligned";
    case ADMM_EHIP: return "ADMM_EHIP: HIP runtime error";
    case ADMM_ENOTPD: return "ADMM_ENOTPD: Gram matrix not positive definite";
    case ADMM_ENONFINITE: return "ADMM_ENONFINITE: non-finite value in H, g or the iterates";
    case ADMM_ESTATE: return "ADMM_ESTATE: call out of order";
    case ADMM_EUNSUPPORTED: return "ADMM_EUNSUPPORTED: combination not built";
    default: return "ADMM: unknown status";
  }
}

const char* admm_last_error(void) { return g_last_error.c_str(); }

int admm_workspace_bytes(int64_t m, int64_t n, int Q, const int64_t* row_off, int P, const int64_t* col_off,
                         int storage, size_t* out_bytes) {
  g_last_error.clear();
  if (!out_bytes) return fail(ADMM_EINVAL, "out_bytes is NULL");
  Geometry geo;
  std::string err;
  int rc = build_geometry(geo, m, n, Q, row_off, P, col_off, storage, err);
  if (rc) return fail(rc, "%s", err.c_str());
  *out_bytes = geo.lay.total;
  return ADMM_OK;
}

namespace {
// Timing model of a plan (admm_choose_split): setup and per-iteration
// seconds as sums of features times per-unit costs (coefficients).
// Setup: FP64 flops; the Gram build's span, ceil(K / 32) K-chunks of one
// tile's workgroup times ceil(tiles / 512) rounds of workgroups (two of its
// 67 KB-LDS workgroups fit each of the 256 CUs; K = n_j, or m_i in the
// direct form); the tiled Cholesky's and triangular inverse's
// serial panel steps (T = tile-padded Gram edge / 64); blocks; fixed.
// Iteration: the bytes of H the single pass streams, weighted by its wave
// load factor (slot groups over row groups) and split by workgroup size
// (512 or 1024 threads); all other algorithmic bytes (all of them for the
// two-pass and direct forms); blocks; fixed.
constexpr int kSetupTerms = 5, kIterTerms = 5;
constexpr int kCoefs = kSetupTerms + kIterTerms;
// Coefficients fitted by non-negative least squares (relative error) to the
// setup and 50-iteration times of all 169 candidate splits of 2160 x 22500
// and 6144 x 32000 on MI355X (complex64): s/flop (69 TFLOP/s), s per span
// unit, s per panel step, s per block, s; s per single-pass byte of H (512-
// and 1024-thread workgroups), s per other byte (7.0 TB/s), s per block, s.
constexpr double kDefaultCoef[kCoefs] = {1.462e-14, 7.313e-06, 3.683e-04, 2.004e-06, 7.954e-04,
                                         7.962e-14, 1.344e-13, 1.436e-13, 1.701e-08, 6.400e-05};

void model_features(const Geometry& geo, double iter_bytes, double flops, double* fs, double* fi) {
  int64_t kmax = 0;
  for (const BlockDesc& d : geo.blocks) kmax = std::max<int64_t>(kmax, geo.direct ? d.mi : d.nj);
  const double tiles = (double)geo.t_gram.size();
  const double nb = (double)geo.blocks.size();
  fs[0] = flops;
  fs[1] = std::ceil((double)kmax / 32.0) * std::ceil(tiles / 512.0);
  fs[2] = geo.max_mt / kTile;
  fs[3] = nb;
  fs[4] = 1.0;
  const double h = (double)geo.lay.h_bytes;
  double hz = 0.0;
  if (geo.fz) {
    int groups = 0;
    const int waves = geo.fzt.bw[geo.Q];
    for (int w = 0; w < waves; ++w) groups += geo.fzt.ngw[w];
    hz = h * (double)(waves * geo.fz_rpl) / (double)std::max(groups, 1);
  }
  fi[0] = geo.fz && geo.fz_nt == 512 ? hz : 0.0;
  fi[1] = geo.fz && geo.fz_nt == 1024 ? hz : 0.0;
  fi[2] = geo.fz ? std::max(0.0, iter_bytes - h) : iter_bytes;
  fi[3] = nb;
  fi[4] = 1.0;
}

double dot_n(const double* a, const double* b, int n) {
  double t = 0.0;
  for (int k = 0; k < n; ++k) t += a[k] * b[k];
  return t;
}

// Cost model of one split (host only; see admm_split_cost).
void split_cost(const Geometry& geo, double* out) {
  const int64_t m = geo.m, n = geo.n;
  const int Q = geo.Q, P = geo.P;
  int64_t mi = 0, nj = 0;
  for (int i = 0; i < Q; ++i) mi = std::max(mi, geo.ro[i + 1] - geo.ro[i]);
  for (int j = 0; j < P; ++j) nj = std::max(nj, geo.co[j + 1] - geo.co[j]);
  // elements one node sends and receives per iteration (Sec. IV, table of
  // exchanged elements; with uneven blocks the largest ones)
  double exch = 0.0;
  if (Q > 1 && P == 1) exch = 2.0 * (double)n;
  else if (Q == 1 && P > 1) exch = (double)P * (double)m;
  else if (Q > 1 && P > 1) exch = (double)P * (double)mi + 2.0 * (double)nj;
  // HBM bytes of one iteration: the four per-iteration kernels' algorithmic bytes
  const double e = elem_bytes(geo.storage), c = 8.0;
  const double h = (double)m * (double)n * e + (geo.storage == ADMM_STORAGE_FP8 ? 4.0 * (double)m * P : 0.0);
  const double vrows = c * P * (double)m, vcols = c * Q * (double)n;
  const bool patch = !geo.t_gpatch.empty();
  double ginv = 0.0, parts = 0.0, flops = 0.0;
  for (const BlockDesc& d : geo.blocks) {
    const double T = d.mt / kTile;
    ginv += T * (T + 1) / 2 * kTile * kTile;
    parts += T * (patch ? std::ceil(T / 4) + 1 : T);
    // FP64 setup: lower half of the Gram matrix (gd (gd + 1) / 2 times the
    // other edge complex multiply-adds), Cholesky, triangular inverse and
    // W^H W (gd^3 / 3 each), 8 real flops per complex multiply-add
    const double a = d.gd, b = geo.direct ? d.mi : d.nj;
    flops += 8.0 * (a * (a + 1) / 2 * b + a * a * a);
  }
  double gemv_n = h + vcols + c * m + (P > 1 ? (P - 1) * vrows + 2 * vrows : vrows);
  double gram = ginv * (geo.inv16 ? 4.0 : c) + 2 * parts * kTile * c + vrows * (P > 1 ? 4 : 3);
  const double gemv_h = h + vrows + geo.KH * vcols;
  // more than 32 replicas do not stay in registers: the z-update reads c and
  // the row-chunk partials a second time
  const double zupd = geo.KH * vcols + 4 * vcols + 2 * c * n + (Q > 32 ? (geo.KH + 1) * vcols : 0.0);
  for (int k = 0; k < 16; ++k) out[k] = 0.0;
  out[0] = exch;
  out[1] = gemv_n + gram + gemv_h + zupd;
  if (geo.direct) {
    // direct form: the residuals of every block (reads g and ghat, writes
    // one row vector per block), their adjoint product, d = the partials +
    // rho (c - u_prev), the Gram apply to d (its pieces are added by the
    // z-update), the z-update (reads the pieces, u_prev and s, writes s, c and
    // u, reads and writes v), the row product ghat = H u
    const double dgp = c * m + 2 * vrows;
    const double rhs = (geo.KH + 3) * vcols;
    gram = ginv * (geo.inv16 ? 4.0 : c) + parts * kTile * c + vcols;
    const double dz = parts * kTile * c + 5 * vcols + 2 * c * n;
    gemv_n = h + vcols + vrows;
    out[1] = dgp + gemv_h + rhs + gram + dz + gemv_n;
  }
  if (geo.fz) {
    // single pass: the slab kernel reads H once, y, c and s, writes c, s, v
    // and its row parts of H c; the row kernel reads the parts and forms r
    const double parts = (double)geo.t_fz.size() * (double)m * c;
    const double fz_slab = h + vrows + 4 * vcols + 2 * c * n + parts;
    const double fz_rows = parts + c * m + (P > 1 ? (P - 1) * vrows + 2 * vrows : vrows);
    out[1] = fz_rows + gram + fz_slab;
  }
  out[2] = flops;
  out[3] = (double)geo.lay.ginv_bytes;
  out[4] = (double)geo.lay.h_bytes;
  out[5] = (double)geo.lay.total;
  out[6] = (double)mi;
  out[7] = (double)nj;
  out[8] = geo.KH;
  out[9] = (double)geo.t_gpatch.size();
  out[10] = geo.fz ? 1.0 : 0.0;
  out[11] = (double)geo.t_fz.size();
  out[12] = geo.direct ? 1.0 : 0.0;
  // features of the timing model (model_features)
  double fs[kSetupTerms], fi[kIterTerms];
  model_features(geo, out[1], out[2], fs, fi);
  out[13] = geo.fz ? (fi[0] + fi[1]) / (double)geo.lay.h_bytes : 0.0;   // single pass: wave load factor
  out[14] = geo.fz ? geo.fz_nt : 0;
  out[15] = fs[1];                                                       // Gram-build span
}
}  // namespace

int admm_split_cost(int64_t m, int64_t n, int Q, const int64_t* row_off, int P, const int64_t* col_off, int storage,
                    double* out16) {
  g_last_error.clear();
  if (!out16) return fail(ADMM_EINVAL, "out is NULL");
  Geometry geo;
  std::string err;
  const int rc = build_geometry(geo, m, n, Q, row_off, P, col_off, storage, err);
  if (rc) return fail(rc, "%s", err.c_str());
  split_cost(geo, out16);
  return ADMM_OK;
}

namespace {
constexpr int kCand[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32};

// Modelled seconds of setup plus `iters` iterations of every candidate equal
// split within the exchange limit, cheapest first.
struct Priced {
  double t;
  int Q, P;
};
void price_candidates(int64_t m, int64_t n, int iters, int storage, double max_exchange, const double* coef,
                      std::vector<Priced>& v) {
  v.clear();
  for (int Q : kCand)
    for (int P : kCand) {
      if (Q > m || P > n) continue;
      Geometry geo;
      std::string err;
      if (build_geometry(geo, m, n, Q, nullptr, P, nullptr, storage, err) != ADMM_OK) continue;
      double c[16];
      split_cost(geo, c);
      if (max_exchange > 0.0 && c[0] > max_exchange) continue;
      double fs[kSetupTerms], fi[kIterTerms];
      model_features(geo, c[1], c[2], fs, fi);
      const double t = dot_n(fs, coef, kSetupTerms) + iters * dot_n(fi, coef + kSetupTerms, kIterTerms);
      v.push_back({t, Q, P});
    }
  std::stable_sort(v.begin(), v.end(), [](const Priced& a, const Priced& b) { return a.t < b.t; });
}

int check_coef(const double* coef) {
  for (int k = 0; k < kCoefs; ++k)
    if (!(coef[k] >= 0.0) || !std::isfinite(coef[k]))
      return fail(ADMM_EINVAL, "coefficient %d must be finite and >= 0", k);
  return ADMM_OK;
}

// Non-negative least squares for a few unknowns: rows of X (nf columns
// `cols` of a row-major matrix with stride ld) against y, relative residuals
// (each row divided by y); an active set that drops the most negative
// coefficient and solves again.  Columns not in `cols` keep their value.
void nnls_small(const std::vector<double>& X, int ld, const std::vector<double>& y, std::vector<int> cols,
                double* coef) {
  const int rows = (int)y.size();
  while (!cols.empty()) {
    const int k = (int)cols.size();
    std::vector<double> A(k * k, 0.0), b(k, 0.0);
    for (int r = 0; r < rows; ++r) {
      const double w = 1.0 / (y[r] * y[r]);
      for (int a = 0; a < k; ++a) {
        b[a] += w * X[r * ld + cols[a]] * y[r];
        for (int c = 0; c < k; ++c) A[a * k + c] += w * X[r * ld + cols[a]] * X[r * ld + cols[c]];
      }
    }
    // scaled Gaussian elimination with partial pivoting (features differ by
    // many orders of magnitude: columns scaled to unit diagonal first)
    std::vector<double> sc(k);
    for (int a = 0; a < k; ++a) sc[a] = A[a * k + a] > 0 ? 1.0 / std::sqrt(A[a * k + a]) : 1.0;
    for (int a = 0; a < k; ++a) {
      b[a] *= sc[a];
      for (int c = 0; c < k; ++c) A[a * k + c] *= sc[a] * sc[c];
    }
    bool singular = false;
    for (int piv = 0; piv < k; ++piv) {
      int best = piv;
      for (int r = piv + 1; r < k; ++r)
        if (std::fabs(A[r * k + piv]) > std::fabs(A[best * k + piv])) best = r;
      if (std::fabs(A[best * k + piv]) < 1e-12) {
        singular = true;
        break;
      }
      if (best != piv) {
        for (int c = 0; c < k; ++c) std::swap(A[piv * k + c], A[best * k + c]);
        std::swap(b[piv], b[best]);
      }
      for (int r = piv + 1; r < k; ++r) {
        const double f = A[r * k + piv] / A[piv * k + piv];
        for (int c = piv; c < k; ++c) A[r * k + c] -= f * A[piv * k + c];
        b[r] -= f * b[piv];
      }
    }
    std::vector<double> x(k, 0.0);
    if (!singular)
      for (int r = k - 1; r >= 0; --r) {
        double t = b[r];
        for (int c = r + 1; c < k; ++c) t -= A[r * k + c] * x[c];
        x[r] = t / A[r * k + r] * 1.0;
      }
    int worst = -1;
    for (int a = 0; a < k; ++a) {
      x[a] *= sc[a];
      if (singular || x[a] < 0.0)
        if (worst < 0 || x[a] < x[worst]) worst = a;
    }
    if (singular) worst = k - 1;   // drop the last column and try again
    if (worst < 0) {
      for (int a = 0; a < k; ++a) coef[cols[a]] = x[a];
      return;
    }
    coef[cols[worst]] = 0.0;
    cols.erase(cols.begin() + worst);
  }
}

// Wall time of one setup and of `its` iterations (after a warm-up solve) of
// split (Q, P) with the given flags, in the caller's workspace.
int time_split(const void* H, const void* g, int64_t m, int64_t n, int Q, int P, int storage, void* ws,
               size_t ws_bytes, void* stream, int its, double* setup_s, double* iter_s, Geometry* geo_out) {
  Geometry geo;
  std::string err;
  int rc = build_geometry(geo, m, n, Q, nullptr, P, nullptr, storage, err);
  if (rc) return fail(rc, "%s", err.c_str());
  if (geo.lay.total > ws_bytes) return ADMM_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  admm_plan* p = nullptr;
  HIP_TRY(hipStreamSynchronize(st));
  auto t0 = std::chrono::steady_clock::now();
  rc = admm_setup(&p, H, m, n, Q, nullptr, P, nullptr, 1.0, 0.0, storage, ws, ws_bytes, stream);
  auto t1 = std::chrono::steady_clock::now();
  if (rc) return rc;
  // v_out in the workspace's KKT staging vector (n_pad >= n complex), not read back
  void* v_out = p->kkt_v;
  rc = admm_solve(p, g, std::min(its, 10), 0.0, 1, v_out, nullptr, nullptr, 0, stream);
  auto t2 = std::chrono::steady_clock::now();
  if (!rc) rc = admm_solve(p, g, its, 0.0, 1, v_out, nullptr, nullptr, 0, stream);
  auto t3 = std::chrono::steady_clock::now();
  if (geo_out) *geo_out = p->geo;
  admm_destroy(p);
  if (rc) return rc;
  *setup_s = std::chrono::duration<double>(t1 - t0).count();
  *iter_s = std::chrono::duration<double>(t3 - t2).count() / its;
  return ADMM_OK;
}
}  // namespace

int admm_model_coefficients(double* coef) {
  g_last_error.clear();
  if (!coef) return fail(ADMM_EINVAL, "coef is NULL");
  for (int k = 0; k < kCoefs; ++k) coef[k] = kDefaultCoef[k];
  return ADMM_OK;
}

int admm_choose_split(int64_t m, int64_t n, int iters, int storage, double max_exchange, const double* coef,
                      int* Q_out, int* P_out, double* model_s) {
  g_last_error.clear();
  if (!Q_out || !P_out) return fail(ADMM_EINVAL, "Q_out and P_out must not be NULL");
  if (iters < 0) return fail(ADMM_EINVAL, "iters must be >= 0");
  if (coef && check_coef(coef)) return ADMM_EINVAL;
  std::vector<Priced> v;
  price_candidates(m, n, iters, storage, max_exchange, coef ? coef : kDefaultCoef, v);
  if (v.empty()) return fail(ADMM_EUNSUPPORTED, "no candidate split meets the exchange limit");
  *Q_out = v[0].Q;
  *P_out = v[0].P;
  if (model_s) *model_s = v[0].t;
  return ADMM_OK;
}

int admm_shortlist(int64_t m, int64_t n, int iters, int storage, double max_exchange, const double* coef, int k,
                   int* Qs, int* Ps, double* model_s, int* count, size_t* max_workspace) {
  g_last_error.clear();
  if (!Qs || !Ps || !count || k < 1) return fail(ADMM_EINVAL, "Qs, Ps, count must not be NULL and k >= 1");
  if (iters < 0) return fail(ADMM_EINVAL, "iters must be >= 0");
  if (coef && check_coef(coef)) return ADMM_EINVAL;
  std::vector<Priced> v;
  price_candidates(m, n, iters, storage, max_exchange, coef ? coef : kDefaultCoef, v);
  const int got = (int)std::min<size_t>(v.size(), (size_t)k);
  size_t ws = 0;
  for (int i = 0; i < got; ++i) {
    Qs[i] = v[i].Q;
    Ps[i] = v[i].P;
    if (model_s) model_s[i] = v[i].t;
    Geometry geo;
    std::string err;
    if (build_geometry(geo, m, n, v[i].Q, nullptr, v[i].P, nullptr, storage, err) == ADMM_OK)
      ws = std::max(ws, geo.lay.total);
  }
  *count = got;
  if (max_workspace) *max_workspace = ws;
  return got ? ADMM_OK : fail(ADMM_EUNSUPPORTED, "no candidate split meets the exchange limit");
}

int admm_calibrate(const void* H, const void* g, int64_t m, int64_t n, int storage, void* workspace,
                   size_t workspace_bytes, void* stream, double* coef) {
  g_last_error.clear();
  if (!H || !g || !coef || !workspace) return fail(ADMM_EINVAL, "H, g, workspace and coef must not be NULL");
  for (int k = 0; k < kCoefs; ++k) coef[k] = kDefaultCoef[k];
  // Probe splits: single-pass plans of moderate and of many blocks, a few
  // large blocks, and the two-pass kernels (the flag), so that work and
  // overhead vary independently across the probes.
  struct Probe {
    int Q, P, flags;
  };
  const Probe probes[] = {{4, 4, 0}, {16, 16, 0}, {2, 1, 0}, {32, 32, 0}, {20, 4, 0}, {4, 4, ADMM_TWO_PASS},
                          {8, 2, 0}};
  std::vector<double> Xs, Xi, ys, yi;
  for (const Probe& pr : probes) {
    const int Q = (int)std::min<int64_t>(pr.Q, m), P = (int)std::min<int64_t>(pr.P, n);
    double su = 0.0, it = 0.0;
    Geometry geo;
    const int rc = time_split(H, g, m, n, Q, P, storage | pr.flags, workspace, workspace_bytes, stream, 20, &su,
                              &it, &geo);
    if (rc == ADMM_EWORKSPACE) continue;   // does not fit the caller's memory: skipped
    if (rc) return rc;
    double c[16], fs[kSetupTerms], fi[kIterTerms];
    split_cost(geo, c);
    model_features(geo, c[1], c[2], fs, fi);
    Xs.insert(Xs.end(), fs, fs + kSetupTerms);
    Xi.insert(Xi.end(), fi, fi + kIterTerms);
    ys.push_back(su);
    yi.push_back(it);
  }
  if (ys.size() < 3) return fail(ADMM_EWORKSPACE, "the workspace holds fewer than three probe splits");
  // The built-in model's structure is kept (it was fitted to 338 measured
  // splits); the probes fit four scale factors of it: setup work (flops,
  // span, panel steps) and setup overhead (blocks, fixed), iteration bytes
  // (the three byte terms) and iteration overhead (blocks, fixed).
  const size_t rows = ys.size();
  std::vector<double> Xs2(rows * 2), Xi2(rows * 2);
  for (size_t r = 0; r < rows; ++r) {
    const double* fs = &Xs[r * kSetupTerms];
    const double* fi = &Xi[r * kIterTerms];
    const double* d = kDefaultCoef;
    Xs2[r * 2] = d[0] * fs[0] + d[1] * fs[1] + d[2] * fs[2];
    Xs2[r * 2 + 1] = d[3] * fs[3] + d[4] * fs[4];
    Xi2[r * 2] = d[5] * fi[0] + d[6] * fi[1] + d[7] * fi[2];
    Xi2[r * 2 + 1] = d[8] * fi[3] + d[9] * fi[4];
  }
  double ss[2] = {1.0, 1.0}, si[2] = {1.0, 1.0};
  nnls_small(Xs2, 2, ys, {0, 1}, ss);
  nnls_small(Xi2, 2, yi, {0, 1}, si);
  const double scale[kCoefs] = {ss[0], ss[0], ss[0], ss[1], ss[1], si[0], si[0], si[0], si[1], si[1]};
  for (int k = 0; k < kCoefs; ++k) coef[k] = kDefaultCoef[k] * scale[k];
  return ADMM_OK;
}

int admm_choose_split_measure(const void* H, const void* g, int64_t m, int64_t n, int iters, int storage,
                              double max_exchange, const double* coef, int shortlist, void* workspace,
                              size_t workspace_bytes, void* stream, int* Q_out, int* P_out, double* measured_s) {
  g_last_error.clear();
  if (!H || !g || !Q_out || !P_out || !workspace) return fail(ADMM_EINVAL, "H, g, workspace, Q_out and P_out must not be NULL");
  if (iters < 0 || shortlist < 1) return fail(ADMM_EINVAL, "iters >= 0 and shortlist >= 1 required");
  if (coef && check_coef(coef)) return ADMM_EINVAL;
  std::vector<Priced> v;
  price_candidates(m, n, iters, storage, max_exchange, coef ? coef : kDefaultCoef, v);
  if (v.empty()) return fail(ADMM_EUNSUPPORTED, "no candidate split meets the exchange limit");
  double best = HUGE_VAL;
  int bq = 0, bp = 0, timed_n = 0;
  for (const Priced& c : v) {
    if (timed_n == shortlist) break;
    double su = 0.0, it = 0.0;
    const int rc = time_split(H, g, m, n, c.Q, c.P, storage, workspace, workspace_bytes, stream, 20, &su, &it,
                              nullptr);
    if (rc == ADMM_EWORKSPACE) continue;
    if (rc) return rc;
    ++timed_n;
    const double t = su + iters * it;
    if (t < best) best = t, bq = c.Q, bp = c.P;
  }
  if (!bq) return fail(ADMM_EWORKSPACE, "no shortlisted split fits the workspace");
  *Q_out = bq;
  *P_out = bp;
  if (measured_s) *measured_s = best;
  return ADMM_OK;
}

int admm_setup(admm_plan** out, const void* H, int64_t m, int64_t n, int Q, const int64_t* row_off, int P,
               const int64_t* col_off, double rho, double lambda, int storage, void* workspace,
               size_t workspace_bytes, void* stream) {
  g_last_error.clear();
  if (!out) return fail(ADMM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!H) return fail(ADMM_EINVAL, "H is NULL");
  if (!(rho > 0.0) || !std::isfinite(rho)) return fail(ADMM_EINVAL, "rho must be finite and > 0");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(ADMM_EINVAL, "lambda must be finite and >= 0");
  admm_plan* p = new admm_plan;
  std::string err;
  int rc = build_geometry(p->geo, m, n, Q, row_off, P, col_off, storage, err);
  if (rc) {
    delete p;
    return fail(rc, "%s", err.c_str());
  }
  storage = p->geo.storage;   // H format (the inverse flag is in geo.inv16)
  const Layout& L = p->geo.lay;
  if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
    delete p;
    return fail(ADMM_EWORKSPACE, "workspace needs %zu bytes at 256-byte alignment (got %zu at %p)", L.total,
                workspace_bytes, workspace);
  }
  p->rho = rho;
  p->lam = lambda;
  p->ws = static_cast<char*>(workspace);
  p->ws_bytes = workspace_bytes;
  p->H = at<float2>(p, L.H);
  p->Ginv = at<float2>(p, L.Ginv);
  p->Ginv16 = p->geo.inv16 ? at<uint32_t>(p, L.Ginv16) : nullptr;
  p->F64a = at<double2>(p, L.F64a);
  p->F64b = at<double2>(p, L.F64b);
  p->c = at<float2>(p, L.c);
  p->s = at<float2>(p, L.s);
  p->v = at<float2>(p, L.v);
  p->part = at<float2>(p, L.part);
  p->gp = at<float2>(p, L.gp);
  p->ghat = at<float2>(p, L.ghat);
  p->r = at<float2>(p, L.r);
  p->y = at<float2>(p, L.y);
  p->d_blocks = at<BlockDesc>(p, L.blocks);
  p->d_cols = at<ColDesc>(p, L.cols);
  p->t_rows = at<int4>(p, L.t_rows);
  p->t_cols = at<int4>(p, L.t_cols);
  p->t_z = at<int4>(p, L.t_z);
  p->t_gram = at<int4>(p, L.t_gram);
  p->t_kadj = at<int4>(p, L.t_kadj);
  p->t_hrows = at<int4>(p, L.t_hrows);
  p->t_wrows = at<int4>(p, L.t_wrows);
  p->t_gpatch = at<int4>(p, L.t_gpatch);
  p->t_gtr = at<int4>(p, L.t_gtr);
  p->gpart = at<float2>(p, L.gpart);
  p->hs.storage = storage;
  p->hs.base = p->ws + L.H;
  p->hs.base_im = storage == ADMM_STORAGE_C64 ? nullptr : p->ws + L.H_im;
  p->hs.row_scale = storage == ADMM_STORAGE_FP8 ? at<float>(p, L.H_scale) : nullptr;
  p->ctl = at<Control>(p, L.ctl);
  p->redpart = at<double>(p, L.redpart);
  p->row_block = at<int64_t>(p, L.row_block);
  p->kkt_e = at<double2>(p, L.kkt_e);
  p->kkt_v = at<float2>(p, L.kkt_v);
  p->kkt_part = at<double2>(p, L.kkt_part);
  p->kkt_max = at<double>(p, L.kkt_max);
  p->vb = at<float2>(p, L.vb);
  p->sb = at<float2>(p, L.sb);
  p->ub = at<float2>(p, L.ub);
  p->ghb = at<float2>(p, L.ghb);
  p->gpb = at<float2>(p, L.gpb);
  p->yb = at<float2>(p, L.yb);
  p->rb = at<float2>(p, L.rb);
  p->gbar = at<double2>(p, L.gbar);
  p->kpart = at<double>(p, L.kpart);
  p->rpart = at<double>(p, L.rpart);
  p->t_fz = at<int4>(p, L.t_fz);
  p->t_fzr = at<int4>(p, L.t_fzr);
  p->fz_colwg = at<int2>(p, L.fz_colwg);
  p->t_dgp = at<int4>(p, L.t_dgp);
  p->dflag = at<int>(p, L.dflag);
  p->fz = p->geo.fzt;
  p->fz.hsl = HStore{p->ws + L.Hs, nullptr, nullptr, ADMM_STORAGE_C64};
  p->fz.fpart = at<float2>(p, L.fpart);
  p->fz.work = p->t_fz;
  p->fz.colwg = p->fz_colwg;
  p->fz.mode = 0;
  {
    static std::atomic<uint64_t> next_serial{1};
    p->serial = next_serial++;
  }
  p->h_row_block.resize(m);
  for (int i = 0; i < Q; ++i)
    for (int64_t r = p->geo.ro[i]; r < p->geo.ro[i + 1]; ++r) p->h_row_block[r] = i;

  hipStream_t st = static_cast<hipStream_t>(stream);
  auto cleanup_fail = [&](int code) {
    delete p;
    return code;
  };
#define SETUP_TRY(expr)                                                                        \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return cleanup_fail(fail(ADMM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)));     \
  } while (0)
  // zero everything the kernels rely on being zero (stores with pads, state, control)
  SETUP_TRY(launch_fill(p->ws + L.H, L.Ginv - L.H, st));
  SETUP_TRY(launch_fill(p->ws + L.Ginv, L.ginv_bytes, st));
  SETUP_TRY(launch_fill(p->ws + L.c, L.total - L.c, st));
  const Geometry& G = p->geo;
  SETUP_TRY(hipMemcpyAsync(p->d_blocks, G.blocks.data(), sizeof(BlockDesc) * G.blocks.size(),
                           hipMemcpyHostToDevice, st));
  SETUP_TRY(hipMemcpyAsync(p->d_cols, G.cols.data(), sizeof(ColDesc) * G.cols.size(), hipMemcpyHostToDevice, st));
  SETUP_TRY(hipMemcpyAsync(p->t_rows, G.t_rows.data(), 16 * G.t_rows.size(), hipMemcpyHostToDevice, st));
  SETUP_TRY(hipMemcpyAsync(p->t_cols, G.t_cols.data(), 16 * G.t_cols.size(), hipMemcpyHostToDevice, st));
  SETUP_TRY(hipMemcpyAsync(p->t_z, G.t_z.data(), 16 * G.t_z.size(), hipMemcpyHostToDevice, st));
  SETUP_TRY(hipMemcpyAsync(p->t_gram, G.t_gram.data(), 16 * G.t_gram.size(), hipMemcpyHostToDevice, st));
  SETUP_TRY(hipMemcpyAsync(p->t_kadj, G.t_kadj.data(), 16 * G.t_kadj.size(), hipMemcpyHostToDevice, st));
  SETUP_TRY(hipMemcpyAsync(p->t_hrows, G.t_hrows.data(), 16 * G.t_hrows.size(), hipMemcpyHostToDevice, st));
  if (!G.t_wrows.empty())
    SETUP_TRY(hipMemcpyAsync(p->t_wrows, G.t_wrows.data(), 16 * G.t_wrows.size(), hipMemcpyHostToDevice, st));
  if (!G.t_gpatch.empty())
    SETUP_TRY(hipMemcpyAsync(p->t_gpatch, G.t_gpatch.data(), 16 * G.t_gpatch.size(), hipMemcpyHostToDevice, st));
  SETUP_TRY(hipMemcpyAsync(p->t_gtr, G.t_gtr.data(), 16 * G.t_gtr.size(), hipMemcpyHostToDevice, st));
  if (G.fz) {
    SETUP_TRY(hipMemcpyAsync(p->t_fz, G.t_fz.data(), 16 * G.t_fz.size(), hipMemcpyHostToDevice, st));
    SETUP_TRY(hipMemcpyAsync(p->fz_colwg, G.fz_colwg.data(), 8 * G.fz_colwg.size(), hipMemcpyHostToDevice, st));
    SETUP_TRY(hipMemcpyAsync(p->t_fzr, G.t_fzr.data(), 16 * G.t_fzr.size(), hipMemcpyHostToDevice, st));
  }
  if (G.direct)
    SETUP_TRY(hipMemcpyAsync(p->t_dgp, G.t_dgp.data(), 16 * G.t_dgp.size(), hipMemcpyHostToDevice, st));
  SETUP_TRY(hipMemcpyAsync(p->row_block, p->h_row_block.data(), 8 * (size_t)m, hipMemcpyHostToDevice, st));
  int max_mi = 0;
  for (auto& d : G.blocks) max_mi = std::max(max_mi, d.mi);
  if (storage == ADMM_STORAGE_C64)
    SETUP_TRY(launch_pack_c64(static_cast<const float2*>(H), n, p->d_blocks, (int)G.blocks.size(), max_mi, p->H,
                              p->ctl, st));
  else
    SETUP_TRY(launch_pack_quant(static_cast<const float2*>(H), m, n, p->d_blocks, (int)G.blocks.size(), max_mi,
                                p->hs, p->ctl, st));
  if (G.fz) SETUP_TRY(launch_pack_slabs(p->hs, p->fz.hsl, p->d_blocks, G.Q, G.P, G.m_pad, p->fz, st));
  SETUP_TRY(launch_gram_build(G, p->d_blocks, p->t_gram, p->hs, rho, p->F64a, st));
  SETUP_TRY(launch_cholesky_inverse(G, p->d_blocks, p->t_gram, p->F64a, p->F64b, p->Ginv, p->ctl, st));
  if (p->Ginv16) SETUP_TRY(launch_to_bf16_pairs(p->Ginv, p->Ginv16, L.ginv_bytes / 8, st));
  Control hc;
  SETUP_TRY(hipMemcpyAsync(&hc, p->ctl, sizeof hc, hipMemcpyDeviceToHost, st));
  SETUP_TRY(hipStreamSynchronize(st));
#undef SETUP_TRY
  if (hc.nonfinite) return cleanup_fail(fail(ADMM_ENONFINITE, "H holds NaN or Inf"));
  if (hc.notpd) return cleanup_fail(fail(ADMM_ENOTPD, "a Gram matrix pivot was not positive"));
  *out = p;
  return ADMM_OK;
}

int admm_set_lambda(admm_plan* p, double lambda) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(ADMM_EINVAL, "lambda must be finite and >= 0");
  p->lam = lambda;
  return ADMM_OK;
}

namespace {

// The launches of one iteration on stream st (kernel events when profiling
// samples iteration k).
int launch_iteration(admm_plan* p, const IterArgs& a, const FzArgs& z, int k, hipStream_t st) {
  const Geometry& G = p->geo;
  int rc;
  const int ngr = (int)G.t_gram.size(), ngt = (int)G.t_gtr.size();
  auto gram = [&](KTime kt) {
    return launch_gram(a, p->t_gram, ngr, p->t_gpatch, (int)G.t_gpatch.size(), p->t_gtr, ngt, st, kt);
  };
  if (G.direct) {
    // Direct form (Sec. III-B) as a correction of the previous u (k_iter.hip):
    // the row residuals (or g') of every block from the estimates, their
    // adjoint product (row-chunk partials), d = H^H r + rho (c - u_ref), the
    // pieces of A^{-1} d, the z- and dual update on u = u_ref + A^{-1} d
    // (which also stores u), and the estimated data ghat = H u.
    IterArgs ah = a, af = a;
    ah.y = a.gp;   // the adjoint product reads g'
    af.c = a.y;    // the row product reads u
    const int nz = (int)G.t_z.size();
    const int src = (!a.Ginv16 && !G.t_gpatch.empty()) ? 1 : 2;
    auto gram_apply = [&](KTime kt) {
      return launch_gram(a, p->t_gram, ngr, p->t_gpatch, (int)G.t_gpatch.size(), p->t_gtr, ngt, st, kt, false);
    };
    if ((rc = timed(p, ADMM_K_DIRECT_GP, k, st, [&](KTime kt) { return launch_direct_gp(a, p->t_dgp, (int)G.t_dgp.size(), st, kt); }))) return rc;
    if ((rc = timed(p, ADMM_K_GEMV_H, k, st, [&](KTime kt) { return launch_gemv_h(ah, p->t_cols, (int)G.t_cols.size(), st, kt); }))) return rc;
    if ((rc = timed(p, ADMM_K_DIRECT_RHS, k, st, [&](KTime kt) { return launch_direct_rhs(a, p->t_z, nz, st, kt); }))) return rc;
    if ((rc = timed(p, ADMM_K_GRAM, k, st, gram_apply))) return rc;
    if ((rc = timed(p, ADMM_K_ZUPDATE, k, st, [&](KTime kt) { return launch_zupdate(a, p->t_z, nz, st, kt, src); }))) return rc;
    if ((rc = timed(p, ADMM_K_GEMV_N, k, st, [&](KTime kt) { return launch_gemv_n(af, p->t_hrows, (int)G.t_hrows.size(), p->t_wrows, (int)G.t_wrows.size(), st, kt); }))) return rc;
  } else if (G.fz) {
    if ((rc = timed(p, ADMM_K_FZ_ROWS, k, st, [&](KTime kt) { return launch_fz_rows(a, z, p->t_fzr, (int)G.t_fzr.size(), st, kt); }))) return rc;
    if ((rc = timed(p, ADMM_K_GRAM, k, st, gram))) return rc;
    if ((rc = timed(p, ADMM_K_FZ_SLAB, k, st, [&](KTime kt) { return launch_fz_slab(a, z, G.fz_nt, G.fz_rpl, st, kt); }))) return rc;
  } else {
    if ((rc = timed(p, ADMM_K_GEMV_N, k, st, [&](KTime kt) { return launch_gemv_n(a, p->t_hrows, (int)G.t_hrows.size(), p->t_wrows, (int)G.t_wrows.size(), st, kt); }))) return rc;
    if ((rc = timed(p, ADMM_K_GRAM, k, st, gram))) return rc;
    if ((rc = timed(p, ADMM_K_GEMV_H, k, st, [&](KTime kt) { return launch_gemv_h(a, p->t_cols, (int)G.t_cols.size(), st, kt); }))) return rc;
    if ((rc = timed(p, ADMM_K_ZUPDATE, k, st, [&](KTime kt) { return launch_zupdate(a, p->t_z, (int)G.t_z.size(), st, kt); }))) return rc;
  }
  return ADMM_OK;
}

// A graph of `chunk` iterations for these arguments (captured again when g,
// the residual history, kappa or the chunk change).
constexpr int kGraphChunk = 10;
int ensure_graph(admm_plan* p, const IterArgs& a, const FzArgs& z, int chunk) {
  if (p->gexec && p->gkey_g == a.g && p->gkey_hist == a.hist && p->gkey_kappa == a.kappa && p->gkey_chunk == chunk)
    return ADMM_OK;
  if (!p->gs) {
    HIP_TRY(hipStreamCreateWithFlags(&p->gs, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&p->gin, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&p->gout, hipEventDisableTiming));
  }
  if (p->gexec) {
    HIP_TRY(hipGraphExecDestroy(p->gexec));
    p->gexec = nullptr;
  }
  HIP_TRY(hipStreamBeginCapture(p->gs, hipStreamCaptureModeThreadLocal));
  int rc = ADMM_OK;
  for (int c = 0; c < chunk && rc == ADMM_OK; ++c) rc = launch_iteration(p, a, z, c, p->gs);
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(p->gs, &gr);
  if (rc) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc;
  }
  if (e != hipSuccess) return fail(ADMM_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(&p->gexec, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e2 != hipSuccess) {
    p->gexec = nullptr;
    return fail(ADMM_EHIP, "graph instantiation failed: %s", hipGetErrorString(e2));
  }
  p->gkey_g = a.g;
  p->gkey_hist = a.hist;
  p->gkey_kappa = a.kappa;
  p->gkey_chunk = chunk;
  return ADMM_OK;
}

}  // namespace

int admm_solve(admm_plan* p, const void* g, int iters, double tol, int check_every, void* v_out, int* iters_done,
               double* resid_hist, int warm, void* stream) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  if (!g || !v_out) return fail(ADMM_EINVAL, "g and v_out must not be NULL");
  if (iters < 0) return fail(ADMM_EINVAL, "iters must be >= 0");
  if (std::isnan(tol)) return fail(ADMM_EINVAL, "tol is NaN");
  if (tol > 0 && check_every < 1) return fail(ADMM_EINVAL, "check_every must be >= 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Geometry& G = p->geo;
  int rc;
  if (!warm && (rc = reset_state(p, st))) return rc;
  HIP_TRY(launch_fill(p->ctl, 16, st));  // iteration counter, pending z-sums flag, error flags
  IterArgs a = iter_args(p, static_cast<const float2*>(g), resid_hist);
  FzArgs z = p->fz;
  if (G.fz) {
    a.nz = (int)G.t_fz.size();   // residual partials: one per slab-pass workgroup
    if (!p->fz_valid && iters > 0) {
      // the workspace's parts of H c belong to another c (state import,
      // recorded solve): one forward-only slab pass
      z.mode = 1;
      HIP_TRY(launch_fz_slab(a, z, G.fz_nt, G.fz_rpl, st));
      z.mode = 0;
      p->fz_valid = true;
    }
  }
  // Runs of `chunk` iterations (check_every with a tolerance) replay one
  // captured graph when graphs are on and no kernel timing is sampled.
  const int chunk = tol > 0 ? check_every : kGraphChunk;
  const bool use_graph = p->graphs && !p->prof && iters >= chunk;
  hipStream_t ws = st;
  if (use_graph) {
    if ((rc = ensure_graph(p, a, z, chunk))) return rc;
    HIP_TRY(hipEventRecord(p->gin, st));
    HIP_TRY(hipStreamWaitEvent(p->gs, p->gin, 0));
    ws = p->gs;
  }
  int done = 0;
  while (done < iters) {
    if (use_graph && iters - done >= chunk) {
      HIP_TRY(hipGraphLaunch(p->gexec, ws));
      done += chunk;
    } else {
      if ((rc = launch_iteration(p, a, z, done, ws))) return rc;
      ++done;
    }
    if (tol > 0 && done % check_every == 0) {
      HIP_TRY(launch_zfinal(a, ws));
      Control hc;
      HIP_TRY(hipMemcpyAsync(&hc, p->ctl, sizeof hc, hipMemcpyDeviceToHost, ws));
      HIP_TRY(hipStreamSynchronize(ws));
      if (hc.nonfinite) break;
      const double Q = G.Q;
      const double rp = std::sqrt(hc.red[kRedRp2]), rd = p->rho * std::sqrt(Q * hc.red[kRedDv2]);
      const double pri = tol * std::max(std::sqrt(hc.red[kRedU2]), std::sqrt(Q * hc.red[kRedV2]));
      const double dua = tol * p->rho * std::sqrt(hc.red[kRedS2]);
      if (rp <= pri && rd <= dua) break;
    }
  }
  if (use_graph) {
    HIP_TRY(hipEventRecord(p->gout, p->gs));
    HIP_TRY(hipStreamWaitEvent(st, p->gout, 0));
  }
  p->k_done += done;
  HIP_TRY(launch_zfinal(a, st));
  HIP_TRY(launch_unpad_cols(p->d_cols, G.P, G.n, p->v, static_cast<float2*>(v_out), 0, 0, 1, 0, st));
  Control hc;
  HIP_TRY(hipMemcpyAsync(&hc, p->ctl, sizeof hc, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (iters_done) *iters_done = done;
  if (hc.nonfinite) return fail(ADMM_ENONFINITE, "a NaN or Inf reached the iterates (check g and rho)");
  return ADMM_OK;
}

int admm_set_graphs(admm_plan* p, int enable) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  p->graphs = enable != 0;
  return ADMM_OK;
}

int admm_tape_bytes(const admm_plan* p, int iters, int interval, size_t* out_bytes) {
  g_last_error.clear();
  if (!p || !out_bytes) return fail(ADMM_EINVAL, "plan and out_bytes must not be NULL");
  if (iters < 1 || interval < 1) return fail(ADMM_EINVAL, "iters and interval must be >= 1");
  *out_bytes = tape_layout(p->geo, iters, interval).total;
  return ADMM_OK;
}

int admm_solve_record(admm_plan* p, const void* g, int iters, int interval, void* tape, size_t tape_bytes,
                      void* v_out, void* stream) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  if (!g || !v_out || !tape) return fail(ADMM_EINVAL, "g, v_out and tape must not be NULL");
  if (iters < 1 || interval < 1) return fail(ADMM_EINVAL, "iters and interval must be >= 1");
  if (p->geo.direct) return fail(ADMM_EUNSUPPORTED, "the reverse sweep is built for the inversion-lemma form only");
  const Geometry& G = p->geo;
  const TapeLayout T = tape_layout(G, iters, interval);
  if (tape_bytes < T.total || (reinterpret_cast<uintptr_t>(tape) & 255))
    return fail(ADMM_EWORKSPACE, "tape needs %zu bytes at 256-byte alignment", T.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* tp = static_cast<char*>(tape);
  int rc;
  if ((rc = reset_state(p, st))) return rc;
  p->fz_valid = false;   // the two-pass kernels below move c
  HIP_TRY(launch_fill(p->ctl, 16, st));
  const IterArgs a = iter_args(p, static_cast<const float2*>(g), nullptr);
  const int nr = (int)G.t_rows.size(), nc = (int)G.t_cols.size(), nz = (int)G.t_z.size();
  const int nh = (int)G.t_hrows.size();
  const int ngr = (int)G.t_gram.size(), ngt = (int)G.t_gtr.size();
  const size_t colv = (size_t)G.n_pad * 8, rowv = (size_t)G.m_pad * 8;
  for (int k = 0; k < iters; ++k) {
    if (k % interval == 0) {
      char* ck = tp + T.ckpt + T.ckpt_stride * (k / interval);
      HIP_TRY(hipMemcpyAsync(ck + T.v, p->v, colv, hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(ck + T.s, p->s, colv * G.Q, hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(ck + T.ghat, p->ghat, rowv * G.P, hipMemcpyDeviceToDevice, st));
    }
    if ((rc = timed(p, ADMM_K_GEMV_N, k, st, [&](KTime kt) { return launch_gemv_n(a, p->t_hrows, nh, p->t_wrows, (int)G.t_wrows.size(), st, kt); }))) return rc;
    if ((rc = timed(p, ADMM_K_GRAM, k, st, [&](KTime kt) { return launch_gram(a, p->t_gram, ngr, p->t_gpatch, (int)G.t_gpatch.size(), p->t_gtr, ngt, st, kt); }))) return rc;
    if ((rc = timed(p, ADMM_K_GEMV_H, k, st, [&](KTime kt) { return launch_gemv_h(a, p->t_cols, nc, st, kt); }))) return rc;
    if ((rc = timed(p, ADMM_K_ZUPDATE, k, st, [&](KTime kt) { return launch_zupdate(a, p->t_z, nz, st, kt); }))) return rc;
  }
  HIP_TRY(launch_zfinal(a, st));
  p->k_done = iters;
  TapeHeader h{};
  h.magic = kTapeMagic;
  h.version = 1;
  h.iters = iters;
  h.interval = interval;
  h.nseg = (iters + interval - 1) / interval;
  h.Q = G.Q;
  h.P = G.P;
  h.m_pad = G.m_pad;
  h.n_pad = G.n_pad;
  h.lam = p->lam;
  h.rho = p->rho;
  h.serial = p->serial;
  HIP_TRY(hipMemcpyAsync(tp, &h, sizeof h, hipMemcpyHostToDevice, st));
  HIP_TRY(launch_unpad_cols(p->d_cols, G.P, G.n, p->v, static_cast<float2*>(v_out), 0, 0, 1, 0, st));
  Control hc;
  HIP_TRY(hipMemcpyAsync(&hc, p->ctl, sizeof hc, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hc.nonfinite) return fail(ADMM_ENONFINITE, "a NaN or Inf reached the iterates");
  return ADMM_OK;
}

int admm_backward(admm_plan* p, const void* g, const void* grad_v, void* tape, void* grad_g,
                  double* grad_lambda, double* grad_rho, void* stream) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  if (!g || !grad_v || !tape || !grad_g || !grad_lambda || !grad_rho)
    return fail(ADMM_EINVAL, "g, grad_v, tape, grad_g, grad_lambda and grad_rho must not be NULL");
  if (p->geo.direct) return fail(ADMM_EUNSUPPORTED, "the reverse sweep is built for the inversion-lemma form only");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Geometry& G = p->geo;
  char* tp = static_cast<char*>(tape);
  TapeHeader h{};
  HIP_TRY(hipMemcpyAsync(&h, tp, sizeof h, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h.magic != kTapeMagic || h.serial != p->serial)
    return fail(ADMM_ESTATE, "the tape was not recorded by this plan (admm_solve_record first)");
  if (h.lam != p->lam || h.rho != p->rho) return fail(ADMM_ESTATE, "lambda changed since the tape was recorded");
  const int K = h.iters, C = h.interval;
  const TapeLayout T = tape_layout(G, K, C);
  const size_t colv = (size_t)G.n_pad * 8, rowv = (size_t)G.m_pad * 8;
  p->fz_valid = false;   // the recomputed forward moves c
  // adjoint state: vb = grad_v, everything else zero
  HIP_TRY(launch_fill(p->ws + G.lay.vb, G.lay.total - G.lay.vb, st));
  HIP_TRY(launch_fill(&p->ctl->kbar, 16, st));
  HIP_TRY(launch_unpad_cols(p->d_cols, G.P, G.n, static_cast<const float2*>(grad_v), p->vb, 0, 0, 1, 1, st));
  HIP_TRY(launch_fill(p->ctl, 16, st));
  IterArgs a = iter_args(p, static_cast<const float2*>(g), nullptr);
  AdjArgs b{};
  b.blocks = p->d_blocks;
  b.cols = p->d_cols;
  b.hs = p->hs;
  b.Ginv = p->Ginv;
  b.Ginv16 = p->Ginv16;
  b.vb = p->vb;
  b.sb = p->sb;
  b.ub = p->ub;
  b.ghb = p->ghb;
  b.gpb = p->gpb;
  b.yb = p->yb;
  b.rb = p->rb;
  b.part = p->part;
  b.gpart = p->gpart;
  b.gbar = p->gbar;
  b.kpart = p->kpart;
  b.rpart = p->rpart;
  b.ctl = p->ctl;
  b.m_pad = G.m_pad;
  b.n_pad = G.n_pad;
  b.Q = G.Q;
  b.P = G.P;
  b.KH = G.KH;
  b.rho = (float)p->rho;
  b.kappa = a.kappa;
  b.cpl = a.cpl;
  const int nr = (int)G.t_rows.size(), nc = (int)G.t_cols.size(), nz = (int)G.t_z.size();
  const int nh = (int)G.t_hrows.size();
  const int ngr = (int)G.t_gram.size(), ngt = (int)G.t_gtr.size();
  float2* yrec = reinterpret_cast<float2*>(tp + T.yrec);
  float2* arec = reinterpret_cast<float2*>(tp + T.arec);
  const size_t ystride = align256(rowv * G.P) / 8, astride = align256(colv) / 8;
  for (int seg = h.nseg - 1; seg >= 0; --seg) {
    const int k0 = seg * C, k1 = std::min(K, k0 + C);
    const char* ck = tp + T.ckpt + T.ckpt_stride * seg;
    HIP_TRY(hipMemcpyAsync(p->v, ck + T.v, colv, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(p->s, ck + T.s, colv * G.Q, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(p->ghat, ck + T.ghat, rowv * G.P, hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_make_c(p->d_cols, G.P, G.Q, G.n_pad, cols_per_load(G.storage), p->v, p->s, p->c, st));
    for (int k = k0; k < k1; ++k) {
      a.y = yrec + ystride * (k - k0);
      a.arec = arec + astride * (k - k0);
      HIP_TRY(launch_gemv_n(a, p->t_hrows, nh, p->t_wrows, (int)G.t_wrows.size(), st));
      HIP_TRY(launch_gram(a, p->t_gram, ngr, p->t_gpatch, (int)G.t_gpatch.size(), p->t_gtr, ngt, st));
      HIP_TRY(launch_gemv_h(a, p->t_cols, nc, st));
      HIP_TRY(launch_zupdate(a, p->t_z, nz, st));
    }
    for (int k = k1 - 1; k >= k0; --k)
      HIP_TRY(launch_adj_iteration(b, G, p->t_hrows, p->t_gram, p->t_gtr, p->t_cols, p->t_z, arec + astride * (k - k0),
                                   yrec + ystride * (k - k0), st));
  }
  HIP_TRY(launch_adj_gflush(b, p->d_blocks, (int)G.blocks.size(), static_cast<float2*>(grad_g), st));
  HIP_TRY(launch_adj_scalars(b, (int)G.t_z.size(), (int)G.t_gtr.size(), st));
  Control hc;
  HIP_TRY(hipMemcpyAsync(&hc, p->ctl, sizeof hc, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const double Q = G.Q;
  *grad_lambda = hc.kbar / (Q * p->rho);
  *grad_rho = hc.rbar - hc.kbar * p->lam / (Q * p->rho * p->rho);
  p->k_done = std::min(K, C);   // the state the last recomputed interval ends in
  if (hc.nonfinite) return fail(ADMM_ENONFINITE, "a NaN or Inf reached the recomputed iterates");
  return ADMM_OK;
}

int admm_get_state(admm_plan* p, void* v, void* s, void* ghat, int* k, void* stream) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Geometry& G = p->geo;
  if (v) HIP_TRY(launch_unpad_cols(p->d_cols, G.P, G.n, p->v, static_cast<float2*>(v), 0, 0, 1, 0, st));
  if (s)
    HIP_TRY(launch_unpad_cols(p->d_cols, G.P, G.n, p->s, static_cast<float2*>(s), G.n_pad, G.n, G.Q, 0, st));
  if (ghat)
    HIP_TRY(launch_unpad_rows(p->d_blocks, (int)G.blocks.size(), G.m, G.m_pad, p->ghat, static_cast<float2*>(ghat),
                              0, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (k) *k = p->k_done;
  return ADMM_OK;
}

int admm_set_state(admm_plan* p, const void* v, const void* s, const void* ghat, int k, void* stream) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  if (!v || !s || !ghat) return fail(ADMM_EINVAL, "v, s and ghat must not be NULL");
  if (k < 0) return fail(ADMM_EINVAL, "k must be >= 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Geometry& G = p->geo;
  int rc;
  if ((rc = reset_state(p, st))) return rc;
  HIP_TRY(launch_unpad_cols(p->d_cols, G.P, G.n, static_cast<const float2*>(v), p->v, 0, 0, 1, 1, st));
  HIP_TRY(launch_unpad_cols(p->d_cols, G.P, G.n, static_cast<const float2*>(s), p->s, G.n, G.n_pad, G.Q, 1, st));
  HIP_TRY(launch_unpad_rows(p->d_blocks, (int)G.blocks.size(), G.m, G.m_pad, static_cast<const float2*>(ghat),
                            p->ghat, 1, st));
  HIP_TRY(launch_make_c(p->d_cols, G.P, G.Q, G.n_pad, cols_per_load(G.storage), p->v, p->s, p->c, st));
  HIP_TRY(hipStreamSynchronize(st));
  p->k_done = k;
  p->fz_valid = false;
  return ADMM_OK;
}

int admm_kkt(admm_plan* p, const void* g, const void* v, double* out, void* stream) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  if (!g || !v || !out) return fail(ADMM_EINVAL, "g, v and out must not be NULL");
  if (!(p->lam > 0.0)) return fail(ADMM_EINVAL, "the KKT check needs lambda > 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Geometry& G = p->geo;
  HIP_TRY(launch_unpad_cols(p->d_cols, G.P, G.n, static_cast<const float2*>(v), p->kkt_v, 0, 0, 1, 1, st));
  HIP_TRY(launch_kkt_all(p->d_blocks, p->d_cols, p->row_block, p->t_kadj, (int)G.t_kadj.size(), p->t_z,
                         (int)G.t_z.size(), G.m, G.n_pad, G.Q, G.P, G.KH, p->hs, static_cast<const float2*>(g),
                         p->kkt_v, p->lam, p->kkt_e, p->kkt_part, p->kkt_max, p->ctl, st));
  Control hc;
  HIP_TRY(hipMemcpyAsync(&hc, p->ctl, sizeof hc, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *out = hc.kkt / p->lam;
  return ADMM_OK;
}

int admm_kkt_noalloc(admm_plan* p, const void* g, const void* v, double* out, void* stream) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  if (!g || !v || !out) return fail(ADMM_EINVAL, "g, v and out must not be NULL");
  if (!(p->lam > 0.0)) return fail(ADMM_EINVAL, "the KKT check needs lambda > 0");
  const Geometry& G = p->geo;
  // the scratch admm_kkt takes from the plan's workspace: v in the padded
  // column space, the FP64 residual g - H v, the FP64 adjoint partials per
  // row chunk and replica, one maximum per final workgroup.  Every entry a
  // kernel reads was written earlier in the same call, so nothing is cleared.
  const size_t colv = (size_t)G.n_pad * 8;
  const size_t off_e = align256(colv);
  const size_t off_part = off_e + align256(16 * (size_t)G.m);
  const size_t off_max = off_part + align256(2 * colv * (size_t)G.Q * (size_t)G.KH);
  const size_t need = off_max + align256(8 * G.t_z.size());
  if (need > kStaticScratchBytes)
    return fail(ADMM_EWORKSPACE, "the KKT check of this plan needs %zu bytes of scratch; the static scratch holds %zu",
                need, kStaticScratchBytes);
  char* sb = nullptr;
  int rc = static_scratch(&sb);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float2* vpad = reinterpret_cast<float2*>(sb);
  HIP_TRY(launch_unpad_cols(p->d_cols, G.P, G.n, static_cast<const float2*>(v), vpad, 0, 0, 1, 1, st));
  HIP_TRY(launch_kkt_all(p->d_blocks, p->d_cols, p->row_block, p->t_kadj, (int)G.t_kadj.size(), p->t_z,
                         (int)G.t_z.size(), G.m, G.n_pad, G.Q, G.P, G.KH, p->hs, static_cast<const float2*>(g), vpad,
                         p->lam, reinterpret_cast<double2*>(sb + off_e), reinterpret_cast<double2*>(sb + off_part),
                         reinterpret_cast<double*>(sb + off_max), p->ctl, st));
  Control hc;
  HIP_TRY(hipMemcpyAsync(&hc, p->ctl, sizeof hc, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *out = hc.kkt / p->lam;
  return ADMM_OK;
}

int admm_hty_absmax(admm_plan* p, const void* g, double* out, void* stream) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  if (!g || !out) return fail(ADMM_EINVAL, "g and out must not be NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Geometry& G = p->geo;
  // the KKT pass with v = 0 and lambda = 0: its per-column value is |(H^H g)_n|
  HIP_TRY(launch_fill(p->kkt_v, (size_t)G.n_pad * sizeof(float2), st));
  HIP_TRY(launch_kkt_all(p->d_blocks, p->d_cols, p->row_block, p->t_kadj, (int)G.t_kadj.size(), p->t_z,
                         (int)G.t_z.size(), G.m, G.n_pad, G.Q, G.P, G.KH, p->hs, static_cast<const float2*>(g),
                         p->kkt_v, 0.0, p->kkt_e, p->kkt_part, p->kkt_max, p->ctl, st));
  Control hc;
  HIP_TRY(hipMemcpyAsync(&hc, p->ctl, sizeof hc, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *out = hc.kkt;
  return ADMM_OK;
}

int admm_get_stored_h(admm_plan* p, void* re_out, void* im_out, float* scale_out, void* stream) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  const Geometry& G = p->geo;
  if (!re_out || (G.storage != ADMM_STORAGE_C64 && !im_out) || (G.storage == ADMM_STORAGE_FP8 && !scale_out))
    return fail(ADMM_EINVAL, "output planes for this storage must not be NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int max_mi = 0;
  for (auto& d : G.blocks) max_mi = std::max(max_mi, d.mi);
  HIP_TRY(launch_export_h(p->hs, G.n, p->d_blocks, (int)G.blocks.size(), max_mi, re_out, im_out, st));
  if (G.storage == ADMM_STORAGE_FP8)
    HIP_TRY(hipMemcpyAsync(scale_out, p->hs.row_scale, 4 * (size_t)G.m, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return ADMM_OK;
}

int admm_profile(admm_plan* p, int enable) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  int rc = drain_profile(p);
  if (rc) return rc;
  for (int k = 0; k < ADMM_K_COUNT; ++k) {
    p->prof_ms[k] = 0;
    p->prof_n[k] = 0;
  }
  if (enable < 0) return fail(ADMM_EINVAL, "enable must be >= 0");
  p->prof = enable != 0;
  p->prof_every = enable > 0 ? enable : 1;
  // Create the events of 64 timed iterations now, so that a timed solve does
  // not create them between its launches.
  while (p->prof && p->pool.size() < (size_t)2 * ADMM_K_COUNT * 64) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    p->pool.push_back(e);
  }
  return ADMM_OK;
}

int admm_profile_read(admm_plan* p, int kernel, double* total_ms, int64_t* launches) {
  g_last_error.clear();
  if (!p) return fail(ADMM_EINVAL, "plan is NULL");
  if (kernel < 0 || kernel >= ADMM_K_COUNT) return fail(ADMM_EINVAL, "unknown kernel id %d", kernel);
  int rc = drain_profile(p);
  if (rc) return rc;
  if (total_ms) *total_ms = p->prof_ms[kernel];
  if (launches) *launches = p->prof_n[kernel];
  return ADMM_OK;
}

int admm_plan_info(const admm_plan* p, int64_t* info) {
  g_last_error.clear();
  if (!p || !info) return fail(ADMM_EINVAL, "plan and info must not be NULL");
  const Geometry& G = p->geo;
  int64_t v[16] = {G.m, G.n, G.Q, G.P, G.storage, G.KH, (int64_t)G.lay.total, (int64_t)G.lay.h_bytes,
                   (int64_t)G.lay.ginv_bytes, p->k_done, G.m_pad, G.n_pad, (int64_t)G.t_gpatch.size(),
                   G.fz ? 1 : 0, (int64_t)G.t_fz.size(), G.direct ? 1 : 0};
  std::memcpy(info, v, sizeof v);
  return ADMM_OK;
}

void admm_destroy(admm_plan* p) {
  if (!p) return;
  drain_profile(p);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->gin) (void)hipEventDestroy(p->gin);
  if (p->gout) (void)hipEventDestroy(p->gout);
  if (p->gs) (void)hipStreamDestroy(p->gs);
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  delete p;
}

}  // extern "C"
