// Views of the stored H for the device kernels, one per storage format.
//
//   FmtC64  complex64, interleaved (re, im)                      8 B / element
//   FmtBF16 bfloat16 real plane + imaginary plane                4 B / element
//   FmtFP8  OCP fp8 e4m3 real + imaginary planes, fp32 row scale 2 B / element
//
// Every block keeps the same element offsets in every plane.  A "lane load"
// reads 16 bytes of each plane: CPL consecutive complex columns.  Row scales
// (FP8) multiply whole rows, so kernels fold them into the vector operands:
//   (diag(s) Hq) c = s o (Hq c),   (diag(s) Hq)^H y = Hq^H (s o y).
#pragma once

#include "common.h"

namespace admm {

typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef unsigned int v4u_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 ldnt4(const float4* p) {
  const v4f_t v = __builtin_nontemporal_load(reinterpret_cast<const v4f_t*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint4 ldnt4u(const void* p) {
  const v4u_t v = __builtin_nontemporal_load(reinterpret_cast<const v4u_t*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float bf16_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

// OCP e4m3 (bias 7, no infinities, max 448) -> fp32 for a byte, exact.
__device__ __forceinline__ float e4m3_to_f32(unsigned b) {
  const unsigned s = (b & 0x80u) << 24;
  const unsigned e = (b >> 3) & 0xfu, m = b & 7u;
  float mag;
  if (e == 0)
    mag = (float)m * 0.001953125f;                                   // m * 2^-9
  else
    mag = __uint_as_float(((e + 120u) << 23) | (m << 20));           // (1+m/8) 2^(e-7)
  return __uint_as_float(__float_as_uint(mag) | s);
}

// Four packed e4m3 bytes -> four fp32 (hardware conversion; gfx950 reads OCP fp8).
__device__ __forceinline__ void e4m3x4_to_f32(unsigned w, float& a, float& b, float& c, float& d) {
  typedef float v2f_t __attribute__((ext_vector_type(2)));
  const v2f_t lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
  const v2f_t hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
  a = lo.x;
  b = lo.y;
  c = hi.x;
  d = hi.y;
}

// Each format: Raw = what one lane load returns (16 B per plane),
// load(e) reads columns e .. e+CPL-1 of a row (e a multiple of CPL),
// decode() turns it into CPL complex values (row scale not applied).
// row(e0) is the view of one row starting at element e0 (wave-uniform
// pointers, kept in scalar registers) and load(row, k) its k-th lane load:
// the 32-bit byte offset k * 16 lets every row share one vector offset.
__device__ __forceinline__ const char* lane_load_at(const char* rowp, uint32_t k) { return rowp + k * 16u; }
struct FmtC64 {
  static constexpr int CPL = 2;
  struct Raw { float4 a; };
  const float2* p;
  __device__ __forceinline__ Raw load(int64_t e) const { return Raw{ldnt4(reinterpret_cast<const float4*>(p + e))}; }
  struct Row { const char* p; };
  __device__ __forceinline__ Row row(int64_t e0) const { return Row{reinterpret_cast<const char*>(p + e0)}; }
  __device__ __forceinline__ static Raw load(const Row& r, uint32_t k) {
    return Raw{ldnt4(reinterpret_cast<const float4*>(lane_load_at(r.p, k)))};
  }
  __device__ __forceinline__ static void decode(const Raw& r, float (&re)[CPL], float (&im)[CPL]) {
    re[0] = r.a.x; im[0] = r.a.y; re[1] = r.a.z; im[1] = r.a.w;
  }
  __device__ __forceinline__ float row_scale(int) const { return 1.f; }
  // one element, dequantised (row scale included), in double
  __device__ __forceinline__ double2 getd(int64_t e, int) const {
    const float2 h = p[e];
    return make_double2(h.x, h.y);
  }
};

struct FmtBF16 {
  static constexpr int CPL = 8;
  struct Raw { uint4 a, b; };
  const uint16_t* re_p;
  const uint16_t* im_p;
  __device__ __forceinline__ Raw load(int64_t e) const { return Raw{ldnt4u(re_p + e), ldnt4u(im_p + e)}; }
  struct Row { const char* re; const char* im; };
  __device__ __forceinline__ Row row(int64_t e0) const {
    return Row{reinterpret_cast<const char*>(re_p + e0), reinterpret_cast<const char*>(im_p + e0)};
  }
  __device__ __forceinline__ static Raw load(const Row& r, uint32_t k) {
    return Raw{ldnt4u(lane_load_at(r.re, k)), ldnt4u(lane_load_at(r.im, k))};
  }
  __device__ __forceinline__ static void decode(const Raw& r, float (&re)[CPL], float (&im)[CPL]) {
    const unsigned aw[4] = {r.a.x, r.a.y, r.a.z, r.a.w}, bw[4] = {r.b.x, r.b.y, r.b.z, r.b.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      re[2 * q] = bf16_lo(aw[q]);
      re[2 * q + 1] = bf16_hi(aw[q]);
      im[2 * q] = bf16_lo(bw[q]);
      im[2 * q + 1] = bf16_hi(bw[q]);
    }
  }
  __device__ __forceinline__ float row_scale(int) const { return 1.f; }
  __device__ __forceinline__ double2 getd(int64_t e, int) const {
    return make_double2(__uint_as_float((unsigned)re_p[e] << 16), __uint_as_float((unsigned)im_p[e] << 16));
  }
};

struct FmtFP8 {
  static constexpr int CPL = 16;
  struct Raw { uint4 a, b; };
  const uint8_t* re_p;
  const uint8_t* im_p;
  const float* scale;   // per global row
  __device__ __forceinline__ Raw load(int64_t e) const { return Raw{ldnt4u(re_p + e), ldnt4u(im_p + e)}; }
  struct Row { const char* re; const char* im; };
  __device__ __forceinline__ Row row(int64_t e0) const {
    return Row{reinterpret_cast<const char*>(re_p + e0), reinterpret_cast<const char*>(im_p + e0)};
  }
  __device__ __forceinline__ static Raw load(const Row& r, uint32_t k) {
    return Raw{ldnt4u(lane_load_at(r.re, k)), ldnt4u(lane_load_at(r.im, k))};
  }
  __device__ __forceinline__ static void decode(const Raw& r, float (&re)[CPL], float (&im)[CPL]) {
    const unsigned aw[4] = {r.a.x, r.a.y, r.a.z, r.a.w}, bw[4] = {r.b.x, r.b.y, r.b.z, r.b.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      e4m3x4_to_f32(aw[q], re[4 * q], re[4 * q + 1], re[4 * q + 2], re[4 * q + 3]);
      e4m3x4_to_f32(bw[q], im[4 * q], im[4 * q + 1], im[4 * q + 2], im[4 * q + 3]);
    }
  }
  __device__ __forceinline__ float row_scale(int grow) const { return scale[grow]; }
  __device__ __forceinline__ double2 getd(int64_t e, int grow) const {
    const double s = scale[grow];
    return make_double2(s * (double)e4m3_to_f32(re_p[e]), s * (double)e4m3_to_f32(im_p[e]));
  }
};

// Build the view of the plan's H store for format F.
template <class F> struct MakeFmt;
template <> struct MakeFmt<FmtC64> {
  __device__ __forceinline__ static FmtC64 make(const HStore& h) {
    return FmtC64{static_cast<const float2*>(h.base)};
  }
};
template <> struct MakeFmt<FmtBF16> {
  __device__ __forceinline__ static FmtBF16 make(const HStore& h) {
    return FmtBF16{static_cast<const uint16_t*>(h.base), static_cast<const uint16_t*>(h.base_im)};
  }
};
template <> struct MakeFmt<FmtFP8> {
  __device__ __forceinline__ static FmtFP8 make(const HStore& h) {
    return FmtFP8{static_cast<const uint8_t*>(h.base), static_cast<const uint8_t*>(h.base_im), h.row_scale};
  }
};

}  // namespace admm
