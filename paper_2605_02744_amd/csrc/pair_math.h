// Device-side pair arithmetic shared by the all-pairs kernels (pairs.hip) and
// the persistent ensemble kernel (ensemble.hip).
#pragma once

#include <type_traits>

#include "common.h"

namespace nb {

enum Mode { kFP64 = NBODY_FP64, kFP32C = NBODY_FP32C, kFP32 = NBODY_FP32 };

// Knuth's TwoSum: (hi, lo) += x with the rounding error of hi + x kept in lo.
template <typename T>
__device__ __forceinline__ void fold(T& hi, T& lo, T x) {
  T s = hi + x;
  T bp = s - hi;
  T e = (hi - (s - bp)) + (x - bp);
  hi = s;
  lo += e;
}

// 1/sqrt(r2) in FP64: the hardware estimate y (about 5e-8 relative) refined in
// one step from the residual h = 1 - r2 y^2 with the binomial series
// (1 - h)^(-1/2) = 1 + h/2 + 3h^2/8 + O(h^3): y += y h (1/2 + 3h/8).  With
// |h| ~ 1e-7 the truncated term (5h^3/16) is ~1e-22, below FP64 rounding, for
// five operations where two Newton steps take eight.
__device__ __forceinline__ double rsqrt64(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double h = fma(-r2 * y, y, 1.0);
  return fma(y * h, fma(0.375, h, 0.5), y);
}

__device__ __forceinline__ float rsqrt32(float r2) { return __builtin_amdgcn_rsqf(r2); }

// Per-mode LDS record of one j-particle and its conversion from FP64.
template <int MODE> struct JRec;

template <> struct JRec<kFP64> {
  double4 p;  // x, y, z, m
  __device__ static JRec make(double x, double y, double z, double m) {
    JRec r; r.p = make_double4(x, y, z, m); return r;
  }
};
template <> struct JRec<kFP32C> {
  float4 h;   // hi parts, mass
  float4 l;   // lo parts
  __device__ static JRec make(double x, double y, double z, double m) {
    JRec r;
    float hx = (float)x, hy = (float)y, hz = (float)z;
    r.h = make_float4(hx, hy, hz, (float)m);
    r.l = make_float4((float)(x - (double)hx), (float)(y - (double)hy), (float)(z - (double)hz), 0.f);
    return r;
  }
};
template <> struct JRec<kFP32> {
  float4 h;
  __device__ static JRec make(double x, double y, double z, double m) {
    JRec r; r.h = make_float4((float)x, (float)y, (float)z, (float)m); return r;
  }
};

// Per-mode i-particle state held in registers.
template <int MODE> struct IPos;
template <> struct IPos<kFP64> {
  double x, y, z;
  __device__ void set(double a, double b, double c) { x = a; y = b; z = c; }
  __device__ void from(const JRec<kFP64>& r) { x = r.p.x; y = r.p.y; z = r.p.z; }
};
template <> struct IPos<kFP32C> {
  float hx, hy, hz, lx, ly, lz;
  __device__ void set(double a, double b, double c) {
    hx = (float)a; hy = (float)b; hz = (float)c;
    lx = (float)(a - (double)hx); ly = (float)(b - (double)hy); lz = (float)(c - (double)hz);
  }
  __device__ void from(const JRec<kFP32C>& r) {
    hx = r.h.x; hy = r.h.y; hz = r.h.z; lx = r.l.x; ly = r.l.y; lz = r.l.z;
  }
};
template <> struct IPos<kFP32> {
  float hx, hy, hz;
  __device__ void set(double a, double b, double c) { hx = (float)a; hy = (float)b; hz = (float)c; }
  __device__ void from(const JRec<kFP32>& r) { hx = r.h.x; hy = r.h.y; hz = r.h.z; }
};

template <int MODE> using Real = typename std::conditional<MODE == kFP64, double, float>::type;

// Displacement d = x_j - x_i per mode.
__device__ __forceinline__ void disp(const JRec<kFP64>& r, const IPos<kFP64>& p, double& dx, double& dy, double& dz) {
  dx = r.p.x - p.x; dy = r.p.y - p.y; dz = r.p.z - p.z;
}
__device__ __forceinline__ void disp(const JRec<kFP32C>& r, const IPos<kFP32C>& p, float& dx, float& dy, float& dz) {
  dx = (r.h.x - p.hx) + (r.l.x - p.lx);
  dy = (r.h.y - p.hy) + (r.l.y - p.ly);
  dz = (r.h.z - p.hz) + (r.l.z - p.lz);
}
// Displacement from the hi parts only (positions rounded to FP32).
__device__ __forceinline__ void disp_hi(const JRec<kFP32C>& r, const IPos<kFP32C>& p, float& dx, float& dy, float& dz) {
  dx = r.h.x - p.hx; dy = r.h.y - p.hy; dz = r.h.z - p.hz;
}
__device__ __forceinline__ void disp(const JRec<kFP32>& r, const IPos<kFP32>& p, float& dx, float& dy, float& dz) {
  dx = r.h.x - p.hx; dy = r.h.y - p.hy; dz = r.h.z - p.hz;
}
__device__ __forceinline__ double jmass(const JRec<kFP64>& r) { return r.p.w; }
__device__ __forceinline__ float jmass(const JRec<kFP32C>& r) { return r.h.w; }
__device__ __forceinline__ float jmass(const JRec<kFP32>& r) { return r.h.w; }
__device__ __forceinline__ double rsq(double r2) { return rsqrt64(r2); }
__device__ __forceinline__ float rsq(float r2) { return rsqrt32(r2); }

// Near-field repair of FP32C pairs (see accel_kernel): a pair closer than
//   d_c(i) = max(max(kNearX, kNearN n^-1/3) |x_i|_inf, kNearEps eps)
// gets a float-float displacement.  Rounding a coordinate to FP32 moves it by
// up to u |x| (u = 2^-24), which changes a pair term m_j d / |d|^3 by about
// 3 u |x| m_j / |d|^3.  The first bound keeps that below 3u / kNearX^3 of the
// pair's own term; the second keeps it below 3u / kNearN^3 of G M / |x|^2 for
// a pair of mass M / n, which matters in small systems, where one pair at the
// radius can outweigh the whole acceleration of particle i.
constexpr float kNearX = 2.0e-2f;
constexpr float kNearN = 0.5f;
constexpr float kNearEps = 2.0f;

// Error estimate of FP32C rows and the threshold of their FP64 rescue (the
// estimate and its use are described in rescue.hip): a block of terms with
// partial sum P and closest non-repaired pair at softened distance d adds
// ((1 + kEstNear |x_i|_inf / d) |P|)^2 to E_i, and the row is recomputed in
// FP64 when kEstC u |G| sqrt(E_i) > kRescueTol |a_i|.  kEstC prices the
// arithmetic of an FP32 term (a few roundings of u); kEstNear the rounding of
// both positions to FP32, about 3 sqrt(3) u (|x_i| + |x_j|) / d relative, in
// units of kEstC u.
constexpr float kEstNear = 1.5f;
constexpr double kEstC = 4.0;
constexpr double kRescueTol = 4.0e-6;
// the flag test as sqrt(E_i) * kRescueScale |G| > |a_i|
constexpr double kRescueScale = kEstC * 5.9604644775390625e-8 / kRescueTol;

// Adds one block's share to the error estimate e (see above).
__device__ __forceinline__ float est_add(float e, float px, float py, float pz, float xinf, float r2nr) {
  const float w = fmaf(kEstNear * xinf, __builtin_amdgcn_rsqf(r2nr), 1.0f);
  return fmaf(w * w, fmaf(px, px, fmaf(py, py, pz * pz)), e);
}

// Squared repair radius of lane particle i (positions given in double) in a
// system of n particles.
__device__ __forceinline__ float near_rc2(double xa, double ya, double za, double eps, int n) {
  const float fx = fmaxf(kNearX, kNearN / cbrtf((float)(n > 0 ? n : 1)));
  const float dc = fmaxf(fx * (float)fmax(fabs(xa), fmax(fabs(ya), fabs(za))), kNearEps * (float)eps);
  return dc * dc + (float)(eps * eps);
}

}  // namespace nb
