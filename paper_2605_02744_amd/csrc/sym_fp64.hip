// Symmetric FP64 acceleration: the plain FP64 path with every unordered pair
// evaluated once and applied to both particles, on the layout of the FP32C
// kernel (sym_pairs.hip): I-blocks of 512 particles, two per lane; J-blocks
// streamed through LDS in tiles of 64 as sub-blocks of 16 stored twice in a
// row, so that at step K lane r meets record (r + K) mod 16; the j-side terms
// of both i of a lane summed and moved to the lane owning that j by a row
// rotation (each double as two 32-bit DPP moves, then an FP64 add); wave sums
// across rows on the LDS pipe; tile sums to per-distance FP64 slots; a half
// ring of block pairs in chunks; FP64 slot sums in a fixed order.  All
// arithmetic is FP64 with the refined inverse square root of the ordered FP64
// kernel; there is no near-field repair to do.  The vector-Jacobian product of
// the acceleration (the adjoint's pairwise VJP) runs on the same layout with
// four FP64 components per particle, acceleration + jerk (Algorithm 3) with
// six and the sixth-order Hermite evaluation (acceleration, jerk, snap) with
// nine.
#include "sym_common.h"

namespace nb {
namespace {

// A double rotated within each row of 16 lanes: lane r gets lane (r - K) mod 16's value.
template <int K>
__device__ __forceinline__ double row_ror64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b & 0xffffffffull), 0x120 + K, 0xF, 0xF, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0x120 + K, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The two 32-bit halves of a double through ds_swizzle / ds_bpermute.
__device__ __forceinline__ double swizzle64_xor16(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_swizzle((int)(unsigned)(b & 0xffffffffull), 0x401F);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_swizzle((int)(unsigned)(b >> 32), 0x401F);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double bpermute64(int addr, double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(b & 0xffffffffull));
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

struct S64Args {
  const double* x;  // [3][n]
  const double* m;  // [n]
  int n, nb, npad, dmax, half, d_lo, T, nparts;  // T: tiles per workgroup
  double eps;
  const double4* rec;  // [npad] staged (x, y, z, m); padding far away and massless
  double* pj;          // [D][3][npad] j-side tile sums of the chunk's distances
  double* pi;          // [nparts][3][npad] i-side sums of the chunk's workgroups
};

struct DSet {
  double x[2], y[2], z[2], mneg[2];
};

template <int K>
__device__ __forceinline__ void step64(const DSet& s, const double4* __restrict__ rowp, double e2,
                                       double (&px)[2], double (&py)[2], double (&pz)[2], double& ajx, double& ajy,
                                       double& ajz) {
  const double4 r = rowp[K];
  double tx = 0.0, ty = 0.0, tz = 0.0;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const double dx = r.x - s.x[u], dy = r.y - s.y[u], dz = r.z - s.z[u];
    const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
    const double ri = rsqrt64(r2);
    const double ri3 = (ri * ri) * ri;
    const double si = r.w * ri3;
    px[u] = fma(si, dx, px[u]);
    py[u] = fma(si, dy, py[u]);
    pz[u] = fma(si, dz, pz[u]);
    const double sj = s.mneg[u] * ri3;
    if (u == 0) { tx = sj * dx; ty = sj * dy; tz = sj * dz; }
    else { tx = fma(sj, dx, tx); ty = fma(sj, dy, ty); tz = fma(sj, dz, tz); }
  }
  if constexpr (K == 0) { ajx += tx; ajy += ty; ajz += tz; }
  else {
    ajx += row_ror64<K>(tx);
    ajy += row_ror64<K>(ty);
    ajz += row_ror64<K>(tz);
  }
}

template <int... K>
__device__ __forceinline__ void sub64(const DSet& s, const double4* __restrict__ rowp, double e2, double (&px)[2],
                                      double (&py)[2], double (&pz)[2], double& ajx, double& ajy, double& ajz,
                                      std::integer_sequence<int, K...>) {
  (step64<K>(s, rowp, e2, px, py, pz, ajx, ajy, ajz), ...);
}

__device__ __forceinline__ void load_dset(const S64Args& A, int g, int t, DSet& s) {
  const int n = A.n;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = g * kSI + u * kSL + t;
    if (i < n) {
      s.x[u] = A.x[i]; s.y[u] = A.x[n + i]; s.z[u] = A.x[2 * n + i];
      s.mneg[u] = -A.m[i];
    } else {
      s.x[u] = s.y[u] = s.z[u] = kFarAway;
      s.mneg[u] = 0.0;
    }
  }
}

__global__ void sym64_stage_kernel(S64Args A, double4* __restrict__ rec) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= A.npad) return;
  const int n = A.n;
  rec[j] = j < n ? make_double4(A.x[j], A.x[n + j], A.x[2 * n + j], A.m[j])
                 : make_double4(kFarAway, kFarAway, kFarAway, 0.0);
}

// Grid: nb * nparts workgroups; workgroup (g, part) takes the distances
// [d_lo + part L, d_lo + (part + 1) L) of I-block g's half ring (d >= 1).
__global__ __launch_bounds__(kSL, 6) void sym64_kernel(S64Args A) {
  __shared__ double4 s_rec[2][4][2 * kSR];  // each sub-block twice in a row
  __shared__ double s_part[3][kSW][kST];
  __shared__ double s_acc_lo[6][kSL];       // the lo halves of the i-side (hi, lo) sums

  const int t = threadIdx.x;
  const int rl = t & (kSR - 1);
  const int wave = t / 64;
  const int lid = xcd_local_index(blockIdx.x, gridDim.x);
  const int g = lid % A.nb;
  const int part = lid / A.nb;
  // this workgroup's tiles: kbeg, kbeg + 1, ... of the chunk, counted from the
  // first tile of distance d_lo (A.T of them, fewer where g's ring ends)
  const int kbeg = part * A.T;
  const int rend = (A.half && g >= A.nb / 2) ? A.dmax : A.dmax + 1;  // g's ring ends before this distance
  const int ntiles = max(0, min(kbeg + A.T, (rend - A.d_lo) * kSTiles) - kbeg);
  const double e2 = A.eps * A.eps;

  DSet s;
  load_dset(A, g, t, s);
  double hx[2] = {0.0, 0.0}, hy[2] = {0.0, 0.0}, hz[2] = {0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 6; ++c) s_acc_lo[c][t] = 0.0;
  const int xor32 = ((t & 63) ^ 32) * 4;

  // the last wave copies tile k into LDS buffer b, one sub-block per copy: lane
  // L brings the half (L & 1) of record (L >> 1) mod 16, so that the 64 lanes'
  // 16-byte pieces lay the sub-block's 16 records out twice in a row
  const unsigned lane_off = (unsigned)((((t & 63) >> 1) & (kSR - 1)) * sizeof(double4) + (t & 1) * 16);
  auto stage = [&](int k, int b) {
    const int rec0 = __builtin_amdgcn_readfirstlane(((g + A.d_lo + (kbeg + k) / kSTiles) % A.nb) * kSI + ((kbeg + k) % kSTiles) * kST);
    const char* base = reinterpret_cast<const char*>(A.rec) + (size_t)rec0 * sizeof(double4);
    unsigned o = lane_off;
    asm volatile("" : "+v"(o));
#pragma unroll
    for (int q = 0; q < 4; ++q)
      __builtin_amdgcn_global_load_lds(base + q * kSR * sizeof(double4) + o, (lds_ptr)&s_rec[b][q][0], 16, 0, 0);
  };

  if (ntiles > 0 && t >= 3 * 64) {
    stage(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();

  for (int k = 0; k < ntiles; ++k) {
    const int b = k & 1;
    const int d = A.d_lo + (kbeg + k) / kSTiles;
    const int tt = (kbeg + k) % kSTiles;
    if (t >= 3 * 64 && k + 1 < ntiles) stage(k + 1, b ^ 1);
    double px[2] = {0.0, 0.0}, py[2] = {0.0, 0.0}, pz[2] = {0.0, 0.0};
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      double ajx = 0.0, ajy = 0.0, ajz = 0.0;
      sub64(s, &s_rec[b][q][rl], e2, px, py, pz, ajx, ajy, ajz, std::make_integer_sequence<int, kSR>{});
      ajx += swizzle64_xor16(ajx);
      ajy += swizzle64_xor16(ajy);
      ajz += swizzle64_xor16(ajz);
      ajx += bpermute64(xor32, ajx);
      ajy += bpermute64(xor32, ajy);
      ajz += bpermute64(xor32, ajz);
      s_part[0][wave][q * kSR + rl] = ajx;
      s_part[1][wave][q * kSR + rl] = ajy;
      s_part[2][wave][q * kSR + rl] = ajz;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      fold(hx[u], s_acc_lo[3 * u][t], px[u]);
      fold(hy[u], s_acc_lo[3 * u + 1][t], py[u]);
      fold(hz[u], s_acc_lo[3 * u + 2][t], pz[u]);
    }
    __syncthreads();
    if (t < 3 * 64) {
      const int c = t / kST, jl = t % kST;
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < kSW; ++w) v += s_part[c][w][jl];
      const int J = (g + d) % A.nb;
      A.pj[((size_t)(d - A.d_lo) * 3 + c) * A.npad + (size_t)J * kSI + tt * kST + jl] = v;
    } else {
      __builtin_amdgcn_s_waitcnt(0);  // the next tile's copies have landed in LDS
    }
    __syncthreads();
  }

  double* o = A.pi + (size_t)part * 3 * A.npad;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const size_t i = (size_t)g * kSI + u * kSL + t;
    o[i] = hx[u] + s_acc_lo[3 * u][t];
    o[A.npad + i] = hy[u] + s_acc_lo[3 * u + 1][t];
    o[2 * (size_t)A.npad + i] = hz[u] + s_acc_lo[3 * u + 2][t];
  }
}

// The block with itself (distance 0), ordered form, i-side only, own pair
// masked when asked.  The gridDim.y workgroups of a block each take a slice of
// its j, and their kDiagG groups of kSL lanes each a part of the slice; group 0
// adds the groups' hi + lo in group order into pd[slice][3][npad].
template <bool EXCL>
__global__ __launch_bounds__(kSL* kDiagG) void sym64_diag_kernel(S64Args A, double* __restrict__ pd) {
  __shared__ double4 s_rec[kSI];
  __shared__ double s_part[kDiagG - 1][3][kSI];
  const int t = threadIdx.x % kSL, grp = threadIdx.x / kSL;
  const int g = blockIdx.x;
  const double e2 = A.eps * A.eps;
  const int span = kSI / ((int)gridDim.y * kDiagG), fl = span < kFold ? span : kFold;
  const int f0 = ((int)blockIdx.y * kDiagG + grp) * span;
  DSet s;
  load_dset(A, g, t, s);
  for (int k = threadIdx.x; k < kSI; k += kSL * kDiagG) s_rec[k] = A.rec[(size_t)g * kSI + k];
  __syncthreads();
  double hx[2] = {0.0, 0.0}, hy[2] = {0.0, 0.0}, hz[2] = {0.0, 0.0};
  double lx[2] = {0.0, 0.0}, ly[2] = {0.0, 0.0}, lz[2] = {0.0, 0.0};
#pragma unroll 1
  for (int f = f0; f < f0 + span; f += fl) {
    double px[2] = {0.0, 0.0}, py[2] = {0.0, 0.0}, pz[2] = {0.0, 0.0};
#pragma unroll 8
    for (int j = f; j < f + fl; ++j) {
      const double4 r = s_rec[j];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const double dx = r.x - s.x[u], dy = r.y - s.y[u], dz = r.z - s.z[u];
        const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
        const double ri = rsqrt64(r2);
        double si = (r.w * ri) * (ri * ri);
        if (EXCL) si = (j == u * kSL + t) ? 0.0 : si;
        px[u] = fma(si, dx, px[u]);
        py[u] = fma(si, dy, py[u]);
        pz[u] = fma(si, dz, pz[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      fold(hx[u], lx[u], px[u]);
      fold(hy[u], ly[u], py[u]);
      fold(hz[u], lz[u], pz[u]);
    }
  }
  if (grp > 0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      s_part[grp - 1][0][u * kSL + t] = hx[u] + lx[u];
      s_part[grp - 1][1][u * kSL + t] = hy[u] + ly[u];
      s_part[grp - 1][2][u * kSL + t] = hz[u] + lz[u];
    }
  }
  __syncthreads();
  if (grp > 0) return;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int k = u * kSL + t;
    const size_t i = (size_t)g * kSI + k;
    double* const pds = pd + (size_t)blockIdx.y * 3 * A.npad;
    double vx = hx[u] + lx[u], vy = hy[u] + ly[u], vz = hz[u] + lz[u];
#pragma unroll
    for (int q = 0; q < kDiagG - 1; ++q) {
      vx += s_part[q][0][k];
      vy += s_part[q][1][k];
      vz += s_part[q][2][k];
    }
    pds[i] = vx;
    pds[A.npad + i] = vy;
    pds[2 * (size_t)A.npad + i] = vz;
  }
}


// ------------------------------------------------ symmetric FP64 VJP
// The vector-Jacobian product of the acceleration on the same layout, in FP64:
// with d = x_j - x_k, r^2 = |d|^2 + eps^2 and u = m_k w_j - m_j w_k, the
// unordered pair {k, j} gives
//   gx_k += r^-3 u - 3 r^-5 (d.u) d,   gm_k -= r^-3 (d . w_j),
//   gx_j -= r^-3 u - 3 r^-5 (d.u) d,   gm_j += r^-3 (d . w_k)
// (d and u both change sign when k and j swap).  Four components per particle
// (gx, gy, gz, gm); cotangents staged as a second record per particle.
constexpr int kV64 = 4;

struct V64Args {
  const double* x;  // [3][n]
  const double* m;  // [n]
  const double* w;  // [3][n] cotangent
  int n, nb, npad, dmax, half, d_lo, T, nparts;
  double eps;
  const double4* rec;   // [npad] staged (x, y, z, m); padding far away and massless
  const double4* recw;  // [npad] staged (wx, wy, wz, 0); padding zero
  double* pj;           // [D][4][npad] j-side tile sums of the chunk's distances
  double* pi;           // [nparts][4][npad] i-side sums of the chunk's workgroups
};

struct VDSet {
  double x[2], y[2], z[2], m[2], wx[2], wy[2], wz[2];
};

__device__ __forceinline__ void load_vdset(const V64Args& A, int g, int t, VDSet& s) {
  const int n = A.n;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = g * kSI + u * kSL + t;
    if (i < n) {
      s.x[u] = A.x[i]; s.y[u] = A.x[n + i]; s.z[u] = A.x[2 * n + i];
      s.m[u] = A.m[i];
      s.wx[u] = A.w[i]; s.wy[u] = A.w[n + i]; s.wz[u] = A.w[2 * n + i];
    } else {
      s.x[u] = s.y[u] = s.z[u] = kFarAway;
      s.m[u] = 0.0;
      s.wx[u] = s.wy[u] = s.wz[u] = 0.0;
    }
  }
}

// One pair's terms for lane particle u against record (r, wj): the k-side
// terms added to p[u], the j-side ones to (ax, ay, az, am).
__device__ __forceinline__ void vjp64_pair(const VDSet& s, int u, const double4& r, const double4& wj, double e2,
                                           double (&p)[2][kV64], double& ax, double& ay, double& az, double& am) {
  const double dx = r.x - s.x[u], dy = r.y - s.y[u], dz = r.z - s.z[u];
  const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
  const double ri = rsqrt64(r2);
  const double ri2 = ri * ri;
  const double r3 = ri2 * ri;
  const double c5 = (-3.0 * ri2) * r3;
  const double ux = fma(s.m[u], wj.x, -(r.w * s.wx[u]));
  const double uy = fma(s.m[u], wj.y, -(r.w * s.wy[u]));
  const double uz = fma(s.m[u], wj.z, -(r.w * s.wz[u]));
  const double cc = c5 * fma(dz, uz, fma(dy, uy, dx * ux));
  p[u][0] = fma(cc, dx, fma(r3, ux, p[u][0]));
  p[u][1] = fma(cc, dy, fma(r3, uy, p[u][1]));
  p[u][2] = fma(cc, dz, fma(r3, uz, p[u][2]));
  ax = fma(-cc, dx, fma(-r3, ux, ax));
  ay = fma(-cc, dy, fma(-r3, uy, ay));
  az = fma(-cc, dz, fma(-r3, uz, az));
  p[u][3] = fma(-r3, fma(dz, wj.z, fma(dy, wj.y, dx * wj.x)), p[u][3]);
  am = fma(r3, fma(dz, s.wz[u], fma(dy, s.wy[u], dx * s.wx[u])), am);
}

template <int K>
__device__ __forceinline__ void vstep64(const VDSet& s, const double4* __restrict__ rowp,
                                        const double4* __restrict__ roww, double e2, double (&p)[2][kV64],
                                        double (&aj)[kV64]) {
  const double4 r = rowp[K];
  const double4 wj = roww[K];
  double ax = 0.0, ay = 0.0, az = 0.0, am = 0.0;
  vjp64_pair(s, 0, r, wj, e2, p, ax, ay, az, am);
  vjp64_pair(s, 1, r, wj, e2, p, ax, ay, az, am);
  // the j met here sits at row position (r + K): its owner is K lanes further on
  if constexpr (K == 0) {
    aj[0] += ax; aj[1] += ay; aj[2] += az; aj[3] += am;
  } else {
    aj[0] += row_ror64<K>(ax);
    aj[1] += row_ror64<K>(ay);
    aj[2] += row_ror64<K>(az);
    aj[3] += row_ror64<K>(am);
  }
}

template <int... K>
__device__ __forceinline__ void vsub64(const VDSet& s, const double4* __restrict__ rowp,
                                       const double4* __restrict__ roww, double e2, double (&p)[2][kV64],
                                       double (&aj)[kV64], std::integer_sequence<int, K...>) {
  (vstep64<K>(s, rowp, roww, e2, p, aj), ...);
}

__global__ void vsym64_stage_kernel(V64Args A, double4* __restrict__ rec, double4* __restrict__ recw) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= A.npad) return;
  const int n = A.n;
  rec[j] = j < n ? make_double4(A.x[j], A.x[n + j], A.x[2 * n + j], A.m[j])
                 : make_double4(kFarAway, kFarAway, kFarAway, 0.0);
  recw[j] = j < n ? make_double4(A.w[j], A.w[n + j], A.w[2 * n + j], 0.0) : make_double4(0.0, 0.0, 0.0, 0.0);
}

// Grid: nb * nparts workgroups; workgroup (g, part) takes tiles kbeg ..
// kbeg + T - 1 of the chunk (fewer where g's ring ends), as sym64_kernel.
__global__ __launch_bounds__(kSL, 3) void vsym64_kernel(V64Args A) {
  __shared__ double4 s_rec[2][4][2 * kSR];  // each sub-block twice in a row
  __shared__ double4 s_w[2][4][2 * kSR];    // cotangents, laid out as s_rec
  __shared__ double s_part[kV64][kSW][kST];
  __shared__ double s_acc_lo[2 * kV64][kSL];  // the lo halves of the i-side (hi, lo) sums

  const int t = threadIdx.x;
  const int rl = t & (kSR - 1);
  const int wave = t / 64;
  const int lid = xcd_local_index(blockIdx.x, gridDim.x);
  const int g = lid % A.nb;
  const int part = lid / A.nb;
  const int kbeg = part * A.T;
  const int rend = (A.half && g >= A.nb / 2) ? A.dmax : A.dmax + 1;  // g's ring ends before this distance
  const int ntiles = max(0, min(kbeg + A.T, (rend - A.d_lo) * kSTiles) - kbeg);
  const double e2 = A.eps * A.eps;

  VDSet s;
  load_vdset(A, g, t, s);
  double h[2][kV64];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < kV64; ++c) h[u][c] = 0.0;
#pragma unroll
  for (int c = 0; c < 2 * kV64; ++c) s_acc_lo[c][t] = 0.0;
  const int xor32 = ((t & 63) ^ 32) * 4;

  // the last wave copies tile k into LDS buffer b, one sub-block per copy: lane
  // L brings the half (L & 1) of record (L >> 1) mod 16, so that the 64 lanes'
  // 16-byte pieces lay the sub-block's 16 records out twice in a row
  const unsigned lane_off = (unsigned)((((t & 63) >> 1) & (kSR - 1)) * sizeof(double4) + (t & 1) * 16);
  auto stage = [&](int k, int b) {
    const int rec0 = __builtin_amdgcn_readfirstlane(((g + A.d_lo + (kbeg + k) / kSTiles) % A.nb) * kSI + ((kbeg + k) % kSTiles) * kST);
    const char* base = reinterpret_cast<const char*>(A.rec) + (size_t)rec0 * sizeof(double4);
    const char* wbase = reinterpret_cast<const char*>(A.recw) + (size_t)rec0 * sizeof(double4);
    unsigned o = lane_off;
    asm volatile("" : "+v"(o));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      __builtin_amdgcn_global_load_lds(base + q * kSR * sizeof(double4) + o, (lds_ptr)&s_rec[b][q][0], 16, 0, 0);
      __builtin_amdgcn_global_load_lds(wbase + q * kSR * sizeof(double4) + o, (lds_ptr)&s_w[b][q][0], 16, 0, 0);
    }
  };

  if (ntiles > 0 && t >= 3 * 64) {
    stage(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();

  for (int k = 0; k < ntiles; ++k) {
    const int b = k & 1;
    const int d = A.d_lo + (kbeg + k) / kSTiles;
    const int tt = (kbeg + k) % kSTiles;
    if (t >= 3 * 64 && k + 1 < ntiles) stage(k + 1, b ^ 1);
    double p[2][kV64];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kV64; ++c) p[u][c] = 0.0;
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      double aj[kV64] = {0.0, 0.0, 0.0, 0.0};
      vsub64(s, &s_rec[b][q][rl], &s_w[b][q][rl], e2, p, aj, std::make_integer_sequence<int, kSR>{});
      // the four rows' sums of the same 16 j
#pragma unroll
      for (int c = 0; c < kV64; ++c) {
        aj[c] += swizzle64_xor16(aj[c]);
        aj[c] += bpermute64(xor32, aj[c]);
        s_part[c][wave][q * kSR + rl] = aj[c];
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kV64; ++c) fold(h[u][c], s_acc_lo[u * kV64 + c][t], p[u][c]);
    __syncthreads();
    {
      // the tile's j-side sums: the 4 wave sums of each j, in wave order
      const int c = t / kST, jl = t % kST;
      double v = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < kSW; ++w2) v += s_part[c][w2][jl];
      const int J = (g + d) % A.nb;
      A.pj[((size_t)(d - A.d_lo) * kV64 + c) * A.npad + (size_t)J * kSI + tt * kST + jl] = v;
    }
    if (t >= 3 * 64) __builtin_amdgcn_s_waitcnt(0);  // the next tile's copies have landed in LDS
    __syncthreads();
  }

  double* o = A.pi + (size_t)part * kV64 * A.npad;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const size_t i = (size_t)g * kSI + u * kSL + t;
#pragma unroll
    for (int c = 0; c < kV64; ++c) o[(size_t)c * A.npad + i] = h[u][c] + s_acc_lo[u * kV64 + c][t];
  }
}

// The block with itself (distance 0): the k-side of all ordered pairs inside
// I-block g, own pair left out (its term is zero: d = 0 and u = 0).  The
// gridDim.y workgroups of a block each take a slice of its j, and their kDiagG
// groups of kSL lanes each a part of the slice; group 0 adds the groups' hi +
// lo in group order into pd[slice][4][npad].
__global__ __launch_bounds__(kSL* kDiagG) void vsym64_diag_kernel(V64Args A, double* __restrict__ pd) {
  __shared__ double4 s_rec[kSI];
  __shared__ double4 s_w[kSI];
  __shared__ double s_part[kDiagG - 1][kV64][kSI];
  const int t = threadIdx.x % kSL, grp = threadIdx.x / kSL;
  const int g = blockIdx.x;
  const double e2 = A.eps * A.eps;
  const int span = kSI / ((int)gridDim.y * kDiagG), fl = span < kFold ? span : kFold;
  const int f0 = ((int)blockIdx.y * kDiagG + grp) * span;
  VDSet s;
  load_vdset(A, g, t, s);
  for (int k = threadIdx.x; k < kSI; k += kSL * kDiagG) {
    s_rec[k] = A.rec[(size_t)g * kSI + k];
    s_w[k] = A.recw[(size_t)g * kSI + k];
  }
  __syncthreads();
  double h[2][kV64], l[2][kV64];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < kV64; ++c) h[u][c] = l[u][c] = 0.0;
#pragma unroll 1
  for (int f = f0; f < f0 + span; f += fl) {
    double p[2][kV64];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kV64; ++c) p[u][c] = 0.0;
#pragma unroll 4
    for (int j = f; j < f + fl; ++j) {
      const double4 r = s_rec[j];
      const double4 wj = s_w[j];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        double q[2][kV64];
#pragma unroll
        for (int c = 0; c < kV64; ++c) q[0][c] = q[1][c] = 0.0;
        double ax = 0.0, ay = 0.0, az = 0.0, am = 0.0;
        vjp64_pair(s, u, r, wj, e2, q, ax, ay, az, am);
        const bool own = j == u * kSL + t;
#pragma unroll
        for (int c = 0; c < kV64; ++c) p[u][c] += own ? 0.0 : q[u][c];
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kV64; ++c) fold(h[u][c], l[u][c], p[u][c]);
  }
  if (grp > 0) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kV64; ++c) s_part[grp - 1][c][u * kSL + t] = h[u][c] + l[u][c];
  }
  __syncthreads();
  if (grp > 0) return;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int k = u * kSL + t;
    const size_t i = (size_t)g * kSI + k;
    double* const pds = pd + (size_t)blockIdx.y * kV64 * A.npad;
#pragma unroll
    for (int c = 0; c < kV64; ++c) {
      double v = h[u][c] + l[u][c];
#pragma unroll
      for (int q = 0; q < kDiagG - 1; ++q) v += s_part[q][c][k];
      pds[(size_t)c * A.npad + i] = v;
    }
  }
}


// ------------------------------------------ symmetric FP64 acceleration + jerk
// Algorithm 3's pair term once per unordered pair, in FP64: with d = x_j - x_i,
// w = v_j - v_i, r^2 = |d|^2 + eps^2 and q = -3 r^-2 (d . w),
//   a_i += m_j r^-3 d,   jerk_i += m_j r^-3 (w + q d),
//   a_j -= m_i r^-3 d,   jerk_j -= m_i r^-3 (w + q d)
// (d and w change sign when i and j swap, q does not).  Six components per
// particle (a, then jerk); velocities staged as a second record per particle.
constexpr int kJ64 = 6;

struct J64Args {
  const double* x;  // [3][n]
  const double* v;  // [3][n]
  const double* m;  // [n]
  int n, nb, npad, dmax, half, d_lo, T, nparts;
  double eps;
  const double4* rec;   // [npad] staged (x, y, z, m); padding far away and massless
  const double4* recv;  // [npad] staged (vx, vy, vz, 0); padding at rest
  double* pj;           // [D][6][npad] j-side tile sums of the chunk's distances
  double* pi;           // [nparts][6][npad] i-side sums of the chunk's workgroups
};

struct JDSet {
  double x[2], y[2], z[2], mneg[2], vx[2], vy[2], vz[2];
};

__device__ __forceinline__ void load_jdset(const J64Args& A, int g, int t, JDSet& s) {
  const int n = A.n;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = g * kSI + u * kSL + t;
    if (i < n) {
      s.x[u] = A.x[i]; s.y[u] = A.x[n + i]; s.z[u] = A.x[2 * n + i];
      s.mneg[u] = -A.m[i];
      s.vx[u] = A.v[i]; s.vy[u] = A.v[n + i]; s.vz[u] = A.v[2 * n + i];
    } else {
      s.x[u] = s.y[u] = s.z[u] = kFarAway;
      s.mneg[u] = 0.0;
      s.vx[u] = s.vy[u] = s.vz[u] = 0.0;
    }
  }
}

// One pair for lane particle u against record (r, vj): the i-side terms are
// added to p[u] (scale m_j), the j-side ones to b (scale -m_i).  The own pair
// (masked with own) adds nothing: its r^-3 and q are replaced by zeros, since
// without softening they are infinite and NaN.
__device__ __forceinline__ void jerk64_pair(const JDSet& s, int u, const double4& r, const double4& vj, double e2,
                                            bool own, double (&p)[2][kJ64], double (&b)[kJ64]) {
  const double dx = r.x - s.x[u], dy = r.y - s.y[u], dz = r.z - s.z[u];
  const double wx = vj.x - s.vx[u], wy = vj.y - s.vy[u], wz = vj.z - s.vz[u];
  const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
  const double ri = rsqrt64(r2);
  const double ri2 = ri * ri;
  const double r3 = own ? 0.0 : ri2 * ri;
  const double q = own ? 0.0 : (-3.0 * ri2) * fma(dz, wz, fma(dy, wy, dx * wx));
  const double tx = fma(q, dx, wx), ty = fma(q, dy, wy), tz = fma(q, dz, wz);
  const double si = r.w * r3;
  const double sj = s.mneg[u] * r3;
  p[u][0] = fma(si, dx, p[u][0]);
  p[u][1] = fma(si, dy, p[u][1]);
  p[u][2] = fma(si, dz, p[u][2]);
  p[u][3] = fma(si, tx, p[u][3]);
  p[u][4] = fma(si, ty, p[u][4]);
  p[u][5] = fma(si, tz, p[u][5]);
  b[0] = fma(sj, dx, b[0]); b[1] = fma(sj, dy, b[1]); b[2] = fma(sj, dz, b[2]);
  b[3] = fma(sj, tx, b[3]); b[4] = fma(sj, ty, b[4]); b[5] = fma(sj, tz, b[5]);
}

template <int K>
__device__ __forceinline__ void jstep64(const JDSet& s, const double4* __restrict__ rowp,
                                        const double4* __restrict__ rowv, double e2, double (&p)[2][kJ64],
                                        double (&aj)[kJ64]) {
  const double4 r = rowp[K];
  const double4 vj = rowv[K];
  double b[kJ64] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  jerk64_pair(s, 0, r, vj, e2, false, p, b);
  jerk64_pair(s, 1, r, vj, e2, false, p, b);
  // the j met here sits at row position (r + K): its owner is K lanes further on
  if constexpr (K == 0) {
#pragma unroll
    for (int c = 0; c < kJ64; ++c) aj[c] += b[c];
  } else {
#pragma unroll
    for (int c = 0; c < kJ64; ++c) aj[c] += row_ror64<K>(b[c]);
  }
}

template <int... K>
__device__ __forceinline__ void jsub64(const JDSet& s, const double4* __restrict__ rowp,
                                       const double4* __restrict__ rowv, double e2, double (&p)[2][kJ64],
                                       double (&aj)[kJ64], std::integer_sequence<int, K...>) {
  (jstep64<K>(s, rowp, rowv, e2, p, aj), ...);
}

__global__ void jsym64_stage_kernel(J64Args A, double4* __restrict__ rec, double4* __restrict__ recv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= A.npad) return;
  const int n = A.n;
  rec[j] = j < n ? make_double4(A.x[j], A.x[n + j], A.x[2 * n + j], A.m[j])
                 : make_double4(kFarAway, kFarAway, kFarAway, 0.0);
  recv[j] = j < n ? make_double4(A.v[j], A.v[n + j], A.v[2 * n + j], 0.0) : make_double4(0.0, 0.0, 0.0, 0.0);
}

// Grid: nb * nparts workgroups; workgroup (g, part) takes tiles kbeg ..
// kbeg + T - 1 of the chunk (fewer where g's ring ends), as sym64_kernel.
__global__ __launch_bounds__(kSL, 2) void jsym64_kernel(J64Args A) {
  __shared__ double4 s_rec[2][4][2 * kSR];  // each sub-block twice in a row
  __shared__ double4 s_v[2][4][2 * kSR];    // velocities, laid out as s_rec
  __shared__ double s_part[kJ64][kSW][kST];
  __shared__ double s_acc_lo[2 * kJ64][kSL];  // the lo halves of the i-side (hi, lo) sums

  const int t = threadIdx.x;
  const int rl = t & (kSR - 1);
  const int wave = t / 64;
  const int lid = xcd_local_index(blockIdx.x, gridDim.x);
  const int g = lid % A.nb;
  const int part = lid / A.nb;
  const int kbeg = part * A.T;
  const int rend = (A.half && g >= A.nb / 2) ? A.dmax : A.dmax + 1;  // g's ring ends before this distance
  const int ntiles = max(0, min(kbeg + A.T, (rend - A.d_lo) * kSTiles) - kbeg);
  const double e2 = A.eps * A.eps;

  JDSet s;
  load_jdset(A, g, t, s);
  double h[2][kJ64];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < kJ64; ++c) h[u][c] = 0.0;
#pragma unroll
  for (int c = 0; c < 2 * kJ64; ++c) s_acc_lo[c][t] = 0.0;
  const int xor32 = ((t & 63) ^ 32) * 4;

  // the last wave copies tile k into LDS buffer b, as in sym64_kernel
  const unsigned lane_off = (unsigned)((((t & 63) >> 1) & (kSR - 1)) * sizeof(double4) + (t & 1) * 16);
  auto stage = [&](int k, int b) {
    const int rec0 = __builtin_amdgcn_readfirstlane(((g + A.d_lo + (kbeg + k) / kSTiles) % A.nb) * kSI + ((kbeg + k) % kSTiles) * kST);
    const char* base = reinterpret_cast<const char*>(A.rec) + (size_t)rec0 * sizeof(double4);
    const char* vbase = reinterpret_cast<const char*>(A.recv) + (size_t)rec0 * sizeof(double4);
    unsigned o = lane_off;
    asm volatile("" : "+v"(o));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      __builtin_amdgcn_global_load_lds(base + q * kSR * sizeof(double4) + o, (lds_ptr)&s_rec[b][q][0], 16, 0, 0);
      __builtin_amdgcn_global_load_lds(vbase + q * kSR * sizeof(double4) + o, (lds_ptr)&s_v[b][q][0], 16, 0, 0);
    }
  };

  if (ntiles > 0 && t >= 3 * 64) {
    stage(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();

  for (int k = 0; k < ntiles; ++k) {
    const int b = k & 1;
    const int d = A.d_lo + (kbeg + k) / kSTiles;
    const int tt = (kbeg + k) % kSTiles;
    if (t >= 3 * 64 && k + 1 < ntiles) stage(k + 1, b ^ 1);
    double p[2][kJ64];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kJ64; ++c) p[u][c] = 0.0;
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      double aj[kJ64] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      jsub64(s, &s_rec[b][q][rl], &s_v[b][q][rl], e2, p, aj, std::make_integer_sequence<int, kSR>{});
      // the four rows' sums of the same 16 j
#pragma unroll
      for (int c = 0; c < kJ64; ++c) {
        aj[c] += swizzle64_xor16(aj[c]);
        aj[c] += bpermute64(xor32, aj[c]);
        s_part[c][wave][q * kSR + rl] = aj[c];
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kJ64; ++c) fold(h[u][c], s_acc_lo[u * kJ64 + c][t], p[u][c]);
    __syncthreads();
    // the tile's j-side sums: the 4 wave sums of each j, in wave order (6 x 64
    // of them over 256 lanes)
    for (int e = t; e < kJ64 * kST; e += kSL) {
      const int c = e / kST, jl = e % kST;
      double v = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < kSW; ++w2) v += s_part[c][w2][jl];
      const int J = (g + d) % A.nb;
      A.pj[((size_t)(d - A.d_lo) * kJ64 + c) * A.npad + (size_t)J * kSI + tt * kST + jl] = v;
    }
    if (t >= 3 * 64) __builtin_amdgcn_s_waitcnt(0);  // the next tile's copies have landed in LDS
    __syncthreads();
  }

  double* o = A.pi + (size_t)part * kJ64 * A.npad;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const size_t i = (size_t)g * kSI + u * kSL + t;
#pragma unroll
    for (int c = 0; c < kJ64; ++c) o[(size_t)c * A.npad + i] = h[u][c] + s_acc_lo[u * kJ64 + c][t];
  }
}

// The block with itself (distance 0): the i-side of all ordered pairs inside
// I-block g, own pair masked when asked, in slices as sym64_diag_kernel; group
// 0 adds the groups' hi + lo in group order into pd[slice][6][npad].
template <bool EXCL>
__global__ __launch_bounds__(kSL* kDiagG) void jsym64_diag_kernel(J64Args A, double* __restrict__ pd) {
  __shared__ double4 s_rec[kSI];
  __shared__ double4 s_v[kSI];
  __shared__ double s_part[kDiagG - 1][kJ64][kSI];
  const int t = threadIdx.x % kSL, grp = threadIdx.x / kSL;
  const int g = blockIdx.x;
  const double e2 = A.eps * A.eps;
  const int span = kSI / ((int)gridDim.y * kDiagG), fl = span < kFold ? span : kFold;
  const int f0 = ((int)blockIdx.y * kDiagG + grp) * span;
  JDSet s;
  load_jdset(A, g, t, s);
  for (int k = threadIdx.x; k < kSI; k += kSL * kDiagG) {
    s_rec[k] = A.rec[(size_t)g * kSI + k];
    s_v[k] = A.recv[(size_t)g * kSI + k];
  }
  __syncthreads();
  double h[2][kJ64], l[2][kJ64];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < kJ64; ++c) h[u][c] = l[u][c] = 0.0;
#pragma unroll 1
  for (int f = f0; f < f0 + span; f += fl) {
    double p[2][kJ64];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kJ64; ++c) p[u][c] = 0.0;
#pragma unroll 2
    for (int j = f; j < f + fl; ++j) {
      const double4 r = s_rec[j];
      const double4 vj = s_v[j];
      double b[kJ64] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // the j side is not needed here
      jerk64_pair(s, 0, r, vj, e2, EXCL && j == t, p, b);
      jerk64_pair(s, 1, r, vj, e2, EXCL && j == kSL + t, p, b);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kJ64; ++c) fold(h[u][c], l[u][c], p[u][c]);
  }
  if (grp > 0) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kJ64; ++c) s_part[grp - 1][c][u * kSL + t] = h[u][c] + l[u][c];
  }
  __syncthreads();
  if (grp > 0) return;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int k = u * kSL + t;
    const size_t i = (size_t)g * kSI + k;
    double* const pds = pd + (size_t)blockIdx.y * kJ64 * A.npad;
#pragma unroll
    for (int c = 0; c < kJ64; ++c) {
      double v = h[u][c] + l[u][c];
#pragma unroll
      for (int q = 0; q < kDiagG - 1; ++q) v += s_part[q][c][k];
      pds[(size_t)c * A.npad + i] = v;
    }
  }
}


// ------------------------------ symmetric FP64 acceleration + jerk + snap
// The sixth-order Hermite pair term once per unordered pair, in FP64: with
// d = x_j - x_i, w = v_j - v_i, u = acc_j - acc_i, s = |d|^2 + eps^2,
// alpha = (d . w) / s and beta = (w . w + d . u) / s + alpha^2,
//   P0 = s^-3/2 d,  P1 = s^-3/2 w - 3 alpha P0,  P2 = s^-3/2 u - 6 alpha P1 - 3 beta P0;
// a_i, jerk_i, snap_i gain m_j (P0, P1, P2) and particle j gets -m_i times the
// same (every term changes sign when i and j swap).  Nine components per
// particle; velocities and accelerations staged as two more records.
constexpr int kS64 = 9;
constexpr int kSDiagG = 2;  // lane groups of the snap's block-diagonal kernel (its registers need 512-lane workgroups)

struct S64SArgs {
  const double* x;    // [3][n]
  const double* v;    // [3][n]
  const double* acc;  // [3][n]
  const double* m;    // [n]
  int n, nb, npad, dmax, half, d_lo, T, nparts;
  double eps;
  const double4* rec;   // [npad] staged (x, y, z, m); padding far away and massless
  const double4* recv;  // [npad] staged (vx, vy, vz, 0); padding at rest
  const double4* reca;  // [npad] staged (ax, ay, az, 0); padding zero
  double* pj;           // [D][9][npad] j-side tile sums of the chunk's distances
  double* pi;           // [nparts][9][npad] i-side sums of the chunk's workgroups
};

struct SDSet {
  double x[2], y[2], z[2], mneg[2], vx[2], vy[2], vz[2], ax[2], ay[2], az[2];
};

__device__ __forceinline__ void load_sdset(const S64SArgs& A, int g, int t, SDSet& s) {
  const int n = A.n;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = g * kSI + u * kSL + t;
    if (i < n) {
      s.x[u] = A.x[i]; s.y[u] = A.x[n + i]; s.z[u] = A.x[2 * n + i];
      s.mneg[u] = -A.m[i];
      s.vx[u] = A.v[i]; s.vy[u] = A.v[n + i]; s.vz[u] = A.v[2 * n + i];
      s.ax[u] = A.acc[i]; s.ay[u] = A.acc[n + i]; s.az[u] = A.acc[2 * n + i];
    } else {
      s.x[u] = s.y[u] = s.z[u] = kFarAway;
      s.mneg[u] = 0.0;
      s.vx[u] = s.vy[u] = s.vz[u] = 0.0;
      s.ax[u] = s.ay[u] = s.az[u] = 0.0;
    }
  }
}

// One pair for lane particle u against record (r, vj, aj4): the i-side terms
// are added to p[u] (scale m_j), the j-side ones to b (scale -m_i).  The own
// pair (masked with own) adds nothing: its s^-3/2, alpha and beta are replaced
// by zeros, since without softening they are infinite or NaN.
__device__ __forceinline__ void snap64_pair(const SDSet& s, int u, const double4& r, const double4& vj,
                                            const double4& aj4, double e2, bool own, double (&p)[2][kS64],
                                            double (&b)[kS64]) {
  const double d[3] = {r.x - s.x[u], r.y - s.y[u], r.z - s.z[u]};
  const double w[3] = {vj.x - s.vx[u], vj.y - s.vy[u], vj.z - s.vz[u]};
  const double q[3] = {aj4.x - s.ax[u], aj4.y - s.ay[u], aj4.z - s.az[u]};
  const double r2 = fma(d[2], d[2], fma(d[1], d[1], fma(d[0], d[0], e2)));
  const double ri = rsqrt64(r2);
  const double sinv = ri * ri;
  const double r3 = own ? 0.0 : sinv * ri;
  const double alpha = own ? 0.0 : fma(d[2], w[2], fma(d[1], w[1], d[0] * w[0])) * sinv;
  const double wwdu = fma(d[2], q[2], fma(d[1], q[1], fma(d[0], q[0], fma(w[2], w[2], fma(w[1], w[1], w[0] * w[0])))));
  const double beta = own ? 0.0 : fma(wwdu, sinv, alpha * alpha);
  const double a3 = -3.0 * alpha, a6 = -6.0 * alpha, b3 = -3.0 * beta;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double p0 = r3 * d[c];
    const double p1 = fma(a3, p0, r3 * w[c]);
    const double p2 = fma(a6, p1, fma(b3, p0, r3 * q[c]));
    p[u][c] = fma(r.w, p0, p[u][c]);
    p[u][3 + c] = fma(r.w, p1, p[u][3 + c]);
    p[u][6 + c] = fma(r.w, p2, p[u][6 + c]);
    b[c] = fma(s.mneg[u], p0, b[c]);
    b[3 + c] = fma(s.mneg[u], p1, b[3 + c]);
    b[6 + c] = fma(s.mneg[u], p2, b[6 + c]);
  }
}

template <int K>
__device__ __forceinline__ void sstep64(const SDSet& s, const double4* __restrict__ rowp,
                                        const double4* __restrict__ rowv, const double4* __restrict__ rowa,
                                        double e2, double (&p)[2][kS64], double (&aj)[kS64]) {
  const double4 r = rowp[K];
  const double4 vj = rowv[K];
  const double4 a4 = rowa[K];
  double b[kS64] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  snap64_pair(s, 0, r, vj, a4, e2, false, p, b);
  snap64_pair(s, 1, r, vj, a4, e2, false, p, b);
  // the j met here sits at row position (r + K): its owner is K lanes further on
  if constexpr (K == 0) {
#pragma unroll
    for (int c = 0; c < kS64; ++c) aj[c] += b[c];
  } else {
#pragma unroll
    for (int c = 0; c < kS64; ++c) aj[c] += row_ror64<K>(b[c]);
  }
}

template <int... K>
__device__ __forceinline__ void ssub64(const SDSet& s, const double4* __restrict__ rowp,
                                       const double4* __restrict__ rowv, const double4* __restrict__ rowa, double e2,
                                       double (&p)[2][kS64], double (&aj)[kS64], std::integer_sequence<int, K...>) {
  (sstep64<K>(s, rowp, rowv, rowa, e2, p, aj), ...);
}

__global__ void ssym64_stage_kernel(S64SArgs A, double4* __restrict__ rec, double4* __restrict__ recv,
                                    double4* __restrict__ reca) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= A.npad) return;
  const int n = A.n;
  const bool in = j < n;
  rec[j] = in ? make_double4(A.x[j], A.x[n + j], A.x[2 * n + j], A.m[j])
              : make_double4(kFarAway, kFarAway, kFarAway, 0.0);
  recv[j] = in ? make_double4(A.v[j], A.v[n + j], A.v[2 * n + j], 0.0) : make_double4(0.0, 0.0, 0.0, 0.0);
  reca[j] = in ? make_double4(A.acc[j], A.acc[n + j], A.acc[2 * n + j], 0.0) : make_double4(0.0, 0.0, 0.0, 0.0);
}

// Grid: nb * nparts workgroups; workgroup (g, part) takes tiles kbeg ..
// kbeg + T - 1 of the chunk (fewer where g's ring ends), as sym64_kernel.
__global__ __launch_bounds__(kSL, 2) void ssym64_kernel(S64SArgs A) {
  __shared__ double4 s_rec[2][4][2 * kSR];  // each sub-block twice in a row
  __shared__ double4 s_v[2][4][2 * kSR];    // velocities, laid out as s_rec
  __shared__ double4 s_a[2][4][2 * kSR];    // accelerations, laid out as s_rec
  __shared__ double s_part[kS64][kSW][kST];
  __shared__ double s_acc_lo[2 * kS64][kSL];  // the lo halves of the i-side (hi, lo) sums

  const int t = threadIdx.x;
  const int rl = t & (kSR - 1);
  const int wave = t / 64;
  const int lid = xcd_local_index(blockIdx.x, gridDim.x);
  const int g = lid % A.nb;
  const int part = lid / A.nb;
  const int kbeg = part * A.T;
  const int rend = (A.half && g >= A.nb / 2) ? A.dmax : A.dmax + 1;  // g's ring ends before this distance
  const int ntiles = max(0, min(kbeg + A.T, (rend - A.d_lo) * kSTiles) - kbeg);
  const double e2 = A.eps * A.eps;

  SDSet s;
  load_sdset(A, g, t, s);
  double h[2][kS64];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < kS64; ++c) h[u][c] = 0.0;
#pragma unroll
  for (int c = 0; c < 2 * kS64; ++c) s_acc_lo[c][t] = 0.0;
  const int xor32 = ((t & 63) ^ 32) * 4;

  // the last wave copies tile k into LDS buffer b, as in sym64_kernel
  const unsigned lane_off = (unsigned)((((t & 63) >> 1) & (kSR - 1)) * sizeof(double4) + (t & 1) * 16);
  auto stage = [&](int k, int b) {
    const int rec0 = __builtin_amdgcn_readfirstlane(((g + A.d_lo + (kbeg + k) / kSTiles) % A.nb) * kSI + ((kbeg + k) % kSTiles) * kST);
    const size_t off = (size_t)rec0 * sizeof(double4);
    const char* base = reinterpret_cast<const char*>(A.rec) + off;
    const char* vbase = reinterpret_cast<const char*>(A.recv) + off;
    const char* abase = reinterpret_cast<const char*>(A.reca) + off;
    unsigned o = lane_off;
    asm volatile("" : "+v"(o));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      __builtin_amdgcn_global_load_lds(base + q * kSR * sizeof(double4) + o, (lds_ptr)&s_rec[b][q][0], 16, 0, 0);
      __builtin_amdgcn_global_load_lds(vbase + q * kSR * sizeof(double4) + o, (lds_ptr)&s_v[b][q][0], 16, 0, 0);
      __builtin_amdgcn_global_load_lds(abase + q * kSR * sizeof(double4) + o, (lds_ptr)&s_a[b][q][0], 16, 0, 0);
    }
  };

  if (ntiles > 0 && t >= 3 * 64) {
    stage(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();

  for (int k = 0; k < ntiles; ++k) {
    const int b = k & 1;
    const int d = A.d_lo + (kbeg + k) / kSTiles;
    const int tt = (kbeg + k) % kSTiles;
    if (t >= 3 * 64 && k + 1 < ntiles) stage(k + 1, b ^ 1);
    double p[2][kS64];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kS64; ++c) p[u][c] = 0.0;
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      double aj[kS64] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      ssub64(s, &s_rec[b][q][rl], &s_v[b][q][rl], &s_a[b][q][rl], e2, p, aj, std::make_integer_sequence<int, kSR>{});
      // the four rows' sums of the same 16 j
#pragma unroll
      for (int c = 0; c < kS64; ++c) {
        aj[c] += swizzle64_xor16(aj[c]);
        aj[c] += bpermute64(xor32, aj[c]);
        s_part[c][wave][q * kSR + rl] = aj[c];
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kS64; ++c) fold(h[u][c], s_acc_lo[u * kS64 + c][t], p[u][c]);
    __syncthreads();
    // the tile's j-side sums: the 4 wave sums of each j, in wave order (9 x 64
    // of them over 256 lanes)
    for (int e = t; e < kS64 * kST; e += kSL) {
      const int c = e / kST, jl = e % kST;
      double v = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < kSW; ++w2) v += s_part[c][w2][jl];
      const int J = (g + d) % A.nb;
      A.pj[((size_t)(d - A.d_lo) * kS64 + c) * A.npad + (size_t)J * kSI + tt * kST + jl] = v;
    }
    if (t >= 3 * 64) __builtin_amdgcn_s_waitcnt(0);  // the next tile's copies have landed in LDS
    __syncthreads();
  }

  double* o = A.pi + (size_t)part * kS64 * A.npad;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const size_t i = (size_t)g * kSI + u * kSL + t;
#pragma unroll
    for (int c = 0; c < kS64; ++c) o[(size_t)c * A.npad + i] = h[u][c] + s_acc_lo[u * kS64 + c][t];
  }
}

// The block with itself (distance 0): the i-side of all ordered pairs inside
// I-block g, own pair masked when asked; the gridDim.y workgroups of a block
// each take a slice of its j and their kSDiagG groups of kSL lanes each a part
// of the slice; group 0 adds the groups' hi + lo in group order into
// pd[slice][9][npad].
template <bool EXCL>
__global__ __launch_bounds__(kSL* kSDiagG) void ssym64_diag_kernel(S64SArgs A, double* __restrict__ pd) {
  __shared__ double4 s_rec[kSI];
  __shared__ double4 s_v[kSI];
  __shared__ double4 s_a[kSI];
  __shared__ double s_part[kSDiagG - 1][kS64][kSI];
  const int t = threadIdx.x % kSL, grp = threadIdx.x / kSL;
  const int g = blockIdx.x;
  const double e2 = A.eps * A.eps;
  const int span = kSI / ((int)gridDim.y * kSDiagG), fl = span < kFold ? span : kFold;
  const int f0 = ((int)blockIdx.y * kSDiagG + grp) * span;
  SDSet s;
  load_sdset(A, g, t, s);
  for (int k = threadIdx.x; k < kSI; k += kSL * kSDiagG) {
    s_rec[k] = A.rec[(size_t)g * kSI + k];
    s_v[k] = A.recv[(size_t)g * kSI + k];
    s_a[k] = A.reca[(size_t)g * kSI + k];
  }
  __syncthreads();
  double h[2][kS64], l[2][kS64];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < kS64; ++c) h[u][c] = l[u][c] = 0.0;
#pragma unroll 1
  for (int f = f0; f < f0 + span; f += fl) {
    double p[2][kS64];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kS64; ++c) p[u][c] = 0.0;
#pragma unroll 1
    for (int j = f; j < f + fl; ++j) {
      const double4 r = s_rec[j];
      const double4 vj = s_v[j];
      const double4 a4 = s_a[j];
      double b[kS64] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // the j side is not needed here
      snap64_pair(s, 0, r, vj, a4, e2, EXCL && j == t, p, b);
      snap64_pair(s, 1, r, vj, a4, e2, EXCL && j == kSL + t, p, b);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kS64; ++c) fold(h[u][c], l[u][c], p[u][c]);
  }
  if (grp > 0) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kS64; ++c) s_part[grp - 1][c][u * kSL + t] = h[u][c] + l[u][c];
  }
  __syncthreads();
  if (grp > 0) return;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int k = u * kSL + t;
    const size_t i = (size_t)g * kSI + k;
    double* const pds = pd + (size_t)blockIdx.y * kS64 * A.npad;
#pragma unroll
    for (int c = 0; c < kS64; ++c) {
      double v = h[u][c] + l[u][c];
#pragma unroll
      for (int q = 0; q < kSDiagG - 1; ++q) v += s_part[q][c][k];
      pds[(size_t)c * A.npad + i] = v;
    }
  }
}

}  // namespace

int launch_sym_accel64(int64_t n, const double* x, const double* m, double* a, double G, double eps, bool excl,
                       const PairConfig& cfg, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  int nb, T, D;
  // per particle: FP64 j-side slot sums per distance, FP64 i-side sums per workgroup,
  // FP64 block-diagonal sums (in pds slices) and one staged double4 record
  const int pds = diag_slices((int)((n + kSI - 1) / kSI));
  sym_plan(n, cfg.launches, 3 * sizeof(double), 3 * sizeof(double), 3 * sizeof(double),
           pds * 3 * (int)sizeof(double) + (int)sizeof(double4), cfg.scratch ? cfg.scratch_bytes : SIZE_MAX, &nb, &T,
           &D);
  const int dmax = nb / 2;
  const int half = (nb % 2 == 0) ? 1 : 0;
  const int64_t npad = (int64_t)nb * kSI;
  const int nparts = D * kSTiles / T;
  const int nchunks = dmax > 0 ? (dmax + D - 1) / D : 0;
  // with two half-ring chunks or more and the library's own workspace, the
  // block-diagonal kernel and the slot sums run on the side stream, and the
  // slots come twice, so that a chunk's pair kernel need not wait for the
  // previous chunk's slot sum (with one chunk the cross-stream waits cost more
  // than the overlap gains: 15 us of a 0.15 ms evaluation at 16384)
  std::unique_lock<std::mutex> side_lk;
  SideStream* side = nchunks >= 2 && !cfg.scratch ? acquire_side_stream(s, side_lk) : nullptr;
  const int nbuf = side ? 2 : 1;
  int st = NBODY_OK;
  const size_t pj_bytes = sizeof(double) * 3 * (size_t)npad * D;
  const size_t pi_bytes = sizeof(double) * 3 * (size_t)npad * nparts;
  const size_t pd_bytes = sizeof(double) * 3 * (size_t)npad * pds;
  const size_t rec_bytes = sizeof(double4) * (size_t)npad;
  const size_t buf_bytes = pj_bytes + pi_bytes;  // one slot set
  char* ws = static_cast<char*>(pair_scratch(cfg, nbuf * buf_bytes + pd_bytes + rec_bytes, &st));
  if (!ws) return st;
  S64Args A;
  A.x = x; A.m = m; A.n = (int)n; A.nb = nb; A.npad = (int)npad; A.dmax = dmax; A.half = half;
  A.T = T; A.nparts = nparts; A.eps = eps; A.d_lo = 1;
  auto slots = [&](int b, S64Args& Q) {
    Q.pj = reinterpret_cast<double*>(ws + (size_t)b * buf_bytes);
    Q.pi = reinterpret_cast<double*>(ws + (size_t)b * buf_bytes + pj_bytes);
  };
  slots(0, A);
  double* pd = reinterpret_cast<double*>(ws + nbuf * buf_bytes);
  double4* rec = reinterpret_cast<double4*>(ws + nbuf * buf_bytes + pd_bytes);
  A.rec = rec;
  sym64_stage_kernel<<<(unsigned)((npad + 255) / 256), 256, 0, s>>>(A, rec);
  NB_LAUNCH_CHECK("sym64_stage_kernel");
  const dim3 dg((unsigned)nb, (unsigned)pds);
  auto diag = [&](hipStream_t ds) -> int {
    if (excl) sym64_diag_kernel<true><<<dg, kSL * kDiagG, 0, ds>>>(A, pd);
    else sym64_diag_kernel<false><<<dg, kSL * kDiagG, 0, ds>>>(A, pd);
    NB_LAUNCH_CHECK("sym64_diag_kernel");
    return NBODY_OK;
  };
  const dim3 rg((unsigned)((n + 255) / 256), 3);
  if (dmax == 0) {
    if ((st = diag(s))) return st;
    sym_reduce_kernel<3, double><<<rg, 256, 0, s>>>((int)n, (int)npad, nb, dmax, half, 1, 0, 0, A.pj, A.pi, pd, a,
                                                    nullptr, G, 1, 1, nullptr, nullptr, nullptr, nullptr, pds);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  }
  auto pair = [&](int c, int b) -> int {
    S64Args B = A;
    slots(b, B);
    B.d_lo = 1 + c * D;
    sym64_kernel<<<(unsigned)nb * (unsigned)nparts, kSL, 0, s>>>(B);
    NB_LAUNCH_CHECK("sym64_kernel");
    return NBODY_OK;
  };
  auto sum = [&](int c, int b, hipStream_t rs) -> int {
    S64Args B = A;
    slots(b, B);
    sym_reduce_kernel<3, double><<<rg, 256, 0, rs>>>((int)n, (int)npad, nb, dmax, half, 1 + c * D, D, nparts, B.pj, B.pi,
                                                     pd, a, nullptr, G, c == 0, c == nchunks - 1, nullptr, nullptr,
                                                     nullptr, nullptr, pds);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  };
  return run_sym_chunks(side, s, nchunks, nbuf, diag, pair, sum);
}

int launch_sym_vjp64(int64_t n, const double* x, const double* m, const double* w, double* gx, double* gm, double G,
                     double eps, const PairConfig& cfg, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  int nb, T, D;
  // per particle: FP64 j-side slot sums per distance and i-side sums per
  // workgroup (4 components), block-diagonal sums (pds slices), two records
  const int pds = diag_slices((int)((n + kSI - 1) / kSI));
  sym_plan(n, cfg.launches, kV64 * sizeof(double), kV64 * sizeof(double), kV64 * sizeof(double),
           pds * kV64 * (int)sizeof(double) + 2 * (int)sizeof(double4), cfg.scratch ? cfg.scratch_bytes : SIZE_MAX, &nb,
           &T, &D);
  const int dmax = nb / 2;
  const int half = (nb % 2 == 0) ? 1 : 0;
  const int64_t npad = (int64_t)nb * kSI;
  const int nparts = D * kSTiles / T;
  const int nchunks = dmax > 0 ? (dmax + D - 1) / D : 0;
  std::unique_lock<std::mutex> side_lk;
  SideStream* side = nchunks >= 2 && !cfg.scratch ? acquire_side_stream(s, side_lk) : nullptr;
  const int nbuf = side ? 2 : 1;
  int st = NBODY_OK;
  const size_t pj_bytes = sizeof(double) * kV64 * (size_t)npad * D;
  const size_t pi_bytes = sizeof(double) * kV64 * (size_t)npad * nparts;
  const size_t pd_bytes = sizeof(double) * kV64 * (size_t)npad * pds;
  const size_t rec_bytes = sizeof(double4) * (size_t)npad;
  const size_t buf_bytes = pj_bytes + pi_bytes;  // one slot set
  char* ws = static_cast<char*>(pair_scratch(cfg, nbuf * buf_bytes + pd_bytes + 2 * rec_bytes, &st));
  if (!ws) return st;
  V64Args A;
  A.x = x; A.m = m; A.w = w; A.n = (int)n; A.nb = nb; A.npad = (int)npad; A.dmax = dmax; A.half = half;
  A.T = T; A.nparts = nparts; A.eps = eps; A.d_lo = 1;
  auto slots = [&](int b, V64Args& Q) {
    Q.pj = reinterpret_cast<double*>(ws + (size_t)b * buf_bytes);
    Q.pi = reinterpret_cast<double*>(ws + (size_t)b * buf_bytes + pj_bytes);
  };
  slots(0, A);
  double* pd = reinterpret_cast<double*>(ws + nbuf * buf_bytes);
  double4* rec = reinterpret_cast<double4*>(ws + nbuf * buf_bytes + pd_bytes);
  double4* recw = rec + npad;
  A.rec = rec;
  A.recw = recw;
  vsym64_stage_kernel<<<(unsigned)((npad + 255) / 256), 256, 0, s>>>(A, rec, recw);
  NB_LAUNCH_CHECK("vsym64_stage_kernel");
  const dim3 dg((unsigned)nb, (unsigned)pds);
  auto diag = [&](hipStream_t ds) -> int {
    vsym64_diag_kernel<<<dg, kSL * kDiagG, 0, ds>>>(A, pd);
    NB_LAUNCH_CHECK("vsym64_diag_kernel");
    return NBODY_OK;
  };
  const dim3 rg((unsigned)((n + 255) / 256), kV64);
  if (dmax == 0) {
    if ((st = diag(s))) return st;
    sym_reduce_kernel<kV64, double><<<rg, 256, 0, s>>>((int)n, (int)npad, nb, dmax, half, 1, 0, 0, A.pj, A.pi, pd, gx,
                                                       gm, G, 1, 1, nullptr, nullptr, nullptr, nullptr, pds);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  }
  auto pair = [&](int c, int b) -> int {
    V64Args B = A;
    slots(b, B);
    B.d_lo = 1 + c * D;
    vsym64_kernel<<<(unsigned)nb * (unsigned)nparts, kSL, 0, s>>>(B);
    NB_LAUNCH_CHECK("vsym64_kernel");
    return NBODY_OK;
  };
  auto sum = [&](int c, int b, hipStream_t rs) -> int {
    V64Args B = A;
    slots(b, B);
    sym_reduce_kernel<kV64, double><<<rg, 256, 0, rs>>>((int)n, (int)npad, nb, dmax, half, 1 + c * D, D, nparts, B.pj,
                                                        B.pi, pd, gx, gm, G, c == 0, c == nchunks - 1, nullptr, nullptr,
                                                        nullptr, nullptr, pds);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  };
  return run_sym_chunks(side, s, nchunks, nbuf, diag, pair, sum);
}


int launch_sym_jerk64(int64_t n, const double* x, const double* v, const double* m, double* a, double* jk, double G,
                      double eps, bool excl, const PairConfig& cfg, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  int nb, T, D;
  // per particle: FP64 j-side slot sums per distance and i-side sums per
  // workgroup (6 components), block-diagonal sums (pds slices), two records
  const int pds = diag_slices((int)((n + kSI - 1) / kSI));
  sym_plan(n, cfg.launches, kJ64 * sizeof(double), kJ64 * sizeof(double), kJ64 * sizeof(double),
           pds * kJ64 * (int)sizeof(double) + 2 * (int)sizeof(double4), cfg.scratch ? cfg.scratch_bytes : SIZE_MAX, &nb,
           &T, &D);
  const int dmax = nb / 2;
  const int half = (nb % 2 == 0) ? 1 : 0;
  const int64_t npad = (int64_t)nb * kSI;
  const int nparts = D * kSTiles / T;
  const int nchunks = dmax > 0 ? (dmax + D - 1) / D : 0;
  std::unique_lock<std::mutex> side_lk;
  SideStream* side = nchunks >= 2 && !cfg.scratch ? acquire_side_stream(s, side_lk) : nullptr;
  const int nbuf = side ? 2 : 1;
  int st = NBODY_OK;
  const size_t pj_bytes = sizeof(double) * kJ64 * (size_t)npad * D;
  const size_t pi_bytes = sizeof(double) * kJ64 * (size_t)npad * nparts;
  const size_t pd_bytes = sizeof(double) * kJ64 * (size_t)npad * pds;
  const size_t rec_bytes = sizeof(double4) * (size_t)npad;
  const size_t buf_bytes = pj_bytes + pi_bytes;  // one slot set
  char* ws = static_cast<char*>(pair_scratch(cfg, nbuf * buf_bytes + pd_bytes + 2 * rec_bytes, &st));
  if (!ws) return st;
  J64Args A;
  A.x = x; A.v = v; A.m = m; A.n = (int)n; A.nb = nb; A.npad = (int)npad; A.dmax = dmax; A.half = half;
  A.T = T; A.nparts = nparts; A.eps = eps; A.d_lo = 1;
  auto slots = [&](int b, J64Args& Q) {
    Q.pj = reinterpret_cast<double*>(ws + (size_t)b * buf_bytes);
    Q.pi = reinterpret_cast<double*>(ws + (size_t)b * buf_bytes + pj_bytes);
  };
  slots(0, A);
  double* pd = reinterpret_cast<double*>(ws + nbuf * buf_bytes);
  double4* rec = reinterpret_cast<double4*>(ws + nbuf * buf_bytes + pd_bytes);
  double4* recv = rec + npad;
  A.rec = rec;
  A.recv = recv;
  jsym64_stage_kernel<<<(unsigned)((npad + 255) / 256), 256, 0, s>>>(A, rec, recv);
  NB_LAUNCH_CHECK("jsym64_stage_kernel");
  const dim3 dg((unsigned)nb, (unsigned)pds);
  auto diag = [&](hipStream_t ds) -> int {
    if (excl) jsym64_diag_kernel<true><<<dg, kSL * kDiagG, 0, ds>>>(A, pd);
    else jsym64_diag_kernel<false><<<dg, kSL * kDiagG, 0, ds>>>(A, pd);
    NB_LAUNCH_CHECK("jsym64_diag_kernel");
    return NBODY_OK;
  };
  const dim3 rg((unsigned)((n + 255) / 256), kJ64);
  if (dmax == 0) {
    if ((st = diag(s))) return st;
    sym_reduce_kernel<kJ64, double><<<rg, 256, 0, s>>>((int)n, (int)npad, nb, dmax, half, 1, 0, 0, A.pj, A.pi, pd, a,
                                                       jk, G, 1, 1, nullptr, nullptr, nullptr, nullptr, pds);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  }
  auto pair = [&](int c, int b) -> int {
    J64Args B = A;
    slots(b, B);
    B.d_lo = 1 + c * D;
    jsym64_kernel<<<(unsigned)nb * (unsigned)nparts, kSL, 0, s>>>(B);
    NB_LAUNCH_CHECK("jsym64_kernel");
    return NBODY_OK;
  };
  auto sum = [&](int c, int b, hipStream_t rs) -> int {
    J64Args B = A;
    slots(b, B);
    sym_reduce_kernel<kJ64, double><<<rg, 256, 0, rs>>>((int)n, (int)npad, nb, dmax, half, 1 + c * D, D, nparts, B.pj,
                                                        B.pi, pd, a, jk, G, c == 0, c == nchunks - 1, nullptr, nullptr,
                                                        nullptr, nullptr, pds);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  };
  return run_sym_chunks(side, s, nchunks, nbuf, diag, pair, sum);
}


int launch_sym_snap64(int64_t n, const double* x, const double* v, const double* acc, const double* m, double* a,
                      double* jk, double* sn, double G, double eps, bool excl, const PairConfig& cfg, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  int nb, T, D;
  // per particle: FP64 j-side slot sums per distance and i-side sums per
  // workgroup (9 components), block-diagonal sums (pds slices), three records
  const int pds = diag_slices((int)((n + kSI - 1) / kSI));
  sym_plan(n, cfg.launches, kS64 * sizeof(double), kS64 * sizeof(double), kS64 * sizeof(double),
           pds * kS64 * (int)sizeof(double) + 3 * (int)sizeof(double4), cfg.scratch ? cfg.scratch_bytes : SIZE_MAX, &nb,
           &T, &D);
  const int dmax = nb / 2;
  const int half = (nb % 2 == 0) ? 1 : 0;
  const int64_t npad = (int64_t)nb * kSI;
  const int nparts = D * kSTiles / T;
  const int nchunks = dmax > 0 ? (dmax + D - 1) / D : 0;
  std::unique_lock<std::mutex> side_lk;
  SideStream* side = nchunks >= 2 && !cfg.scratch ? acquire_side_stream(s, side_lk) : nullptr;
  const int nbuf = side ? 2 : 1;
  int st = NBODY_OK;
  const size_t pj_bytes = sizeof(double) * kS64 * (size_t)npad * D;
  const size_t pi_bytes = sizeof(double) * kS64 * (size_t)npad * nparts;
  const size_t pd_bytes = sizeof(double) * kS64 * (size_t)npad * pds;
  const size_t rec_bytes = sizeof(double4) * (size_t)npad;
  const size_t buf_bytes = pj_bytes + pi_bytes;  // one slot set
  char* ws = static_cast<char*>(pair_scratch(cfg, nbuf * buf_bytes + pd_bytes + 3 * rec_bytes, &st));
  if (!ws) return st;
  S64SArgs A;
  A.x = x; A.v = v; A.acc = acc; A.m = m; A.n = (int)n; A.nb = nb; A.npad = (int)npad; A.dmax = dmax;
  A.half = half; A.T = T; A.nparts = nparts; A.eps = eps; A.d_lo = 1;
  auto slots = [&](int b, S64SArgs& Q) {
    Q.pj = reinterpret_cast<double*>(ws + (size_t)b * buf_bytes);
    Q.pi = reinterpret_cast<double*>(ws + (size_t)b * buf_bytes + pj_bytes);
  };
  slots(0, A);
  double* pd = reinterpret_cast<double*>(ws + nbuf * buf_bytes);
  double4* rec = reinterpret_cast<double4*>(ws + nbuf * buf_bytes + pd_bytes);
  double4* recv = rec + npad;
  double4* reca = recv + npad;
  A.rec = rec;
  A.recv = recv;
  A.reca = reca;
  ssym64_stage_kernel<<<(unsigned)((npad + 255) / 256), 256, 0, s>>>(A, rec, recv, reca);
  NB_LAUNCH_CHECK("ssym64_stage_kernel");
  const dim3 dg((unsigned)nb, (unsigned)pds);
  auto diag = [&](hipStream_t ds) -> int {
    if (excl) ssym64_diag_kernel<true><<<dg, kSL * kSDiagG, 0, ds>>>(A, pd);
    else ssym64_diag_kernel<false><<<dg, kSL * kSDiagG, 0, ds>>>(A, pd);
    NB_LAUNCH_CHECK("ssym64_diag_kernel");
    return NBODY_OK;
  };
  const dim3 rg((unsigned)((n + 255) / 256), kS64);
  if (dmax == 0) {
    if ((st = diag(s))) return st;
    sym_reduce_kernel<kS64, double><<<rg, 256, 0, s>>>((int)n, (int)npad, nb, dmax, half, 1, 0, 0, A.pj, A.pi, pd, a,
                                                       jk, G, 1, 1, nullptr, nullptr, nullptr, nullptr, pds, sn);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  }
  auto pair = [&](int c, int b) -> int {
    S64SArgs B = A;
    slots(b, B);
    B.d_lo = 1 + c * D;
    ssym64_kernel<<<(unsigned)nb * (unsigned)nparts, kSL, 0, s>>>(B);
    NB_LAUNCH_CHECK("ssym64_kernel");
    return NBODY_OK;
  };
  auto sum = [&](int c, int b, hipStream_t rs) -> int {
    S64SArgs B = A;
    slots(b, B);
    sym_reduce_kernel<kS64, double><<<rg, 256, 0, rs>>>((int)n, (int)npad, nb, dmax, half, 1 + c * D, D, nparts, B.pj,
                                                        B.pi, pd, a, jk, G, c == 0, c == nchunks - 1, nullptr, nullptr,
                                                        nullptr, nullptr, pds, sn);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  };
  return run_sym_chunks(side, s, nchunks, nbuf, diag, pair, sum);
}

}  // namespace nb
