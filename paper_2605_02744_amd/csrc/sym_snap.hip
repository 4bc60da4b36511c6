// Symmetric acceleration + jerk + snap (the pair term of a sixth-order
// Hermite evaluation, Sec. 2.1, evaluated once per unordered pair).  Particles
// move along x_k(t) = x_k + v_k t + acc_k t^2 / 2; with d = x_j - x_i,
// w = v_j - v_i, u = acc_j - acc_i, s = |d|^2 + eps^2, alpha = (d . w) / s and
// beta = (w . w + d . u) / s + alpha^2, the pair's terms per unit mass are
//   P0 = s^-3/2 d,  P1 = s^-3/2 w - 3 alpha P0,
//   P2 = s^-3/2 u - 6 alpha P1 - 3 beta P0,
// and a_i, jerk_i, snap_i gain m_j (P0, P1, P2).  When i and j swap, d, w and u
// change sign while alpha and beta do not, so every term changes sign: the
// same evaluation gives a_j, jerk_j, snap_j their -m_i (P0, P1, P2).
// Same layout as the symmetric acceleration (sym_pairs.hip) and the symmetric
// acceleration + jerk (sym_jerk.hip); nine components travel.  FP32C: rounded
// positions with the near-field correction for both sides, velocities and
// accelerations rounded to FP32 as in the ordered kernel.
#include "sym_common.h"

namespace nb {
namespace {

constexpr int kSC = 9;  // components per particle: a (3), jerk (3), snap (3)

struct SSet {
  float x[2], y[2], z[2], mneg[2], vx[2], vy[2], vz[2], ax[2], ay[2], az[2];
};

// The pair's terms per unit mass at displacement d, velocity difference w and
// acceleration difference u: P0, P1, P2 as above, component c at p[3 k + c].
__device__ __forceinline__ void snap_terms(float dx, float dy, float dz, float wx, float wy, float wz, float ux,
                                           float uy, float uz, float e2, float (&p)[kSC]) {
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
  const float ri = rsqrt32(r2);
  const float sinv = ri * ri;
  const float r3 = sinv * ri;
  const float alpha = fmaf(dz, wz, fmaf(dy, wy, dx * wx)) * sinv;
  const float wwdu = fmaf(dz, uz, fmaf(dy, uy, fmaf(dx, ux, fmaf(wz, wz, fmaf(wy, wy, wx * wx)))));
  const float beta = fmaf(wwdu, sinv, alpha * alpha);
  const float a3 = -3.0f * alpha, a6 = -6.0f * alpha, b3 = -3.0f * beta;
  const float d[3] = {dx, dy, dz}, w[3] = {wx, wy, wz}, u[3] = {ux, uy, uz};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    p[c] = r3 * d[c];
    p[3 + c] = fmaf(a3, p[c], r3 * w[c]);
    p[6 + c] = fmaf(a6, p[3 + c], fmaf(b3, p[c], r3 * u[c]));
  }
}

// One step of a sub-block: both i of the lane against record (r + K).
template <int K, bool NEAR>
__device__ __forceinline__ void ssym_step(const SSet& s, const float4* __restrict__ rowp,
                                          const float4* __restrict__ rowv, const float4* __restrict__ rowa, float e2,
                                          float (&p)[2][kSC], float (&r2min)[2], float (&aj)[kSC]) {
  const float4 r = rowp[K];
  const float4 vj = rowv[K];
  const float4 acj = rowa[K];
  float b[kSC];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const float dx = r.x - s.x[u], dy = r.y - s.y[u], dz = r.z - s.z[u];
    float t[kSC];
    snap_terms(dx, dy, dz, vj.x - s.vx[u], vj.y - s.vy[u], vj.z - s.vz[u], acj.x - s.ax[u], acj.y - s.ay[u],
               acj.z - s.az[u], e2, t);
#pragma unroll
    for (int c = 0; c < kSC; ++c) {
      p[u][c] = fmaf(r.w, t[c], p[u][c]);
      b[c] = u == 0 ? s.mneg[u] * t[c] : fmaf(s.mneg[u], t[c], b[c]);
    }
    if constexpr (NEAR) r2min[u] = fminf(r2min[u], fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2))));
  }
  // the j met here sits at row position (r + K): its owner is K lanes further on
  if constexpr (K == 0) {
#pragma unroll
    for (int c = 0; c < kSC; ++c) aj[c] += b[c];
  } else {
#pragma unroll
    for (int c = 0; c < kSC; ++c) aj[c] += row_ror<K>(b[c]);
  }
}

template <bool NEAR, int... K>
__device__ __forceinline__ void ssym_sub(const SSet& s, const float4* __restrict__ rowp,
                                         const float4* __restrict__ rowv, const float4* __restrict__ rowa, float e2,
                                         float (&p)[2][kSC], float (&r2min)[2], float (&aj)[kSC],
                                         std::integer_sequence<int, K...>) {
  (ssym_step<K, NEAR>(s, rowp, rowv, rowa, e2, p, r2min, aj), ...);
}

// Loads the two i of lane t of I-block g (padding: far away, massless, at
// rest) and their flag radii^2 (PAIR: also covering the j's own radius, as in
// the acceleration; -1 for padding).  The velocities come from A.w, the
// accelerations from A.u.
template <bool PAIR>
__device__ __forceinline__ void load_sset(const SymArgs& A, int g, int t, SSet& s, float (&thr)[2]) {
  const int n = A.n;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = g * kSI + u * kSL + t;
    thr[u] = -1.f;
    if (i < n) {
      const double xa = A.x[i], ya = A.x[n + i], za = A.x[2 * n + i];
      s.x[u] = (float)xa; s.y[u] = (float)ya; s.z[u] = (float)za;
      s.mneg[u] = -(float)A.m[i];
      s.vx[u] = (float)A.w[i]; s.vy[u] = (float)A.w[n + i]; s.vz[u] = (float)A.w[2 * n + i];
      s.ax[u] = (float)A.u[i]; s.ay[u] = (float)A.u[n + i]; s.az[u] = (float)A.u[2 * n + i];
      thr[u] = sym_rc2(xa, ya, za, A.eps, PAIR ? A.fx / (1.0f - A.fx) * 1.0001f : A.fx);
    } else {
      s.x[u] = s.y[u] = s.z[u] = (float)kFarAway;
      s.mneg[u] = 0.f;
      s.vx[u] = s.vy[u] = s.vz[u] = 0.f;
      s.ax[u] = s.ay[u] = s.az[u] = 0.f;
    }
  }
}

// The j-records of all npad particles: (x, y, z, m) rounded to FP32, the
// velocities (rw) and accelerations (ru) rounded to FP32, and the lo parts with
// the repair radius^2 (-1 without the repair); padding past n far away,
// massless, at rest.
template <bool NEAR>
__global__ void ssym_stage_kernel(SymArgs A, float4* __restrict__ rhi, float4* __restrict__ rv,
                                  float4* __restrict__ ra, float4* __restrict__ rlo) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= A.npad) return;
  const int n = A.n;
  float4 hi, vv, aa, lo;
  if (j < n) {
    const double xa = A.x[j], ya = A.x[n + j], za = A.x[2 * n + j];
    hi = make_float4((float)xa, (float)ya, (float)za, (float)A.m[j]);
    vv = make_float4((float)A.w[j], (float)A.w[n + j], (float)A.w[2 * n + j], 0.f);
    aa = make_float4((float)A.u[j], (float)A.u[n + j], (float)A.u[2 * n + j], 0.f);
    lo = make_float4((float)(xa - (double)hi.x), (float)(ya - (double)hi.y), (float)(za - (double)hi.z),
                     NEAR ? sym_rc2(xa, ya, za, A.eps, A.fx) : -1.f);
  } else {
    hi = make_float4((float)kFarAway, (float)kFarAway, (float)kFarAway, 0.f);
    vv = aa = make_float4(0.f, 0.f, 0.f, 0.f);
    lo = make_float4(0.f, 0.f, 0.f, -1.f);
  }
  rhi[j] = hi;
  rv[j] = vv;
  ra[j] = aa;
  rlo[j] = lo;
}

// Near-field correction of one lane's tile (FP32C): every pair of the lane's
// two i with the tile's 64 j closer than the larger repair radius of its two
// particles gets (float-float term - rounded term) added, times m_j to the
// lane's i-side sums p and times -m_i to the wave's j-side sums of the tile
// (part: components kSW * kST apart).  The j are visited in the rotated order
// of the pair loop, so at each step the lanes of a row touch distinct j; the
// four rows of the wave, which share the slots, take turns.
__device__ __forceinline__ void ssym_repair(const SymArgs& A, int g, int t, int rl, float e2, const SSet& s,
                                            float (&p)[2][kSC], const float4* hi, const float4* vr, const float4* ar,
                                            const float4* lo, float* part) {
  const int n = A.n;
  const int wrow = (t & 63) / kSR;
  float rc[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = g * kSI + u * kSL + t;
    rc[u] = i < n ? sym_rc2(A.x[i], A.x[n + i], A.x[2 * n + i], A.eps, A.fx) : -1.f;
  }
  for (int jj = 0; jj < kST; ++jj) {
    const int q = jj / kSR;
    const int jl = q * kSR + ((rl + jj) & (kSR - 1));
    const float4 rh = hi[q * 2 * kSR + (jl % kSR)];
    const float4 vj = vr[q * 2 * kSR + (jl % kSR)];
    const float4 acj = ar[q * 2 * kSR + (jl % kSR)];
    const float4 rlj = lo[jl];
    float c[kSC];
#pragma unroll
    for (int k = 0; k < kSC; ++k) c[k] = 0.f;
    bool any = false;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const float dx = rh.x - s.x[u], dy = rh.y - s.y[u], dz = rh.z - s.z[u];
      const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
      if (rc[u] >= 0.f && r2 < fmaxf(rc[u], rlj.w)) {
        const int i = g * kSI + u * kSL + t;
        const double xa = A.x[i], ya = A.x[n + i], za = A.x[2 * n + i];
        const float ex = dx + (rlj.x - (float)(xa - (double)s.x[u]));
        const float ey = dy + (rlj.y - (float)(ya - (double)s.y[u]));
        const float ez = dz + (rlj.z - (float)(za - (double)s.z[u]));
        const float wx = vj.x - s.vx[u], wy = vj.y - s.vy[u], wz = vj.z - s.vz[u];
        const float ux = acj.x - s.ax[u], uy = acj.y - s.ay[u], uz = acj.z - s.az[u];
        float tr[kSC], tf[kSC];
        snap_terms(dx, dy, dz, wx, wy, wz, ux, uy, uz, e2, tr);
        snap_terms(ex, ey, ez, wx, wy, wz, ux, uy, uz, e2, tf);
#pragma unroll
        for (int k = 0; k < kSC; ++k) {
          const float dk = tf[k] - tr[k];
          p[u][k] = fmaf(rh.w, dk, p[u][k]);
          c[k] = fmaf(s.mneg[u], dk, c[k]);
        }
        any = true;
      }
    }
    for (int r = 0; r < 4; ++r) {
      if (wrow == r && any) {
#pragma unroll
        for (int k = 0; k < kSC; ++k) part[k * kSW * kST + jl] += c[k];
      }
      wave_sync();  // one row's turn ends before the next row reads the sums
    }
  }
}

// Grid: nb * nparts workgroups; workgroup (g, part) takes the tiles
// [part T, (part + 1) T) of I-block g's half ring in this chunk (d >= 1).
template <bool NEAR>
__global__ __launch_bounds__(kSL, 3) void ssym_kernel(SymArgs A) {
  __shared__ float4 s_hi[2][4][2 * kSR];  // (x, y, z, m) hi parts, each sub-block twice
  __shared__ float4 s_v[2][4][2 * kSR];   // velocities, laid out as s_hi
  __shared__ float4 s_a[2][4][2 * kSR];   // accelerations, laid out as s_hi
  __shared__ float4 s_lo[2][kST];         // (x, y, z) lo parts and the repair radius^2 of j
  __shared__ float s_part[kSC][kSW][kST];
  __shared__ float s_acc_lo[2 * kSC][kSL];  // the lo halves of the i-side (hi, lo) sums

  const int t = threadIdx.x;
  const int rl = t & (kSR - 1);
  const int wave = t / 64;
  const int lid = xcd_local_index(blockIdx.x, gridDim.x);
  const int g = lid % A.nb;
  const int part = lid / A.nb;
  // this workgroup's tiles: kbeg, kbeg + 1, ... of the chunk, counted from the
  // first tile of distance d_lo (A.T of them, fewer where g's ring ends)
  const int kbeg = part * A.T;
  const int ntiles = max(0, min(kbeg + A.T, (ring_end(A, g) - A.d_lo) * kSTiles) - kbeg);
  const float e2 = (float)(A.eps * A.eps);

  SSet s;
  float thr[2];
  load_sset<true>(A, g, t, s, thr);
  float h[2][kSC];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < kSC; ++c) h[u][c] = 0.f;
#pragma unroll
  for (int c = 0; c < 2 * kSC; ++c) s_acc_lo[c][t] = 0.f;
  const int xor32 = ((t & 63) ^ 32) * 4;

  // the last wave copies tile k's staged records into LDS buffer b (global to
  // LDS, no registers held); lanes 0-15 and 16-31 fetch the first sub-block of
  // a pair, 32-47 and 48-63 the second, laying each sub-block out twice
  const unsigned lane_hi = (unsigned)((((t & 63) >> 5) * kSR + (t & (kSR - 1))) * sizeof(float4));
  const unsigned lane_lo = (unsigned)((t & 63) * sizeof(float4));
  auto stage = [&](int k, int b) {
    const int rec0 = __builtin_amdgcn_readfirstlane(((g + A.d_lo + (kbeg + k) / kSTiles) % A.nb) * kSI +
                                                    ((kbeg + k) % kSTiles) * kST);
    const size_t base = (size_t)rec0 * sizeof(float4);
    const char* hb = reinterpret_cast<const char*>(A.rhi) + base;
    const char* vb = reinterpret_cast<const char*>(A.rw) + base;
    const char* ab = reinterpret_cast<const char*>(A.ru) + base;
    const char* lb = reinterpret_cast<const char*>(A.rlo) + base;
    // the lane offsets enter each address afresh (hidden from loop-invariant
    // hoisting), so that every copy is scalar base + 32-bit lane offset
    unsigned oh = lane_hi, ol = lane_lo;
    asm volatile("" : "+v"(oh), "+v"(ol));
    __builtin_amdgcn_global_load_lds(hb + oh, (lds_ptr)&s_hi[b][0][0], 16, 0, 0);
    __builtin_amdgcn_global_load_lds(hb + 2 * kSR * sizeof(float4) + oh, (lds_ptr)&s_hi[b][2][0], 16, 0, 0);
    __builtin_amdgcn_global_load_lds(vb + oh, (lds_ptr)&s_v[b][0][0], 16, 0, 0);
    __builtin_amdgcn_global_load_lds(vb + 2 * kSR * sizeof(float4) + oh, (lds_ptr)&s_v[b][2][0], 16, 0, 0);
    __builtin_amdgcn_global_load_lds(ab + oh, (lds_ptr)&s_a[b][0][0], 16, 0, 0);
    __builtin_amdgcn_global_load_lds(ab + 2 * kSR * sizeof(float4) + oh, (lds_ptr)&s_a[b][2][0], 16, 0, 0);
    __builtin_amdgcn_global_load_lds(lb + ol, (lds_ptr)&s_lo[b][0], 16, 0, 0);
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
    float p[2][kSC];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kSC; ++c) p[u][c] = 0.f;
    float r2min[2] = {3.0e38f, 3.0e38f};
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      float aj[kSC];
#pragma unroll
      for (int c = 0; c < kSC; ++c) aj[c] = 0.f;
      ssym_sub<NEAR>(s, &s_hi[b][q][rl], &s_v[b][q][rl], &s_a[b][q][rl], e2, p, r2min, aj,
                     std::make_integer_sequence<int, kSR>{});
      // the four rows' sums of the same 16 j, as in the acceleration
#pragma unroll
      for (int c = 0; c < kSC; ++c) {
        aj[c] += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(aj[c]), 0x401F));
        aj[c] += __int_as_float(__builtin_amdgcn_ds_bpermute(xor32, __float_as_int(aj[c])));
        s_part[c][wave][q * kSR + rl] = aj[c];
      }
    }
    if constexpr (NEAR) {
      if (r2min[0] < thr[0] || r2min[1] < thr[1])
        ssym_repair(A, g, t, rl, e2, s, p, &s_hi[b][0][0], &s_v[b][0][0], &s_a[b][0][0], &s_lo[b][0],
                    &s_part[0][wave][0]);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kSC; ++c) fold(h[u][c], s_acc_lo[u * kSC + c][t], p[u][c]);
    __syncthreads();
    {
      // the tile's j-side sums: the 4 wave sums of each j, in wave order; the
      // nine components of 64 j take the 256 lanes' three passes
      const int J = (g + d) % A.nb;
      for (int e = t; e < kSC * kST; e += kSL) {
        const int c = e / kST, jl = e % kST;
        float v = 0.f;
#pragma unroll
        for (int w2 = 0; w2 < kSW; ++w2) v += s_part[c][w2][jl];
        A.pj[((size_t)(d - A.d_lo) * kSC + c) * A.npad + (size_t)J * kSI + tt * kST + jl] = v;
      }
    }
    if (t >= 3 * 64) __builtin_amdgcn_s_waitcnt(0);  // the next tile's copies have landed in LDS
    __syncthreads();
  }

  // the i-side sums of this workgroup
  double* o = A.pi + (size_t)part * kSC * A.npad;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const size_t i = (size_t)g * kSI + u * kSL + t;
#pragma unroll
    for (int c = 0; c < kSC; ++c) o[(size_t)c * A.npad + i] = (double)h[u][c] + (double)s_acc_lo[u * kSC + c][t];
  }
}

// The block with itself (distance 0): the i-side of all ordered pairs inside
// I-block g, record broadcast to every lane, with the near-field correction of
// the ordered kernel (pairs closer than particle i's repair radius).  The own
// pair is left out (its terms are zero, and without softening undefined).
// The gridDim.y workgroups of a block each take a slice of its j, and their
// kDiagG groups of kSL lanes each a part of the slice; group 0 adds the
// groups' hi + lo in group order into pd[slice][9][npad].
template <bool NEAR>
__global__ __launch_bounds__(kSL* kDiagG) void ssym_diag_kernel(SymArgs A, double* __restrict__ pd) {
  __shared__ float4 s_hi[kSI];
  __shared__ float4 s_v[kSI];
  __shared__ float4 s_a[kSI];
  __shared__ float4 s_lo[kSI];
  __shared__ double s_part[kDiagG - 1][kSC][kSI];
  const int t = threadIdx.x % kSL, grp = threadIdx.x / kSL;
  const int g = blockIdx.x;
  const float e2 = (float)(A.eps * A.eps);
  const int span = kSI / ((int)gridDim.y * kDiagG), fl = span < kFold ? span : kFold;
  const int f0 = ((int)blockIdx.y * kDiagG + grp) * span;
  SSet s;
  float thr[2];
  load_sset<false>(A, g, t, s, thr);
  for (int k = threadIdx.x; k < kSI; k += kSL * kDiagG) {
    const size_t j = (size_t)g * kSI + k;
    s_hi[k] = A.rhi[j];
    s_v[k] = A.rw[j];
    s_a[k] = A.ru[j];
    s_lo[k] = A.rlo[j];
  }
  __syncthreads();
  float h[2][kSC], l[2][kSC];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < kSC; ++c) h[u][c] = l[u][c] = 0.f;
#pragma unroll 1
  for (int f = f0; f < f0 + span; f += fl) {
    float p[2][kSC];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kSC; ++c) p[u][c] = 0.f;
    float r2min[2] = {3.0e38f, 3.0e38f};
#pragma unroll 4
    for (int j = f; j < f + fl; ++j) {
      const float4 r = s_hi[j];
      const float4 vj = s_v[j];
      const float4 acj = s_a[j];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const float dx = r.x - s.x[u], dy = r.y - s.y[u], dz = r.z - s.z[u];
        float tt[kSC];
        snap_terms(dx, dy, dz, vj.x - s.vx[u], vj.y - s.vy[u], vj.z - s.vz[u], acj.x - s.ax[u], acj.y - s.ay[u],
                   acj.z - s.az[u], e2, tt);
        const bool self = j == u * kSL + t;
#pragma unroll
        for (int c = 0; c < kSC; ++c) p[u][c] = fmaf(self ? 0.f : r.w, self ? 0.f : tt[c], p[u][c]);
        if constexpr (NEAR) r2min[u] = fminf(r2min[u], self ? 3.0e38f : fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2))));
      }
    }
    if constexpr (NEAR) {
      if (r2min[0] < thr[0] || r2min[1] < thr[1]) {
        for (int j = f; j < f + fl; ++j) {
          const float4 rh = s_hi[j];
          const float4 vj = s_v[j];
          const float4 acj = s_a[j];
          const float4 lo = s_lo[j];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const float dx = rh.x - s.x[u], dy = rh.y - s.y[u], dz = rh.z - s.z[u];
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
            const float4 li = s_lo[u * kSL + t];
            if (li.w >= 0.f && r2 < li.w && j != u * kSL + t) {
              const float wx = vj.x - s.vx[u], wy = vj.y - s.vy[u], wz = vj.z - s.vz[u];
              const float ux = acj.x - s.ax[u], uy = acj.y - s.ay[u], uz = acj.z - s.az[u];
              float tr[kSC], tf[kSC];
              snap_terms(dx, dy, dz, wx, wy, wz, ux, uy, uz, e2, tr);
              snap_terms(dx + (lo.x - li.x), dy + (lo.y - li.y), dz + (lo.z - li.z), wx, wy, wz, ux, uy, uz, e2, tf);
#pragma unroll
              for (int c = 0; c < kSC; ++c) p[u][c] = fmaf(rh.w, tf[c] - tr[c], p[u][c]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kSC; ++c) fold(h[u][c], l[u][c], p[u][c]);
  }
  if (grp > 0) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kSC; ++c) s_part[grp - 1][c][u * kSL + t] = (double)h[u][c] + (double)l[u][c];
  }
  __syncthreads();
  if (grp > 0) return;
  double* const pds = pd + (size_t)blockIdx.y * kSC * A.npad;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int k = u * kSL + t;
    const size_t i = (size_t)g * kSI + k;
#pragma unroll
    for (int c = 0; c < kSC; ++c) {
      double v = (double)h[u][c] + (double)l[u][c];
#pragma unroll
      for (int q = 0; q < kDiagG - 1; ++q) v += s_part[q][c][k];
      pds[(size_t)c * A.npad + i] = v;
    }
  }
}

}  // namespace

int launch_sym_snap(int64_t n, const double* x, const double* v, const double* acc, const double* m, double* a,
                    double* jk, double* sn, double G, double eps, int precision, bool excl, const PairConfig& cfg,
                    hipStream_t s) {
  if (n == 0) return NBODY_OK;
  if (precision != kFP32C && precision != kFP32)
    return set_error(NBODY_EUNSUPPORTED, "symmetric acceleration + jerk + snap kernel: FP32C and FP32 only");
  if (n > (int64_t(1) << 30)) return set_error(NBODY_EINVAL, "symmetric acceleration + jerk + snap kernel: n too large");
  int nb, T, D;
  // per particle: FP32 j-side slot sums per distance, FP64 i-side sums per workgroup,
  // FP64 block-diagonal sums (in pds slices) and four staged float4 records
  const int pds = diag_slices((int)((n + kSI - 1) / kSI));
  sym_plan(n, cfg.launches, kSC * sizeof(float), kSC * sizeof(float), kSC * sizeof(double),
           pds * kSC * (int)sizeof(double) + 4 * (int)sizeof(float4), cfg.scratch ? cfg.scratch_bytes : SIZE_MAX, &nb,
           &T, &D);
  const int dmax = nb / 2;
  const int half = (nb % 2 == 0) ? 1 : 0;
  const int64_t npad = (int64_t)nb * kSI;
  const int nparts = D * kSTiles / T;
  const int nchunks = dmax > 0 ? (dmax + D - 1) / D : 0;
  // with two half-ring chunks or more and the library's own workspace, the
  // block-diagonal kernel and the slot sums run on the side stream, and the
  // slots come twice (see sym_pairs.hip)
  std::unique_lock<std::mutex> side_lk;
  SideStream* side = nchunks >= 2 && !cfg.scratch ? acquire_side_stream(s, side_lk) : nullptr;
  const int nbuf = side ? 2 : 1;
  int st = NBODY_OK;
  const size_t pj_bytes = sizeof(float) * kSC * (size_t)npad * D;
  const size_t pi_bytes = sizeof(double) * kSC * (size_t)npad * nparts;
  const size_t pd_bytes = sizeof(double) * kSC * (size_t)npad * pds;
  const size_t rec_bytes = sizeof(float4) * (size_t)npad;
  const size_t buf_bytes = pj_bytes + pi_bytes;  // one slot set
  char* ws = static_cast<char*>(pair_scratch(cfg, nbuf * buf_bytes + pd_bytes + 4 * rec_bytes, &st));
  if (!ws) return st;
  SymArgs A;
  A.pe = nullptr;
  A.pw = nullptr;
  A.x = x; A.m = m; A.w = v; A.u = acc; A.n = (int)n; A.nb = nb; A.npad = (int)npad; A.dmax = dmax; A.half = half;
  A.T = T; A.nparts = nparts; A.eps = eps; A.d_lo = 1;
  A.fx = std::max(kNearX, kNearN / std::cbrt((float)n));
  auto slots = [&](int b, SymArgs& Q) {
    Q.pj = reinterpret_cast<float*>(ws + (size_t)b * buf_bytes);
    Q.pi = reinterpret_cast<double*>(ws + (size_t)b * buf_bytes + pj_bytes);
  };
  slots(0, A);
  double* pd = reinterpret_cast<double*>(ws + nbuf * buf_bytes);
  float4* rhi = reinterpret_cast<float4*>(ws + nbuf * buf_bytes + pd_bytes);
  float4* rv = rhi + npad;
  float4* ra = rv + npad;
  float4* rlo = ra + npad;
  A.rhi = rhi;
  A.rw = rv;
  A.ru = ra;
  A.rlo = rlo;
  const bool near = precision == kFP32C;
  const unsigned sg = (unsigned)((npad + 255) / 256);
  if (near) ssym_stage_kernel<true><<<sg, 256, 0, s>>>(A, rhi, rv, ra, rlo);
  else ssym_stage_kernel<false><<<sg, 256, 0, s>>>(A, rhi, rv, ra, rlo);
  NB_LAUNCH_CHECK("ssym_stage_kernel");
  // the own pair is always left out of the block-diagonal sums, so exclude_self needs no variant
  (void)excl;
  const dim3 dg((unsigned)nb, (unsigned)pds);
  auto diag = [&](hipStream_t ds) -> int {
    if (near) ssym_diag_kernel<true><<<dg, kSL * kDiagG, 0, ds>>>(A, pd);
    else ssym_diag_kernel<false><<<dg, kSL * kDiagG, 0, ds>>>(A, pd);
    NB_LAUNCH_CHECK("ssym_diag_kernel");
    return NBODY_OK;
  };
  const dim3 rg((unsigned)((n + 255) / 256), kSC);
  if (dmax == 0) {
    if ((st = diag(s))) return st;
    sym_reduce_kernel<kSC, float><<<rg, 256, 0, s>>>((int)n, (int)npad, nb, dmax, half, 1, 0, 0, A.pj, A.pi, pd, a, jk, G,
                                              1, 1, nullptr, nullptr, nullptr, nullptr, pds, sn);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  }
  auto pair = [&](int c, int b) -> int {
    SymArgs B = A;
    slots(b, B);
    B.d_lo = 1 + c * D;
    const unsigned grid = (unsigned)nb * (unsigned)nparts;
    if (near) ssym_kernel<true><<<grid, kSL, 0, s>>>(B);
    else ssym_kernel<false><<<grid, kSL, 0, s>>>(B);
    NB_LAUNCH_CHECK("ssym_kernel");
    return NBODY_OK;
  };
  auto sum = [&](int c, int b, hipStream_t rs) -> int {
    SymArgs B = A;
    slots(b, B);
    sym_reduce_kernel<kSC, float><<<rg, 256, 0, rs>>>((int)n, (int)npad, nb, dmax, half, 1 + c * D, D, nparts, B.pj, B.pi,
                                               pd, a, jk, G, c == 0, c == nchunks - 1, nullptr, nullptr, nullptr,
                                               nullptr, pds, sn);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  };
  return run_sym_chunks(side, s, nchunks, nbuf, diag, pair, sum);
}

}  // namespace nb
