// Symmetric vector-Jacobian product of the acceleration: every unordered pair
// {k, j} is evaluated once and serves both particles.  With d = x_j - x_k,
// r^2 = |d|^2 + eps^2 and u = m_k w_j - m_j w_k, the pair gives
//   gx_k += r^-3 u - 3 r^-5 (d.u) d,   gm_k -= r^-3 (d . w_j),
// and, since d and u both change sign when k and j swap,
//   gx_j -= r^-3 u - 3 r^-5 (d.u) d,   gm_j += r^-3 (d . w_k).
// Same layout as the symmetric acceleration (sym_pairs.hip): I-blocks of 512
// particles, two per lane; J-blocks streamed through LDS in tiles of 64 as
// sub-blocks of 16 stored twice in a row; the j-side terms of both i of a lane
// summed and moved to the lane owning that j by a DPP row rotation fused into
// the add; wave sums across rows on the LDS pipe; tile sums to per-distance
// slots; a half ring of block pairs in chunks; FP64 slot sums in a fixed
// order.  Four components (gx, gy, gz, gm) travel where the force has three.
// FP32C: rounded positions with the near-field correction for both sides.
#include "sym_common.h"

namespace nb {
namespace {

constexpr int kVC = 4;  // components per particle: gx, gy, gz, gm

struct VSet {
  float x[2], y[2], z[2], m[2], wx[2], wy[2], wz[2];
};

// The pair terms for particle k (mass mk, cotangent wk) and record j at
// displacement d: t = the k-side gx term, qk = the k-side gm term, qj = the
// j-side gm term (the j-side gx term is -t).
__device__ __forceinline__ void vjp_terms(float dx, float dy, float dz, float e2, float mk, float wkx, float wky,
                                          float wkz, float mj, float wjx, float wjy, float wjz, float (&t)[3],
                                          float& qk, float& qj) {
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
  const float ri = rsqrt32(r2);
  const float ri2 = ri * ri;
  const float r3 = ri2 * ri;
  const float c5 = (-3.0f * ri2) * r3;
  const float ux = fmaf(mk, wjx, -(mj * wkx));
  const float uy = fmaf(mk, wjy, -(mj * wky));
  const float uz = fmaf(mk, wjz, -(mj * wkz));
  const float cc = c5 * fmaf(dz, uz, fmaf(dy, uy, dx * ux));
  t[0] = fmaf(cc, dx, r3 * ux);
  t[1] = fmaf(cc, dy, r3 * uy);
  t[2] = fmaf(cc, dz, r3 * uz);
  qk = -r3 * fmaf(dz, wjz, fmaf(dy, wjy, dx * wjx));
  qj = r3 * fmaf(dz, wkz, fmaf(dy, wky, dx * wkx));
}

// One step of a sub-block: both k of the lane against record (r + K).
template <int K, bool NEAR>
__device__ __forceinline__ void vsym_step(const VSet& s, const float4* __restrict__ rowp,
                                          const float4* __restrict__ roww, float e2, float (&p)[2][kVC],
                                          float (&r2min)[2], float (&aj)[kVC]) {
  const float4 r = rowp[K];
  const float4 wj = roww[K];
  float ax = 0.f, ay = 0.f, az = 0.f, am = 0.f;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const float dx = r.x - s.x[u], dy = r.y - s.y[u], dz = r.z - s.z[u];
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
    const float ri = rsqrt32(r2);
    const float ri2 = ri * ri;
    const float r3 = ri2 * ri;
    const float c5 = (-3.0f * ri2) * r3;
    const float ux = fmaf(s.m[u], wj.x, -(r.w * s.wx[u]));
    const float uy = fmaf(s.m[u], wj.y, -(r.w * s.wy[u]));
    const float uz = fmaf(s.m[u], wj.z, -(r.w * s.wz[u]));
    const float cc = c5 * fmaf(dz, uz, fmaf(dy, uy, dx * ux));
    p[u][0] = fmaf(cc, dx, fmaf(r3, ux, p[u][0]));
    p[u][1] = fmaf(cc, dy, fmaf(r3, uy, p[u][1]));
    p[u][2] = fmaf(cc, dz, fmaf(r3, uz, p[u][2]));
    ax = fmaf(-cc, dx, fmaf(-r3, ux, ax));
    ay = fmaf(-cc, dy, fmaf(-r3, uy, ay));
    az = fmaf(-cc, dz, fmaf(-r3, uz, az));
    p[u][3] = fmaf(-r3, fmaf(dz, wj.z, fmaf(dy, wj.y, dx * wj.x)), p[u][3]);
    am = fmaf(r3, fmaf(dz, s.wz[u], fmaf(dy, s.wy[u], dx * s.wx[u])), am);
    if constexpr (NEAR) r2min[u] = fminf(r2min[u], r2);
  }
  // the j met here sits at row position (r + K): its owner is K lanes further on
  if constexpr (K == 0) {
    aj[0] += ax; aj[1] += ay; aj[2] += az; aj[3] += am;
  } else {
    aj[0] += row_ror<K>(ax);
    aj[1] += row_ror<K>(ay);
    aj[2] += row_ror<K>(az);
    aj[3] += row_ror<K>(am);
  }
}

template <bool NEAR, int... K>
__device__ __forceinline__ void vsym_sub(const VSet& s, const float4* __restrict__ rowp,
                                         const float4* __restrict__ roww, float e2, float (&p)[2][kVC],
                                         float (&r2min)[2], float (&aj)[kVC], std::integer_sequence<int, K...>) {
  (vsym_step<K, NEAR>(s, rowp, roww, e2, p, r2min, aj), ...);
}

// Loads the two k of lane t of I-block g (padding: far away, massless, zero
// cotangent) and their flag radii^2 (PAIR: also covering the j's own radius,
// as in the acceleration; -1 for padding).
template <bool PAIR>
__device__ __forceinline__ void load_vset(const SymArgs& A, int g, int t, VSet& s, float (&thr)[2]) {
  const int n = A.n;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = g * kSI + u * kSL + t;
    thr[u] = -1.f;
    if (i < n) {
      const double xa = A.x[i], ya = A.x[n + i], za = A.x[2 * n + i];
      s.x[u] = (float)xa; s.y[u] = (float)ya; s.z[u] = (float)za;
      s.m[u] = (float)A.m[i];
      s.wx[u] = (float)A.w[i]; s.wy[u] = (float)A.w[n + i]; s.wz[u] = (float)A.w[2 * n + i];
      thr[u] = sym_rc2(xa, ya, za, A.eps, PAIR ? A.fx / (1.0f - A.fx) * 1.0001f : A.fx);
    } else {
      s.x[u] = s.y[u] = s.z[u] = (float)kFarAway;
      s.m[u] = 0.f;
      s.wx[u] = s.wy[u] = s.wz[u] = 0.f;
    }
  }
}

template <bool NEAR>
__global__ void vsym_stage_kernel(SymArgs A, float4* __restrict__ rhi, float4* __restrict__ rw,
                                  float4* __restrict__ rlo) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= A.npad) return;
  const int n = A.n;
  float4 hi, wv, lo;
  if (j < n) {
    const double xa = A.x[j], ya = A.x[n + j], za = A.x[2 * n + j];
    hi = make_float4((float)xa, (float)ya, (float)za, (float)A.m[j]);
    wv = make_float4((float)A.w[j], (float)A.w[n + j], (float)A.w[2 * n + j], 0.f);
    lo = make_float4((float)(xa - (double)hi.x), (float)(ya - (double)hi.y), (float)(za - (double)hi.z),
                     NEAR ? sym_rc2(xa, ya, za, A.eps, A.fx) : -1.f);
  } else {
    hi = make_float4((float)kFarAway, (float)kFarAway, (float)kFarAway, 0.f);
    wv = make_float4(0.f, 0.f, 0.f, 0.f);
    lo = make_float4(0.f, 0.f, 0.f, -1.f);
  }
  rhi[j] = hi;
  rw[j] = wv;
  rlo[j] = lo;
}

// Near-field correction of one lane's tile (FP32C): every pair of the lane's
// two k with the tile's 64 j closer than the larger repair radius of its two
// particles gets (float-float term - rounded term) added, to the lane's k-side
// sums p and to the wave's j-side sums of the tile (part: components kSW * kST
// apart).  The j are visited in the rotated order of the pair loop, so at each
// step the lanes of a row touch distinct j; the four rows of the wave, which
// share the slots, take turns.
__device__ __forceinline__ void vsym_repair(const SymArgs& A, int g, int t, int rl, float e2, const VSet& s,
                                            float (&p)[2][kVC], const float4* hi, const float4* wr, const float4* lo,
                                            float* part) {
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
    const float4 wj = wr[q * 2 * kSR + (jl % kSR)];
    const float4 rlj = lo[jl];
    float c[kVC] = {0.f, 0.f, 0.f, 0.f};
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
        float tr[3], tf[3], qkr, qjr, qkf, qjf;
        vjp_terms(dx, dy, dz, e2, s.m[u], s.wx[u], s.wy[u], s.wz[u], rh.w, wj.x, wj.y, wj.z, tr, qkr, qjr);
        vjp_terms(ex, ey, ez, e2, s.m[u], s.wx[u], s.wy[u], s.wz[u], rh.w, wj.x, wj.y, wj.z, tf, qkf, qjf);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          p[u][k] += tf[k] - tr[k];
          c[k] -= tf[k] - tr[k];
        }
        p[u][3] += qkf - qkr;
        c[3] += qjf - qjr;
      }
    }
    for (int r = 0; r < 4; ++r) {
      if (wrow == r && (c[0] != 0.f || c[1] != 0.f || c[2] != 0.f || c[3] != 0.f)) {
#pragma unroll
        for (int k = 0; k < kVC; ++k) part[k * kSW * kST + jl] += c[k];
      }
      wave_sync();  // one row's turn ends before the next row reads the sums
    }
  }
}

// Grid: nb * nparts workgroups; workgroup (g, part) takes the distances
// [d_lo + part L, d_lo + (part + 1) L) of I-block g's half ring (d >= 1).
template <bool NEAR>
__global__ __launch_bounds__(kSL, 6) void vsym_kernel(SymArgs A) {
  __shared__ float4 s_hi[2][4][2 * kSR];  // (x, y, z, m) hi parts, each sub-block twice
  __shared__ float4 s_w[2][4][2 * kSR];   // cotangents, laid out as s_hi
  __shared__ float4 s_lo[2][kST];         // (x, y, z) lo parts and the repair radius^2 of j
  __shared__ float s_part[kVC][kSW][kST];
  __shared__ float s_acc_lo[2 * kVC][kSL];  // the lo halves of the k-side (hi, lo) sums

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

  VSet s;
  float thr[2];
  load_vset<true>(A, g, t, s, thr);
  float h[2][kVC];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < kVC; ++c) h[u][c] = 0.f;
#pragma unroll
  for (int c = 0; c < 2 * kVC; ++c) s_acc_lo[c][t] = 0.f;
  const int xor32 = ((t & 63) ^ 32) * 4;

  // the last wave copies tile k's staged records into LDS buffer b (global to
  // LDS, no registers held); lanes 0-15 and 16-31 fetch the first sub-block of
  // a pair, 32-47 and 48-63 the second, laying each sub-block out twice
  const unsigned lane_hi = (unsigned)((((t & 63) >> 5) * kSR + (t & (kSR - 1))) * sizeof(float4));
  const unsigned lane_lo = (unsigned)((t & 63) * sizeof(float4));
  auto stage = [&](int k, int b) {
    const int rec0 = __builtin_amdgcn_readfirstlane(((g + A.d_lo + (kbeg + k) / kSTiles) % A.nb) * kSI + ((kbeg + k) % kSTiles) * kST);
    const size_t base = (size_t)rec0 * sizeof(float4);
    const char* hb = reinterpret_cast<const char*>(A.rhi) + base;
    const char* wb = reinterpret_cast<const char*>(A.rw) + base;
    const char* lb = reinterpret_cast<const char*>(A.rlo) + base;
    // the lane offsets enter each address afresh (hidden from loop-invariant
    // hoisting), so that every copy is scalar base + 32-bit lane offset
    unsigned oh = lane_hi, ol = lane_lo;
    asm volatile("" : "+v"(oh), "+v"(ol));
    __builtin_amdgcn_global_load_lds(hb + oh, (lds_ptr)&s_hi[b][0][0], 16, 0, 0);
    __builtin_amdgcn_global_load_lds(hb + 2 * kSR * sizeof(float4) + oh, (lds_ptr)&s_hi[b][2][0], 16, 0, 0);
    __builtin_amdgcn_global_load_lds(wb + oh, (lds_ptr)&s_w[b][0][0], 16, 0, 0);
    __builtin_amdgcn_global_load_lds(wb + 2 * kSR * sizeof(float4) + oh, (lds_ptr)&s_w[b][2][0], 16, 0, 0);
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
    float p[2][kVC];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kVC; ++c) p[u][c] = 0.f;
    float r2min[2] = {3.0e38f, 3.0e38f};
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      float aj[kVC] = {0.f, 0.f, 0.f, 0.f};
      vsym_sub<NEAR>(s, &s_hi[b][q][rl], &s_w[b][q][rl], e2, p, r2min, aj, std::make_integer_sequence<int, kSR>{});
      // the four rows' sums of the same 16 j, as in the acceleration
#pragma unroll
      for (int c = 0; c < kVC; ++c) {
        aj[c] += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(aj[c]), 0x401F));
        aj[c] += __int_as_float(__builtin_amdgcn_ds_bpermute(xor32, __float_as_int(aj[c])));
        s_part[c][wave][q * kSR + rl] = aj[c];
      }
    }
    if constexpr (NEAR) {
      if (r2min[0] < thr[0] || r2min[1] < thr[1])
        vsym_repair(A, g, t, rl, e2, s, p, &s_hi[b][0][0], &s_w[b][0][0], &s_lo[b][0], &s_part[0][wave][0]);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kVC; ++c) fold(h[u][c], s_acc_lo[u * kVC + c][t], p[u][c]);
    __syncthreads();
    {
      // the tile's j-side sums: the 4 wave sums of each j, in wave order
      const int c = t / kST, jl = t % kST;
      float v = 0.f;
#pragma unroll
      for (int w2 = 0; w2 < kSW; ++w2) v += s_part[c][w2][jl];
      const int J = (g + d) % A.nb;
      A.pj[((size_t)(d - A.d_lo) * kVC + c) * A.npad + (size_t)J * kSI + tt * kST + jl] = v;
    }
    if (t >= 3 * 64) __builtin_amdgcn_s_waitcnt(0);  // the next tile's copies have landed in LDS
    __syncthreads();
  }

  // the k-side sums of this workgroup
  double* o = A.pi + (size_t)part * kVC * A.npad;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const size_t i = (size_t)g * kSI + u * kSL + t;
#pragma unroll
    for (int c = 0; c < kVC; ++c) o[(size_t)c * A.npad + i] = (double)h[u][c] + (double)s_acc_lo[u * kVC + c][t];
  }
}

// The block with itself (distance 0): the k-side of all ordered pairs inside
// I-block g, record broadcast to every lane, with the near-field correction.
// The own pair is always left out: its term is zero (d = 0 and u = 0), which
// the fused u would not reproduce exactly.  The gridDim.y workgroups of a block
// each take a slice of its j, and their kDiagG groups of kSL lanes each a part
// of the slice; group 0 adds the groups' hi + lo in group order into
// pd[slice][4][npad].
template <bool NEAR>
__global__ __launch_bounds__(kSL* kDiagG) void vsym_diag_kernel(SymArgs A, double* __restrict__ pd) {
  __shared__ float4 s_hi[kSI];
  __shared__ float4 s_w[kSI];
  __shared__ float4 s_lo[kSI];
  __shared__ double s_part[kDiagG - 1][kVC][kSI];
  const int t = threadIdx.x % kSL, grp = threadIdx.x / kSL;
  const int g = blockIdx.x;
  const float e2 = (float)(A.eps * A.eps);
  const int span = kSI / ((int)gridDim.y * kDiagG), fl = span < kFold ? span : kFold;
  const int f0 = ((int)blockIdx.y * kDiagG + grp) * span;
  VSet s;
  float thr[2];
  load_vset<false>(A, g, t, s, thr);
  for (int k = threadIdx.x; k < kSI; k += kSL * kDiagG) {
    const size_t j = (size_t)g * kSI + k;
    s_hi[k] = A.rhi[j];
    s_w[k] = A.rw[j];
    s_lo[k] = A.rlo[j];
  }
  __syncthreads();
  float h[2][kVC], l[2][kVC];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < kVC; ++c) h[u][c] = l[u][c] = 0.f;
#pragma unroll 1
  for (int f = f0; f < f0 + span; f += fl) {
    float p[2][kVC];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kVC; ++c) p[u][c] = 0.f;
    float r2min[2] = {3.0e38f, 3.0e38f};
#pragma unroll 8
    for (int j = f; j < f + fl; ++j) {
      const float4 r = s_hi[j];
      const float4 wj = s_w[j];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const float dx = r.x - s.x[u], dy = r.y - s.y[u], dz = r.z - s.z[u];
        float tk[3], qk, qj;
        vjp_terms(dx, dy, dz, e2, s.m[u], s.wx[u], s.wy[u], s.wz[u], r.w, wj.x, wj.y, wj.z, tk, qk, qj);
        const bool self = j == u * kSL + t;
#pragma unroll
        for (int c = 0; c < 3; ++c) p[u][c] += self ? 0.f : tk[c];
        p[u][3] += self ? 0.f : qk;
        if constexpr (NEAR) r2min[u] = fminf(r2min[u], fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2))));
      }
    }
    if constexpr (NEAR) {
      if (r2min[0] < thr[0] || r2min[1] < thr[1]) {
        for (int j = f; j < f + fl; ++j) {
          const float4 rh = s_hi[j];
          const float4 wj = s_w[j];
          const float4 lo = s_lo[j];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const float dx = rh.x - s.x[u], dy = rh.y - s.y[u], dz = rh.z - s.z[u];
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
            const float rc = s_lo[u * kSL + t].w;
            if (rc >= 0.f && r2 < rc && j != u * kSL + t) {
              const float4 li = s_lo[u * kSL + t];
              float tr[3], tf[3], qkr, qjr, qkf, qjf;
              vjp_terms(dx, dy, dz, e2, s.m[u], s.wx[u], s.wy[u], s.wz[u], rh.w, wj.x, wj.y, wj.z, tr, qkr, qjr);
              vjp_terms(dx + (lo.x - li.x), dy + (lo.y - li.y), dz + (lo.z - li.z), e2, s.m[u], s.wx[u], s.wy[u],
                        s.wz[u], rh.w, wj.x, wj.y, wj.z, tf, qkf, qjf);
#pragma unroll
              for (int c = 0; c < 3; ++c) p[u][c] += tf[c] - tr[c];
              p[u][3] += qkf - qkr;
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kVC; ++c) fold(h[u][c], l[u][c], p[u][c]);
  }
  if (grp > 0) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < kVC; ++c) s_part[grp - 1][c][u * kSL + t] = (double)h[u][c] + (double)l[u][c];
  }
  __syncthreads();
  if (grp > 0) return;
  double* const pds = pd + (size_t)blockIdx.y * kVC * A.npad;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int k = u * kSL + t;
    const size_t i = (size_t)g * kSI + k;
#pragma unroll
    for (int c = 0; c < kVC; ++c) {
      double v = (double)h[u][c] + (double)l[u][c];
#pragma unroll
      for (int q = 0; q < kDiagG - 1; ++q) v += s_part[q][c][k];
      pds[(size_t)c * A.npad + i] = v;
    }
  }
}

}  // namespace

int launch_sym_vjp(int64_t n, const double* x, const double* m, const double* w, double* gx, double* gm, double G,
                   double eps, int precision, bool excl, const PairConfig& cfg, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  if (precision != kFP32C && precision != kFP32)
    return set_error(NBODY_EUNSUPPORTED, "symmetric VJP kernel: FP32C and FP32 only");
  int nb, T, D;
  // per particle: FP32 j-side slot sums per distance, FP64 i-side sums per workgroup,
  // FP64 block-diagonal sums (in pds slices) and three staged float4 records
  const int pds = diag_slices((int)((n + kSI - 1) / kSI));
  sym_plan(n, cfg.launches, kVC * sizeof(float), kVC * sizeof(float), kVC * sizeof(double),
           pds * kVC * (int)sizeof(double) + 3 * (int)sizeof(float4), cfg.scratch ? cfg.scratch_bytes : SIZE_MAX, &nb,
           &T, &D);
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
  const size_t pj_bytes = sizeof(float) * kVC * (size_t)npad * D;
  const size_t pi_bytes = sizeof(double) * kVC * (size_t)npad * nparts;
  const size_t pd_bytes = sizeof(double) * kVC * (size_t)npad * pds;
  const size_t rec_bytes = sizeof(float4) * (size_t)npad;
  const size_t buf_bytes = pj_bytes + pi_bytes;  // one slot set
  char* ws = static_cast<char*>(pair_scratch(cfg, nbuf * buf_bytes + pd_bytes + 3 * rec_bytes, &st));
  if (!ws) return st;
  SymArgs A;
  A.pe = nullptr;
  A.pw = nullptr;
  A.x = x; A.m = m; A.w = w; A.n = (int)n; A.nb = nb; A.npad = (int)npad; A.dmax = dmax; A.half = half;
  A.T = T; A.nparts = nparts; A.eps = eps; A.d_lo = 1;
  A.fx = std::max(kNearX, kNearN / std::cbrt((float)n));
  auto slots = [&](int b, SymArgs& Q) {
    Q.pj = reinterpret_cast<float*>(ws + (size_t)b * buf_bytes);
    Q.pi = reinterpret_cast<double*>(ws + (size_t)b * buf_bytes + pj_bytes);
  };
  slots(0, A);
  double* pd = reinterpret_cast<double*>(ws + nbuf * buf_bytes);
  float4* rhi = reinterpret_cast<float4*>(ws + nbuf * buf_bytes + pd_bytes);
  float4* rw = rhi + npad;
  float4* rlo = rw + npad;
  A.rhi = rhi;
  A.rw = rw;
  A.rlo = rlo;
  const bool near = precision == kFP32C;
  const unsigned sg = (unsigned)((npad + 255) / 256);
  if (near) vsym_stage_kernel<true><<<sg, 256, 0, s>>>(A, rhi, rw, rlo);
  else vsym_stage_kernel<false><<<sg, 256, 0, s>>>(A, rhi, rw, rlo);
  NB_LAUNCH_CHECK("vsym_stage_kernel");
  // the own pair is always left out of the block-diagonal sums, so exclude_self needs no variant
  (void)excl;
  const dim3 dg((unsigned)nb, (unsigned)pds);
  auto diag = [&](hipStream_t ds) -> int {
    if (near) vsym_diag_kernel<true><<<dg, kSL * kDiagG, 0, ds>>>(A, pd);
    else vsym_diag_kernel<false><<<dg, kSL * kDiagG, 0, ds>>>(A, pd);
    NB_LAUNCH_CHECK("vsym_diag_kernel");
    return NBODY_OK;
  };
  const dim3 rg((unsigned)((n + 255) / 256), kVC);
  if (dmax == 0) {
    if ((st = diag(s))) return st;
    sym_reduce_kernel<kVC, float><<<rg, 256, 0, s>>>((int)n, (int)npad, nb, dmax, half, 1, 0, 0, A.pj, A.pi, pd, gx, gm, G,
                                              1, 1, nullptr, nullptr, nullptr, nullptr, pds);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  }
  auto pair = [&](int c, int b) -> int {
    SymArgs B = A;
    slots(b, B);
    B.d_lo = 1 + c * D;
    const unsigned grid = (unsigned)nb * (unsigned)nparts;
    if (near) vsym_kernel<true><<<grid, kSL, 0, s>>>(B);
    else vsym_kernel<false><<<grid, kSL, 0, s>>>(B);
    NB_LAUNCH_CHECK("vsym_kernel");
    return NBODY_OK;
  };
  auto sum = [&](int c, int b, hipStream_t rs) -> int {
    SymArgs B = A;
    slots(b, B);
    sym_reduce_kernel<kVC, float><<<rg, 256, 0, rs>>>((int)n, (int)npad, nb, dmax, half, 1 + c * D, D, nparts, B.pj, B.pi,
                                               pd, gx, gm, G, c == 0, c == nchunks - 1, nullptr, nullptr, nullptr,
                                               nullptr, pds);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
    return NBODY_OK;
  };
  return run_sym_chunks(side, s, nchunks, nbuf, diag, pair, sum);
}

}  // namespace nb
