// Symmetric all-pairs acceleration: every unordered pair {i, j} is evaluated
// once and its term is applied to both particles (a_i gets m_j d r^-3, a_j gets
// -m_i d r^-3, the pairwise antisymmetry of Eq. 1), which halves the inverse
// square roots, displacements and squared distances of the ordered kernel.
//
// Layout on the chip:
//   * a workgroup of 256 lanes holds an I-block of 512 particles, two per lane
//     (lane t owns i = 512 g + t and 512 g + 256 + t), and streams J-blocks of
//     512 particles through LDS in tiles of 64;
//   * the lanes form 16 rows of 16.  A tile is 4 sub-blocks of 16 records, each
//     stored twice in a row in LDS, so that at step K (0..15) lane r of a row
//     reads record (r + K) of the sub-block at an immediate offset: over 16
//     steps every lane meets all 16 records, and at each step the 16 lanes of a
//     row meet 16 different j;
//   * the i-side terms stay in the lane; the j-side terms of a step (both i of
//     the lane summed first) belong to the lane that met that j at step 0 and
//     move there through a row rotation (DPP row_ror) fused into the add;
//   * after a sub-block the four rows of a wave hold j-side sums for the same
//     16 j; they are added across rows on the LDS pipe (swizzle, permute) and
//     stored per wave; after the tile the 4 wave sums of each j are added in
//     wave order and the tile's sum is written to a per-distance slot in HBM; a
//     reduction kernel adds the slots in a fixed order in FP64, so results are
//     reproducible;
//   * block pairs are visited once on a half ring: I-block g meets the J-blocks
//     g + d (mod nb) for d = 1 .. nb/2 (d = nb/2 only for g < nb/2 when nb is
//     even); d = 0 is the block with itself, evaluated in the ordered form (the
//     i-side only, over all 512 j, the own pair masked when asked);
//   * the half ring is cut into chunks of D distances, one launch and one
//     reduction each, so the slot buffers stay bounded whatever N is.
// FP32C (positions rounded to FP32 plus the near-field repair of the ordered
// kernel: pairs closer than the larger repair radius of their two particles get
// float-float displacements, for both sides) and FP32 (no repair) are built.
#include <mutex>

#include "sym_common.h"

namespace nb {
namespace {

struct ISet {
  float x[2], y[2], z[2], mneg[2];
};

// One step of a sub-block: both i of the lane against record (r + K).
template <int K, bool NEAR>
__device__ __forceinline__ void sym_step(const ISet& s, const float4* __restrict__ rowp, float e2, float (&px)[2],
                                         float (&py)[2], float (&pz)[2], float (&r2min)[2], float& ajx,
                                         float& ajy, float& ajz) {
  const float4 r = rowp[K];
  float tx = 0.f, ty = 0.f, tz = 0.f;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const float dx = r.x - s.x[u], dy = r.y - s.y[u], dz = r.z - s.z[u];
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
    const float ri = rsqrt32(r2);
    const float ri3 = (ri * ri) * ri;
    const float si = r.w * ri3;
    px[u] = fmaf(si, dx, px[u]);
    py[u] = fmaf(si, dy, py[u]);
    pz[u] = fmaf(si, dz, pz[u]);
    if constexpr (NEAR) r2min[u] = fminf(r2min[u], r2);
    const float sj = s.mneg[u] * ri3;
    if (u == 0) { tx = sj * dx; ty = sj * dy; tz = sj * dz; }
    else { tx = fmaf(sj, dx, tx); ty = fmaf(sj, dy, ty); tz = fmaf(sj, dz, tz); }
  }
  // the j met here sits at row position (r + K): its owner, the lane that met it
  // at step 0, is K lanes further on
  if constexpr (K == 0) {
    ajx += tx; ajy += ty; ajz += tz;
  } else {
    ajx += row_ror<K>(tx);
    ajy += row_ror<K>(ty);
    ajz += row_ror<K>(tz);
  }
}

template <bool NEAR, int... K>
__device__ __forceinline__ void sym_sub(const ISet& s, const float4* __restrict__ rowp, float e2, float (&px)[2],
                                        float (&py)[2], float (&pz)[2], float (&r2min)[2], float& ajx,
                                        float& ajy, float& ajz, std::integer_sequence<int, K...>) {
  (sym_step<K, NEAR>(s, rowp, e2, px, py, pz, r2min, ajx, ajy, ajz), ...);
}

// Loads the two i of lane t of I-block g (padding i: far away and massless, so
// they add nothing to any j) and, per i, the squared radius that flags a tile
// for the repair (-1 for padding).  PAIR: radii that also hold every pair
// inside the j's own repair radius, since the pair serves both particles:
// |d| < f |x_j| with |x_j| <= |x_i| + |d| gives |d| < f / (1 - f) |x_i| (f is at
// most 1/2; the eps term is the same for both particles).
template <bool PAIR>
__device__ __forceinline__ void load_iset(const SymArgs& A, int g, int t, ISet& s, float (&thr)[2]) {
  const int n = A.n;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = g * kSI + u * kSL + t;
    thr[u] = -1.f;
    if (i < n) {
      const double xa = A.x[i], ya = A.x[n + i], za = A.x[2 * n + i];
      s.x[u] = (float)xa; s.y[u] = (float)ya; s.z[u] = (float)za;
      s.mneg[u] = -(float)A.m[i];
      thr[u] = sym_rc2(xa, ya, za, A.eps, PAIR ? A.fx / (1.0f - A.fx) * 1.0001f : A.fx);
    } else {
      s.x[u] = s.y[u] = s.z[u] = (float)kFarAway;
      s.mneg[u] = 0.f;
    }
  }
}

// Float-float term minus rounded-position term of the pair (i, j), times m:
// the near-field correction (FP32C), for i with m = m_j and for j with m = -m_i.
__device__ __forceinline__ void near_delta(float dx, float dy, float dz, float r2, float ex, float ey, float ez,
                                           float e2, float& fx, float& fy, float& fz) {
  const float ri = rsqrt32(r2);
  const float ri3 = (ri * ri) * ri;
  const float q2 = fmaf(ez, ez, fmaf(ey, ey, fmaf(ex, ex, e2)));
  const float qi = rsqrt32(q2);
  const float qi3 = (qi * qi) * qi;
  fx = fmaf(qi3, ex, -(ri3 * dx));
  fy = fmaf(qi3, ey, -(ri3 * dy));
  fz = fmaf(qi3, ez, -(ri3 * dz));
}

// The j-records of all npad particles (padding past n: far away, massless,
// never repaired), converted once per evaluation so that the force kernel's
// tiles are plain 16-byte copies.
template <bool NEAR>
__global__ void sym_stage_kernel(SymArgs A, float4* __restrict__ rhi, float4* __restrict__ rlo, int* __restrict__ zc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (zc && j == 0) *zc = 0;  // the rescue's count of flagged rows
  if (j >= A.npad) return;
  float4 hi, lo;
  const int n = A.n;
  if (j < n) {
    const double xa = A.x[j], ya = A.x[n + j], za = A.x[2 * n + j];
    hi = make_float4((float)xa, (float)ya, (float)za, (float)A.m[j]);
    lo = make_float4((float)(xa - (double)hi.x), (float)(ya - (double)hi.y), (float)(za - (double)hi.z),
                     NEAR ? sym_rc2(xa, ya, za, A.eps, A.fx) : -1.f);
  } else {
    hi = make_float4((float)kFarAway, (float)kFarAway, (float)kFarAway, 0.f);
    lo = make_float4(0.f, 0.f, 0.f, -1.f);
  }
  rhi[j] = hi;
  rlo[j] = lo;
}

struct P6 {
  float x0, x1, y0, y1, z0, z1;
};

// Near-field repair of one lane's tile (FP32C): for every pair of the lane's
// two i with the tile's 64 j closer than the larger repair radius of its two
// particles, the rounded-position term is replaced by the float-float one: in
// the lane's i-side sums p (returned) and in the wave's j-side sums of the tile
// (part: the wave's slots, components kSW * kST apart).  The j are visited in
// the rotated order of the pair loop, so at each step the lanes of a row touch
// distinct j; the four rows of the wave, which share the slots, take turns.
// r2nr receives, per i, the smallest squared distance of the tile's pairs that
// keep their rounded-position terms (for the error estimate of the rescue).
__device__ __forceinline__ P6 sym_repair(const double* __restrict__ x, int n, double eps, float fx, int g, int t, int rl,
                                         float e2, ISet s, P6 p, const float4* hi, const float4* lo, float* part,
                                         float (&r2nr)[2]) {
  const int wrow = (t & 63) / kSR;
  float px[2] = {p.x0, p.x1}, py[2] = {p.y0, p.y1}, pz[2] = {p.z0, p.z1};
  float rc[2];
  r2nr[0] = r2nr[1] = 3.0e38f;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = g * kSI + u * kSL + t;
    rc[u] = i < n ? sym_rc2(x[i], x[n + i], x[2 * n + i], eps, fx) : -1.f;
  }
  for (int jj = 0; jj < kST; ++jj) {
    const int q = jj / kSR;
    const int jl = q * kSR + ((rl + jj) & (kSR - 1));
    const float4 rh = hi[q * 2 * kSR + (jl % kSR)];
    const float4 rl4 = lo[jl];
    float cx = 0.f, cy = 0.f, cz = 0.f;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const float dx = rh.x - s.x[u], dy = rh.y - s.y[u], dz = rh.z - s.z[u];
      const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
      if (!(r2 < fmaxf(rc[u], rl4.w))) r2nr[u] = fminf(r2nr[u], r2);
      if (rc[u] >= 0.f && r2 < fmaxf(rc[u], rl4.w)) {
        const int i = g * kSI + u * kSL + t;
        const double xa = x[i], ya = x[n + i], za = x[2 * n + i];
        const float ex = dx + (rl4.x - (float)(xa - (double)s.x[u]));
        const float ey = dy + (rl4.y - (float)(ya - (double)s.y[u]));
        const float ez = dz + (rl4.z - (float)(za - (double)s.z[u]));
        float fx3, fy3, fz3;
        near_delta(dx, dy, dz, r2, ex, ey, ez, e2, fx3, fy3, fz3);
        px[u] = fmaf(rh.w, fx3, px[u]);
        py[u] = fmaf(rh.w, fy3, py[u]);
        pz[u] = fmaf(rh.w, fz3, pz[u]);
        cx = fmaf(s.mneg[u], fx3, cx);
        cy = fmaf(s.mneg[u], fy3, cy);
        cz = fmaf(s.mneg[u], fz3, cz);
      }
    }
    for (int r = 0; r < 4; ++r) {
      if (wrow == r && (cx != 0.f || cy != 0.f || cz != 0.f)) {
        part[jl] += cx;
        part[kSW * kST + jl] += cy;
        part[2 * kSW * kST + jl] += cz;
      }
      wave_sync();  // one row's turn ends before the next row reads the sums
    }
  }
  return P6{px[0], px[1], py[0], py[1], pz[0], pz[1]};
}

// Grid: nb * nparts workgroups; workgroup (g, part) takes the distances
// [d_lo + part L, d_lo + (part + 1) L) of I-block g's half ring (d >= 1).
template <bool NEAR, bool EST>
__global__ __launch_bounds__(kSL, 7) void sym_accel_kernel(SymArgs A) {
  __shared__ float4 s_hi[2][4][2 * kSR];  // (x, y, z, m) hi parts, each sub-block twice
  __shared__ float4 s_lo[2][kST];         // (x, y, z) lo parts and the repair radius^2 of j
  __shared__ float s_part[3][kSW][kST];
  __shared__ float s_acc_lo[6][kSL];      // the lo halves of the i-side (hi, lo) sums
  __shared__ float s_est[2][kSL];         // the i-side error estimates (EST)
  __shared__ float s_pmin[kSW];           // the tile's smallest non-repaired squared distance per wave (EST)

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
  const int n = A.n;
  const float e2 = (float)(A.eps * A.eps);

  ISet s;
  float thr[2];
  load_iset<true>(A, g, t, s, thr);
  float hx[2] = {0.f, 0.f}, hy[2] = {0.f, 0.f}, hz[2] = {0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 6; ++c) s_acc_lo[c][t] = 0.f;
  s_est[0][t] = s_est[1][t] = 0.f;
  // lane address for the exchange across the two halves of a wave
  const int xor32 = ((t & 63) ^ 32) * 4;

  // the last wave copies tile k's staged records into LDS buffer b, straight
  // from global memory to LDS (no registers held): one 16-byte record per lane
  // and copy, lanes in order.  Lanes 0-15 and 16-31 both fetch the first
  // sub-block of a pair, lanes 32-47 and 48-63 the second, which lays each
  // sub-block out twice in a row; a third copy fetches the lo records.
  // per-lane byte offsets within a tile (the tile's base is uniform)
  const unsigned lane_hi = (unsigned)((((t & 63) >> 5) * kSR + (t & (kSR - 1))) * sizeof(float4));
  const unsigned lane_lo = (unsigned)((t & 63) * sizeof(float4));
  auto stage = [&](int k, int b) {
    // the tile's first record, kept scalar (an address in VGPR pairs would cost
    // registers the pair loop needs)
    const int rec0 = __builtin_amdgcn_readfirstlane(((g + A.d_lo + (kbeg + k) / kSTiles) % A.nb) * kSI + ((kbeg + k) % kSTiles) * kST);
    const size_t base = (size_t)rec0 * sizeof(float4);
    const char* hb = reinterpret_cast<const char*>(A.rhi) + base;
    const char* lb = reinterpret_cast<const char*>(A.rlo) + base;
    // the lane offsets enter each address afresh (an empty asm statement hides
    // them from loop-invariant hoisting), so that every copy takes the form
    // scalar base + 32-bit lane offset instead of a 64-bit per-lane pointer
    unsigned oh = lane_hi, ol = lane_lo;
    asm volatile("" : "+v"(oh), "+v"(ol));
    __builtin_amdgcn_global_load_lds(hb + oh, (lds_ptr)&s_hi[b][0][0], 16, 0, 0);
    __builtin_amdgcn_global_load_lds(hb + 2 * kSR * sizeof(float4) + oh, (lds_ptr)&s_hi[b][2][0], 16, 0, 0);
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
    // the next tile's records travel while this one is evaluated (buffer b ^ 1
    // was last read in tile k - 1, before the barrier that ended it)
    if (t >= 3 * 64 && k + 1 < ntiles) stage(k + 1, b ^ 1);
    float px[2] = {0.f, 0.f}, py[2] = {0.f, 0.f}, pz[2] = {0.f, 0.f};
    float r2min[2] = {3.0e38f, 3.0e38f};
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      float ajx = 0.f, ajy = 0.f, ajz = 0.f;
      sym_sub<NEAR>(s, &s_hi[b][q][rl], e2, px, py, pz, r2min, ajx, ajy, ajz, std::make_integer_sequence<int, kSR>{});
      // the four rows' sums of the same 16 j: rows (0 + 1) and (2 + 3) by a
      // swizzle, then the two halves by a permute, after which all four rows
      // hold the same totals and store the same values (no branch in the loop)
      ajx += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(ajx), 0x401F));
      ajy += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(ajy), 0x401F));
      ajz += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(ajz), 0x401F));
      ajx += __int_as_float(__builtin_amdgcn_ds_bpermute(xor32, __float_as_int(ajx)));
      ajy += __int_as_float(__builtin_amdgcn_ds_bpermute(xor32, __float_as_int(ajy)));
      ajz += __int_as_float(__builtin_amdgcn_ds_bpermute(xor32, __float_as_int(ajz)));
      s_part[0][wave][q * kSR + rl] = ajx;
      s_part[1][wave][q * kSR + rl] = ajy;
      s_part[2][wave][q * kSR + rl] = ajz;
    }
    if constexpr (NEAR) {
      // rare: a pair of this tile may be closer than the larger repair radius
      // of its two particles
      if (r2min[0] < thr[0] || r2min[1] < thr[1]) {
        const P6 r = sym_repair(A.x, n, A.eps, A.fx, g, t, rl, e2, s, P6{px[0], px[1], py[0], py[1], pz[0], pz[1]},
                                &s_hi[b][0][0], &s_lo[b][0], &s_part[0][wave][0], r2min);
        px[0] = r.x0; px[1] = r.x1; py[0] = r.y0; py[1] = r.y1; pz[0] = r.z0; pz[1] = r.z1;
      }
      // the error estimate of the rescue: this tile's partial sums, weighted by
      // the distance of their closest pair left in rounded positions (r2min
      // holds it after the repair); for the far side, the wave's smallest such
      // distance over the whole tile, a lower bound of every j's own
      if constexpr (EST) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const float xinf = fmaxf(fabsf(s.x[u]), fmaxf(fabsf(s.y[u]), fabsf(s.z[u])));
          s_est[u][t] = est_add(s_est[u][t], px[u], py[u], pz[u], xinf, r2min[u]);
        }
        float tm = fminf(r2min[0], r2min[1]);
        tm = fminf(tm, row_ror<8>(tm));
        tm = fminf(tm, row_ror<4>(tm));
        tm = fminf(tm, row_ror<2>(tm));
        tm = fminf(tm, row_ror<1>(tm));
        tm = fminf(tm, __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(tm), 0x401F)));
        tm = fminf(tm, __int_as_float(__builtin_amdgcn_ds_bpermute(xor32, __float_as_int(tm))));
        if ((t & 63) == 0) s_pmin[wave] = tm;
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      fold(hx[u], s_acc_lo[3 * u][t], px[u]);
      fold(hy[u], s_acc_lo[3 * u + 1][t], py[u]);
      fold(hz[u], s_acc_lo[3 * u + 2][t], pz[u]);
    }
    __syncthreads();
    if (t < 2 * kST && (t < kST || EST)) {
      // the tile's j-side sums: the 4 wave sums of each j, in wave order; the
      // first wave writes them, the second (EST) their share of the estimate
      const int jl = t % kST;
      float v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v[c] = 0.f;
#pragma unroll
        for (int w = 0; w < kSW; ++w) v[c] += s_part[c][w][jl];
      }
      const int J = (g + d) % A.nb;
      const size_t col = (size_t)J * kSI + tt * kST + jl;
      if (t < kST) {
#pragma unroll
        for (int c = 0; c < 3; ++c) A.pj[((size_t)(d - A.d_lo) * 3 + c) * A.npad + col] = v[c];
      } else if constexpr (EST) {
        // the far side's share of j's error estimate: this tile's sum over the
        // workgroup's i, weighted by the smallest distance of the tile's pairs
        // left in rounded positions (over all its j: a lower bound of j's own
        // closest such pair); a pair closer than j's own repair radius was
        // repaired, so that radius bounds the distance from below too
        float dm = s_pmin[0];
#pragma unroll
        for (int w = 1; w < kSW; ++w) dm = fminf(dm, s_pmin[w]);
        const float4 rj = s_hi[b][jl / kSR][jl % kSR];
        const float xinf = fmaxf(fabsf(rj.x), fmaxf(fabsf(rj.y), fabsf(rj.z)));
        const float wj = fmaf(kEstNear * xinf, rsqrt32(fmaxf(dm, s_lo[b][jl].w)), 1.0f);
        A.pw[(size_t)(d - A.d_lo) * A.npad + col] = wj * wj * fmaf(v[0], v[0], fmaf(v[1], v[1], v[2] * v[2]));
      }
    } else if (t >= 3 * 64) {
      __builtin_amdgcn_s_waitcnt(0);  // the next tile's copies have landed in LDS
    }
    __syncthreads();
  }

  // the i-side sums of this workgroup
  double* o = A.pi + (size_t)part * 3 * A.npad;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const size_t i = (size_t)g * kSI + u * kSL + t;
    o[i] = (double)hx[u] + (double)s_acc_lo[3 * u][t];
    o[A.npad + i] = (double)hy[u] + (double)s_acc_lo[3 * u + 1][t];
    o[2 * (size_t)A.npad + i] = (double)hz[u] + (double)s_acc_lo[3 * u + 2][t];
    if (EST) A.pe[(size_t)part * A.npad + i] = s_est[u][t];
  }
}

// The block with itself (distance 0): the i-side of all ordered pairs inside
// I-block g, in the ordered form (the LDS record broadcast to every lane), with
// the own pair masked when asked and the near-field repair of the force kernel.
// The gridDim.y workgroups of a block each take a slice of its j, and their
// kDiagG groups of kSL lanes each a part of the slice (so that the launch has
// several waves per SIMD); group 0 adds the groups' hi + lo in group order and
// writes the slice's sums into pd[slice][3][npad] (ed[slice][npad]).
template <bool NEAR, bool EXCL>
__global__ __launch_bounds__(kSL* kDiagG) void sym_diag_kernel(SymArgs A, double* __restrict__ pd,
                                                                float* __restrict__ ed) {
  __shared__ float4 s_hi[kSI];
  __shared__ float4 s_lo[kSI];
  __shared__ double s_part[kDiagG - 1][3][kSI];
  __shared__ float s_epart[kDiagG - 1][kSI];
  const int t = threadIdx.x % kSL, grp = threadIdx.x / kSL;
  const int g = blockIdx.x;
  const float e2 = (float)(A.eps * A.eps);
  // this lane group's j: a run of span records, folded fl at a time
  const int span = kSI / ((int)gridDim.y * kDiagG), fl = span < kFold ? span : kFold;
  const int f0 = ((int)blockIdx.y * kDiagG + grp) * span;
  ISet s;
  float thr[2];
  load_iset<false>(A, g, t, s, thr);
  for (int k = threadIdx.x; k < kSI; k += kSL * kDiagG) {
    s_hi[k] = A.rhi[(size_t)g * kSI + k];
    s_lo[k] = A.rlo[(size_t)g * kSI + k];
  }
  __syncthreads();
  float hx[2] = {0.f, 0.f}, hy[2] = {0.f, 0.f}, hz[2] = {0.f, 0.f};
  float lx[2] = {0.f, 0.f}, ly[2] = {0.f, 0.f}, lz[2] = {0.f, 0.f};
  float rc[2], ea[2] = {0.f, 0.f};
#pragma unroll
  for (int u = 0; u < 2; ++u) rc[u] = s_lo[u * kSL + t].w;
#pragma unroll 1
  for (int f = f0; f < f0 + span; f += fl) {
    float px[2] = {0.f, 0.f}, py[2] = {0.f, 0.f}, pz[2] = {0.f, 0.f};
    float r2min[2] = {3.0e38f, 3.0e38f};
#pragma unroll 16
    for (int j = f; j < f + fl; ++j) {
      const float4 r = s_hi[j];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const float dx = r.x - s.x[u], dy = r.y - s.y[u], dz = r.z - s.z[u];
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
        const float ri = rsqrt32(r2);
        float si = (r.w * ri) * (ri * ri);
        if (EXCL) si = (j == u * kSL + t) ? 0.f : si;
        px[u] = fmaf(si, dx, px[u]);
        py[u] = fmaf(si, dy, py[u]);
        pz[u] = fmaf(si, dz, pz[u]);
        if constexpr (NEAR) r2min[u] = fminf(r2min[u], r2);
      }
    }
    if constexpr (NEAR) {
      if (r2min[0] < thr[0] || r2min[1] < thr[1]) {
        float r2nr[2] = {3.0e38f, 3.0e38f};
        for (int j = f; j < f + fl; ++j) {
          const float4 rh = s_hi[j];
          const float4 lo = s_lo[j];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const float dx = rh.x - s.x[u], dy = rh.y - s.y[u], dz = rh.z - s.z[u];
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
            if (!(r2 < rc[u]) && j != u * kSL + t) r2nr[u] = fminf(r2nr[u], r2);
            if (rc[u] >= 0.f && r2 < rc[u] && j != u * kSL + t) {
              const float4 li = s_lo[u * kSL + t];
              float fx, fy, fz;
              near_delta(dx, dy, dz, r2, dx + (lo.x - li.x), dy + (lo.y - li.y), dz + (lo.z - li.z), e2, fx, fy, fz);
              px[u] = fmaf(rh.w, fx, px[u]);
              py[u] = fmaf(rh.w, fy, py[u]);
              pz[u] = fmaf(rh.w, fz, pz[u]);
            }
          }
        }
        r2min[0] = r2nr[0];
        r2min[1] = r2nr[1];
      }
      if (ed) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const float xinf = fmaxf(fabsf(s.x[u]), fmaxf(fabsf(s.y[u]), fabsf(s.z[u])));
          ea[u] = est_add(ea[u], px[u], py[u], pz[u], xinf, r2min[u]);
        }
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
      s_part[grp - 1][0][u * kSL + t] = (double)hx[u] + (double)lx[u];
      s_part[grp - 1][1][u * kSL + t] = (double)hy[u] + (double)ly[u];
      s_part[grp - 1][2][u * kSL + t] = (double)hz[u] + (double)lz[u];
      s_epart[grp - 1][u * kSL + t] = ea[u];
    }
  }
  __syncthreads();
  if (grp > 0) return;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int k = u * kSL + t;
    const size_t i = (size_t)g * kSI + k;
    double* const pds = pd + (size_t)blockIdx.y * 3 * A.npad;
    double vx = (double)hx[u] + (double)lx[u], vy = (double)hy[u] + (double)ly[u], vz = (double)hz[u] + (double)lz[u];
    float e = ea[u];
#pragma unroll
    for (int q = 0; q < kDiagG - 1; ++q) {
      vx += s_part[q][0][k];
      vy += s_part[q][1][k];
      vz += s_part[q][2][k];
      e += s_epart[q][k];
    }
    pds[i] = vx;
    pds[A.npad + i] = vy;
    pds[2 * (size_t)A.npad + i] = vz;
    if (NEAR && ed) ed[(size_t)blockIdx.y * A.npad + i] = e;
  }
}

constexpr int kSideDev = 64;
std::mutex g_side_mu;
SideStream g_side[kSideDev];

void destroy_side(SideStream& S) {
  for (hipEvent_t* e : {&S.stage, &S.pair[0], &S.pair[1], &S.red[0], &S.red[1], &S.join})
    if (*e) {
      (void)hipEventDestroy(*e);
      *e = nullptr;
    }
  if (S.side) (void)hipStreamDestroy(S.side);
  S.side = nullptr;
}

}  // namespace

SideStream* acquire_side_stream(hipStream_t s, std::unique_lock<std::mutex>& lk) {
  const int dev = current_device();
  if (dev < 0 || dev >= kSideDev) return nullptr;
  lk = std::unique_lock<std::mutex>(g_side_mu);
  SideStream& S = g_side[dev];
  if (S.side) return &S;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  bool ok = hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone &&
            hipStreamCreateWithFlags(&S.side, hipStreamNonBlocking) == hipSuccess;
  for (hipEvent_t* e : {&S.stage, &S.pair[0], &S.pair[1], &S.red[0], &S.red[1], &S.join})
    ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    destroy_side(S);
    lk.unlock();
    return nullptr;
  }
  return &S;
}

void release_side_streams() {
  std::lock_guard<std::mutex> lk(g_side_mu);
  int prev = 0;
  (void)hipGetDevice(&prev);
  for (int d = 0; d < kSideDev; ++d)
    if (g_side[d].side) {
      (void)hipSetDevice(d);
      (void)hipStreamSynchronize(g_side[d].side);
      destroy_side(g_side[d]);
    }
  (void)hipSetDevice(prev);
}

int launch_sym_accel(int64_t n, const double* x, const double* m, double* a, double G, double eps, int precision,
                     bool excl, const PairConfig& cfg, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  if (precision != kFP32C && precision != kFP32)
    return set_error(NBODY_EUNSUPPORTED, "symmetric pair kernel: FP32C and FP32 only");
  if (n > (int64_t(1) << 30)) return set_error(NBODY_EINVAL, "symmetric pair kernel: n too large");
  const bool near = precision == kFP32C;
  const bool rescue = near && cfg.rescue;
  int nb, T, D;
  // per particle: FP32 j-side slot sums (and, for the rescue, an FP32 error estimate)
  // per distance, FP64 i-side sums (and an FP32 estimate) per workgroup, FP64
  // block-diagonal sums, two staged float4 records and, for the rescue, two FP32
  // estimates and a list entry; the list's count takes 64 more ints
  const int est_fixed = rescue ? 2 * (int)sizeof(float) + (int)sizeof(int) : 0;
  const size_t count_bytes = rescue ? 64 * sizeof(int) : 0;
  const int est_part = rescue ? (int)sizeof(float) : 0;
  const int est_slot = rescue ? (int)sizeof(float) : 0;
  // the block-diagonal sums (and estimate shares) come in pds slices
  const int pds = diag_slices((int)((n + kSI - 1) / kSI));
  sym_plan(n, cfg.launches, 3 * sizeof(float) + est_slot, 3 * sizeof(float), 3 * sizeof(double) + est_part,
           pds * (3 * (int)sizeof(double) + (rescue ? (int)sizeof(float) : 0)) + 2 * sizeof(float4) + est_fixed -
               (rescue ? (int)sizeof(float) : 0),
           cfg.scratch ? cfg.scratch_bytes - count_bytes : SIZE_MAX, &nb, &T, &D);
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
  const size_t pj_bytes = sizeof(float) * 3 * (size_t)npad * D;
  const size_t pi_bytes = sizeof(double) * 3 * (size_t)npad * nparts;
  const size_t pd_bytes = sizeof(double) * 3 * (size_t)npad * pds;
  const size_t rec_bytes = sizeof(float4) * (size_t)npad;
  const size_t pe_bytes = rescue ? sizeof(float) * (size_t)npad * nparts : 0;
  const size_t pw_bytes = rescue ? sizeof(float) * (size_t)npad * D : 0;
  const size_t eo_bytes = rescue ? sizeof(float) * (1 + pds) * (size_t)npad : 0;  // eo [npad], ed [pds][npad]
  const size_t list_bytes = rescue ? sizeof(int) * (size_t)npad + count_bytes : 0;  // the count, then the list
  const size_t buf_bytes = pj_bytes + pi_bytes + pe_bytes + pw_bytes;  // one set of slots
  char* ws = static_cast<char*>(
      pair_scratch(cfg, nbuf * buf_bytes + pd_bytes + 2 * rec_bytes + eo_bytes + list_bytes, &st));
  if (!ws) return st;
  SymArgs A;
  A.x = x; A.m = m; A.n = (int)n; A.nb = nb; A.npad = (int)npad; A.dmax = dmax; A.half = half;
  A.T = T; A.nparts = nparts; A.eps = eps; A.d_lo = 1;
  A.fx = std::max(kNearX, kNearN / std::cbrt((float)n));
  // slot set b: pj, pi, pe, pw
  auto slots = [&](int b, SymArgs& Q) {
    char* q = ws + (size_t)b * buf_bytes;
    Q.pj = reinterpret_cast<float*>(q);
    Q.pi = reinterpret_cast<double*>(q + pj_bytes);
    Q.pe = rescue ? reinterpret_cast<float*>(q + pj_bytes + pi_bytes) : nullptr;
    Q.pw = rescue ? reinterpret_cast<float*>(q + pj_bytes + pi_bytes + pe_bytes) : nullptr;
  };
  slots(0, A);
  char* fixed = ws + nbuf * buf_bytes;
  double* pd = reinterpret_cast<double*>(fixed);
  float4* rhi = reinterpret_cast<float4*>(fixed + pd_bytes);
  float4* rlo = rhi + npad;
  char* tail = fixed + pd_bytes + 2 * rec_bytes;
  A.rhi = rhi;
  A.rlo = rlo;
  float* eo = rescue ? reinterpret_cast<float*>(tail) : nullptr;
  float* ed = rescue ? eo + npad : nullptr;
  int* list = rescue ? reinterpret_cast<int*>(tail + eo_bytes) : nullptr;
  const unsigned sg = (unsigned)((npad + 255) / 256);
  if (near) sym_stage_kernel<true><<<sg, 256, 0, s>>>(A, rhi, rlo, list);
  else sym_stage_kernel<false><<<sg, 256, 0, s>>>(A, rhi, rlo, list);
  NB_LAUNCH_CHECK("sym_stage_kernel");
  const dim3 dg((unsigned)nb, (unsigned)pds);
  auto diag = [&](hipStream_t ds) -> int {
    if (near) {
      if (excl) sym_diag_kernel<true, true><<<dg, kSL * kDiagG, 0, ds>>>(A, pd, ed);
      else sym_diag_kernel<true, false><<<dg, kSL * kDiagG, 0, ds>>>(A, pd, ed);
    } else {
      if (excl) sym_diag_kernel<false, true><<<dg, kSL * kDiagG, 0, ds>>>(A, pd, ed);
      else sym_diag_kernel<false, false><<<dg, kSL * kDiagG, 0, ds>>>(A, pd, ed);
    }
    NB_LAUNCH_CHECK("sym_diag_kernel");
    return NBODY_OK;
  };
  const dim3 rg((unsigned)((n + 255) / 256), 3);
  if (dmax == 0) {
    if ((st = diag(s))) return st;
    sym_reduce_kernel<3, float><<<rg, 256, 0, s>>>((int)n, (int)npad, nb, dmax, half, 1, 0, 0, A.pj, A.pi, pd, a, nullptr, G,
                                            1, 1, A.pe, A.pw, ed, eo, pds);
    NB_LAUNCH_CHECK("sym_reduce_kernel");
  } else {
    auto pair = [&](int c, int b) -> int {
      SymArgs B = A;
      slots(b, B);
      B.d_lo = 1 + c * D;
      const unsigned grid = (unsigned)nb * (unsigned)nparts;
      if (rescue) sym_accel_kernel<true, true><<<grid, kSL, 0, s>>>(B);
      else if (near) sym_accel_kernel<true, false><<<grid, kSL, 0, s>>>(B);
      else sym_accel_kernel<false, false><<<grid, kSL, 0, s>>>(B);
      NB_LAUNCH_CHECK("sym_accel_kernel");
      return NBODY_OK;
    };
    auto sum = [&](int c, int b, hipStream_t rs) -> int {
      SymArgs B = A;
      slots(b, B);
      sym_reduce_kernel<3, float><<<rg, 256, 0, rs>>>((int)n, (int)npad, nb, dmax, half, 1 + c * D, D, nparts, B.pj, B.pi,
                                               pd, a, nullptr, G, c == 0, c == nchunks - 1, B.pe, B.pw, ed, eo, pds);
      NB_LAUNCH_CHECK("sym_reduce_kernel");
      return NBODY_OK;
    };
    if ((st = run_sym_chunks(side, s, nchunks, nbuf, diag, pair, sum))) return st;
  }
  if (rescue) return launch_rescue(n, x, m, eps, G, excl, eo, 1, (size_t)npad, a, list + 64, list, s);
  return NBODY_OK;
}

}  // namespace nb
