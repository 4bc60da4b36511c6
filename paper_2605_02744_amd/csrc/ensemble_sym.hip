// Symmetric per-step ensemble (nbody_config.bsplit = 4; FP32C and FP32).
//
// Every unordered pair of a system is evaluated once and its term applied to
// both particles (the antisymmetry of Eq. 1), as in the single-system symmetric
// kernel, but at the size of one wave, so that systems of 64 to a few thousand
// particles fill the chip.  Each system is cut into blocks of 64 particles
// (lane t owns particle t of a block); block b meets
//   * itself at distance 0, in the ordered form (the i-side of every ordered
//     pair, the own pair masked when asked);
//   * the blocks b + d (mod nb_c) of its system for d = 1 .. nb_c / 2 (d = nb_c / 2
//     only for b < nb_c / 2 when nb_c is even), each pair once.  The lanes form
//     4 rows of 16 and a J-block is 4 sub-blocks of 16 records, each stored
//     twice in a row in LDS, so that at step K lane r of every row reads record
//     (r + K) of the sub-block at an immediate offset.  The i-side terms stay
//     in the lane; the j-side term of a step belongs to the lane that met that
//     j at step 0 and moves there through a DPP row rotation fused into the
//     add; after a sub-block the four rows' sums of its 16 j are added on the
//     LDS pipe; the J-block's 64 sums go to the system's slot for distance d.
// A block's distances are cut into parts of a few distances; an item is one
// part, evaluated by one wave, so that the items of the largest systems are
// not much longer than the rest.  Each step is three launches: publish (the
// kicks, the drift and the pair records of the new positions), force (each
// item's i-side sums into a for the first part, else into its part's slot;
// the j-side sums into the distance slots) and reduce (per particle, its part
// sums in part order, then its distance slots in distance order, in FP64,
// times G), so results are reproducible.  Items are placed longest first over
// the workgroups and a workgroup's waves take its items from an LDS counter.
// FP32C positions are rounded to FP32 and the near-field rule of the ordered
// kernels applies: in the ordered block a pair closer than particle i's repair
// radius, in a block pair a pair closer than the larger radius of its two
// particles, gets float-float displacements.
// With the FP64 rescue (FP32C), each sum of 64 terms that a wave forms also
// adds its share to the row's rounding-error estimate (rescue.hip): the i-side
// sums of the ordered block and of every block pair, weighted by the lane's
// closest pair left in rounded positions, into per-part estimate slots; for
// the j-side sums of a block pair the wave records only the closest such pair
// of the whole block pair (one wave reduction, a lower bound of each j's own),
// and the reduction, which reads each j-side sum anyway, weights it with that
// distance.  The reduction then lists the rows whose estimate is too large
// against |a_i| per system, and the batched rescue recomputes those rows in
// FP64.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <queue>
#include <vector>

#include "sym_common.h"

namespace nb {
namespace {

constexpr int kEBlock = 1024;          // lanes per workgroup
constexpr int kEWaves = kEBlock / 64;  // waves (items in flight) per workgroup
constexpr int kEOcc = 8;               // waves per SIMD the force kernel is built for (<= 64 VGPRs)
constexpr int kEMaxPerCu = 2;          // resident workgroups per CU at most
constexpr size_t kESlotCap = size_t(1) << 30;  // bytes of j-side slots a plan may hold

// A block of 64 particles of a system, or (in the force kernel's work list)
// one part of its distances: [d0, d1), distance 0 being the block with itself.
struct EItem {
  int sys;   // system
  int b;     // block of 64 particles within the system
  int ni;    // particles in the block
  int d0, d1;
  int part;  // index of the part among the block's parts
};

// Per-system geometry: particles [o, o + nc) of the concatenated arrays, nb
// blocks of 64, j-side slots [dmax][3][nb * 64] floats from sbase, i-side
// slots [parts - 1][3][nb * 64] doubles from ibase for the parts after the
// first (a block's distances cut into parts of lp); with the rescue, the
// i-side error estimates [parts][nb * 64] floats from iebase (every part) and
// per block pair its closest pair left in rounded positions (squared),
// [dmax][nb] floats from wbase, indexed by distance and J-block.
struct ESys {
  int64_t o;
  int64_t sbase;
  int64_t ibase;
  int64_t iebase;
  int64_t wbase;
  double eps;
  int nc, nb, dmax, half;
  float fx;  // repair-radius factor max(kNearX, kNearN nc^-1/3)
  int lp;
};

// End of block b's distances: 0 (itself) .. dend - 1.
__host__ __device__ inline int esym_dend(const ESys& S, int b) {
  return (S.half && b >= S.nb / 2) ? S.dmax : S.dmax + 1;
}

// kicks = 0: records only; 1: v += h a, x += dt v; 2: v += h a twice (the
// closing half-kick of the previous step and the opening one of this step,
// rounded separately), x += dt v.  Then the pair records of the new position:
// hi = (x, y, z, m) rounded to FP32, lo = (x - hi, y - hi, z - hi, repair
// radius^2, or -1 without the repair).
// With rcnt (the rescue): clears the ncl per-system counts of flagged rows.
template <bool NEAR>
__global__ void esym_publish_kernel(int nblocks, const EItem* __restrict__ blocks, const ESys* __restrict__ sys,
                                    int64_t total, double* __restrict__ x, double* __restrict__ v,
                                    const double* __restrict__ a, const double* __restrict__ m,
                                    float4* __restrict__ rhi, float4* __restrict__ rlo, double h, double dt,
                                    int kicks, int* __restrict__ rcnt, int ncl) {
  if (rcnt)
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncl; c += gridDim.x * blockDim.x) rcnt[c] = 0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < (int64_t)nblocks * 64;
       g += (int64_t)gridDim.x * blockDim.x) {
    const EItem it = blocks[g >> 6];
    const int lane = (int)(g & 63);
    if (lane >= it.ni) continue;
    const ESys& S = sys[it.sys];
    const int64_t i = S.o + (int64_t)it.b * 64 + lane;
    double xn[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t e = d * total + i;
      if (kicks > 0) {
        const double ae = a[e];
        double ve = fma(h, ae, v[e]);
        if (kicks > 1) ve = fma(h, ae, ve);
        v[e] = ve;
        xn[d] = fma(dt, ve, x[e]);
        x[e] = xn[d];
      } else {
        xn[d] = x[e];
      }
    }
    const float4 hi = make_float4((float)xn[0], (float)xn[1], (float)xn[2], (float)m[i]);
    rhi[i] = hi;
    rlo[i] = make_float4((float)(xn[0] - (double)hi.x), (float)(xn[1] - (double)hi.y), (float)(xn[2] - (double)hi.z),
                         NEAR ? sym_rc2(xn[0], xn[1], xn[2], S.eps, S.fx) : -1.f);
  }
}

__global__ void esym_kick_kernel(int64_t total, double* __restrict__ v, const double* __restrict__ a, double h) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 3 * total; e += (int64_t)gridDim.x * blockDim.x)
    v[e] = fma(h, a[e], v[e]);
}

// One step of a sub-block: the lane's i against record (r + K) of its row.
template <int K, bool NEAR>
__device__ __forceinline__ void esym_step(const float4& ip, float mneg, const float4* __restrict__ rowp, float e2,
                                          float& px, float& py, float& pz, float& r2m, float& ajx, float& ajy,
                                          float& ajz) {
  const float4 r = rowp[K];
  const float dx = r.x - ip.x, dy = r.y - ip.y, dz = r.z - ip.z;
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
  const float ri = rsqrt32(r2);
  const float ri3 = (ri * ri) * ri;
  const float si = r.w * ri3;
  px = fmaf(si, dx, px);
  py = fmaf(si, dy, py);
  pz = fmaf(si, dz, pz);
  if constexpr (NEAR) r2m = fminf(r2m, r2);
  const float sj = mneg * ri3;
  const float tx = sj * dx, ty = sj * dy, tz = sj * dz;
  // the j met here sits at row position (r + K): its owner is K lanes further on
  if constexpr (K == 0) { ajx += tx; ajy += ty; ajz += tz; }
  else {
    ajx += row_ror<K>(tx);
    ajy += row_ror<K>(ty);
    ajz += row_ror<K>(tz);
  }
}

template <bool NEAR, int... K>
__device__ __forceinline__ void esym_sub(const float4& ip, float mneg, const float4* __restrict__ rowp, float e2,
                                         float& px, float& py, float& pz, float& r2m, float& ajx, float& ajy,
                                         float& ajz, std::integer_sequence<int, K...>) {
  (esym_step<K, NEAR>(ip, mneg, rowp, e2, px, py, pz, r2m, ajx, ajy, ajz), ...);
}

// EST (FP32C with the rescue): the i-side shares of the error estimate into
// iest, each block pair's closest pair left in rounded positions into wslots.
template <bool NEAR, bool EXCL, bool EST>
__global__ __launch_bounds__(kEBlock, kEOcc) void esym_force_kernel(
    const ESys* __restrict__ sys, const EItem* __restrict__ items, const int* __restrict__ wg_off,
    const int* __restrict__ wg_list, const float4* __restrict__ rhi, const float4* __restrict__ rlo,
    double* __restrict__ a, double* __restrict__ islot, float* __restrict__ slots, int64_t total,
    float* __restrict__ iest, float* __restrict__ wslots) {
  static_assert(NEAR || !EST, "the estimate belongs to FP32C");
  __shared__ float4 s_hi[kEWaves][4][2 * kSR];  // (x, y, z, m) hi parts, each sub-block twice
  __shared__ float4 s_lo[kEWaves][64];          // lo parts and the repair radius^2
  __shared__ float s_j[kEWaves][3][64];         // the block pair's j-side sums
  __shared__ int next_item;
  const int t = threadIdx.x;
  const int wv = t >> 6, lane = t & 63, rl = lane & (kSR - 1), row = lane >> 4;
  const int xor32 = (lane ^ 32) * 4;
  const int q0 = wg_off[blockIdx.x], q1 = wg_off[blockIdx.x + 1];
  if (t == 0) next_item = 0;
  __syncthreads();
  for (;;) {
    int k = 0;
    if (lane == 0) k = atomicAdd(&next_item, 1);
    k = __builtin_amdgcn_readfirstlane(k);
    if (k >= q1 - q0) break;
    const EItem it = items[wg_list[q0 + k]];
    const ESys& S = sys[it.sys];
    const int nc = S.nc, nb = S.nb;
    const float4* hs = rhi + S.o;
    const float4* ls = rlo + S.o;
    const float e2 = (float)(S.eps * S.eps);
    const int il = it.b * 64 + lane;
    const bool valid = lane < it.ni;
    // padding (past the system's end): far away, massless, never repaired
    auto load = [&](int j, float4& rh, float4& rq) {
      if (j < nc) {
        rh = hs[j];
        rq = ls[j];
      } else {
        rh = make_float4((float)kFarAway, (float)kFarAway, (float)kFarAway, 0.f);
        rq = make_float4(0.f, 0.f, 0.f, -1.f);
      }
    };
    float4 ip, iq;
    load(valid ? il : nc, ip, iq);
    const float mneg = -ip.w;
    // flags a block pair for the repair: every pair inside the larger radius of
    // its two particles is inside this one (|d| < f |x_j| with |x_j| <= |x_i| + |d|
    // gives |d| < f / (1 - f) |x_i|; the eps term is the same for both)
    const float thr = (NEAR && valid)
                          ? sym_rc2((double)ip.x, (double)ip.y, (double)ip.z, S.eps, S.fx / (1.0f - S.fx) * 1.0001f)
                          : -1.f;
    auto fetch = [&](int J, float4& rh, float4& rq) { load(J * 64 + lane, rh, rq); };
    auto put = [&](const float4& rh, const float4& rq) {
      wave_sync();
      s_hi[wv][row][rl] = rh;
      s_hi[wv][row][rl + kSR] = rh;
      s_lo[wv][lane] = rq;
      wave_sync();
    };
    float hx = 0.f, hy = 0.f, hz = 0.f, lx = 0.f, ly = 0.f, lz = 0.f;
    float eacc = 0.f;  // the lane's i-side share of its row's error estimate (EST)
    // |x_i|_inf, formed where it is used (cheaper than a register held over the item)
    auto xinf = [&]() { return fmaxf(fabsf(ip.x), fmaxf(fabsf(ip.y), fabsf(ip.z))); };
    float4 nh, nq;
    const int r0 = it.d0 > 0 ? it.d0 : 1;  // first distance of the ring in this part
    if (it.d0 == 0) {
      fetch(it.b, nh, nq);
      put(nh, nq);
    }
    if (r0 < it.d1) fetch(it.b + r0 < nb ? it.b + r0 : it.b + r0 - nb, nh, nq);
    if (it.d0 == 0) {
      // the block with itself: ordered pairs, i-side only
      float px = 0.f, py = 0.f, pz = 0.f, r2min = 3.0e38f;
#pragma unroll 16
      for (int jj = 0; jj < 64; ++jj) {
        const float4 r = s_hi[wv][jj >> 4][jj & (kSR - 1)];
        const float dx = r.x - ip.x, dy = r.y - ip.y, dz = r.z - ip.z;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
        const float ri = rsqrt32(r2);
        float sc = (r.w * ri) * (ri * ri);
        if constexpr (EXCL) sc = jj == lane ? 0.f : sc;
        px = fmaf(sc, dx, px);
        py = fmaf(sc, dy, py);
        pz = fmaf(sc, dz, pz);
        if constexpr (NEAR) r2min = fminf(r2min, jj == lane ? 3.0e38f : r2);
      }
      if constexpr (NEAR) {
        if (r2min < iq.w) {
          // rare: redo the block with float-float displacements for the pairs
          // closer than particle i's repair radius
          float qx = 0.f, qy = 0.f, qz = 0.f, r2nr = 3.0e38f;
          for (int jj = 0; jj < 64; ++jj) {
            const float4 r = s_hi[wv][jj >> 4][jj & (kSR - 1)];
            const float4 q = s_lo[wv][jj];
            float dx = r.x - ip.x, dy = r.y - ip.y, dz = r.z - ip.z;
            float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
            if (r2 < iq.w) {
              dx += q.x - iq.x;
              dy += q.y - iq.y;
              dz += q.z - iq.z;
              r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
            } else if (jj != lane) {
              r2nr = fminf(r2nr, r2);
            }
            const float ri = rsqrt32(r2);
            float sc = (r.w * ri) * (ri * ri);
            if constexpr (EXCL) sc = jj == lane ? 0.f : sc;
            qx = fmaf(sc, dx, qx);
            qy = fmaf(sc, dy, qy);
            qz = fmaf(sc, dz, qz);
          }
          px = qx;
          py = qy;
          pz = qz;
          r2min = r2nr;
        }
        // the block's share of the estimate, weighted by its closest pair left
        // in rounded positions
        if constexpr (EST) eacc = est_add(eacc, px, py, pz, xinf(), r2min);
      }
      fold(hx, lx, px);
      fold(hy, ly, py);
      fold(hz, lz, pz);
    }
    const size_t npad = (size_t)nb * 64;
#pragma unroll 1
    for (int d = r0; d < it.d1; ++d) {
      const int J = it.b + d < nb ? it.b + d : it.b + d - nb;
      put(nh, nq);
      if (d + 1 < it.d1) fetch(J + 1 < nb ? J + 1 : J + 1 - nb, nh, nq);
      float px = 0.f, py = 0.f, pz = 0.f, r2m = 3.0e38f;
#pragma unroll 1
      for (int q = 0; q < 4; ++q) {
        float ajx = 0.f, ajy = 0.f, ajz = 0.f;
        esym_sub<NEAR>(ip, mneg, &s_hi[wv][q][rl], e2, px, py, pz, r2m, ajx, ajy, ajz,
                       std::make_integer_sequence<int, kSR>{});
        // the four rows' sums of the same 16 j: rows (0 + 1) and (2 + 3) by a
        // swizzle, then the two halves by a permute; every row then holds the
        // totals and stores the same values
        ajx += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(ajx), 0x401F));
        ajy += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(ajy), 0x401F));
        ajz += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(ajz), 0x401F));
        ajx += __int_as_float(__builtin_amdgcn_ds_bpermute(xor32, __float_as_int(ajx)));
        ajy += __int_as_float(__builtin_amdgcn_ds_bpermute(xor32, __float_as_int(ajy)));
        ajz += __int_as_float(__builtin_amdgcn_ds_bpermute(xor32, __float_as_int(ajz)));
        s_j[wv][0][q * kSR + rl] = ajx;
        s_j[wv][1][q * kSR + rl] = ajy;
        s_j[wv][2][q * kSR + rl] = ajz;
      }
      if constexpr (NEAR) {
        wave_sync();
        float r2nr = r2m;  // a lane without a repair keeps all its pairs in rounded positions
        if (r2m < thr) {
          r2nr = 3.0e38f;
          // rare: for every pair of the lane's i closer than the larger repair
          // radius of its two particles, the rounded-position term is replaced
          // by the float-float one on both sides.  The j are visited in the
          // rotated order of the pair loop, so at each step the lanes of a row
          // touch distinct j; the four rows, which share the j, take turns.
          for (int jj = 0; jj < 64; ++jj) {
            const int q = jj >> 4;
            const int jl = q * kSR + ((rl + jj) & (kSR - 1));
            const float4 r = s_hi[wv][q][jl & (kSR - 1)];
            const float4 ql = s_lo[wv][jl];
            const float dx = r.x - ip.x, dy = r.y - ip.y, dz = r.z - ip.z;
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
            float cx = 0.f, cy = 0.f, cz = 0.f;
            if (!(r2 < fmaxf(iq.w, ql.w))) r2nr = fminf(r2nr, r2);
            if (r2 < fmaxf(iq.w, ql.w)) {
              const float ex = dx + (ql.x - iq.x), ey = dy + (ql.y - iq.y), ez = dz + (ql.z - iq.z);
              const float ri = rsqrt32(r2);
              const float ri3 = (ri * ri) * ri;
              const float q2 = fmaf(ez, ez, fmaf(ey, ey, fmaf(ex, ex, e2)));
              const float qi = rsqrt32(q2);
              const float qi3 = (qi * qi) * qi;
              // float-float term minus rounded term, per unit mass
              const float fx3 = fmaf(qi3, ex, -(ri3 * dx));
              const float fy3 = fmaf(qi3, ey, -(ri3 * dy));
              const float fz3 = fmaf(qi3, ez, -(ri3 * dz));
              px = fmaf(r.w, fx3, px);
              py = fmaf(r.w, fy3, py);
              pz = fmaf(r.w, fz3, pz);
              cx = mneg * fx3;
              cy = mneg * fy3;
              cz = mneg * fz3;
            }
            for (int rr = 0; rr < 4; ++rr) {
              if (row == rr && (cx != 0.f || cy != 0.f || cz != 0.f)) {
                s_j[wv][0][jl] += cx;
                s_j[wv][1][jl] += cy;
                s_j[wv][2][jl] += cz;
              }
              wave_sync();  // one row's turn ends before the next row reads the sums
            }
          }
        }
        if constexpr (EST) {
          eacc = est_add(eacc, px, py, pz, xinf(), r2nr);
          // the wave's minimum: within each row of 16 by rotations, then rows
          // (0 + 1) and (2 + 3) by a swizzle, then the two halves by a permute
          float tm = r2nr;
          tm = fminf(tm, row_ror<8>(tm));
          tm = fminf(tm, row_ror<4>(tm));
          tm = fminf(tm, row_ror<2>(tm));
          tm = fminf(tm, row_ror<1>(tm));
          tm = fminf(tm, __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(tm), 0x401F)));
          tm = fminf(tm, __int_as_float(__builtin_amdgcn_ds_bpermute(xor32, __float_as_int(tm))));
          if (lane == 0) wslots[S.wbase + (size_t)(d - 1) * nb + J] = tm;
        }
      }
      fold(hx, lx, px);
      fold(hy, ly, py);
      fold(hz, lz, pz);
      wave_sync();
      float* dst = slots + S.sbase + (size_t)(d - 1) * 3 * npad + (size_t)J * 64 + lane;
      dst[0] = s_j[wv][0][lane];
      dst[npad] = s_j[wv][1][lane];
      dst[2 * npad] = s_j[wv][2][lane];
    }
    if (valid) {
      // part 0 (the one with the block itself) writes a, unscaled; the others their slots
      double* o = it.part == 0 ? a + S.o + il : islot + S.ibase + (size_t)(it.part - 1) * 3 * npad + il;
      const size_t st = it.part == 0 ? (size_t)total : npad;
      o[0] = (double)hx + (double)lx;
      o[st] = (double)hy + (double)ly;
      o[2 * st] = (double)hz + (double)lz;
      if constexpr (EST) iest[S.iebase + (size_t)it.part * npad + il] = eacc;
    }
  }
}

// a = G (the particle's i-side sums in part order, part 0 in a itself, + its
// j-side slots in distance order), in FP64;
// one thread per (particle, component: blockIdx.y), the slots loaded eight at
// a time.  Only the largest distance can be missing: the slot of a block whose
// partner at distance dmax lies in the upper half of an even ring (that block
// pair is visited from the lower half only, where it is distance dmax the
// other way).
__global__ void esym_reduce_kernel(int nblocks, const EItem* __restrict__ blocks, const ESys* __restrict__ sys,
                                   int64_t total, const double* __restrict__ islot, const float* __restrict__ slots,
                                   double* __restrict__ a, double G) {
  const int c = blockIdx.y;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < (int64_t)nblocks * 64;
       g += (int64_t)gridDim.x * blockDim.x) {
    const EItem it = blocks[g >> 6];
    const int lane = (int)(g & 63);
    if (lane >= it.ni) continue;
    const ESys& S = sys[it.sys];
    const int p = it.b * 64 + lane;
    const int64_t i = S.o + p;
    const size_t npad = (size_t)S.nb * 64;
    int dn = S.dmax;
    if (S.half && dn > 0) {
      int src = it.b - S.dmax;
      if (src < 0) src += S.nb;
      if (src >= S.nb / 2) --dn;
    }
    const size_t stride = 3 * npad;
    const int np = (esym_dend(S, it.b) + S.lp - 1) / S.lp;
    const double* iq = islot + S.ibase + c * npad + p;
    double acc = a[c * total + i];
    for (int k = 1; k < np; ++k) acc += iq[(size_t)(k - 1) * stride];
    const float* q = slots + S.sbase + c * npad + p;
    int d = 0;
    for (; d + 8 <= dn; d += 8) {
      float f[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) f[u] = q[(size_t)(d + u) * stride];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += (double)f[u];
    }
    for (; d < dn; ++d) acc += (double)q[(size_t)d * stride];
    a[c * total + i] = G * acc;
  }
}

// The same sums with the rescue's estimate, one thread per particle (the three
// components read together, each added in the order above, so the forces equal
// those of esym_reduce_kernel bitwise).  The row's estimate adds its i-side
// shares in part order, then per distance the far side's share: the j-side sum
// of the slot, weighted by the closest pair of its block pair left in rounded
// positions, or by the particle's own repair radius where that is larger
// (pairs inside it were repaired).  A row whose estimate is too large against
// |a_i| (see rescue.hip) is appended to its system's list for the batched
// rescue (rlist from the system's first particle on, system-local indices,
// rcnt[system] rows; one atomic add per wave, a wave being one block of 64 of
// one system).
__global__ void esym_reduce_est_kernel(int nblocks, const EItem* __restrict__ blocks, const ESys* __restrict__ sys,
                                       int64_t total, const double* __restrict__ islot,
                                       const float* __restrict__ slots, const float* __restrict__ iest,
                                       const float* __restrict__ wslots, const float4* __restrict__ rhi,
                                       const float4* __restrict__ rlo, double* __restrict__ a, double G,
                                       int* __restrict__ rcnt, int* __restrict__ rlist) {
  // the grid stride is a whole number of waves, so every wave stays one block
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < (int64_t)nblocks * 64;
       g += (int64_t)gridDim.x * blockDim.x) {
    const EItem it = blocks[g >> 6];
    const int lane = (int)(g & 63);
    const ESys& S = sys[it.sys];
    const int p = it.b * 64 + lane;
    bool flag = false;
    if (lane < it.ni) {
      const int64_t i = S.o + p;
      const size_t npad = (size_t)S.nb * 64;
      int dn = S.dmax;
      if (S.half && dn > 0) {
        int src = it.b - S.dmax;
        if (src < 0) src += S.nb;
        if (src >= S.nb / 2) --dn;
      }
      const size_t stride = 3 * npad;
      const int np = (esym_dend(S, it.b) + S.lp - 1) / S.lp;
      double ax = a[i], ay = a[total + i], az = a[2 * total + i];
      const double* iq = islot + S.ibase + p;
      for (int k = 1; k < np; ++k) {
        const double* o = iq + (size_t)(k - 1) * stride;
        ax += o[0];
        ay += o[npad];
        az += o[2 * npad];
      }
      float e = 0.f;
      for (int k = 0; k < np; ++k) e += iest[S.iebase + (size_t)k * npad + p];
      const float4 rh = rhi[i];
      const float rc = rlo[i].w;
      const float xw = kEstNear * fmaxf(fabsf(rh.x), fmaxf(fabsf(rh.y), fabsf(rh.z)));
      const float* q = slots + S.sbase + p;
      const float* wq = wslots + S.wbase + it.b;
#pragma unroll 4
      for (int d = 0; d < dn; ++d) {
        const float* qd = q + (size_t)d * stride;
        const float fx = qd[0], fy = qd[npad], fz = qd[2 * npad];
        const float w = fmaf(xw, rsqrt32(fmaxf(wq[(size_t)d * S.nb], rc)), 1.0f);
        ax += (double)fx;
        ay += (double)fy;
        az += (double)fz;
        e = fmaf(w * w, fmaf(fx, fx, fmaf(fy, fy, fz * fz)), e);
      }
      ax *= G;
      ay *= G;
      az *= G;
      a[i] = ax;
      a[total + i] = ay;
      a[2 * total + i] = az;
      flag = sqrt((double)e) * (kRescueScale * fabs(G)) > sqrt(ax * ax + ay * ay + az * az);
    }
    const unsigned long long mask = __ballot(flag);
    if (mask) {
      int base = 0;
      if (lane == 0) base = atomicAdd(&rcnt[it.sys], __popcll(mask));
      base = __shfl(base, 0, 64);
      if (flag) rlist[S.o + base + __popcll(mask & ((1ull << lane) - 1ull))] = p;
    }
  }
}

// ------------------------------------------------------------------ plans
struct EPlan {
  std::vector<int64_t> off;
  std::vector<double> eps;
  int precision = 0, device = 0, ncl = 0, nwg = 0, nblocks = 0;
  int64_t total = 0;
  ESys* d_sys = nullptr;
  EItem* d_blocks = nullptr;  // one per block of 64 (publish, reduce)
  EItem* d_items = nullptr;   // the parts (force)
  double* d_islot = nullptr;
  int* d_wg_off = nullptr;
  int* d_wg_list = nullptr;
  float4* d_rhi = nullptr;
  float4* d_rlo = nullptr;
  float* d_slots = nullptr;
  // FP32C: the rescue's estimate slots, the systems' offsets and softenings
  // on the device, and the per-system lists of flagged rows
  float* d_iest = nullptr;
  float* d_wslots = nullptr;
  int64_t* d_off = nullptr;
  double* d_eps = nullptr;
  int* d_rcnt = nullptr;   // ncl
  int* d_rlist = nullptr;  // total
};

std::mutex g_eplan_mu;
std::vector<EPlan*> g_eplans;

void free_eplan(EPlan* p) {
  for (void* q : {(void*)p->d_sys, (void*)p->d_blocks, (void*)p->d_items, (void*)p->d_islot, (void*)p->d_wg_off,
                  (void*)p->d_wg_list, (void*)p->d_rhi, (void*)p->d_rlo, (void*)p->d_slots, (void*)p->d_iest,
                  (void*)p->d_wslots, (void*)p->d_off, (void*)p->d_eps, (void*)p->d_rcnt, (void*)p->d_rlist})
    if (q) (void)hipFree(q);
  delete p;
}

template <typename T>
bool eupload(T** dst, const std::vector<T>& src) {
  const size_t bytes = sizeof(T) * std::max<size_t>(1, src.size());
  if (hipMalloc(dst, bytes) != hipSuccess) return false;
  return src.empty() || hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) == hipSuccess;
}

// Bytes of j-side slots the layout needs: per system, dmax distances x 3
// components x its padded particle count, in FP32.
size_t esym_slot_bytes(int32_t ncl, const int64_t* off) {
  size_t f = 0;
  for (int c = 0; c < ncl; ++c) {
    const int64_t nb = (off[c + 1] - off[c] + 63) / 64;
    f += (size_t)(nb / 2) * 3 * (size_t)nb * 64;
  }
  return f * sizeof(float);
}

// Blocks: every system cut into blocks of 64.  Items: each block's distances
// 0 .. dend - 1 cut into parts of lp, lp chosen so that the parts number about
// four per wave the launch holds (whole half rings of the largest systems would
// leave a few long items at the end of the step).  An item's cost is 48 for
// its ordered block (64 pairs per lane at about 3/4 of a symmetric step) plus
// 64 per ring distance plus a fixed 32; items go longest first to the least
// loaded workgroup, and each workgroup's list stays in decreasing cost (the
// order its waves take them in).
int build_eplan(int32_t ncl, const int64_t* off, const double* eps, int precision, int device, EPlan** out) {
  EPlan* p = new EPlan();
  p->off.assign(off, off + ncl + 1);
  p->eps.assign(eps, eps + ncl);
  p->precision = precision;
  p->device = device;
  p->ncl = ncl;
  p->total = off[ncl];
  int per_cu = kEMaxPerCu;
  for (const void* f : {reinterpret_cast<const void*>(&esym_force_kernel<true, false, false>),
                        reinterpret_cast<const void*>(&esym_force_kernel<true, true, false>),
                        reinterpret_cast<const void*>(&esym_force_kernel<true, false, true>),
                        reinterpret_cast<const void*>(&esym_force_kernel<true, true, true>)}) {
    int k = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, f, kEBlock, 0) != hipSuccess) {
      (void)hipGetLastError();
      k = 1;
    }
    per_cu = std::min(per_cu, k);
  }
  per_cu = std::max(1, per_cu);
  const int cap_wg = std::max(1, per_cu * cu_count(device));
  std::vector<ESys> sys(std::max(1, ncl));
  int64_t work = 0;  // block distances (the ordered block counted as one)
  for (int c = 0; c < ncl; ++c) {
    const int64_t nb = (off[c + 1] - off[c] + 63) / 64;
    work += nb * (nb / 2) + nb - ((nb % 2 == 0) ? nb / 2 : 0);
  }
  const int lp = (int)std::max<int64_t>(4, std::min<int64_t>(64, work / (4 * (int64_t)cap_wg * kEWaves)));
  std::vector<EItem> blocks, items;
  std::vector<double> cost;
  int64_t sbase = 0, ibase = 0, iebase = 0, wbase = 0;
  for (int c = 0; c < ncl; ++c) {
    const int64_t nc = off[c + 1] - off[c];
    ESys& S = sys[c];
    S.o = off[c];
    S.sbase = sbase;
    S.ibase = ibase;
    S.iebase = iebase;
    S.wbase = wbase;
    S.eps = eps[c];
    S.nc = (int)nc;
    S.nb = (int)((nc + 63) / 64);
    S.dmax = S.nb / 2;
    S.half = S.nb % 2 == 0 ? 1 : 0;
    S.fx = std::max(kNearX, kNearN / std::cbrt((float)std::max<int64_t>(1, nc)));
    S.lp = lp;
    sbase += (int64_t)S.dmax * 3 * S.nb * 64;
    ibase += (int64_t)((S.dmax + 1 + lp - 1) / lp - 1) * 3 * S.nb * 64;
    iebase += (int64_t)((S.dmax + 1 + lp - 1) / lp) * S.nb * 64;
    wbase += (int64_t)S.dmax * S.nb;
    for (int b = 0; b < S.nb; ++b) {
      const int ni = (int)std::min<int64_t>(64, nc - (int64_t)b * 64);
      const int dend = esym_dend(S, b);
      blocks.push_back(EItem{c, b, ni, 0, dend, 0});
      for (int d0 = 0, part = 0; d0 < dend; d0 += lp, ++part) {
        const int d1 = std::min(dend, d0 + lp);
        items.push_back(EItem{c, b, ni, d0, d1, part});
        cost.push_back((d0 == 0 ? 48.0 : 0.0) + 64.0 * (d1 - std::max(d0, 1)) + 32.0);
      }
    }
  }
  const int nwg = std::max(1, std::min<int>((int)((items.size() + kEWaves - 1) / kEWaves), cap_wg));
  std::vector<int> order(items.size());
  for (size_t k = 0; k < items.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int u, int w) { return cost[u] > cost[w]; });
  std::vector<std::vector<int>> lists(nwg);
  using Slot = std::pair<double, int>;
  std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
  for (int w = 0; w < nwg; ++w) heap.push({0.0, w});
  for (int k : order) {
    Slot sl = heap.top();
    heap.pop();
    lists[sl.second].push_back(k);
    heap.push({sl.first + cost[k], sl.second});
  }
  std::vector<int> wg_off(nwg + 1, 0), wg_list;
  for (int w = 0; w < nwg; ++w) {
    wg_list.insert(wg_list.end(), lists[w].begin(), lists[w].end());
    wg_off[w + 1] = (int)wg_list.size();
  }
  p->nwg = nwg;
  p->nblocks = (int)blocks.size();
  const size_t nrec = (size_t)std::max<int64_t>(1, p->total);
  bool ok = eupload(&p->d_sys, sys) && eupload(&p->d_blocks, blocks) && eupload(&p->d_items, items) &&
            hipMalloc(&p->d_islot, sizeof(double) * (size_t)std::max<int64_t>(1, ibase)) == hipSuccess && eupload(&p->d_wg_off, wg_off) &&
            eupload(&p->d_wg_list, wg_list) && hipMalloc(&p->d_rhi, nrec * sizeof(float4)) == hipSuccess &&
            hipMalloc(&p->d_rlo, nrec * sizeof(float4)) == hipSuccess &&
            hipMalloc(&p->d_slots, sizeof(float) * (size_t)std::max<int64_t>(1, sbase)) == hipSuccess;
  if (ok && precision == NBODY_FP32C)
    ok = hipMalloc(&p->d_iest, sizeof(float) * (size_t)std::max<int64_t>(1, iebase)) == hipSuccess &&
         hipMalloc(&p->d_wslots, sizeof(float) * (size_t)std::max<int64_t>(1, wbase)) == hipSuccess &&
         eupload(&p->d_off, p->off) && eupload(&p->d_eps, p->eps) &&
         hipMalloc(&p->d_rcnt, sizeof(int) * (size_t)std::max(1, ncl)) == hipSuccess &&
         hipMalloc(&p->d_rlist, sizeof(int) * nrec) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_eplan(p);
    return set_error(NBODY_ENOMEM, "batched: plan upload failed");
  }
  *out = p;
  return NBODY_OK;
}

EPlan* find_eplan(int32_t ncl, const int64_t* off, const double* eps, int precision, int device) {
  for (EPlan* p : g_eplans) {
    if (p->device != device || p->precision != precision || p->ncl != ncl) continue;
    if (std::equal(p->off.begin(), p->off.end(), off) && std::equal(p->eps.begin(), p->eps.end(), eps)) return p;
  }
  return nullptr;
}

// EST (FP32C with the rescue): each step's force also keeps the error
// estimate, the reduction lists the flagged rows, and the batched rescue
// recomputes them in FP64 before the next kick.
template <bool NEAR, bool EST>
int launch_esteps(const EPlan* p, double* x, double* v, double* a, const double* m, double dt, int64_t nsteps,
                  double G, bool acc_valid, bool excl, hipStream_t s) {
  if (p->total == 0 || (nsteps == 0 && acc_valid)) return NBODY_OK;
  const double h = 0.5 * dt;
  const unsigned ew = (unsigned)std::min<int64_t>(((int64_t)p->nblocks * 64 + 255) / 256, 4096);
  const unsigned kw = (unsigned)std::min<int64_t>((3 * p->total + 255) / 256, 4096);
  int* rcnt = EST ? p->d_rcnt : nullptr;
  auto step = [&](int kicks) -> int {
    esym_publish_kernel<NEAR><<<ew, 256, 0, s>>>(p->nblocks, p->d_blocks, p->d_sys, p->total, x, v, a, m, p->d_rhi,
                                                  p->d_rlo, h, dt, kicks, rcnt, p->ncl);
    NB_LAUNCH_CHECK("esym_publish_kernel");
    if (excl)
      esym_force_kernel<NEAR, true, EST><<<p->nwg, kEBlock, 0, s>>>(p->d_sys, p->d_items, p->d_wg_off, p->d_wg_list,
                                                                    p->d_rhi, p->d_rlo, a, p->d_islot, p->d_slots,
                                                                    p->total, p->d_iest, p->d_wslots);
    else
      esym_force_kernel<NEAR, false, EST><<<p->nwg, kEBlock, 0, s>>>(p->d_sys, p->d_items, p->d_wg_off, p->d_wg_list,
                                                                     p->d_rhi, p->d_rlo, a, p->d_islot, p->d_slots,
                                                                     p->total, p->d_iest, p->d_wslots);
    NB_LAUNCH_CHECK("esym_force_kernel");
    if constexpr (EST) {
      esym_reduce_est_kernel<<<ew, 256, 0, s>>>(p->nblocks, p->d_blocks, p->d_sys, p->total, p->d_islot, p->d_slots,
                                                p->d_iest, p->d_wslots, p->d_rhi, p->d_rlo, a, G, p->d_rcnt,
                                                p->d_rlist);
      NB_LAUNCH_CHECK("esym_reduce_est_kernel");
      return launch_ens_rescue(p->ncl, p->d_off, p->d_eps, p->total, x, m, G, excl, p->d_rcnt, p->d_rlist, a, s);
    }
    esym_reduce_kernel<<<dim3(ew, 3), 256, 0, s>>>(p->nblocks, p->d_blocks, p->d_sys, p->total, p->d_islot,
                                                   p->d_slots, a, G);
    NB_LAUNCH_CHECK("esym_reduce_kernel");
    return NBODY_OK;
  };
  int st;
  if (!acc_valid && (st = step(0))) return st;
  for (int64_t k = 0; k < nsteps; ++k)
    if ((st = step(k == 0 ? 1 : 2))) return st;
  if (nsteps > 0) {
    esym_kick_kernel<<<kw, 256, 0, s>>>(p->total, v, a, h);
    NB_LAUNCH_CHECK("esym_kick_kernel");
  }
  return NBODY_OK;
}

}  // namespace

int run_batched_stream(int32_t ncl, const int64_t* off, const double* eps, double* x, double* v, double* a,
                       const double* m, double dt, int64_t nsteps, double G, int precision, bool excl,
                       bool acc_valid, int bitem, bool per_step, bool rescue, hipStream_t s);

// Mode 4.  FP64, and layouts whose slots would exceed kESlotCap, run the
// ordered per-step wave items (mode 3) instead; FP32C takes the rescue as
// asked in either form.
int run_batched_sym(int32_t ncl, const int64_t* off, const double* eps, double* x, double* v, double* a,
                    const double* m, double dt, int64_t nsteps, double G, int precision, bool excl, bool acc_valid,
                    bool rescue, hipStream_t s) {
  if (precision == NBODY_FP64 || esym_slot_bytes(ncl, off) > kESlotCap)
    return run_batched_stream(ncl, off, eps, x, v, a, m, dt, nsteps, G, precision, excl, acc_valid, 64, true, rescue,
                              s);
  for (int c = 0; c < ncl; ++c)
    if (off[c + 1] - off[c] > (int64_t(1) << 24))
      return set_error(NBODY_EUNSUPPORTED, "batched: a system of more than 2^24 particles");
  const int device = current_device();
  std::lock_guard<std::mutex> lk(g_eplan_mu);
  EPlan* p = find_eplan(ncl, off, eps, precision, device);
  if (!p) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return set_error(NBODY_EINVAL, "batched: the plan for this layout must be built by one call outside stream capture");
    int st = build_eplan(ncl, off, eps, precision, device, &p);
    if (st) return st;
    g_eplans.push_back(p);
  }
  if (precision == NBODY_FP32C && rescue)
    return launch_esteps<true, true>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, s);
  if (precision == NBODY_FP32C) return launch_esteps<true, false>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, s);
  return launch_esteps<false, false>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, s);
}

// The untuned default takes the symmetric items when the layout's block pairs
// outnumber its blocks (its systems mostly span several blocks of 64): a
// layout of single-block systems has no pair to save and would only pay the
// third launch.
bool sym_ensemble_default(int32_t ncl, const int64_t* off) {
  int64_t blocks = 0, ring = 0;
  for (int c = 0; c < ncl; ++c) {
    const int64_t nb = (off[c + 1] - off[c] + 63) / 64;
    blocks += nb;
    ring += nb * (nb / 2) - ((nb % 2 == 0) ? nb / 2 : 0);
  }
  return ring >= blocks && esym_slot_bytes(ncl, off) <= kESlotCap;
}

void release_sym_ensemble_plans() {
  std::lock_guard<std::mutex> lk(g_eplan_mu);
  for (EPlan* p : g_eplans) free_eplan(p);
  g_eplans.clear();
}

}  // namespace nb
