// All-pairs kernels of libnbody_accel: acceleration, its vector-Jacobian
// product, and the pair potential used by the diagnostics.
//
// Shape of every kernel (the MI355X counterpart of the paper's read / compute /
// write pipeline, Sec. 3.1 and Algorithms 1-2):
//   * one i-particle per lane (IPL of them per lane, strided by the block size
//     so loads and stores stay coalesced); a workgroup of 256 lanes owns
//     256 * IPL consecutive i's and a contiguous j-range (the grid's y index
//     splits the j-range when there are too few i-blocks to fill 256 CUs);
//   * the j-range is streamed through LDS in tiles of 256 records, double
//     buffered: while the tile in LDS is consumed, the next tile's FP64 values
//     are already in flight from global memory to registers, and are converted
//     and written to the other LDS buffer before the single barrier per tile;
//   * every lane reads the same LDS record (a broadcast, no bank conflicts) and
//     applies it to its IPL i-particles with the pair arithmetic of App. A,
//     Algorithm 3: displacement, squared distance (+ eps^2), inverse square
//     root, cube, weight times cube, accumulate;
//   * partial sums of kFold terms are kept in plain arithmetic and folded into
//     a (hi, lo) pair with Knuth's TwoSum, so the j-sum is compensated at a
//     cost of a few operations per 64 pairs;
//   * the tile loader converts the caller's FP64 SoA positions on the fly, so
//     no staging pass or staging buffer exists: FP32C keeps each coordinate as
//     hi = fl32(x), lo = fl32(x - hi) and forms x_j - x_i = (hi_j - hi_i) +
//     (lo_j - lo_i), where the first difference is exact for nearby pairs
//     (Sterbenz) -- the only place where FP32 positions lose accuracy.
// Padding j-records (past the j-range) sit at kFarAway with zero mass, so they
// contribute exactly zero without a bounds test in the inner loop.
#include "pair_math.h"

namespace nb {
namespace {

// Loads the record of j (or padding if j >= je) from the caller's FP64 arrays.
template <int MODE>
__device__ __forceinline__ JRec<MODE> load_rec(const double* __restrict__ x, const double* __restrict__ m,
                                               int n, int j, int je) {
  if (j < je) return JRec<MODE>::make(x[j], x[n + j], x[2 * n + j], m[j]);
  return JRec<MODE>::make(kFarAway, kFarAway, kFarAway, 0.0);
}

// ============================================================== acceleration
// Near-field repair of the FP32C force: pairs are evaluated from positions
// rounded to FP32 (12 VALU operations per pair instead of 18 with float-float
// displacements), and every lane tracks the smallest squared distance it met
// in each block of kFold j-particles.  Rounding a coordinate to FP32 moves it
// by up to 2^-24 |x|, which only matters for pairs much closer than |x|; when
// a block holds a pair closer than d_c(i) = max(kNearX |x_i|, kNearEps eps),
// that lane rescans the block and replaces the term of each such pair by its
// term from float-float displacements.  Such blocks are rare (a pair closer
// than a few eps, or the block of the lane's own pair), so the force costs one
// extra min per pair and keeps float-float accuracy.

// Grid: (ceil(n / (256*IPL)), split).  Block y handles j in [y*chunk, min(n, (y+1)*chunk)).
// split == 1: writes G*(hi+lo) to a[c*n+i].  split > 1: writes hi+lo to
// part[(y*3+c)*n+i] and a second kernel sums the slices in order.
// NEAR (FP32C only): rounded-position pairs with the near-field repair above;
// otherwise FP32C uses float-float displacements for every pair.  With NEAR
// and est != nullptr, the row's rounding-error estimate over this slice (one
// share per fold block, see rescue.hip) goes to est[y*n+i].
template <int MODE, int IPL, bool EXCL, bool NEAR>
__global__ __launch_bounds__(kBlock) void accel_kernel(int n, const double* __restrict__ x,
                                                       const double* __restrict__ m, double eps, double G,
                                                       int chunk, double* __restrict__ out, float* __restrict__ est,
                                                       int* __restrict__ zc) {
  using R = Real<MODE>;
  static_assert(!NEAR || MODE == kFP32C, "the near-field repair needs float-float records");
  __shared__ JRec<MODE> tile[2][kTile];
  const int t = threadIdx.x;
  if (zc && blockIdx.x == 0 && blockIdx.y == 0 && t == 0) *zc = 0;  // the rescue's count of flagged rows
  const int ibase = blockIdx.x * (kBlock * IPL) + t;
  const int js = blockIdx.y * chunk;
  const int je = min(n, js + chunk);
  const R e2 = (R)(eps * eps);

  IPos<MODE> pi[IPL];
  int iidx[IPL];
  R rc2[IPL];
  float xinf[IPL], eacc[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    int i = ibase + k * kBlock;
    iidx[k] = i;
    int ic = i < n ? i : n - 1;
    const double xa = x[ic], ya = x[n + ic], za = x[2 * n + ic];
    pi[k].set(xa, ya, za);
    rc2[k] = (R)near_rc2(xa, ya, za, eps, n);
    xinf[k] = (float)fmax(fabs(xa), fmax(fabs(ya), fabs(za)));
    eacc[k] = 0.f;
  }
  R hx[IPL], hy[IPL], hz[IPL], lx[IPL], ly[IPL], lz[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) hx[k] = hy[k] = hz[k] = lx[k] = ly[k] = lz[k] = R(0);

  const int ntiles = (je - js + kTile - 1) / kTile;
  if (ntiles > 0) tile[0][t] = load_rec<MODE>(x, m, n, js + t, je);
  __syncthreads();
  for (int tt = 0; tt < ntiles; ++tt) {
    const int jt = js + tt * kTile;
    // records past je are zero-mass padding: skip whole fold blocks of them
    const int fend = min(kTile, (je - jt + kFold - 1) / kFold * kFold);
    const bool more = tt + 1 < ntiles;
    // prefetch the next tile's FP64 values while this tile is consumed
    double nx = 0, ny = 0, nz = 0, nm = 0;
    const int jn = jt + kTile + t;
    if (more && jn < je) { nx = x[jn]; ny = x[n + jn]; nz = x[2 * n + jn]; nm = m[jn]; }
    const JRec<MODE>* cur = tile[tt & 1];
#pragma unroll 1
    for (int f = 0; f < fend; f += kFold) {
      R px[IPL], py[IPL], pz[IPL], r2min[IPL];
#pragma unroll
      for (int k = 0; k < IPL; ++k) {
        px[k] = py[k] = pz[k] = R(0);
        r2min[k] = R(3.0e38f);
      }
#pragma unroll 16
      for (int jj = f; jj < f + kFold; ++jj) {
        const JRec<MODE> r = cur[jj];
        const R mj = jmass(r);
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          R dx, dy, dz;
          if constexpr (NEAR) disp_hi(r, pi[k], dx, dy, dz);
          else disp(r, pi[k], dx, dy, dz);
          R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
          R ri = rsq(r2);
          R s = (mj * ri) * (ri * ri);
          if (EXCL) s = (jt + jj == iidx[k]) ? R(0) : s;
          px[k] = fma(s, dx, px[k]);
          py[k] = fma(s, dy, py[k]);
          pz[k] = fma(s, dz, pz[k]);
          if constexpr (NEAR) r2min[k] = fminf(r2min[k], r2);
        }
      }
      if constexpr (NEAR) {
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          // rare: the block holds a pair closer than the repair radius (the
          // lane's own pair, r2 = eps^2, always is one): for every such pair
          // other than the own pair, replace its term from rounded positions
          // by its term from float-float displacements
          if (r2min[k] < rc2[k]) {
            // the closest pair left in rounded positions, for the error estimate
            R r2nr = R(3.0e38f);
            for (int jj = f; jj < f + kFold; ++jj) {
              const JRec<MODE> r = cur[jj];
              R dx, dy, dz;
              disp_hi(r, pi[k], dx, dy, dz);
              const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
              if (r2 >= rc2[k]) r2nr = fminf(r2nr, r2);
              if (r2 < rc2[k] && jt + jj != iidx[k]) {
                const R ri = rsq(r2);
                const R s = (jmass(r) * ri) * (ri * ri);
                R ex, ey, ez;
                disp(r, pi[k], ex, ey, ez);
                const R q2 = fma(ez, ez, fma(ey, ey, fma(ex, ex, e2)));
                const R qi = rsq(q2);
                const R t = (jmass(r) * qi) * (qi * qi);
                px[k] = fma(t, ex, fma(-s, dx, px[k]));
                py[k] = fma(t, ey, fma(-s, dy, py[k]));
                pz[k] = fma(t, ez, fma(-s, dz, pz[k]));
              }
            }
            r2min[k] = r2nr;
          }
          if (est) eacc[k] = est_add(eacc[k], px[k], py[k], pz[k], xinf[k], r2min[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < IPL; ++k) {
        fold(hx[k], lx[k], px[k]);
        fold(hy[k], ly[k], py[k]);
        fold(hz[k], lz[k], pz[k]);
      }
    }
    if (more) {
      tile[(tt + 1) & 1][t] = (jn < je) ? JRec<MODE>::make(nx, ny, nz, nm)
                                        : JRec<MODE>::make(kFarAway, kFarAway, kFarAway, 0.0);
    }
    __syncthreads();
  }

  const bool direct = gridDim.y == 1;
  double* o = direct ? out : out + (size_t)blockIdx.y * 3 * n;
  const double scale = direct ? G : 1.0;
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    const int i = iidx[k];
    if (i < n) {
      o[i] = scale * ((double)hx[k] + (double)lx[k]);
      o[n + i] = scale * ((double)hy[k] + (double)ly[k]);
      o[2 * n + i] = scale * ((double)hz[k] + (double)lz[k]);
      if (NEAR && est) est[(size_t)blockIdx.y * n + i] = eacc[k];
    }
  }
}

// Sums `split` slices of `cnt` partials in slice order (TwoSum across slices)
// and scales by G; entries e < n0 go to out0[e], e < n1 to out1[e - n0] and
// the rest to out2[e - n1].
__global__ void sum_slices_kernel(int64_t cnt, int split, const double* __restrict__ part, double G,
                                  int64_t n0, double* __restrict__ out0, int64_t n1, double* __restrict__ out1,
                                  double* __restrict__ out2) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  double s = 0.0, c = 0.0;
  for (int y = 0; y < split; ++y) {
    double v = part[(size_t)y * cnt + e];
    double t = s + v;
    double bp = t - s;
    c += (s - (t - bp)) + (v - bp);
    s = t;
  }
  if (e < n0) out0[e] = G * (s + c);
  else if (e < n1) out1[e - n0] = G * (s + c);
  else out2[e - n1] = G * (s + c);
}

// ============================================================== VJP
// j-record for the VJP: the acceleration record plus the cotangent w_j.
template <int MODE> struct WRec {
  JRec<MODE> r;
  typename std::conditional<MODE == kFP64, double4, float4>::type w;
};

template <int MODE>
__device__ __forceinline__ WRec<MODE> load_wrec(const double* __restrict__ x, const double* __restrict__ m,
                                                const double* __restrict__ w, int n, int j, int je) {
  using R = Real<MODE>;
  WRec<MODE> o;
  if (j < je) {
    o.r = JRec<MODE>::make(x[j], x[n + j], x[2 * n + j], m[j]);
    o.w.x = (R)w[j]; o.w.y = (R)w[n + j]; o.w.z = (R)w[2 * n + j]; o.w.w = R(0);
  } else {
    o.r = JRec<MODE>::make(kFarAway, kFarAway, kFarAway, 0.0);
    o.w.x = o.w.y = o.w.z = o.w.w = R(0);
  }
  return o;
}

// u = m_k w_j - m_j w_k without contraction, so that u is exactly zero for j == k.
template <typename R>
__device__ __forceinline__ R cross_weight(R mk, R wj, R mj, R wk) {
#pragma clang fp contract(off)
  R a = mk * wj;
  R b = mj * wk;
  return a - b;
}

// One VJP pair term for lane particle k and record j, displacement d = x_j - x_k:
//   g += r^-3 u - 3 r^-5 (d.u) d,  gm -= r^-3 (d . w_j),  u = m_k w_j - m_j w_k.
template <typename R>
__device__ __forceinline__ R vjp_pair(R dx, R dy, R dz, R e2, R mj, R wjx, R wjy, R wjz, R mk, R wkx, R wky,
                                      R wkz, bool self, R& px, R& py, R& pz, R& pm) {
  R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
  R ri = rsq(r2);
  R ri2 = ri * ri;
  R r3 = ri2 * ri;
  R r5 = r3 * ri2;
  r3 = self ? R(0) : r3;
  r5 = self ? R(0) : r5;
  R ux = cross_weight(mk, wjx, mj, wkx);
  R uy = cross_weight(mk, wjy, mj, wky);
  R uz = cross_weight(mk, wjz, mj, wkz);
  R du = fma(dz, uz, fma(dy, uy, dx * ux));
  R c = R(3) * r5 * du;
  px = fma(-c, dx, fma(r3, ux, px));
  py = fma(-c, dy, fma(r3, uy, py));
  pz = fma(-c, dz, fma(r3, uz, pz));
  R dw = fma(dz, wjz, fma(dy, wjy, dx * wjx));
  pm = fma(-r3, dw, pm);
  return r2;
}

// gx_k = G sum_j [ r^-3 u - 3 r^-5 (d.u) d ],  gm_k = -G sum_j r^-3 (d . w_j),
// d = x_j - x_k, u = m_k w_j - m_j w_k, r^2 = |d|^2 + eps^2.
// split == 1: writes G * sums to gx (3n) and gm (n).
// split > 1: writes slice y's unscaled 4n partials (gx then gm) at part + y*4n.
// NEAR (FP32C only): rounded-position pairs with the near-field repair of the
// force kernel; otherwise FP32C uses float-float displacements for every pair.
template <int MODE, int IPL, bool EXCL, bool NEAR>
__global__ __launch_bounds__(kBlock) void vjp_kernel(int n, const double* __restrict__ x,
                                                     const double* __restrict__ m,
                                                     const double* __restrict__ w, double eps, double G,
                                                     int chunk, double* __restrict__ gx,
                                                     double* __restrict__ gm, double* __restrict__ part) {
  using R = Real<MODE>;
  static_assert(!NEAR || MODE == kFP32C, "the near-field repair needs float-float records");
  __shared__ WRec<MODE> tile[2][kTile];
  const int t = threadIdx.x;
  const int ibase = blockIdx.x * (kBlock * IPL) + t;
  const int js = blockIdx.y * chunk;
  const int je = min(n, js + chunk);
  const R e2 = (R)(eps * eps);

  IPos<MODE> pi[IPL];
  R mk[IPL], wkx[IPL], wky[IPL], wkz[IPL], rc2[IPL];
  int iidx[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    int i = ibase + k * kBlock;
    iidx[k] = i;
    int ic = i < n ? i : n - 1;
    const double xa = x[ic], ya = x[n + ic], za = x[2 * n + ic];
    pi[k].set(xa, ya, za);
    mk[k] = (R)m[ic];
    wkx[k] = (R)w[ic]; wky[k] = (R)w[n + ic]; wkz[k] = (R)w[2 * n + ic];
    rc2[k] = (R)near_rc2(xa, ya, za, eps, n);
  }
  R hx[IPL], hy[IPL], hz[IPL], hm[IPL], lx[IPL], ly[IPL], lz[IPL], lm[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) hx[k] = hy[k] = hz[k] = hm[k] = lx[k] = ly[k] = lz[k] = lm[k] = R(0);

  const int ntiles = (je - js + kTile - 1) / kTile;
  if (ntiles > 0) tile[0][t] = load_wrec<MODE>(x, m, w, n, js + t, je);
  __syncthreads();
  for (int tt = 0; tt < ntiles; ++tt) {
    const int jt = js + tt * kTile;
    // records past je are zero-mass padding: skip whole fold blocks of them
    const int fend = min(kTile, (je - jt + kFold - 1) / kFold * kFold);
    const bool more = tt + 1 < ntiles;
    WRec<MODE> nxt;
    if (more) nxt = load_wrec<MODE>(x, m, w, n, jt + kTile + t, je);
    const WRec<MODE>* cur = tile[tt & 1];
#pragma unroll 1
    for (int f = 0; f < fend; f += kFold) {
      R px[IPL], py[IPL], pz[IPL], pm[IPL], r2min[IPL];
#pragma unroll
      for (int k = 0; k < IPL; ++k) {
        px[k] = py[k] = pz[k] = pm[k] = R(0);
        r2min[k] = R(3.0e38f);
      }
#pragma unroll 8
      for (int jj = f; jj < f + kFold; ++jj) {
        const WRec<MODE> q = cur[jj];
        const R mj = jmass(q.r);
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          R dx, dy, dz;
          if constexpr (NEAR) disp_hi(q.r, pi[k], dx, dy, dz);
          else disp(q.r, pi[k], dx, dy, dz);
          const R r2 = vjp_pair<R>(dx, dy, dz, e2, mj, q.w.x, q.w.y, q.w.z, mk[k], wkx[k], wky[k], wkz[k],
                                   EXCL && (jt + jj == iidx[k]), px[k], py[k], pz[k], pm[k]);
          if constexpr (NEAR) r2min[k] = fminf(r2min[k], r2);
        }
      }
      if constexpr (NEAR) {
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          bool close = r2min[k] < rc2[k];  // a close pair other than the lane's own, as in accel_kernel
          if (close && (unsigned)(iidx[k] - (jt + f)) < (unsigned)kFold) {
            close = false;
            for (int jj = f; jj < f + kFold; ++jj) {
              R dx, dy, dz;
              disp_hi(cur[jj].r, pi[k], dx, dy, dz);
              const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
              close = close || (r2 < rc2[k] && jt + jj != iidx[k]);
            }
          }
          if (close) {
            // rare: redo this block for lane k with float-float displacements for the close pairs
            R qx = 0, qy = 0, qz = 0, qm = 0;
            for (int jj = f; jj < f + kFold; ++jj) {
              const WRec<MODE> q = cur[jj];
              R dx, dy, dz;
              disp_hi(q.r, pi[k], dx, dy, dz);
              const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
              if (r2 < rc2[k]) disp(q.r, pi[k], dx, dy, dz);
              vjp_pair<R>(dx, dy, dz, e2, jmass(q.r), q.w.x, q.w.y, q.w.z, mk[k], wkx[k], wky[k], wkz[k],
                          EXCL && (jt + jj == iidx[k]), qx, qy, qz, qm);
            }
            px[k] = qx;
            py[k] = qy;
            pz[k] = qz;
            pm[k] = qm;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < IPL; ++k) {
        fold(hx[k], lx[k], px[k]);
        fold(hy[k], ly[k], py[k]);
        fold(hz[k], lz[k], pz[k]);
        fold(hm[k], lm[k], pm[k]);
      }
    }
    if (more) tile[(tt + 1) & 1][t] = nxt;
    __syncthreads();
  }

  const bool direct = gridDim.y == 1;
  double* o = direct ? gx : part + (size_t)blockIdx.y * 4 * n;
  double* om = direct ? gm : o + 3 * (size_t)n;
  const double scale = direct ? G : 1.0;
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    const int i = iidx[k];
    if (i < n) {
      o[i] = scale * ((double)hx[k] + (double)lx[k]);
      o[n + i] = scale * ((double)hy[k] + (double)ly[k]);
      o[2 * n + i] = scale * ((double)hz[k] + (double)lz[k]);
      om[i] = scale * ((double)hm[k] + (double)lm[k]);
    }
  }
}

// ============================================================== acceleration + jerk
// App. A, Algorithm 3 in full: per pair r_ij, v_ij, t_j = m_j r^-3,
// A = -3 r^-2, v_r = r_ij . v_ij, q = A v_r; a += t_j r_ij and
// jerk += t_j (v_ij + q r_ij), with r^2 = |r_ij|^2 + eps^2.  Records carry the
// position record plus the velocity (FP32 velocities in the FP32 modes).
// FP32C uses the near-field repair of accel_kernel: displacements from
// FP32-rounded positions, and a block of kFold j's holding a pair closer than
// the lane's repair radius is redone with float-float displacements for those
// pairs.  split == 1 writes G*sums to a and jk; split > 1 writes slice y's
// unscaled 6n partials (a then jerk) at part + y*6n.
template <typename R>
__device__ __forceinline__ R jerk_pair(R dx, R dy, R dz, R wx, R wy, R wz, R mj, R e2, bool self, R* pa, R* pj) {
  const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
  const R ri = rsq(r2);
  R ri2 = ri * ri;
  R tj = (mj * ri) * ri2;                            // t_j = p_w,j r^-3
  if (self) {
    tj = R(0);
    ri2 = R(0);
  }
  const R vr = fma(dz, wz, fma(dy, wy, dx * wx));    // v_r = r . v
  const R qq = R(-3) * ri2 * vr;                     // q = A v_r, A = -3 r^-2
  pa[0] = fma(tj, dx, pa[0]);
  pa[1] = fma(tj, dy, pa[1]);
  pa[2] = fma(tj, dz, pa[2]);
  pj[0] = fma(tj, fma(qq, dx, wx), pj[0]);
  pj[1] = fma(tj, fma(qq, dy, wy), pj[1]);
  pj[2] = fma(tj, fma(qq, dz, wz), pj[2]);
  return r2;
}

template <int MODE, int IPL, bool EXCL>
__global__ __launch_bounds__(kBlock) void jerk_kernel(int n, const double* __restrict__ x,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ m, double eps, double G,
                                                      int chunk, double* __restrict__ a, double* __restrict__ jk,
                                                      double* __restrict__ part) {
  using R = Real<MODE>;
  constexpr bool kNear = MODE == kFP32C;
  __shared__ WRec<MODE> tile[2][kTile];
  const int t = threadIdx.x;
  const int ibase = blockIdx.x * (kBlock * IPL) + t;
  const int js = blockIdx.y * chunk;
  const int je = min(n, js + chunk);
  const R e2 = (R)(eps * eps);

  IPos<MODE> pi[IPL];
  R vx[IPL], vy[IPL], vz[IPL], rc2[IPL];
  int iidx[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    int i = ibase + k * kBlock;
    iidx[k] = i;
    int ic = i < n ? i : n - 1;
    const double xa = x[ic], ya = x[n + ic], za = x[2 * n + ic];
    pi[k].set(xa, ya, za);
    rc2[k] = (R)near_rc2(xa, ya, za, eps, n);
    vx[k] = (R)v[ic]; vy[k] = (R)v[n + ic]; vz[k] = (R)v[2 * n + ic];
  }
  R ah[3][IPL], al[3][IPL], jh[3][IPL], jl[3][IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) ah[c][k] = al[c][k] = jh[c][k] = jl[c][k] = R(0);

  const int ntiles = (je - js + kTile - 1) / kTile;
  if (ntiles > 0) tile[0][t] = load_wrec<MODE>(x, m, v, n, js + t, je);
  __syncthreads();
  for (int tt = 0; tt < ntiles; ++tt) {
    const int jt = js + tt * kTile;
    // records past je are zero-mass padding: skip whole fold blocks of them
    const int fend = min(kTile, (je - jt + kFold - 1) / kFold * kFold);
    const bool more = tt + 1 < ntiles;
    WRec<MODE> nxt;
    if (more) nxt = load_wrec<MODE>(x, m, v, n, jt + kTile + t, je);
    const WRec<MODE>* cur = tile[tt & 1];
#pragma unroll 1
    for (int f = 0; f < fend; f += kFold) {
      R pa[IPL][3], pj[IPL][3], r2min[IPL];
#pragma unroll
      for (int k = 0; k < IPL; ++k) {
        r2min[k] = R(3.0e38f);
#pragma unroll
        for (int c = 0; c < 3; ++c) pa[k][c] = pj[k][c] = R(0);
      }
#pragma unroll 8
      for (int jj = f; jj < f + kFold; ++jj) {
        const WRec<MODE> q = cur[jj];
        const R mj = jmass(q.r);
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          R dx, dy, dz;
          if constexpr (kNear) disp_hi(q.r, pi[k], dx, dy, dz);
          else disp(q.r, pi[k], dx, dy, dz);
          const R r2 = jerk_pair<R>(dx, dy, dz, q.w.x - vx[k], q.w.y - vy[k], q.w.z - vz[k], mj, e2,
                                    EXCL && (jt + jj == iidx[k]), pa[k], pj[k]);
          if constexpr (kNear) r2min[k] = fminf(r2min[k], r2);
        }
      }
      if constexpr (kNear) {
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          // in the block holding the lane's own pair, rescan for another close pair
          bool close = r2min[k] < rc2[k];
          if (close && (unsigned)(iidx[k] - (jt + f)) < (unsigned)kFold) {
            close = false;
            for (int jj = f; jj < f + kFold; ++jj) {
              R dx, dy, dz;
              disp_hi(cur[jj].r, pi[k], dx, dy, dz);
              const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
              close = close || (r2 < rc2[k] && jt + jj != iidx[k]);
            }
          }
          if (close) {
            // rare: redo this block for lane k with float-float displacements for the close pairs
            R qa[3] = {R(0), R(0), R(0)}, qj[3] = {R(0), R(0), R(0)};
            for (int jj = f; jj < f + kFold; ++jj) {
              const WRec<MODE> q = cur[jj];
              R dx, dy, dz;
              disp_hi(q.r, pi[k], dx, dy, dz);
              const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
              if (r2 < rc2[k]) disp(q.r, pi[k], dx, dy, dz);
              jerk_pair<R>(dx, dy, dz, q.w.x - vx[k], q.w.y - vy[k], q.w.z - vz[k], jmass(q.r), e2,
                           EXCL && (jt + jj == iidx[k]), qa, qj);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              pa[k][c] = qa[c];
              pj[k][c] = qj[c];
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < IPL; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          fold(ah[c][k], al[c][k], pa[k][c]);
          fold(jh[c][k], jl[c][k], pj[k][c]);
        }
    }
    if (more) tile[(tt + 1) & 1][t] = nxt;
    __syncthreads();
  }

  const bool direct = gridDim.y == 1;
  double* oa = direct ? a : part + (size_t)blockIdx.y * 6 * n;
  double* oj = direct ? jk : oa + 3 * (size_t)n;
  const double scale = direct ? G : 1.0;
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    const int i = iidx[k];
    if (i < n) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        oa[c * n + i] = scale * ((double)ah[c][k] + (double)al[c][k]);
        oj[c * n + i] = scale * ((double)jh[c][k] + (double)jl[c][k]);
      }
    }
  }
}

// ============================================================== potential
// phi_i = sum_{j != i} m_j / sqrt(|d|^2 + eps^2) in FP64, self pair excluded by
// index.  split == 1: writes scale * phi at out; split > 1: the unscaled slice
// y at out + y*n.
__global__ __launch_bounds__(kBlock) void potential_kernel(int n, const double* __restrict__ x,
                                                           const double* __restrict__ m, double eps,
                                                           double scale, int chunk, double* __restrict__ out) {
  __shared__ double4 tile[2][kTile];
  const int t = threadIdx.x;
  const int i = blockIdx.x * kBlock + t;
  const int ic = i < n ? i : n - 1;
  const int js = blockIdx.y * chunk;
  const int je = min(n, js + chunk);
  const double e2 = eps * eps;
  const double xi = x[ic], yi = x[n + ic], zi = x[2 * n + ic];
  double hp = 0, lp = 0;
  const int ntiles = (je - js + kTile - 1) / kTile;
  auto ld = [&](int j) {
    return j < je ? make_double4(x[j], x[n + j], x[2 * n + j], m[j])
                  : make_double4(kFarAway, kFarAway, kFarAway, 0.0);
  };
  if (ntiles > 0) tile[0][t] = ld(js + t);
  __syncthreads();
  for (int tt = 0; tt < ntiles; ++tt) {
    const int jt = js + tt * kTile;
    // records past je are zero-mass padding: skip whole fold blocks of them
    const int fend = min(kTile, (je - jt + kFold - 1) / kFold * kFold);
    const bool more = tt + 1 < ntiles;
    double4 nxt = make_double4(0, 0, 0, 0);
    if (more) nxt = ld(jt + kTile + t);
    const double4* cur = tile[tt & 1];
#pragma unroll 1
    for (int f = 0; f < fend; f += kFold) {
      double p = 0;
#pragma unroll 8
      for (int jj = f; jj < f + kFold; ++jj) {
        const double4 r = cur[jj];
        double dx = r.x - xi, dy = r.y - yi, dz = r.z - zi;
        double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
        double v = r.w * rsqrt64(r2);
        p += (jt + jj == i) ? 0.0 : v;
      }
      fold(hp, lp, p);
    }
    if (more) tile[(tt + 1) & 1][t] = nxt;
    __syncthreads();
  }
  if (i < n) out[(size_t)blockIdx.y * n + i] = gridDim.y == 1 ? scale * (hp + lp) : hp + lp;
}

// ============================================================== acceleration + jerk + snap
// The evaluation of a sixth-order Hermite step (Sec. 2.1): along paths of
// constant acceleration, the pair term P = t_j d (d = x_j - x_i,
// t_j = m_j s^-3/2, s = |d|^2 + eps^2) has the derivatives
//   P'  = t_j w - 3 alpha P,                  alpha = (d . w) / s
//   P'' = t_j u - 6 alpha P' - 3 beta P,      beta  = (w . w + d . u) / s + alpha^2
// with w = v_j - v_i and u = acc_j - acc_i; a, jerk and snap are G times their
// sums.  Records carry the position record plus velocity and acceleration
// (FP32 velocity and acceleration differences in the FP32 modes; FP32C with
// the near-field repair of accel_kernel).  split == 1 writes G*sums to a, jk
// and sn; split > 1 writes slice y's unscaled 9n partials (a, jerk, snap) at
// part + y*9n.
template <int MODE> struct SRec {
  using V4 = typename std::conditional<MODE == kFP64, double4, float4>::type;
  JRec<MODE> r;
  V4 v;
  V4 u;
};

template <int MODE>
__device__ __forceinline__ SRec<MODE> load_srec(const double* __restrict__ x, const double* __restrict__ m,
                                                const double* __restrict__ v, const double* __restrict__ acc,
                                                int n, int j, int je) {
  using R = Real<MODE>;
  SRec<MODE> o;
  if (j < je) {
    o.r = JRec<MODE>::make(x[j], x[n + j], x[2 * n + j], m[j]);
    o.v.x = (R)v[j]; o.v.y = (R)v[n + j]; o.v.z = (R)v[2 * n + j]; o.v.w = R(0);
    o.u.x = (R)acc[j]; o.u.y = (R)acc[n + j]; o.u.z = (R)acc[2 * n + j]; o.u.w = R(0);
  } else {
    o.r = JRec<MODE>::make(kFarAway, kFarAway, kFarAway, 0.0);
    o.v.x = o.v.y = o.v.z = o.v.w = R(0);
    o.u.x = o.u.y = o.u.z = o.u.w = R(0);
  }
  return o;
}

template <typename R>
__device__ __forceinline__ R snap_pair(const R* d, const R* w, const R* u, R mj, R e2, bool self, R* pa, R* pj,
                                       R* ps) {
  const R r2 = fma(d[2], d[2], fma(d[1], d[1], fma(d[0], d[0], e2)));
  const R ri = rsq(r2);
  R sinv = ri * ri;
  R tj = (mj * ri) * sinv;
  if (self) {
    tj = R(0);
    sinv = R(0);
  }
  const R alpha = fma(d[2], w[2], fma(d[1], w[1], d[0] * w[0])) * sinv;
  const R wwdu = fma(d[2], u[2], fma(d[1], u[1], fma(d[0], u[0], fma(w[2], w[2], fma(w[1], w[1], w[0] * w[0])))));
  const R beta = fma(wwdu, sinv, alpha * alpha);
  const R a3 = R(-3) * alpha;
  const R b3 = R(-3) * beta;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const R P0 = tj * d[c];
    const R P1 = fma(a3, P0, tj * w[c]);
    const R P2 = fma(R(2) * a3, P1, fma(b3, P0, tj * u[c]));
    pa[c] += P0;
    pj[c] += P1;
    ps[c] += P2;
  }
  return r2;
}

template <int MODE, int IPL, bool EXCL>
__global__ __launch_bounds__(kBlock) void snap_kernel(int n, const double* __restrict__ x,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ acc,
                                                      const double* __restrict__ m, double eps, double G,
                                                      int chunk, double* __restrict__ a, double* __restrict__ jk,
                                                      double* __restrict__ sn, double* __restrict__ part) {
  using R = Real<MODE>;
  constexpr bool kNear = MODE == kFP32C;
  __shared__ SRec<MODE> tile[2][kTile];
  const int t = threadIdx.x;
  const int ibase = blockIdx.x * (kBlock * IPL) + t;
  const int js = blockIdx.y * chunk;
  const int je = min(n, js + chunk);
  const R e2 = (R)(eps * eps);

  IPos<MODE> pi[IPL];
  R vi[3][IPL], ui[3][IPL], rc2[IPL];
  int iidx[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    int i = ibase + k * kBlock;
    iidx[k] = i;
    int ic = i < n ? i : n - 1;
    const double xa = x[ic], ya = x[n + ic], za = x[2 * n + ic];
    pi[k].set(xa, ya, za);
    rc2[k] = (R)near_rc2(xa, ya, za, eps, n);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      vi[c][k] = (R)v[c * n + ic];
      ui[c][k] = (R)acc[c * n + ic];
    }
  }
  R ah[3][IPL], al[3][IPL], jh[3][IPL], jl[3][IPL], sh[3][IPL], sl[3][IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) ah[c][k] = al[c][k] = jh[c][k] = jl[c][k] = sh[c][k] = sl[c][k] = R(0);

  const int ntiles = (je - js + kTile - 1) / kTile;
  if (ntiles > 0) tile[0][t] = load_srec<MODE>(x, m, v, acc, n, js + t, je);
  __syncthreads();
  for (int tt = 0; tt < ntiles; ++tt) {
    const int jt = js + tt * kTile;
    // records past je are zero-mass padding: skip whole fold blocks of them
    const int fend = min(kTile, (je - jt + kFold - 1) / kFold * kFold);
    const bool more = tt + 1 < ntiles;
    SRec<MODE> nxt;
    if (more) nxt = load_srec<MODE>(x, m, v, acc, n, jt + kTile + t, je);
    const SRec<MODE>* cur = tile[tt & 1];
#pragma unroll 1
    for (int f = 0; f < fend; f += kFold) {
      R pa[IPL][3], pj[IPL][3], ps[IPL][3], r2min[IPL];
#pragma unroll
      for (int k = 0; k < IPL; ++k) {
        r2min[k] = R(3.0e38f);
#pragma unroll
        for (int c = 0; c < 3; ++c) pa[k][c] = pj[k][c] = ps[k][c] = R(0);
      }
#pragma unroll 4
      for (int jj = f; jj < f + kFold; ++jj) {
        const SRec<MODE> q = cur[jj];
        const R mj = jmass(q.r);
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          R d[3];
          if constexpr (kNear) disp_hi(q.r, pi[k], d[0], d[1], d[2]);
          else disp(q.r, pi[k], d[0], d[1], d[2]);
          const R w[3] = {q.v.x - vi[0][k], q.v.y - vi[1][k], q.v.z - vi[2][k]};
          const R u[3] = {q.u.x - ui[0][k], q.u.y - ui[1][k], q.u.z - ui[2][k]};
          const R r2 = snap_pair<R>(d, w, u, mj, e2, EXCL && (jt + jj == iidx[k]), pa[k], pj[k], ps[k]);
          if constexpr (kNear) r2min[k] = fminf(r2min[k], r2);
        }
      }
      if constexpr (kNear) {
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          // in the block holding the lane's own pair, rescan for another close pair
          bool close = r2min[k] < rc2[k];
          if (close && (unsigned)(iidx[k] - (jt + f)) < (unsigned)kFold) {
            close = false;
            for (int jj = f; jj < f + kFold; ++jj) {
              R dx, dy, dz;
              disp_hi(cur[jj].r, pi[k], dx, dy, dz);
              const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
              close = close || (r2 < rc2[k] && jt + jj != iidx[k]);
            }
          }
          if (close) {
            // rare: redo this block for lane k with float-float displacements for the close pairs
            R qa[3] = {R(0), R(0), R(0)}, qj[3] = {R(0), R(0), R(0)}, qs[3] = {R(0), R(0), R(0)};
            for (int jj = f; jj < f + kFold; ++jj) {
              const SRec<MODE> q = cur[jj];
              R d[3];
              disp_hi(q.r, pi[k], d[0], d[1], d[2]);
              const R r2 = fma(d[2], d[2], fma(d[1], d[1], fma(d[0], d[0], e2)));
              if (r2 < rc2[k]) disp(q.r, pi[k], d[0], d[1], d[2]);
              const R w[3] = {q.v.x - vi[0][k], q.v.y - vi[1][k], q.v.z - vi[2][k]};
              const R u[3] = {q.u.x - ui[0][k], q.u.y - ui[1][k], q.u.z - ui[2][k]};
              snap_pair<R>(d, w, u, jmass(q.r), e2, EXCL && (jt + jj == iidx[k]), qa, qj, qs);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              pa[k][c] = qa[c];
              pj[k][c] = qj[c];
              ps[k][c] = qs[c];
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < IPL; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          fold(ah[c][k], al[c][k], pa[k][c]);
          fold(jh[c][k], jl[c][k], pj[k][c]);
          fold(sh[c][k], sl[c][k], ps[k][c]);
        }
    }
    if (more) tile[(tt + 1) & 1][t] = nxt;
    __syncthreads();
  }

  const bool direct = gridDim.y == 1;
  double* oa = direct ? a : part + (size_t)blockIdx.y * 9 * n;
  double* oj = direct ? jk : oa + 3 * (size_t)n;
  double* os = direct ? sn : oa + 6 * (size_t)n;
  const double scale = direct ? G : 1.0;
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    const int i = iidx[k];
    if (i < n) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        oa[c * n + i] = scale * ((double)ah[c][k] + (double)al[c][k]);
        oj[c * n + i] = scale * ((double)jh[c][k] + (double)jl[c][k]);
        os[c * n + i] = scale * ((double)sh[c][k] + (double)sl[c][k]);
      }
    }
  }
}

// ============================================================== launch helpers
// j-slices are whole fold blocks (64 records), so that small systems can be
// spread over more workgroups than they have 256-record tiles
inline int split_chunk(int64_t n, int split) {
  int64_t c = (n + split - 1) / split;
  c = (c + kFold - 1) / kFold * kFold;
  return (int)(c > 0 ? c : kFold);
}
inline int effective_split(int64_t n, int split) {
  int chunk = split_chunk(n, split);
  return (int)((n + chunk - 1) / chunk);
}

template <int MODE, int IPL>
int accel_dispatch(int64_t n, const double* x, const double* m, double* a, double G, double eps,
                   bool excl, int split, const PairConfig& cfg, hipStream_t s) {
  const int chunk = split_chunk(n, split);
  const int sp = effective_split(n, split);
  dim3 grid((unsigned)((n + kBlock * IPL - 1) / (kBlock * IPL)), (unsigned)sp);
  constexpr bool kNear = MODE == kFP32C;
  const bool rescue = kNear && cfg.rescue;
  // scratch: the slices' partial sums (split > 1), then for the rescue the
  // slices' error estimates, the list of flagged rows and its count
  const size_t part_bytes = sp > 1 ? sizeof(double) * 3 * (size_t)n * sp : 0;
  const size_t est_bytes = rescue ? (sizeof(float) * (size_t)n * sp + 255) / 256 * 256 : 0;
  const size_t list_bytes = rescue ? sizeof(int) * ((size_t)n + 64) : 0;
  int st = NBODY_OK;
  char* ws = nullptr;
  if (part_bytes + est_bytes + list_bytes > 0) {
    ws = static_cast<char*>(pair_scratch(cfg, part_bytes + est_bytes + list_bytes, &st));
    if (!ws) return st;
  }
  double* out = sp > 1 ? reinterpret_cast<double*>(ws) : a;
  float* est = rescue ? reinterpret_cast<float*>(ws + part_bytes) : nullptr;
  int* list = rescue ? reinterpret_cast<int*>(ws + part_bytes + est_bytes) : nullptr;
  if (excl)
    accel_kernel<MODE, IPL, true, kNear><<<grid, kBlock, 0, s>>>((int)n, x, m, eps, G, chunk, out, est, list);
  else
    accel_kernel<MODE, IPL, false, kNear><<<grid, kBlock, 0, s>>>((int)n, x, m, eps, G, chunk, out, est, list);
  NB_LAUNCH_CHECK("accel_kernel");
  if (sp > 1) {
    const int64_t cnt = 3 * n;
    sum_slices_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(cnt, sp, out, G, cnt, a, cnt, nullptr, nullptr);
    NB_LAUNCH_CHECK("sum_slices_kernel");
  }
  if (rescue) return launch_rescue(n, x, m, eps, G, excl, est, sp, (size_t)n, a, list + 64, list, s);
  return NBODY_OK;
}

template <int MODE, int IPL>
int vjp_dispatch(int64_t n, const double* x, const double* m, const double* w, double* gx, double* gm,
                 double G, double eps, bool excl, int split, hipStream_t s) {
  const int chunk = split_chunk(n, split);
  const int sp = effective_split(n, split);
  dim3 grid((unsigned)((n + kBlock * IPL - 1) / (kBlock * IPL)), (unsigned)sp);
  int st = NBODY_OK;
  double* part = nullptr;
  if (sp > 1) {
    part = static_cast<double*>(workspace(current_device(), 0, sizeof(double) * 4 * (size_t)n * sp, &st));
    if (!part) return st;
  }
  constexpr bool kNear = MODE == kFP32C;
  if (excl)
    vjp_kernel<MODE, IPL, true, kNear><<<grid, kBlock, 0, s>>>((int)n, x, m, w, eps, G, chunk, gx, gm, part);
  else
    vjp_kernel<MODE, IPL, false, kNear><<<grid, kBlock, 0, s>>>((int)n, x, m, w, eps, G, chunk, gx, gm, part);
  NB_LAUNCH_CHECK("vjp_kernel");
  if (sp > 1) {
    const int64_t cnt = 4 * n;
    sum_slices_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(cnt, sp, part, G, 3 * n, gx, cnt, gm, nullptr);
    NB_LAUNCH_CHECK("sum_slices_kernel");
  }
  return NBODY_OK;
}

template <int MODE, int IPL>
int jerk_dispatch(int64_t n, const double* x, const double* v, const double* m, double* a, double* jk, double G,
                  double eps, bool excl, int split, hipStream_t s) {
  const int chunk = split_chunk(n, split);
  const int sp = effective_split(n, split);
  dim3 grid((unsigned)((n + kBlock * IPL - 1) / (kBlock * IPL)), (unsigned)sp);
  int st = NBODY_OK;
  double* part = nullptr;
  if (sp > 1) {
    part = static_cast<double*>(workspace(current_device(), 0, sizeof(double) * 6 * (size_t)n * sp, &st));
    if (!part) return st;
  }
  if (excl)
    jerk_kernel<MODE, IPL, true><<<grid, kBlock, 0, s>>>((int)n, x, v, m, eps, G, chunk, a, jk, part);
  else
    jerk_kernel<MODE, IPL, false><<<grid, kBlock, 0, s>>>((int)n, x, v, m, eps, G, chunk, a, jk, part);
  NB_LAUNCH_CHECK("jerk_kernel");
  if (sp > 1) {
    const int64_t cnt = 6 * n;
    sum_slices_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(cnt, sp, part, G, 3 * n, a, cnt, jk, nullptr);
    NB_LAUNCH_CHECK("sum_slices_kernel");
  }
  return NBODY_OK;
}

template <int MODE, int IPL>
int snap_dispatch(int64_t n, const double* x, const double* v, const double* acc, const double* m, double* a,
                  double* jk, double* sn, double G, double eps, bool excl, int split, hipStream_t s) {
  const int chunk = split_chunk(n, split);
  const int sp = effective_split(n, split);
  dim3 grid((unsigned)((n + kBlock * IPL - 1) / (kBlock * IPL)), (unsigned)sp);
  int st = NBODY_OK;
  double* part = nullptr;
  if (sp > 1) {
    part = static_cast<double*>(workspace(current_device(), 0, sizeof(double) * 9 * (size_t)n * sp, &st));
    if (!part) return st;
  }
  if (excl)
    snap_kernel<MODE, IPL, true><<<grid, kBlock, 0, s>>>((int)n, x, v, acc, m, eps, G, chunk, a, jk, sn, part);
  else
    snap_kernel<MODE, IPL, false><<<grid, kBlock, 0, s>>>((int)n, x, v, acc, m, eps, G, chunk, a, jk, sn, part);
  NB_LAUNCH_CHECK("snap_kernel");
  if (sp > 1) {
    const int64_t cnt = 9 * n;
    sum_slices_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(cnt, sp, part, G, 3 * n, a, 6 * n, jk, sn);
    NB_LAUNCH_CHECK("sum_slices_kernel");
  }
  return NBODY_OK;
}

}  // namespace

int launch_accel_jerk_snap(int64_t n, const double* x, const double* v, const double* acc, const double* m,
                           double* a, double* jk, double* sn, double G, double eps, int precision, bool excl,
                           const PairConfig& cfg, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  if (cfg.sym_snap && precision != kFP64)
    return launch_sym_snap(n, x, v, acc, m, a, jk, sn, G, eps, precision, excl, cfg, s);
  if (cfg.sym_snap64 && precision == kFP64) return launch_sym_snap64(n, x, v, acc, m, a, jk, sn, G, eps, excl, cfg, s);
  const int split = cfg.split < 1 ? 1 : cfg.split;
  switch (precision) {
    case kFP64: return snap_dispatch<kFP64, 1>(n, x, v, acc, m, a, jk, sn, G, eps, excl, split, s);
    case kFP32C: return snap_dispatch<kFP32C, 1>(n, x, v, acc, m, a, jk, sn, G, eps, excl, split, s);
    case kFP32: return snap_dispatch<kFP32, 1>(n, x, v, acc, m, a, jk, sn, G, eps, excl, split, s);
  }
  return set_error(NBODY_EINVAL, "unknown precision");
}

int launch_accel_jerk(int64_t n, const double* x, const double* v, const double* m, double* a, double* jk, double G,
                      double eps, int precision, bool excl, const PairConfig& cfg, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  if (cfg.sym_jerk && precision != kFP64) return launch_sym_jerk(n, x, v, m, a, jk, G, eps, precision, excl, cfg, s);
  if (cfg.sym_jerk64 && precision == kFP64) return launch_sym_jerk64(n, x, v, m, a, jk, G, eps, excl, cfg, s);
  const int split = cfg.split < 1 ? 1 : cfg.split;
  const bool one = cfg.ipl <= 1;
  switch (precision) {
    case kFP64: return one ? jerk_dispatch<kFP64, 1>(n, x, v, m, a, jk, G, eps, excl, split, s)
                           : jerk_dispatch<kFP64, 2>(n, x, v, m, a, jk, G, eps, excl, split, s);
    case kFP32C: return one ? jerk_dispatch<kFP32C, 1>(n, x, v, m, a, jk, G, eps, excl, split, s)
                            : jerk_dispatch<kFP32C, 2>(n, x, v, m, a, jk, G, eps, excl, split, s);
    case kFP32: return one ? jerk_dispatch<kFP32, 1>(n, x, v, m, a, jk, G, eps, excl, split, s)
                           : jerk_dispatch<kFP32, 2>(n, x, v, m, a, jk, G, eps, excl, split, s);
  }
  return set_error(NBODY_EINVAL, "unknown precision");
}

int launch_accel(int64_t n, const double* x, const double* m, double* a, double G, double eps,
                 int precision, bool excl, const PairConfig& cfg, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  if (cfg.sym) {
    if (precision == kFP64) return launch_sym_accel64(n, x, m, a, G, eps, excl, cfg, s);
    return launch_sym_accel(n, x, m, a, G, eps, precision, excl, cfg, s);
  }
  const int split = cfg.split < 1 ? 1 : cfg.split;
#define NB_ACC(MODE, IPL) return accel_dispatch<MODE, IPL>(n, x, m, a, G, eps, excl, split, cfg, s)
  switch (precision) {
    case kFP64:
      if (cfg.ipl == 1) NB_ACC(kFP64, 1);
      if (cfg.ipl == 2) NB_ACC(kFP64, 2);
      NB_ACC(kFP64, 4);
    case kFP32C:
      if (cfg.ipl == 1) NB_ACC(kFP32C, 1);
      if (cfg.ipl == 2) NB_ACC(kFP32C, 2);
      NB_ACC(kFP32C, 4);
    case kFP32:
      if (cfg.ipl == 1) NB_ACC(kFP32, 1);
      if (cfg.ipl == 2) NB_ACC(kFP32, 2);
      NB_ACC(kFP32, 4);
  }
#undef NB_ACC
  return set_error(NBODY_EINVAL, "unknown precision");
}

int launch_vjp(int64_t n, const double* x, const double* m, const double* w, double* gx, double* gm,
               double G, double eps, int precision, bool excl, const PairConfig& cfg, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  if (cfg.sym_vjp && precision != kFP64) return launch_sym_vjp(n, x, m, w, gx, gm, G, eps, precision, excl, cfg, s);
  if (cfg.sym_vjp64 && precision == kFP64) return launch_sym_vjp64(n, x, m, w, gx, gm, G, eps, cfg, s);
  const int split = cfg.split < 1 ? 1 : cfg.split;
  // The VJP keeps twice the accumulators of the force, so it runs at most 2 i per lane.
  const bool one = cfg.ipl <= 1;
#define NB_VJP(MODE) return one ? vjp_dispatch<MODE, 1>(n, x, m, w, gx, gm, G, eps, excl, split, s) \
                               : vjp_dispatch<MODE, 2>(n, x, m, w, gx, gm, G, eps, excl, split, s)
  switch (precision) {
    case kFP64: NB_VJP(kFP64);
    case kFP32C: NB_VJP(kFP32C);
    case kFP32: NB_VJP(kFP32);
  }
#undef NB_VJP
  return set_error(NBODY_EINVAL, "unknown precision");
}

// scale * phi_i (FP64) into phi[n]; the energy diagnostics use scale = 1,
// nbody_potential scale = -G.
int launch_potential(int64_t n, const double* x, const double* m, double eps, double scale, double* phi,
                     int split, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  const int chunk = split_chunk(n, split);
  const int sp = effective_split(n, split);
  dim3 grid((unsigned)((n + kBlock - 1) / kBlock), (unsigned)sp);
  int st = NBODY_OK;
  double* part = phi;
  if (sp > 1) {
    part = static_cast<double*>(workspace(current_device(), 0, sizeof(double) * (size_t)n * sp, &st));
    if (!part) return st;
  }
  potential_kernel<<<grid, kBlock, 0, s>>>((int)n, x, m, eps, scale, chunk, part);
  NB_LAUNCH_CHECK("potential_kernel");
  if (sp > 1) {
    sum_slices_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, sp, part, scale, n, phi, n, nullptr, nullptr);
    NB_LAUNCH_CHECK("sum_slices_kernel");
  }
  return NBODY_OK;
}

}  // namespace nb
