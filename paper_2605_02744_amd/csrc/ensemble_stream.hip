// Streamed persistent ensemble integrator (nbody_config.bsplit = 2).
//
// Many independent softened systems advanced for all KDK steps in ONE launch,
// with the work cut finer than whole systems so that no CU waits on one large
// system.  Every system is split into items of at most 1024 i-particles; a
// 1024-lane workgroup evaluates one item at a time, small systems with their
// lanes in j-groups (up to 16 groups of 64), streaming the system's pair
// records through a double-buffered LDS
// tile as the single-system force kernel does, and combining the groups'
// (hi, lo) sums through LDS in group order.  Items are assigned
// longest-processing-time first over the workgroups that can be resident at
// once (two per CU at <= 64 VGPRs: 8 waves per SIMD, the occupancy of the
// single-system kernel).
//
// The loop is step-major.  In every round each workgroup
//   A. kick-drifts the particles it owns (one lane per particle, FP64 state in
//      global memory), writes their pair records to the round's half of a
//      double-buffered record array, and publishes: every wave waits for its
//      stores, then after a barrier one lane issues an agent-scope release
//      fence and increments its items' system counters;
//   B. one lane polls (bounded) until every system it holds items of has all
//      its items published for this round, then issues one agent-scope
//      acquire fence, and after a barrier the workgroup evaluates its items.
// Agent-scope fences write back or invalidate a whole XCD's L2, and the L2
// serialises them (about 0.3 us each, measured): one release and one acquire
// per workgroup per round, and few large workgroups, keep their cost small.
// Phase A never waits, so all publications of a round happen once every
// workgroup has finished the previous round's phase B; with every workgroup
// resident this cannot deadlock.  Record buffers alternate by round: a
// workgroup rewrites a buffer only after all readers of that system have
// published the next round, i.e. finished reading it.  A wait that exceeds
// its bound (a workgroup that never became resident) makes the workgroup
// publish NaN records from then on, so every system coupled to it ends NaN
// instead of silently wrong, and the kernel still terminates.  The bound is
// wall-clock time (the 100 MHz real-time counter), set per plan from its
// largest per-workgroup pair count at a pessimistic 10^8 pairs/s plus 2 s, so
// that a legitimately long round (systems of millions of particles) never
// trips it.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <queue>
#include <vector>

#include "pair_math.h"

namespace nb {
namespace {

constexpr int kSBlock = 1024;           // lanes per workgroup
constexpr int kSMaxPerCu = 2;           // resident workgroups per CU at most
constexpr int kSWaves = 8;              // waves per SIMD the kernel is built for (<= 64 VGPRs)

struct SItem {
  int sys;  // system
  int i0;   // first particle of the item (system-local)
  int ni;   // particles in the item, <= kSBlock / js
  int js;   // j-groups: 1, 2, 4, 8 or 16
};

template <int MODE> struct SPart { Real<MODE> hx, lx, hy, ly, hz, lz; };

template <int MODE, bool EXCL>
__global__ __launch_bounds__(kSBlock, kSWaves) void ens_stream_kernel(
    const int64_t* __restrict__ off, const double* __restrict__ epsv, const int* __restrict__ nparts,
    const SItem* __restrict__ items, const int* __restrict__ wg_off, const int* __restrict__ wg_list,
    double* __restrict__ x, double* __restrict__ v, double* __restrict__ a, const double* __restrict__ m,
    JRec<MODE>* __restrict__ xrec, int* __restrict__ cnt, int64_t total, double dt, int64_t nsteps, double G,
    int acc_valid, uint64_t wait_ticks) {
  using R = Real<MODE>;
  constexpr bool kNear = MODE == kFP32C;
  static_assert(sizeof(SPart<MODE>) * kSBlock <= sizeof(JRec<MODE>) * 2 * kSBlock, "group partials alias the tiles");
  __shared__ JRec<MODE> tile[2][kSBlock];
  __shared__ int lds_bad;
  SPart<MODE>* gpart = reinterpret_cast<SPart<MODE>*>(&tile[0][0]);
  const int t = threadIdx.x;
  const double h = 0.5 * dt;
  const int q0 = wg_off[blockIdx.x], q1 = wg_off[blockIdx.x + 1];
  bool bad = false;  // a wait of this workgroup timed out (uniform)

  const int64_t rounds = nsteps + (acc_valid ? 0 : 1);
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t s = acc_valid ? r : r - 1;  // step of this round; -1: the initial evaluation
    JRec<MODE>* xb = xrec + (size_t)(r & 1) * total;
    // ---- phase A: kick-drift the owned particles and publish their records
    for (int q = q0; q < q1; ++q) {
      const SItem it = items[wg_list[q]];
      const int64_t o = off[it.sys];
      if (t < it.ni) {
        const int64_t i = o + it.i0 + t;
        double xn[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int64_t e = d * total + i;
          if (s >= 0) {
            double ve = v[e];
            const double ae = a[e];
            ve = fma(h, ae, ve);
            if (s > 0) ve = fma(h, ae, ve);  // closing half-kick of the previous step, rounded separately
            v[e] = ve;
            xn[d] = fma(dt, ve, x[e]);
            x[e] = xn[d];
          } else {
            xn[d] = x[e];
          }
        }
        xb[i] = bad ? JRec<MODE>::make(NAN, NAN, NAN, NAN) : JRec<MODE>::make(xn[0], xn[1], xn[2], m[i]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have completed
    __syncthreads();
    if (t == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      for (int q = q0; q < q1; ++q)
        __hip_atomic_fetch_add(cnt + items[wg_list[q]].sys, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // ---- wait until every item of every system held here has published this round.
      // Counters wrap modulo 2^32 and are never more than one round ahead of `want`;
      // after one expired wait the workgroup stops waiting (its results are NaN anyway).
      int ok = bad ? 0 : 1;
      for (int q = q0; q < q1 && ok; ++q) {
        const int sys = items[wg_list[q]].sys;
        const unsigned want = (unsigned)nparts[sys] * (unsigned)(r + 1);
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while (ok && (int)((unsigned)__hip_atomic_load(cnt + sys, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                           want) < 0) {
          if (__builtin_amdgcn_s_memrealtime() - t0 > wait_ticks) ok = 0;
          else __builtin_amdgcn_s_sleep(1);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      lds_bad = ok ? 0 : 1;
    }
    __syncthreads();
    bad = bad || lds_bad != 0;

    // ---- phase B: evaluate the items
    for (int q = q0; q < q1; ++q) {
      const SItem it = items[wg_list[q]];
      const int64_t o = off[it.sys];
      const int nc = (int)(off[it.sys + 1] - o);
      const JRec<MODE>* src = xb + o;
      const int gsz = kSBlock / it.js;
      const int g = t / gsz, l = t - g * gsz;
      const int il = l < it.ni ? l : it.ni - 1;
      const int ii = it.i0 + il;  // system-local index of the lane's particle
      const int iself = l < it.ni ? ii : -1;
      const bool wave_live = (l & ~63) < it.ni;  // gsz is a multiple of 64: uniform per wave
      const double eps = epsv[it.sys];
      const R e2 = (R)(eps * eps);
      IPos<MODE> pi;
      pi.from(src[ii]);
      R rc2 = R(0);
      if constexpr (kNear) rc2 = near_rc2(pi.hx, pi.hy, pi.hz, eps, nc);
      R hx = 0, hy = 0, hz = 0, lx = 0, ly = 0, lz = 0;
      const int ntiles = (nc + kSBlock - 1) / kSBlock;
      tile[0][t] = t < nc ? src[t] : JRec<MODE>::make(kFarAway, kFarAway, kFarAway, 0.0);
      __syncthreads();
      for (int tt = 0; tt < ntiles; ++tt) {
        const int jt = tt * kSBlock;
        const bool more = tt + 1 < ntiles;
        JRec<MODE> nxt;
        if (more) {
          const int jn = jt + kSBlock + t;
          nxt = jn < nc ? src[jn] : JRec<MODE>::make(kFarAway, kFarAway, kFarAway, 0.0);
        }
        const JRec<MODE>* cur = tile[tt & 1];
        // this group's slice of the tile's valid records: the records are dealt
        // to the groups in equal runs of whole fold blocks, [g*cs, (g+1)*cs), so
        // a partly filled tile still spreads over the groups; a run never
        // reaches past the tile's last fold block (cs and g*cs are multiples of
        // kFold), and records past nc are zero-mass padding.
        // A wave none of whose lanes owns a particle of the item skips the pairs
        // (it still stages tiles and meets the barriers), leaving the SIMD to the others.
        const int cntt = min(kSBlock, nc - jt);
        const int cs = ((cntt + it.js - 1) / it.js + kFold - 1) / kFold * kFold;
        const int j0 = g * cs;
        const int cntg = wave_live ? max(0, min(cs, cntt - j0)) : 0;
        const int fend = j0 + (cntg + kFold - 1) / kFold * kFold;
#pragma unroll 1
        for (int f = j0; f < fend; f += kFold) {
          R px = 0, py = 0, pz = 0, r2min = R(3.0e38f);
#pragma unroll 16
          for (int jj = f; jj < f + kFold; ++jj) {
            const JRec<MODE> rj = cur[jj];
            R dx, dy, dz;
            if constexpr (kNear) disp_hi(rj, pi, dx, dy, dz);
            else disp(rj, pi, dx, dy, dz);
            const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
            const R ri = rsq(r2);
            R sc = (jmass(rj) * ri) * (ri * ri);
            if constexpr (EXCL) sc = (jt + jj == iself) ? R(0) : sc;
            px = fma(sc, dx, px);
            py = fma(sc, dy, py);
            pz = fma(sc, dz, pz);
            if constexpr (kNear) r2min = fminf(r2min, r2);
          }
          if constexpr (kNear) {
            // the lane's own pair always has r2 = eps^2: in its block, rescan for another close pair
            bool close = r2min < rc2;
            if (close && (unsigned)(iself - (jt + f)) < (unsigned)kFold) {
              close = false;
              for (int jj = f; jj < f + kFold; ++jj) {
                R dx, dy, dz;
                disp_hi(cur[jj], pi, dx, dy, dz);
                const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
                close = close || (r2 < rc2 && jt + jj != iself);
              }
            }
            if (close) {
              // rare: redo this block with float-float displacements for the close pairs
              R qx = 0, qy = 0, qz = 0;
              for (int jj = f; jj < f + kFold; ++jj) {
                const JRec<MODE> rj = cur[jj];
                R dx, dy, dz;
                disp_hi(rj, pi, dx, dy, dz);
                R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
                if (r2 < rc2) {
                  disp(rj, pi, dx, dy, dz);
                  r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
                }
                const R ri = rsq(r2);
                R sc = (jmass(rj) * ri) * (ri * ri);
                if constexpr (EXCL) sc = (jt + jj == iself) ? R(0) : sc;
                qx = fma(sc, dx, qx);
                qy = fma(sc, dy, qy);
                qz = fma(sc, dz, qz);
              }
              px = qx;
              py = qy;
              pz = qz;
            }
          }
          fold(hx, lx, px);
          fold(hy, ly, py);
          fold(hz, lz, pz);
        }
        if (more) tile[(tt + 1) & 1][t] = nxt;
        __syncthreads();
      }
      // combine the j-groups in group order (the tiles are free: gpart aliases them)
      if (g > 0) gpart[(g - 1) * gsz + l] = SPart<MODE>{hx, lx, hy, ly, hz, lz};
      __syncthreads();
      if (g == 0) {
        for (int gg = 1; gg < it.js; ++gg) {
          const SPart<MODE> p = gpart[(gg - 1) * gsz + l];
          fold(hx, lx, p.hx); lx += p.lx;
          fold(hy, ly, p.hy); ly += p.ly;
          fold(hz, lz, p.hz); lz += p.lz;
        }
        if (l < it.ni) {
          const int64_t i = o + ii;
          a[i] = G * ((double)hx + (double)lx);
          a[total + i] = G * ((double)hy + (double)ly);
          a[2 * total + i] = G * ((double)hz + (double)lz);
        }
      }
      __syncthreads();  // before the next item's tile reuses the LDS
    }
  }
  // closing half-kick of the last step; a workgroup whose wait timed out marks its particles NaN
  for (int q = q0; q < q1; ++q) {
    const SItem it = items[wg_list[q]];
    if (t < it.ni) {
      const int64_t i = off[it.sys] + it.i0 + t;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int64_t e = d * total + i;
        if (bad) {
          x[e] = NAN;
          v[e] = NAN;
          a[e] = NAN;
        } else if (nsteps > 0) {
          v[e] = fma(h, a[e], v[e]);
        }
      }
    }
  }
}

// ------------------------------------------------------------- wave items
// Items of at most 64 particles (bitem = 64), each evaluated by ONE wave
// against its system's whole j-range.  The wave streams the system's pair
// records through its own 64-record LDS slot (records written and read by
// the same wave, so no workgroup barrier inside an item).  Items are placed
// longest first over the workgroups; inside a workgroup the waves take the
// next item of its list (longest first) from an LDS counter as they become
// free, so the SIMD arbiter's preference for older waves, which makes
// statically assigned waves of equal cost finish up to 1.7x apart, costs
// nothing, and the workgroup ends a round with its shortest items.  Phase A
// and the closing half-kick deal the workgroup's items to its waves
// statically.  The round protocol is the one above, per workgroup (one
// release, one acquire): wave 0 publishes for every system the workgroup
// holds items of, one lane per system, and waits for all of them the same
// way.
constexpr int kWWaves = kSBlock / 64;  // waves per workgroup

// Orders this wave's LDS accesses around a rewrite of its slot (LDS
// instructions of one wave execute in order; this keeps the compiler from
// moving reads and writes across the point).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FP64 pairs need more than the 64 VGPRs of 8 waves per SIMD; they run at 4
// (one workgroup per CU) without spilling.
template <int MODE> constexpr int wave_kernel_waves() { return MODE == kFP64 ? 4 : kSWaves; }

template <int MODE, bool EXCL>
__global__ __launch_bounds__(kSBlock, wave_kernel_waves<MODE>()) void ens_wave_kernel(
    const int64_t* __restrict__ off, const double* __restrict__ epsv, const int* __restrict__ nparts,
    const SItem* __restrict__ items, const int* __restrict__ wg_off, const int* __restrict__ wg_list,
    const int* __restrict__ ws_off, const int2* __restrict__ ws_sys, double* __restrict__ x,
    double* __restrict__ v, double* __restrict__ a, const double* __restrict__ m, JRec<MODE>* __restrict__ xrec,
    int* __restrict__ cnt, int64_t total, double dt, int64_t nsteps, double G, int acc_valid, uint64_t wait_ticks) {
  using R = Real<MODE>;
  constexpr bool kNear = MODE == kFP32C;
  __shared__ JRec<MODE> slot[kWWaves][64];
  __shared__ int lds_bad;
  __shared__ int next_item;
  const int t = threadIdx.x;
  const int wv = t >> 6, lane = t & 63;
  const int q0 = wg_off[blockIdx.x], q1 = wg_off[blockIdx.x + 1];
  const int s0 = ws_off[blockIdx.x], s1 = ws_off[blockIdx.x + 1];
  JRec<MODE>* buf = slot[wv];
  const double h = 0.5 * dt;
  bool bad = false;  // a wait of this workgroup timed out (uniform)

  const int64_t rounds = nsteps + (acc_valid ? 0 : 1);
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t s = acc_valid ? r : r - 1;  // step of this round; -1: the initial evaluation
    JRec<MODE>* xb = xrec + (size_t)(r & 1) * total;
    // ---- phase A: kick-drift the workgroup's particles (items dealt to the waves) and publish their records
    for (int q = q0 + wv; q < q1; q += kWWaves) {
      const SItem it = items[wg_list[q]];
      if (lane < it.ni) {
        const int64_t i = off[it.sys] + it.i0 + lane;
        double xn[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int64_t e = d * total + i;
          if (s >= 0) {
            double ve = v[e];
            const double ae = a[e];
            ve = fma(h, ae, ve);
            if (s > 0) ve = fma(h, ae, ve);  // closing half-kick of the previous step, rounded separately
            v[e] = ve;
            xn[d] = fma(dt, ve, x[e]);
            x[e] = xn[d];
          } else {
            xn[d] = x[e];
          }
        }
        xb[i] = bad ? JRec<MODE>::make(NAN, NAN, NAN, NAN) : JRec<MODE>::make(xn[0], xn[1], xn[2], m[i]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have completed
    __syncthreads();
    if (wv == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      for (int k = s0 + lane; k < s1; k += 64)
        __hip_atomic_fetch_add(cnt + ws_sys[k].x, ws_sys[k].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // ---- wait, one lane per held system, until every item of it has published this round
      int ok = bad ? 0 : 1;
      for (int k = s0 + lane; k < s1 && ok; k += 64) {
        const int sys = ws_sys[k].x;
        const unsigned want = (unsigned)nparts[sys] * (unsigned)(r + 1);
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while ((int)((unsigned)__hip_atomic_load(cnt + sys, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - want) < 0) {
          if (__builtin_amdgcn_s_memrealtime() - t0 > wait_ticks) { ok = 0; break; }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      const bool all_ok = __ballot(!ok) == 0;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (lane == 0) {
        lds_bad = all_ok ? 0 : 1;
        next_item = 0;
      }
    }
    __syncthreads();
    bad = bad || lds_bad != 0;

    // ---- phase B: each wave takes the workgroup's next item and evaluates it
    // against its system's whole j-range
    for (;;) {
      int k = 0;
      if (lane == 0) k = atomicAdd(&next_item, 1);
      k = __builtin_amdgcn_readfirstlane(k);
      if (k >= q1 - q0) break;
      const SItem it = items[wg_list[q0 + k]];
      const int64_t o = off[it.sys];
      const int nc = (int)(off[it.sys + 1] - o);
      const JRec<MODE>* src = xb + o;
      const int ii = it.i0 + (lane < it.ni ? lane : it.ni - 1);  // system-local index of the lane's particle
      const int iself = lane < it.ni ? ii : -1;
      const double eps = epsv[it.sys];
      const R e2 = (R)(eps * eps);
      IPos<MODE> pi;
      pi.from(src[ii]);
      R rc2 = R(0);
      if constexpr (kNear) rc2 = near_rc2(pi.hx, pi.hy, pi.hz, eps, nc);
      R hx = 0, hy = 0, hz = 0, lx = 0, ly = 0, lz = 0;
      JRec<MODE> nxt = lane < nc ? src[lane] : JRec<MODE>::make(kFarAway, kFarAway, kFarAway, 0.0);
#pragma unroll 1
      for (int jt = 0; jt < nc; jt += 64) {
        wave_lds_sync();  // the previous block's reads are done
        buf[lane] = nxt;
        wave_lds_sync();  // the block is in the slot
        if (jt + 64 < nc) {
          const int jn = jt + 64 + lane;
          nxt = jn < nc ? src[jn] : JRec<MODE>::make(kFarAway, kFarAway, kFarAway, 0.0);
        }
        // OWN: the block holding the lanes' own particles (the item's 64
        // particles are one aligned block of its system): there the own pair,
        // whose r2 is eps^2, is left out of the near-field minimum
        // FULL: 64 records; otherwise the system's last, partly filled block,
        // of which only the cnt valid records are applied
        auto block = [&](auto own_tag, auto full_tag, int cnt) {
          constexpr bool kOwn = decltype(own_tag)::value;
          constexpr bool kFull = decltype(full_tag)::value;
          const int jend = kFull ? 64 : cnt;
          R px = 0, py = 0, pz = 0, r2min = R(3.0e38f);
#pragma unroll 16
          for (int jj = 0; jj < jend; ++jj) {
            const JRec<MODE> rj = buf[jj];
            R dx, dy, dz;
            if constexpr (kNear) disp_hi(rj, pi, dx, dy, dz);
            else disp(rj, pi, dx, dy, dz);
            const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
            const R ri = rsq(r2);
            R sc = (jmass(rj) * ri) * (ri * ri);
            if constexpr (EXCL) sc = (jt + jj == iself) ? R(0) : sc;
            px = fma(sc, dx, px);
            py = fma(sc, dy, py);
            pz = fma(sc, dz, pz);
            if constexpr (kNear) r2min = fminf(r2min, (kOwn && jt + jj == ii) ? R(3.0e38f) : r2);
          }
          if constexpr (kNear) {
            if (r2min < rc2) {
              // rare: redo this block with float-float displacements for the close pairs
              R qx = 0, qy = 0, qz = 0;
              for (int jj = 0; jj < jend; ++jj) {
                const JRec<MODE> rj = buf[jj];
                R dx, dy, dz;
                disp_hi(rj, pi, dx, dy, dz);
                R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
                if (r2 < rc2) {
                  disp(rj, pi, dx, dy, dz);
                  r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
                }
                const R ri = rsq(r2);
                R sc = (jmass(rj) * ri) * (ri * ri);
                if constexpr (EXCL) sc = (jt + jj == iself) ? R(0) : sc;
                qx = fma(sc, dx, qx);
                qy = fma(sc, dy, qy);
                qz = fma(sc, dz, qz);
              }
              px = qx;
              py = qy;
              pz = qz;
            }
          }
          fold(hx, lx, px);
          fold(hy, ly, py);
          fold(hz, lz, pz);
        };
        const int cnt = nc - jt;
        if (cnt >= 64) {
          if (jt == it.i0) block(std::true_type{}, std::true_type{}, 64);
          else block(std::false_type{}, std::true_type{}, 64);
        } else {
          if (jt == it.i0) block(std::true_type{}, std::false_type{}, cnt);
          else block(std::false_type{}, std::false_type{}, cnt);
        }
      }
      if (lane < it.ni) {
        const int64_t i = o + ii;
        a[i] = G * ((double)hx + (double)lx);
        a[total + i] = G * ((double)hy + (double)ly);
        a[2 * total + i] = G * ((double)hz + (double)lz);
      }
    }
    __syncthreads();  // the accelerations are visible to the waves that kick these particles next
  }
  // closing half-kick of the last step; a workgroup whose wait timed out marks its particles NaN
  for (int q = q0 + wv; q < q1; q += kWWaves) {
    const SItem it = items[wg_list[q]];
    if (lane < it.ni) {
      const int64_t i = off[it.sys] + it.i0 + lane;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int64_t e = d * total + i;
        if (bad) {
          x[e] = NAN;
          v[e] = NAN;
          a[e] = NAN;
        } else if (nsteps > 0) {
          v[e] = fma(h, a[e], v[e]);
        }
      }
    }
  }
}

// ----------------------------------------------------- wave items, per step
// The same items without the persistent loop: every step is two launches,
// ens_publish_kernel (the kicks and the drift of every particle, and its pair
// record) and ens_waveforce_kernel (each workgroup's waves take its items from
// an LDS counter and write the accelerations).  The kernel boundary is the
// step's synchronisation, so no workgroup waits for another and nothing needs
// every workgroup resident at once; the price is two launches per step.

// kicks = 0: publish only; 1: v += h a, x += dt v; 2: v += h a twice (closing
// half-kick of the previous step, opening half-kick of this one, rounded
// separately), x += dt v.  Then the pair record of the new position.
// With rcnt (FP32C with the rescue): the per-system counts of flagged rows
// start the step at zero.
template <int MODE>
__global__ void ens_publish_kernel(int64_t total, double* __restrict__ x, double* __restrict__ v,
                                   const double* __restrict__ a, const double* __restrict__ m,
                                   JRec<MODE>* __restrict__ xrec, double h, double dt, int kicks,
                                   int* __restrict__ rcnt, int ncl) {
  if (rcnt)
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncl; c += gridDim.x * blockDim.x) rcnt[c] = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
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
    xrec[i] = JRec<MODE>::make(xn[0], xn[1], xn[2], m[i]);
  }
}

__global__ void ens_kick_kernel(int64_t total, double* __restrict__ v, const double* __restrict__ a, double h) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 3 * total; e += (int64_t)gridDim.x * blockDim.x)
    v[e] = fma(h, a[e], v[e]);
}

// With rcnt (FP32C with the rescue): the wave keeps each row's rounding-error
// estimate (one share per block of 64 j, as the pair kernels do; see
// rescue.hip) and appends the rows whose estimate is too large to its system's
// list (rlist from the system's first particle on, rcnt[system] rows; one
// atomic add per wave reserves the places), for ens_rescue_kernel.
template <int MODE, bool EXCL>
__global__ __launch_bounds__(kSBlock, wave_kernel_waves<MODE>()) void ens_waveforce_kernel(
    const int64_t* __restrict__ off, const double* __restrict__ epsv, const SItem* __restrict__ items,
    const int* __restrict__ wg_off, const int* __restrict__ wg_list, const JRec<MODE>* __restrict__ xrec,
    double* __restrict__ a, int64_t total, double G, int* __restrict__ rcnt, int* __restrict__ rlist) {
  using R = Real<MODE>;
  constexpr bool kNear = MODE == kFP32C;
  __shared__ JRec<MODE> slot[kWWaves][64];
  __shared__ int next_item;
  const int t = threadIdx.x;
  const int wv = t >> 6, lane = t & 63;
  const int q0 = wg_off[blockIdx.x], q1 = wg_off[blockIdx.x + 1];
  JRec<MODE>* buf = slot[wv];
  if (t == 0) next_item = 0;
  __syncthreads();
  for (;;) {
    int k = 0;
    if (lane == 0) k = atomicAdd(&next_item, 1);
    k = __builtin_amdgcn_readfirstlane(k);
    if (k >= q1 - q0) break;
    const SItem it = items[wg_list[q0 + k]];
    const int64_t o = off[it.sys];
    const int nc = (int)(off[it.sys + 1] - o);
    const JRec<MODE>* src = xrec + o;
    const int ii = it.i0 + (lane < it.ni ? lane : it.ni - 1);
    const int iself = lane < it.ni ? ii : -1;
    const double eps = epsv[it.sys];
    const R e2 = (R)(eps * eps);
    IPos<MODE> pi;
    pi.from(src[ii]);
    R rc2 = R(0);
    float xinf = 0.f, eacc = 0.f;
    if constexpr (kNear) {
      rc2 = near_rc2(pi.hx, pi.hy, pi.hz, eps, nc);
      xinf = fmaxf(fabsf(pi.hx), fmaxf(fabsf(pi.hy), fabsf(pi.hz)));
    }
    R hx = 0, hy = 0, hz = 0, lx = 0, ly = 0, lz = 0;
    JRec<MODE> nxt = lane < nc ? src[lane] : JRec<MODE>::make(kFarAway, kFarAway, kFarAway, 0.0);
#pragma unroll 1
    for (int jt = 0; jt < nc; jt += 64) {
      wave_lds_sync();
      buf[lane] = nxt;
      wave_lds_sync();
      if (jt + 64 < nc) {
        const int jn = jt + 64 + lane;
        nxt = jn < nc ? src[jn] : JRec<MODE>::make(kFarAway, kFarAway, kFarAway, 0.0);
      }
      auto block = [&](auto own_tag, auto full_tag, int cnt) {
        constexpr bool kOwn = decltype(own_tag)::value;
        constexpr bool kFull = decltype(full_tag)::value;
        const int jend = kFull ? 64 : cnt;
        R px = 0, py = 0, pz = 0, r2min = R(3.0e38f);
#pragma unroll 16
        for (int jj = 0; jj < jend; ++jj) {
          const JRec<MODE> rj = buf[jj];
          R dx, dy, dz;
          if constexpr (kNear) disp_hi(rj, pi, dx, dy, dz);
          else disp(rj, pi, dx, dy, dz);
          const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
          const R ri = rsq(r2);
          R sc = (jmass(rj) * ri) * (ri * ri);
          if constexpr (EXCL) sc = (jt + jj == iself) ? R(0) : sc;
          px = fma(sc, dx, px);
          py = fma(sc, dy, py);
          pz = fma(sc, dz, pz);
          if constexpr (kNear) r2min = fminf(r2min, (kOwn && jt + jj == ii) ? R(3.0e38f) : r2);
        }
        if constexpr (kNear) {
          if (r2min < rc2) {
            // rare: redo this block with float-float displacements for the close pairs
            R qx = 0, qy = 0, qz = 0, r2nr = R(3.0e38f);
            for (int jj = 0; jj < jend; ++jj) {
              const JRec<MODE> rj = buf[jj];
              R dx, dy, dz;
              disp_hi(rj, pi, dx, dy, dz);
              R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
              if (r2 < rc2) {
                disp(rj, pi, dx, dy, dz);
                r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
              } else {
                r2nr = fminf(r2nr, r2);
              }
              const R ri = rsq(r2);
              R sc = (jmass(rj) * ri) * (ri * ri);
              if constexpr (EXCL) sc = (jt + jj == iself) ? R(0) : sc;
              qx = fma(sc, dx, qx);
              qy = fma(sc, dy, qy);
              qz = fma(sc, dz, qz);
            }
            px = qx;
            py = qy;
            pz = qz;
            r2min = r2nr;
          }
          if (rcnt) eacc = est_add(eacc, px, py, pz, xinf, r2min);
        }
        fold(hx, lx, px);
        fold(hy, ly, py);
        fold(hz, lz, pz);
      };
      const int cnt = nc - jt;
      if (cnt >= 64) {
        if (jt == it.i0) block(std::true_type{}, std::true_type{}, 64);
        else block(std::false_type{}, std::true_type{}, 64);
      } else {
        if (jt == it.i0) block(std::true_type{}, std::false_type{}, cnt);
        else block(std::false_type{}, std::false_type{}, cnt);
      }
    }
    const double ax = G * ((double)hx + (double)lx), ay = G * ((double)hy + (double)ly),
                 az = G * ((double)hz + (double)lz);
    bool flag = false;
    if (lane < it.ni) {
      const int64_t i = o + ii;
      a[i] = ax;
      a[total + i] = ay;
      a[2 * total + i] = az;
      if (kNear && rcnt) flag = sqrt((double)eacc) * (kRescueScale * fabs(G)) > sqrt(ax * ax + ay * ay + az * az);
    }
    if constexpr (kNear) {
      const unsigned long long mask = __ballot(flag);
      if (mask) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&rcnt[it.sys], __popcll(mask));
        base = __shfl(base, 0, 64);
        if (flag) rlist[o + base + __popcll(mask & ((1ull << lane) - 1ull))] = ii;
      }
    }
  }
}

// The FP64 rescue of the rows the force kernel flagged: kRSplit workgroups
// per system (kRWaves waves each) share its listed rows, kRRow rows per wave
// and pass, workgroup p taking the passes p, p + kRSplit, ...; each stages
// the system's FP64 positions and masses in LDS (kRStage records at a time; a
// system that fits is staged once) unless it has no rows, and lane l of a wave
// takes j = l, l + 64, ... of each stage; the lane sums are added by a
// butterfly, so the result does not depend on the list's order or the grid.
constexpr int kRWaves = 8;
constexpr int kRRow = 2;
constexpr int kRStage = 2048;
constexpr int kRSplit = 8;
template <bool EXCL>
__global__ __launch_bounds__(64 * kRWaves) void ens_rescue_kernel(const int64_t* __restrict__ off,
                                                                  const double* __restrict__ epsv, int64_t total,
                                                                  const double* __restrict__ x,
                                                                  const double* __restrict__ m, double G,
                                                                  const int* __restrict__ rcnt,
                                                                  const int* __restrict__ rlist,
                                                                  double* __restrict__ a) {
  __shared__ double sj[4][kRStage];
  const int c = blockIdx.x;
  const int nf = rcnt[c];
  constexpr int kPass = kRWaves * kRRow;
  if ((int)blockIdx.y * kPass >= nf) return;
  const int t = threadIdx.x, wave = t / 64, lane = t % 64;
  const int64_t o = off[c];
  const int nc = (int)(off[c + 1] - o);
  const double e2 = epsv[c] * epsv[c];
  auto stage = [&](int c0) {
    const int cn = min(kRStage, nc - c0);
    for (int j = t; j < cn; j += 64 * kRWaves) {
      sj[0][j] = x[o + c0 + j];
      sj[1][j] = x[total + o + c0 + j];
      sj[2][j] = x[2 * total + o + c0 + j];
      sj[3][j] = m[o + c0 + j];
    }
  };
  const bool once = nc <= kRStage;
  if (once) {
    stage(0);
    __syncthreads();
  }
  for (int g0 = blockIdx.y * kPass; g0 < nf; g0 += kRSplit * kPass) {
    int li[kRRow];
    double xi[kRRow], yi[kRRow], zi[kRRow], sx[kRRow], sy[kRRow], sz[kRRow];
#pragma unroll
    for (int k = 0; k < kRRow; ++k) {
      const int r = g0 + wave * kRRow + k;
      li[k] = r < nf ? rlist[o + r] : -1;
      const int64_t i = o + (li[k] < 0 ? 0 : li[k]);
      xi[k] = x[i];
      yi[k] = x[total + i];
      zi[k] = x[2 * total + i];
      sx[k] = sy[k] = sz[k] = 0.0;
    }
    for (int c0 = 0; c0 < nc; c0 += kRStage) {
      if (!once) {
        __syncthreads();  // the previous stage has been read
        stage(c0);
        __syncthreads();
      }
      if (li[0] < 0) continue;
      const int cn = min(kRStage, nc - c0);
#pragma unroll 2
      for (int j = lane; j < cn; j += 64) {
        const double xj = sj[0][j], yj = sj[1][j], zj = sj[2][j], mj = sj[3][j];
#pragma unroll
        for (int k = 0; k < kRRow; ++k) {
          const double dx = xj - xi[k], dy = yj - yi[k], dz = zj - zi[k];
          const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
          const double rr = rsqrt64(r2);
          double sc = (mj * rr) * (rr * rr);
          if (EXCL && c0 + j == li[k]) sc = 0.0;
          sx[k] = fma(sc, dx, sx[k]);
          sy[k] = fma(sc, dy, sy[k]);
          sz[k] = fma(sc, dz, sz[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kRRow; ++k) {
      for (int w = 32; w > 0; w >>= 1) {
        sx[k] += __shfl_xor(sx[k], w, 64);
        sy[k] += __shfl_xor(sy[k], w, 64);
        sz[k] += __shfl_xor(sz[k], w, 64);
      }
      if (lane == 0 && li[k] >= 0) {
        const int64_t i = o + li[k];
        a[i] = G * sx[k];
        a[total + i] = G * sy[k];
        a[2 * total + i] = G * sz[k];
      }
    }
  }
}

__global__ void zero_counters_kernel(int* c, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) c[i] = 0;
}

// ------------------------------------------------------------------ plans
struct SPlan {
  std::vector<int64_t> off;
  std::vector<double> eps;
  int precision = 0, device = 0, nwg = 0, ncl = 0, bitem = 0;
  int64_t total = 0;
  uint64_t wait_ticks = 0;  // bound of one counter wait, 100 MHz ticks
  int64_t* d_off = nullptr;
  double* d_eps = nullptr;
  int* d_nparts = nullptr;
  SItem* d_items = nullptr;
  int* d_wg_off = nullptr;   // per workgroup: offsets into d_wg_list
  int* d_wg_list = nullptr;
  int* d_ws_off = nullptr;   // wave items: per workgroup, offsets into d_ws_sys
  int2* d_ws_sys = nullptr;  // wave items: (system, items of it held by the workgroup)
  void* d_xrec = nullptr;
  int* d_cnt = nullptr;
  int* d_rcnt = nullptr;   // per-step wave items, FP32C: flagged rows per system (ncl)
  int* d_rlist = nullptr;  // and their lists (total, each system's from its first particle on)
};

std::mutex g_splan_mu;
std::vector<SPlan*> g_splans;

void free_splan(SPlan* p) {
  for (void* q : {(void*)p->d_off, (void*)p->d_eps, (void*)p->d_nparts, (void*)p->d_items, (void*)p->d_wg_off,
                  (void*)p->d_wg_list, (void*)p->d_ws_off, (void*)p->d_ws_sys, p->d_xrec, (void*)p->d_cnt,
                  (void*)p->d_rcnt, (void*)p->d_rlist})
    if (q) (void)hipFree(q);
  delete p;
}

template <typename T>
bool supload(T** dst, const std::vector<T>& src) {
  const size_t bytes = sizeof(T) * std::max<size_t>(1, src.size());
  if (hipMalloc(dst, bytes) != hipSuccess) return false;
  return src.empty() || hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) == hipSuccess;
}

// Workgroups of the kernel that fit on one CU at once (both EXCL variants), at most kSMaxPerCu.
template <typename K>
int resident_per_cu(K k0, K k1) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(k0), kSBlock, 0) != hipSuccess)
    nb = 1;
  int nb2 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, reinterpret_cast<const void*>(k1), kSBlock, 0) != hipSuccess)
    nb2 = 1;
  (void)hipGetLastError();
  return std::max(1, std::min(kSMaxPerCu, std::min(nb, nb2)));
}

template <int MODE>
int resident_per_cu() {
  return resident_per_cu(&ens_stream_kernel<MODE, false>, &ens_stream_kernel<MODE, true>);
}

// j-records one lane applies per round for an item of a system of nc
// particles with js j-groups: each tile's valid records are dealt to the
// groups in equal runs of whole fold blocks (as in ens_stream_kernel).
double item_rounds(int64_t nc, int js) {
  double w = 0.0;
  for (int64_t jt = 0; jt < nc; jt += kSBlock) {
    const int64_t cnt = std::min<int64_t>(kSBlock, nc - jt);
    w += (double)(((cnt + js - 1) / js + kFold - 1) / kFold * kFold);
  }
  return w;
}

// Items: a system of nc <= 256 particles is one item whose lanes split j into
// js = 16, 8 or 4 groups (nc <= 64, 128, 256); larger systems are cut into
// ceil(nc / bitem) near-equal items with 1024 / bitem j-groups (bitem = 1024,
// one group, unless configured: measured on the 512-cluster workload, 1024
// gave 1.18 ms per step, 512 1.21 and 256 1.25).  Cost of an item per round:
// its j-iterations per lane plus a fixed overhead, i.e. its duration, since a
// workgroup runs its items one after the other (weighting by the item's live
// waves instead, a measure of its share of SIMD throughput, was measured
// 46 % slower on the 512-cluster workload).
template <int MODE>
int build_splan(int32_t ncl, const int64_t* off, const double* eps, int precision, int device, int bitem,
                SPlan** out) {
  SPlan* p = new SPlan();
  p->off.assign(off, off + ncl + 1);
  p->eps.assign(eps, eps + ncl);
  p->precision = precision;
  p->device = device;
  p->ncl = ncl;
  p->bitem = bitem;
  p->total = off[ncl];
  const int item_max = bitem > 0 ? bitem : 1024;
  std::vector<SItem> items;
  std::vector<double> cost;
  std::vector<int> nparts(ncl, 0);
  for (int c = 0; c < ncl; ++c) {
    const int64_t nc = off[c + 1] - off[c];
    if (nc <= 0) continue;
    if (nc > (int64_t(1) << 24)) {
      delete p;
      return set_error(NBODY_EUNSUPPORTED, "batched: a system of more than 2^24 particles");
    }
    const int js = nc <= 64 ? 16 : nc <= 128 ? 8 : nc <= 256 ? 4 : kSBlock / item_max;
    const int cap = kSBlock / js;
    const int P = (int)((nc + cap - 1) / cap);
    const int per = (int)((nc + P - 1) / P);
    for (int k = 0; k < P; ++k) {
      const int i0 = k * per;
      const int ni = (int)std::min<int64_t>(per, nc - i0);
      if (ni <= 0) continue;
      items.push_back(SItem{c, i0, ni, js});
      cost.push_back(item_rounds(nc, js) + 96.0);
      ++nparts[c];
    }
  }
  const int cap_wg = std::max(1, resident_per_cu<MODE>() * cu_count(device));
  const int nwg = std::max(1, std::min<int>((int)items.size(), cap_wg));
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
  double maxpairs = 0.0;
  for (int w = 0; w < nwg; ++w) {
    wg_list.insert(wg_list.end(), lists[w].begin(), lists[w].end());
    wg_off[w + 1] = (int)wg_list.size();
    double pairs = 0.0;
    for (int k : lists[w]) pairs += (double)items[k].ni * (double)(off[items[k].sys + 1] - off[items[k].sys]);
    maxpairs = std::max(maxpairs, pairs);
  }
  p->nwg = nwg;
  // a counter wait lasts at most about one round of the busiest workgroup
  p->wait_ticks = (uint64_t)(1.0e8 * (2.0 + maxpairs / 1.0e8));
  bool ok = supload(&p->d_off, p->off) && supload(&p->d_eps, p->eps) && supload(&p->d_nparts, nparts) &&
            supload(&p->d_items, items) && supload(&p->d_wg_off, wg_off) && supload(&p->d_wg_list, wg_list) &&
            hipMalloc(&p->d_xrec, 2 * (size_t)std::max<int64_t>(1, p->total) * sizeof(JRec<MODE>)) == hipSuccess &&
            hipMalloc(&p->d_cnt, sizeof(int) * (size_t)std::max(1, ncl)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_splan(p);
    return set_error(NBODY_ENOMEM, "batched: plan upload failed");
  }
  *out = p;
  return NBODY_OK;
}

// Plan of wave items (bitem = 64): every system is cut into items of 64
// consecutive particles (the last one shorter); an item's cost per round is
// its system's j-range padded to blocks of 64 plus a fixed per-item overhead
// (the own-block rescan and the item set-up); items are placed longest first
// on the least loaded workgroup.
template <int MODE>
int build_wplan(int32_t ncl, const int64_t* off, const double* eps, int precision, int device, SPlan** out) {
  SPlan* p = new SPlan();
  p->off.assign(off, off + ncl + 1);
  p->eps.assign(eps, eps + ncl);
  p->precision = precision;
  p->device = device;
  p->ncl = ncl;
  p->bitem = 64;
  p->total = off[ncl];
  std::vector<SItem> items;
  std::vector<double> cost;
  std::vector<int> nparts(ncl, 0);
  for (int c = 0; c < ncl; ++c) {
    const int64_t nc = off[c + 1] - off[c];
    if (nc <= 0) continue;
    if (nc > (int64_t(1) << 24)) {
      delete p;
      return set_error(NBODY_EUNSUPPORTED, "batched: a system of more than 2^24 particles");
    }
    for (int64_t i0 = 0; i0 < nc; i0 += 64) {
      items.push_back(SItem{c, (int)i0, (int)std::min<int64_t>(64, nc - i0), 1});
      cost.push_back((double)((nc + 63) / 64 * 64) + 48.0);
      ++nparts[c];
    }
  }
  const int cap_wg = std::max(1, resident_per_cu(&ens_wave_kernel<MODE, false>, &ens_wave_kernel<MODE, true>) *
                                     cu_count(device));
  const int nwg = std::max(1, std::min<int>((int)((items.size() + kWWaves - 1) / kWWaves), cap_wg));
  std::vector<int> order(items.size());
  for (size_t k = 0; k < items.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int u, int w) { return cost[u] > cost[w]; });
  // longest first over the workgroups; each list stays in decreasing cost,
  // the order in which the workgroup's waves take its items
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
  // per workgroup: the systems it holds items of, with the number of such items
  std::vector<int> ws_off(nwg + 1, 0);
  std::vector<int2> ws_sys;
  double maxpairs = 0.0;
  for (int b = 0; b < nwg; ++b) {
    std::vector<std::pair<int, int>> held;
    for (int k : lists[b]) held.push_back({items[k].sys, 1});
    std::sort(held.begin(), held.end());
    for (size_t k = 0; k < held.size();) {
      size_t e = k;
      while (e < held.size() && held[e].first == held[k].first) ++e;
      ws_sys.push_back(make_int2(held[k].first, (int)(e - k)));
      k = e;
    }
    ws_off[b + 1] = (int)ws_sys.size();
  }
  for (int b = 0; b < nwg; ++b) {
    double pairs = 0.0;
    for (int k : lists[b]) pairs += 64.0 * (double)(off[items[k].sys + 1] - off[items[k].sys]);
    maxpairs = std::max(maxpairs, pairs);
  }
  p->nwg = nwg;
  p->wait_ticks = (uint64_t)(1.0e8 * (2.0 + maxpairs / 1.0e8));
  bool ok = supload(&p->d_off, p->off) && supload(&p->d_eps, p->eps) && supload(&p->d_nparts, nparts) &&
            supload(&p->d_items, items) && supload(&p->d_wg_off, wg_off) && supload(&p->d_wg_list, wg_list) &&
            supload(&p->d_ws_off, ws_off) && supload(&p->d_ws_sys, ws_sys) &&
            hipMalloc(&p->d_xrec, 2 * (size_t)std::max<int64_t>(1, p->total) * sizeof(JRec<MODE>)) == hipSuccess &&
            hipMalloc(&p->d_cnt, sizeof(int) * (size_t)std::max(1, ncl)) == hipSuccess &&
            (MODE != kFP32C ||
             (hipMalloc(&p->d_rcnt, sizeof(int) * (size_t)std::max(1, ncl)) == hipSuccess &&
              hipMalloc(&p->d_rlist, sizeof(int) * (size_t)std::max<int64_t>(1, p->total)) == hipSuccess));
  if (!ok) {
    (void)hipGetLastError();
    free_splan(p);
    return set_error(NBODY_ENOMEM, "batched: plan upload failed");
  }
  *out = p;
  return NBODY_OK;
}

SPlan* find_splan(int32_t ncl, const int64_t* off, const double* eps, int precision, int device, int bitem) {
  for (SPlan* p : g_splans) {
    if (p->device != device || p->precision != precision || p->ncl != ncl || p->bitem != bitem) continue;
    if (std::equal(p->off.begin(), p->off.end(), off) && std::equal(p->eps.begin(), p->eps.end(), eps)) return p;
  }
  return nullptr;
}

template <int MODE>
int launch_splan(const SPlan* p, double* x, double* v, double* a, const double* m, double dt, int64_t nsteps,
                 double G, bool acc_valid, bool excl, hipStream_t s) {
  if (p->total == 0 || (nsteps == 0 && acc_valid)) return NBODY_OK;
  zero_counters_kernel<<<1, 256, 0, s>>>(p->d_cnt, std::max(1, p->ncl));
  NB_LAUNCH_CHECK("zero_counters_kernel");
  auto* rec = static_cast<JRec<MODE>*>(p->d_xrec);
  if (p->bitem == 64) {
    if (excl)
      ens_wave_kernel<MODE, true><<<p->nwg, kSBlock, 0, s>>>(p->d_off, p->d_eps, p->d_nparts, p->d_items, p->d_wg_off,
                                                             p->d_wg_list, p->d_ws_off, p->d_ws_sys, x, v, a, m, rec,
                                                             p->d_cnt, p->total, dt, nsteps, G, acc_valid ? 1 : 0,
                                                             p->wait_ticks);
    else
      ens_wave_kernel<MODE, false><<<p->nwg, kSBlock, 0, s>>>(p->d_off, p->d_eps, p->d_nparts, p->d_items, p->d_wg_off,
                                                              p->d_wg_list, p->d_ws_off, p->d_ws_sys, x, v, a, m, rec,
                                                              p->d_cnt, p->total, dt, nsteps, G, acc_valid ? 1 : 0,
                                                              p->wait_ticks);
    NB_LAUNCH_CHECK("ens_wave_kernel");
    return NBODY_OK;
  }
  if (excl)
    ens_stream_kernel<MODE, true><<<p->nwg, kSBlock, 0, s>>>(p->d_off, p->d_eps, p->d_nparts, p->d_items,
                                                               p->d_wg_off, p->d_wg_list, x, v, a, m, rec, p->d_cnt,
                                                               p->total, dt, nsteps, G, acc_valid ? 1 : 0, p->wait_ticks);
  else
    ens_stream_kernel<MODE, false><<<p->nwg, kSBlock, 0, s>>>(p->d_off, p->d_eps, p->d_nparts, p->d_items,
                                                                p->d_wg_off, p->d_wg_list, x, v, a, m, rec, p->d_cnt,
                                                                p->total, dt, nsteps, G, acc_valid ? 1 : 0, p->wait_ticks);
  NB_LAUNCH_CHECK("ens_stream_kernel");
  return NBODY_OK;
}

template <int MODE>
int launch_wsteps(const SPlan* p, double* x, double* v, double* a, const double* m, double dt, int64_t nsteps,
                  double G, bool acc_valid, bool excl, bool rescue, hipStream_t s) {
  if (p->total == 0 || (nsteps == 0 && acc_valid)) return NBODY_OK;
  auto* rec = static_cast<JRec<MODE>*>(p->d_xrec);
  const double h = 0.5 * dt;
  const unsigned ew = (unsigned)std::min<int64_t>((p->total + 255) / 256, 4096);
  // FP32C with the rescue: the force kernel lists each system's flagged rows
  // (counts cleared by the publish kernel) and ens_rescue_kernel recomputes them
  int* rcnt = rescue && MODE == kFP32C ? p->d_rcnt : nullptr;
  int* rlist = rcnt ? p->d_rlist : nullptr;
  auto force = [&]() -> int {
    if (excl)
      ens_waveforce_kernel<MODE, true><<<p->nwg, kSBlock, 0, s>>>(p->d_off, p->d_eps, p->d_items, p->d_wg_off,
                                                                  p->d_wg_list, rec, a, p->total, G, rcnt, rlist);
    else
      ens_waveforce_kernel<MODE, false><<<p->nwg, kSBlock, 0, s>>>(p->d_off, p->d_eps, p->d_items, p->d_wg_off,
                                                                   p->d_wg_list, rec, a, p->total, G, rcnt, rlist);
    NB_LAUNCH_CHECK("ens_waveforce_kernel");
    if (rcnt) return launch_ens_rescue(p->ncl, p->d_off, p->d_eps, p->total, x, m, G, excl, rcnt, rlist, a, s);
    return NBODY_OK;
  };
  int st;
  if (!acc_valid) {
    ens_publish_kernel<MODE><<<ew, 256, 0, s>>>(p->total, x, v, a, m, rec, h, dt, 0, rcnt, p->ncl);
    NB_LAUNCH_CHECK("ens_publish_kernel");
    if ((st = force())) return st;
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    ens_publish_kernel<MODE><<<ew, 256, 0, s>>>(p->total, x, v, a, m, rec, h, dt, k == 0 ? 1 : 2, rcnt, p->ncl);
    NB_LAUNCH_CHECK("ens_publish_kernel");
    if ((st = force())) return st;
  }
  if (nsteps > 0) {
    ens_kick_kernel<<<ew, 256, 0, s>>>(p->total, v, a, h);
    NB_LAUNCH_CHECK("ens_kick_kernel");
  }
  return NBODY_OK;
}

}  // namespace

int launch_ens_rescue(int32_t ncl, const int64_t* d_off, const double* d_eps, int64_t total, const double* x,
                      const double* m, double G, bool excl, const int* rcnt, const int* rlist, double* a,
                      hipStream_t s) {
  if (ncl <= 0) return NBODY_OK;
  if (excl)
    ens_rescue_kernel<true><<<dim3(ncl, kRSplit), 64 * kRWaves, 0, s>>>(d_off, d_eps, total, x, m, G, rcnt, rlist, a);
  else
    ens_rescue_kernel<false><<<dim3(ncl, kRSplit), 64 * kRWaves, 0, s>>>(d_off, d_eps, total, x, m, G, rcnt, rlist, a);
  NB_LAUNCH_CHECK("ens_rescue_kernel");
  return NBODY_OK;
}

int run_batched_stream(int32_t ncl, const int64_t* off, const double* eps, double* x, double* v, double* a,
                       const double* m, double dt, int64_t nsteps, double G, int precision, bool excl,
                       bool acc_valid, int bitem, bool per_step, bool rescue, hipStream_t s) {
  const int device = current_device();
  // automatic item size: items of 64 particles evaluated by one wave each (faster than
  // items of 1024 on every measured layout but one, 64 x 4096, where it is 2 % slower)
  if (bitem == 0 || per_step) bitem = 64;
  std::lock_guard<std::mutex> lk(g_splan_mu);
  SPlan* p = find_splan(ncl, off, eps, precision, device, bitem);
  if (!p) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return set_error(NBODY_EINVAL, "batched: the plan for this layout must be built by one call outside stream capture");
    int st;
    if (bitem == 64) {
      if (precision == NBODY_FP64) st = build_wplan<NBODY_FP64>(ncl, off, eps, precision, device, &p);
      else if (precision == NBODY_FP32C) st = build_wplan<NBODY_FP32C>(ncl, off, eps, precision, device, &p);
      else st = build_wplan<NBODY_FP32>(ncl, off, eps, precision, device, &p);
    } else if (precision == NBODY_FP64) {
      st = build_splan<NBODY_FP64>(ncl, off, eps, precision, device, bitem, &p);
    } else if (precision == NBODY_FP32C) {
      st = build_splan<NBODY_FP32C>(ncl, off, eps, precision, device, bitem, &p);
    } else {
      st = build_splan<NBODY_FP32>(ncl, off, eps, precision, device, bitem, &p);
    }
    if (st) return st;
    g_splans.push_back(p);
  }
  if (per_step) {
    if (precision == NBODY_FP64)
      return launch_wsteps<NBODY_FP64>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, false, s);
    if (precision == NBODY_FP32C)
      return launch_wsteps<NBODY_FP32C>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, rescue, s);
    return launch_wsteps<NBODY_FP32>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, false, s);
  }
  if (precision == NBODY_FP64) return launch_splan<NBODY_FP64>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, s);
  if (precision == NBODY_FP32C) return launch_splan<NBODY_FP32C>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, s);
  return launch_splan<NBODY_FP32>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, s);
}

void release_stream_plans() {
  std::lock_guard<std::mutex> lk(g_splan_mu);
  for (SPlan* p : g_splans) free_splan(p);
  g_splans.clear();
}

}  // namespace nb
