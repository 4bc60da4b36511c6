// Persistent ensemble integrator: many independent softened systems of uneven
// size advanced for all KDK steps inside ONE kernel launch.
//
// Work is a list of items per workgroup (one workgroup per CU; 1024 lanes for
// the FP32 pair modes, 512 for FP64).  An item is a whole system, or one of P
// equal i-ranges of a system too costly for one CU (the plan splits the
// largest systems so that no CU carries much more than the average load).
// Pair arithmetic is that of the single-system kernel (FP32C: rounded-position
// pairs with the float-float near-field repair).  For every item and step:
//   1. kick-drift of the owned FP64 state (closing half-kick of the previous
//      step and opening half-kick of this one, rounded separately as in
//      nbody_step); the new positions go straight into LDS as pair records;
//   2. a split item also publishes its records in a global exchange buffer,
//      signals its step after an agent-scope release fence, waits (bounded)
//      for the other parts' signals, acquires and copies their records into
//      LDS;
//   3. every lane evaluates its i-particles against all records of the system
//      in LDS with the same pair arithmetic and compensated folds as the
//      single-system kernel; small systems, which cannot fill the lanes,
//      split their j-range over lane groups and combine the groups' (hi, lo)
//      sums through LDS in group order;
// then a final closing half-kick.  Deadlock freedom: every workgroup holds at
// most one split item and processes it first, all workgroups are resident
// (grid <= CUs, one workgroup per CU), and every wait is bounded; on a timeout
// the item's state is set to NaN and the workgroup moves on.
#include <cmath>
#include <map>
#include <mutex>
#include <queue>
#include <vector>

#include "pair_math.h"

namespace nb {
namespace {

template <int MODE> constexpr int ens_block() { return MODE == kFP64 ? 512 : 1024; }
template <int MODE> constexpr int ens_max_ipl() { return MODE == kFP64 ? 8 : 4; }
constexpr int kMaxSys = 4096;            // particles per system
constexpr int kPass = 4;                 // most i-particles evaluated together in one pass over j
constexpr size_t kLdsLimit = 160 * 1024;
// wall-clock bound of one wait for a partner flag, in ticks of the 100 MHz
// real-time counter (10 s; a round of LDS-resident systems takes milliseconds)
constexpr uint64_t kWaitTicks = 1000000000ull;

template <int MODE> struct Part { Real<MODE> hx, lx, hy, ly, hz, lz; };

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) / 16 * 16; }

// Lane mapping of an item: ni i-particles of a system of nc particles.
struct Map { int ipl, js; };

__host__ __device__ inline int map_gsz(int ni, int ipl) { return ((ni + ipl - 1) / ipl + 63) / 64 * 64; }

template <int MODE>
size_t lds_bytes(int nc, int ni, Map mp) {
  size_t b = align16((size_t)nc * sizeof(JRec<MODE>));
  if (mp.js > 1) b += (size_t)(mp.js - 1) * mp.ipl * map_gsz(ni, mp.ipl) * sizeof(Part<MODE>);
  return b;
}

// Chooses (ipl, js) minimising the per-lane pair count; returns the cost in
// pair-iterations per lane per step (plus a fixed per-step overhead).
template <int MODE>
bool choose_map(int nc, int ni, Map* out, double* cost) {
  constexpr int block = ens_block<MODE>();
  bool found = false;
  double best = 0;
  for (int ipl = 1; ipl <= ens_max_ipl<MODE>(); ++ipl) {
    const int gsz = map_gsz(ni, ipl);
    if (gsz > block) continue;
    for (int js = 1; js * gsz <= block && js <= 16 && (js == 1 || ipl <= kPass); js *= 2) {
      Map mp{ipl, js};
      if (lds_bytes<MODE>(nc, ni, mp) > kLdsLimit) continue;
      const double c = (double)ipl * ((nc + js - 1) / js) + 48.0 + (js > 1 ? 16.0 * js : 0.0);
      if (!found || c < best) { best = c; *out = mp; found = true; }
    }
  }
  *cost = best;
  return found;
}

// Device description of one work item.
struct Item {
  int sys;      // system index
  int part;     // part index within the system
  int nparts;   // 1 = whole system
  int map;      // ipl | js << 8
};

struct SysView {
  int nc, ni, i0, ipl, js, gsz, g, l, j0, j1;
  int64_t T;
};

// Accelerations of the item's i-particles (i0 + l + k*gsz, k = kb .. kb+IPL-1)
// from all records of the system in LDS.  FP32C uses the near-field repair of
// the single-system kernel: pairs from FP32-rounded positions, and a block of
// kFold j's holding a pair closer than the lane's repair radius is redone with
// float-float displacements for those pairs.
template <int MODE, int IPL, bool EXCL>
__device__ void system_force(const SysView& sv, int kb, const JRec<MODE>* __restrict__ rec,
                             Part<MODE>* __restrict__ part, double eps, double G,
                             double* __restrict__ A) {
  using R = Real<MODE>;
  constexpr bool kNear = MODE == kFP32C;
  const R e2 = (R)(eps * eps);
  IPos<MODE> pi[IPL];
  int ii[IPL];
  R rc2[IPL];
  R hx[IPL], hy[IPL], hz[IPL], lx[IPL], ly[IPL], lz[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    const int il = sv.l + (kb + k) * sv.gsz;
    const int i = sv.i0 + (il < sv.ni ? il : sv.ni - 1);
    ii[k] = il < sv.ni ? i : -1;
    pi[k].from(rec[i]);
    if constexpr (kNear) rc2[k] = near_rc2(pi[k].hx, pi[k].hy, pi[k].hz, eps, sv.nc);
    hx[k] = hy[k] = hz[k] = lx[k] = ly[k] = lz[k] = R(0);
  }
  for (int f = sv.j0; f < sv.j1; f += kFold) {
    const int fe = min(sv.j1, f + kFold);
    R px[IPL], py[IPL], pz[IPL], r2min[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      px[k] = py[k] = pz[k] = R(0);
      r2min[k] = R(3.0e38f);
    }
#pragma unroll 2
    for (int j = f; j < fe; ++j) {
      const JRec<MODE> r = rec[j];
      const R mj = jmass(r);
#pragma unroll
      for (int k = 0; k < IPL; ++k) {
        R dx, dy, dz;
        if constexpr (kNear) disp_hi(r, pi[k], dx, dy, dz);
        else disp(r, pi[k], dx, dy, dz);
        R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
        R ri = rsq(r2);
        R s = (mj * ri) * (ri * ri);
        if constexpr (EXCL) s = (j == ii[k]) ? R(0) : s;
        px[k] = fma(s, dx, px[k]);
        py[k] = fma(s, dy, py[k]);
        pz[k] = fma(s, dz, pz[k]);
        if constexpr (kNear) r2min[k] = fminf(r2min[k], r2);
      }
    }
    if constexpr (kNear) {
#pragma unroll
      for (int k = 0; k < IPL; ++k) {
        // the lane's own pair (zero displacement) always sets r2min = eps^2:
        // in the block holding it, rescan for a close pair other than that one
        bool close = r2min[k] < rc2[k];
        if (close && ii[k] >= f && ii[k] < fe) {
          close = false;
          for (int j = f; j < fe; ++j) {
            R dx, dy, dz;
            disp_hi(rec[j], pi[k], dx, dy, dz);
            const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
            close = close || (r2 < rc2[k] && j != ii[k]);
          }
        }
        if (close) {
          R qx = 0, qy = 0, qz = 0;
          for (int j = f; j < fe; ++j) {
            const JRec<MODE> r = rec[j];
            R dx, dy, dz;
            disp_hi(r, pi[k], dx, dy, dz);
            R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
            if (r2 < rc2[k]) {
              disp(r, pi[k], dx, dy, dz);
              r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
            }
            R ri = rsq(r2);
            R s = (jmass(r) * ri) * (ri * ri);
            if constexpr (EXCL) s = (j == ii[k]) ? R(0) : s;
            qx = fma(s, dx, qx);
            qy = fma(s, dy, qy);
            qz = fma(s, dz, qz);
          }
          px[k] = qx;
          py[k] = qy;
          pz[k] = qz;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      fold(hx[k], lx[k], px[k]);
      fold(hy[k], ly[k], py[k]);
      fold(hz[k], lz[k], pz[k]);
    }
  }
  if (sv.js > 1) {
    if (sv.g > 0 && sv.g < sv.js) {
#pragma unroll
      for (int k = 0; k < IPL; ++k)
        part[((size_t)(sv.g - 1) * IPL + k) * sv.gsz + sv.l] = Part<MODE>{hx[k], lx[k], hy[k], ly[k], hz[k], lz[k]};
    }
    __syncthreads();
    if (sv.g == 0) {
      for (int gg = 1; gg < sv.js; ++gg) {
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          const Part<MODE> q = part[((size_t)(gg - 1) * IPL + k) * sv.gsz + sv.l];
          fold(hx[k], lx[k], q.hx); lx[k] += q.lx;
          fold(hy[k], ly[k], q.hy); ly[k] += q.ly;
          fold(hz[k], lz[k], q.hz); lz[k] += q.lz;
        }
      }
    }
  }
  if (sv.g == 0) {
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int i = ii[k];
      if (i >= 0) {
        A[i] = G * ((double)hx[k] + (double)lx[k]);
        A[sv.T + i] = G * ((double)hy[k] + (double)ly[k]);
        A[2 * sv.T + i] = G * ((double)hz[k] + (double)lz[k]);
      }
    }
  }
}

template <int MODE>
__device__ __forceinline__ void system_force_pass(const SysView& sv, int kb, int cnt, const JRec<MODE>* rec,
                                                  Part<MODE>* part, double eps, double G, int excl, double* A) {
  // the self-pair mask costs two instructions per pair: compiled in only for
  // eps = 0, where the zero-displacement self pair would give 0 * inf
  if (excl) {
    switch (cnt) {
      case 1: system_force<MODE, 1, true>(sv, kb, rec, part, eps, G, A); break;
      case 2: system_force<MODE, 2, true>(sv, kb, rec, part, eps, G, A); break;
      case 3: system_force<MODE, 3, true>(sv, kb, rec, part, eps, G, A); break;
      default: system_force<MODE, 4, true>(sv, kb, rec, part, eps, G, A); break;
    }
  } else {
    switch (cnt) {
      case 1: system_force<MODE, 1, false>(sv, kb, rec, part, eps, G, A); break;
      case 2: system_force<MODE, 2, false>(sv, kb, rec, part, eps, G, A); break;
      case 3: system_force<MODE, 3, false>(sv, kb, rec, part, eps, G, A); break;
      default: system_force<MODE, 4, false>(sv, kb, rec, part, eps, G, A); break;
    }
  }
}

template <int MODE>
__device__ __forceinline__ void system_force_all(const SysView& sv, int pass, const JRec<MODE>* rec,
                                                 Part<MODE>* part, double eps, double G, int excl, double* A) {
  // with a j-split (js > 1) all of the lane's i-particles go in one pass, as
  // the LDS reduction of the groups' partial sums expects
  const int w = sv.js > 1 ? kPass : pass;
  for (int kb = 0; kb < sv.ipl; kb += w) system_force_pass<MODE>(sv, kb, min(w, sv.ipl - kb), rec, part, eps, G, excl, A);
}

// Publishes this part's records (already in LDS), signals round r, waits for
// the other parts' round r and copies their records into LDS.  Returns false
// (for the whole workgroup) if a partner did not arrive in time.
template <int MODE>
__device__ bool exchange(const SysView& sv, const Item& it, int64_t o, JRec<MODE>* rec,
                         JRec<MODE>* __restrict__ xrec, int* __restrict__ flags, int flag_base, int r,
                         int* lds_ok) {
  const int t = threadIdx.x;
  JRec<MODE>* xb = xrec + (size_t)(r & 1) * sv.T + o;
  for (int i = sv.i0 + t; i < sv.i0 + sv.ni; i += blockDim.x) xb[i] = rec[i];
  // Agent-scope fences write back / invalidate a whole XCD's L2 and are
  // serialised there, so one lane issues them for the workgroup: every wave
  // first waits for its own stores, then after the barrier lane 0 releases,
  // signals, polls the partners with relaxed loads and acquires once.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (t == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(flags + flag_base + it.part, r + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    for (int p = 0; p < it.nparts && ok; ++p) {
      if (p == it.part) continue;
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      while (__hip_atomic_load(flags + flag_base + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < r + 1) {
        if (__builtin_amdgcn_s_memrealtime() - t0 > kWaitTicks) { ok = 0; break; }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *lds_ok = ok;
  }
  __syncthreads();
  const bool ok = *lds_ok != 0;
  if (ok) {
    for (int j = t; j < sv.nc; j += blockDim.x)
      if (j < sv.i0 || j >= sv.i0 + sv.ni) rec[j] = xb[j];
  }
  __syncthreads();
  return ok;
}

// One launch integrates every item of the plan for nsteps KDK steps.  The FP64
// state of particle i is read and written in global memory only by the lane
// that owns it (group 0, lane (i - i0) % gsz of the item holding i).
template <int MODE>
__global__ __launch_bounds__(ens_block<MODE>()) void ensemble_kernel(
    const int64_t* __restrict__ off, const double* __restrict__ epsv, const Item* __restrict__ items,
    const int* __restrict__ flag_base, const int* __restrict__ wg_off, const int* __restrict__ wg_list,
    double* __restrict__ x, double* __restrict__ v, double* __restrict__ a, const double* __restrict__ m,
    JRec<MODE>* __restrict__ xrec, int* __restrict__ flags, int64_t total, double dt, int64_t nsteps, double G,
    int acc_valid, int excl, int pass) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int lds_ok;
  JRec<MODE>* rec = reinterpret_cast<JRec<MODE>*>(smem);
  const int t = threadIdx.x;
  const double h = 0.5 * dt;

  for (int q = wg_off[blockIdx.x]; q < wg_off[blockIdx.x + 1]; ++q) {
    const Item it = items[wg_list[q]];
    const int64_t o = off[it.sys];
    SysView sv;
    sv.nc = (int)(off[it.sys + 1] - o);
    if (sv.nc <= 0) continue;
    const int np = (sv.nc + it.nparts - 1) / it.nparts;
    sv.i0 = min(sv.nc, it.part * np);
    sv.ni = min(sv.nc, sv.i0 + np) - sv.i0;
    if (sv.ni <= 0) continue;
    sv.T = total;
    sv.ipl = it.map & 0xff;
    sv.js = it.map >> 8;
    sv.gsz = map_gsz(sv.ni, sv.ipl);
    sv.g = t / sv.gsz;
    sv.l = t - sv.g * sv.gsz;
    const int jc = (sv.nc + sv.js - 1) / sv.js;
    sv.j0 = sv.g < sv.js ? min(sv.nc, sv.g * jc) : sv.nc;
    sv.j1 = sv.g < sv.js ? min(sv.nc, sv.j0 + jc) : sv.nc;
    const double eps = epsv[it.sys];
    Part<MODE>* part = reinterpret_cast<Part<MODE>*>(smem + align16((size_t)sv.nc * sizeof(JRec<MODE>)));
    double* X = x + o;
    double* V = v + o;
    double* A = a + o;
    const double* M = m + o;
    const bool owner = sv.g == 0;
    const bool split = it.nparts > 1;
    const int fb = split ? flag_base[it.sys] : 0;
    int round = 0;
    bool ok = true;

    if (!acc_valid) {
      if (owner)
        for (int k = 0; k < sv.ipl; ++k) {
          const int il = sv.l + k * sv.gsz;
          if (il < sv.ni) {
            const int i = sv.i0 + il;
            rec[i] = JRec<MODE>::make(X[i], X[total + i], X[2 * total + i], M[i]);
          }
        }
      __syncthreads();
      if (split) ok = exchange<MODE>(sv, it, o, rec, xrec, flags, fb, round++, &lds_ok);
      if (ok) system_force_all<MODE>(sv, pass, rec, part, eps, G, excl, A);
      __syncthreads();
    }
    for (int64_t s = 0; s < nsteps && ok; ++s) {
      const int nk = s == 0 ? 1 : 2;
      if (owner)
        for (int k = 0; k < sv.ipl; ++k) {
          const int il = sv.l + k * sv.gsz;
          if (il < sv.ni) {
            const int i = sv.i0 + il;
            double xn[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const int64_t e = d * total + i;
              double ve = V[e];
              const double ae = A[e];
              for (int kk = 0; kk < nk; ++kk) ve = fma(h, ae, ve);
              V[e] = ve;
              xn[d] = fma(dt, ve, X[e]);
              X[e] = xn[d];
            }
            rec[i] = JRec<MODE>::make(xn[0], xn[1], xn[2], M[i]);
          }
        }
      __syncthreads();
      if (split) ok = exchange<MODE>(sv, it, o, rec, xrec, flags, fb, round++, &lds_ok);
      if (ok) system_force_all<MODE>(sv, pass, rec, part, eps, G, excl, A);
      __syncthreads();
    }
    if (owner)
      for (int k = 0; k < sv.ipl; ++k) {
        const int il = sv.l + k * sv.gsz;
        if (il < sv.ni) {
          const int i = sv.i0 + il;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int64_t e = d * total + i;
            if (!ok) {
              X[e] = NAN;
              V[e] = NAN;
              A[e] = NAN;
            } else if (nsteps > 0) {
              V[e] = fma(h, A[e], V[e]);
            }
          }
        }
      }
    __syncthreads();
  }
}

__global__ void zero_flags_kernel(int* flags, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) flags[i] = 0;
}

// ------------------------------------------------------------------ plans
struct Plan {
  std::vector<int64_t> off;
  std::vector<double> eps;
  bool allow_split = true;
  int precision = 0;
  int device = 0;
  int nwg = 0;
  int nflags = 0;
  size_t lds = 0;
  int64_t total = 0;
  int64_t* d_off = nullptr;
  double* d_eps = nullptr;
  Item* d_items = nullptr;
  int* d_flag_base = nullptr;
  int* d_wg_off = nullptr;
  int* d_wg_list = nullptr;
  void* d_xrec = nullptr;
  int* d_flags = nullptr;
};

std::mutex g_plan_mu;
std::vector<Plan*> g_plans;

void free_plan(Plan* p) {
  for (void* q : {(void*)p->d_off, (void*)p->d_eps, (void*)p->d_items, (void*)p->d_flag_base, (void*)p->d_wg_off,
                  (void*)p->d_wg_list, p->d_xrec, (void*)p->d_flags})
    if (q) (void)hipFree(q);
  delete p;
}

template <typename T>
bool upload(T** dst, const std::vector<T>& src) {
  const size_t bytes = sizeof(T) * std::max<size_t>(1, src.size());
  if (hipMalloc(dst, bytes) != hipSuccess) return false;
  return src.empty() || hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) == hipSuccess;
}

// Builds the work plan.  With splitting allowed, a system whose cost exceeds
// the per-CU average T is split into P = ceil(cost / T) <= 4 parts; the items
// are then assigned longest-processing-time first, each to the least loaded
// workgroup, except that a workgroup takes at most one split item, which goes
// first in its list (so that every part of a system runs concurrently).
template <int MODE>
int build_plan(int32_t ncl, const int64_t* off, const double* eps, int precision, int device, bool allow_split,
               Plan** out) {
  Plan* p = new Plan();
  p->off.assign(off, off + ncl + 1);
  p->eps.assign(eps, eps + ncl);
  p->precision = precision;
  p->device = device;
  p->allow_split = allow_split;
  p->total = off[ncl];
  std::vector<double> cost(ncl, 0.0);
  std::vector<Map> whole(ncl);
  size_t lds = 16;
  double sum = 0;
  for (int c = 0; c < ncl; ++c) {
    const int64_t nc = off[c + 1] - off[c];
    if (nc == 0) { whole[c] = Map{1, 1}; continue; }
    if (nc > kMaxSys || !choose_map<MODE>((int)nc, (int)nc, &whole[c], &cost[c])) {
      delete p;
      return set_error(NBODY_EUNSUPPORTED, "batched: system " + std::to_string(c) + " of " + std::to_string(nc) +
                                               " particles exceeds the persistent kernel's capacity (" +
                                               std::to_string(kMaxSys) + ")");
    }
    sum += cost[c];
    lds = std::max(lds, lds_bytes<MODE>((int)nc, (int)nc, whole[c]));
  }
  const int nwg = std::max(1, std::min<int>(ncl, cu_count(device)));
  const double avg = sum / nwg;
  std::vector<int> order(ncl);
  for (int c = 0; c < ncl; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int u, int w) { return cost[u] > cost[w]; });

  std::vector<Item> items;
  std::vector<double> icost;
  std::vector<int> flag_base(ncl, 0);
  int nflags = 0;
  for (int c : order) {
    const int nc = (int)(off[c + 1] - off[c]);
    int P = 1;
    if (allow_split && nwg > 1 && nc >= 512 && cost[c] > avg) P = std::min(4, (int)std::ceil(cost[c] / avg));
    if (P > 1 && nflags + P > nwg) P = 1;
    Map mp{1, 1};
    double pc = 0;
    if (P > 1 && !choose_map<MODE>(nc, (nc + P - 1) / P, &mp, &pc)) P = 1;
    if (P == 1) {
      items.push_back(Item{c, 0, 1, whole[c].ipl | (whole[c].js << 8)});
      icost.push_back(cost[c]);
      continue;
    }
    flag_base[c] = nflags;
    nflags += P;
    for (int q = 0; q < P; ++q) {
      items.push_back(Item{c, q, P, mp.ipl | (mp.js << 8)});
      icost.push_back(pc + 32.0);  // the exchange adds a little per step
    }
    lds = std::max(lds, lds_bytes<MODE>(nc, (nc + P - 1) / P, mp));
  }
  std::vector<int> korder(items.size());
  for (size_t k = 0; k < items.size(); ++k) korder[k] = (int)k;
  std::stable_sort(korder.begin(), korder.end(), [&](int u, int w) { return icost[u] > icost[w]; });
  std::vector<std::vector<int>> lists(nwg);
  std::vector<double> load(nwg, 0.0);
  std::vector<char> has_split(nwg, 0);
  for (int k : korder) {
    const bool sp = items[k].nparts > 1;
    int best = -1;
    for (int w = 0; w < nwg; ++w) {
      if (sp && has_split[w]) continue;
      if (best < 0 || load[w] < load[best]) best = w;
    }
    if (sp) {
      has_split[best] = 1;
      lists[best].insert(lists[best].begin(), k);
    } else {
      lists[best].push_back(k);
    }
    load[best] += icost[k];
  }
  std::vector<int> wg_off(nwg + 1, 0), wg_list;
  for (int w = 0; w < nwg; ++w) {
    wg_list.insert(wg_list.end(), lists[w].begin(), lists[w].end());
    wg_off[w + 1] = (int)wg_list.size();
  }
  p->nwg = nwg;
  p->lds = lds;
  p->nflags = nflags;
  std::vector<double> epsv(eps, eps + ncl);
  bool ok = upload(&p->d_off, p->off) && upload(&p->d_eps, epsv) && upload(&p->d_items, items) &&
            upload(&p->d_flag_base, flag_base) && upload(&p->d_wg_off, wg_off) && upload(&p->d_wg_list, wg_list);
  if (ok && nflags > 0) {
    ok = hipMalloc(&p->d_xrec, 2 * (size_t)p->total * sizeof(JRec<MODE>)) == hipSuccess &&
         hipMalloc(&p->d_flags, sizeof(int) * nflags) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    free_plan(p);
    return set_error(NBODY_ENOMEM, "batched: plan upload failed");
  }
  *out = p;
  return NBODY_OK;
}

Plan* find_plan(int32_t ncl, const int64_t* off, const double* eps, int precision, int device, bool allow_split) {
  for (Plan* p : g_plans) {
    if (p->device != device || p->precision != precision || (int)p->eps.size() != ncl ||
        p->allow_split != allow_split)
      continue;
    if (std::equal(p->off.begin(), p->off.end(), off) && std::equal(p->eps.begin(), p->eps.end(), eps)) return p;
  }
  return nullptr;
}

template <int MODE>
int launch_plan(const Plan* p, double* x, double* v, double* a, const double* m, double dt, int64_t nsteps,
                double G, bool acc_valid, bool excl, int bpass, hipStream_t s) {
  const int pass = bpass > 0 ? bpass : kPass;
  NB_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&ensemble_kernel<MODE>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lds));
  if (p->nflags > 0) {
    zero_flags_kernel<<<1, 256, 0, s>>>(p->d_flags, p->nflags);
    NB_LAUNCH_CHECK("zero_flags_kernel");
  }
  ensemble_kernel<MODE><<<p->nwg, ens_block<MODE>(), p->lds, s>>>(
      p->d_off, p->d_eps, p->d_items, p->d_flag_base, p->d_wg_off, p->d_wg_list, x, v, a, m,
      static_cast<JRec<MODE>*>(p->d_xrec), p->d_flags, p->total, dt, nsteps, G, acc_valid ? 1 : 0, excl ? 1 : 0,
      pass);
  NB_LAUNCH_CHECK("ensemble_kernel");
  return NBODY_OK;
}

}  // namespace

int run_batched_stream(int32_t ncl, const int64_t* off, const double* eps, double* x, double* v, double* a,
                       const double* m, double dt, int64_t nsteps, double G, int precision, bool excl,
                       bool acc_valid, int bitem, bool per_step, bool rescue, hipStream_t s);

int run_batched_sym(int32_t ncl, const int64_t* off, const double* eps, double* x, double* v, double* a,
                    const double* m, double dt, int64_t nsteps, double G, int precision, bool excl, bool acc_valid,
                    bool rescue, hipStream_t s);

int run_batched(int32_t ncl, const int64_t* off, const double* eps, double* x, double* v, double* a,
                const double* m, double dt, int64_t nsteps, double G, int precision, bool excl, bool acc_valid,
                const BatchConfig& bc, hipStream_t s) {
  if (bc.mode == 4)
    return run_batched_sym(ncl, off, eps, x, v, a, m, dt, nsteps, G, precision, excl, acc_valid, bc.rescue != 0, s);
  if (bc.mode == 2 || bc.mode == 3)
    return run_batched_stream(ncl, off, eps, x, v, a, m, dt, nsteps, G, precision, excl, acc_valid, bc.item,
                              bc.mode == 3, bc.rescue != 0, s);
  const int device = current_device();
  const bool allow_split = bc.mode == 1;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  Plan* p = find_plan(ncl, off, eps, precision, device, allow_split);
  if (!p) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return set_error(NBODY_EINVAL, "batched: the plan for this layout must be built by one call outside stream capture");
    int st;
    if (precision == NBODY_FP64) st = build_plan<NBODY_FP64>(ncl, off, eps, precision, device, allow_split, &p);
    else if (precision == NBODY_FP32C) st = build_plan<NBODY_FP32C>(ncl, off, eps, precision, device, allow_split, &p);
    else st = build_plan<NBODY_FP32>(ncl, off, eps, precision, device, allow_split, &p);
    if (st) return st;
    g_plans.push_back(p);
  }
  if (precision == NBODY_FP64)
    return launch_plan<NBODY_FP64>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, bc.pass, s);
  if (precision == NBODY_FP32C)
    return launch_plan<NBODY_FP32C>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, bc.pass, s);
  return launch_plan<NBODY_FP32>(p, x, v, a, m, dt, nsteps, G, acc_valid, excl, bc.pass, s);
}

void release_batched_plans() {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  for (Plan* p : g_plans) free_plan(p);
  g_plans.clear();
}

}  // namespace nb
