// Persistent ensemble integrator: many independent softened systems of uneven
// size advanced for all KDK steps inside ONE kernel launch.
//
// Each 512-lane workgroup (8 waves, one workgroup per CU) owns whole systems
// from a host-built longest-processing-time plan and integrates each of them
// for every step before taking the next, so no communication between
// workgroups is ever needed.  Per step and system:
//   1. kick-drift of the FP64 state (closing half-kick of the previous step and
//      opening half-kick of this one, rounded separately as in nbody_step), and
//      the new positions written straight into LDS as pair records;
//   2. barrier; every lane evaluates its i-particles against the system's
//      records in LDS with the same pair arithmetic and compensated folds as
//      the single-system kernel;
//   3. small systems, which cannot fill 512 lanes with i-particles, split
//      their j-range over lane groups, and the partial (hi, lo) sums of the
//      groups are combined through LDS in group order;
// then a final closing half-kick.  The mapping of a system onto the lanes
// (i-particles per lane `ipl`, j-groups `js`) is chosen per system on the
// host to minimise its per-lane pair count.
#include <cmath>
#include <map>
#include <mutex>
#include <queue>
#include <vector>

#include "pair_math.h"

namespace nb {
namespace {

constexpr int kEnsBlock = 512;
constexpr int kMaxIpl = 8;   // i-particles per lane
constexpr int kPass = 4;     // i-particles evaluated together in one pass over j
constexpr size_t kLdsLimit = 160 * 1024;

template <int MODE> struct Part { Real<MODE> hx, lx, hy, ly, hz, lz; };

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) / 16 * 16; }

// Per-system lane mapping, packed as ipl | js << 8.
struct Map { int ipl, js; };

template <int MODE>
size_t lds_bytes(int nc, Map mp) {
  const int gsz = ((nc + mp.ipl - 1) / mp.ipl + 63) / 64 * 64;
  size_t b = align16((size_t)nc * sizeof(JRec<MODE>));
  if (mp.js > 1) b += (size_t)(mp.js - 1) * mp.ipl * gsz * sizeof(Part<MODE>);
  return b;
}

template <int MODE>
bool choose_map(int nc, Map* out, double* cost) {
  bool found = false;
  double best = 0;
  for (int ipl = 1; ipl <= kMaxIpl; ++ipl) {
    const int gsz = ((nc + ipl - 1) / ipl + 63) / 64 * 64;
    if (gsz > kEnsBlock) continue;
    for (int js = 1; js * gsz <= kEnsBlock && js <= 16 && (js == 1 || ipl <= kPass); js *= 2) {
      Map mp{ipl, js};
      if (lds_bytes<MODE>(nc, mp) > kLdsLimit) continue;
      // per-lane pair iterations plus a per-step overhead for the kick,
      // staging and barriers, in the same units
      const double c = (double)ipl * ((nc + js - 1) / js) + 48.0 + (js > 1 ? 16.0 * js : 0.0);
      if (!found || c < best) { best = c; *out = mp; found = true; }
    }
  }
  *cost = best;
  return found;
}

// Per-system view of the lane mapping, shared by the phases of one step.
struct SysView {
  int nc, ipl, js, gsz, g, l, j0, j1;
  int64_t T;
};

// Accelerations of one system from the records in LDS, for the lane's
// i-particles k = kb .. kb+IPL-1 (i = l + k*gsz).  Lanes of group 0 write a_i;
// other groups (only when js > 1, which implies kb == 0) hand their partial
// sums to group 0 through LDS.
template <int MODE, int IPL>
__device__ void system_force(const SysView& sv, int kb, const JRec<MODE>* __restrict__ rec,
                             Part<MODE>* __restrict__ part, Real<MODE> e2, double G, int excl,
                             double* __restrict__ A) {
  using R = Real<MODE>;
  IPos<MODE> pi[IPL];
  int ii[IPL];
  R hx[IPL], hy[IPL], hz[IPL], lx[IPL], ly[IPL], lz[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    const int i = sv.l + (kb + k) * sv.gsz;
    ii[k] = i;
    pi[k].from(rec[i < sv.nc ? i : sv.nc - 1]);
    hx[k] = hy[k] = hz[k] = lx[k] = ly[k] = lz[k] = R(0);
  }
  for (int f = sv.j0; f < sv.j1; f += kFold) {
    const int fe = min(sv.j1, f + kFold);
    R px[IPL], py[IPL], pz[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) px[k] = py[k] = pz[k] = R(0);
#pragma unroll 2
    for (int j = f; j < fe; ++j) {
      const JRec<MODE> r = rec[j];
      const R mj = jmass(r);
#pragma unroll
      for (int k = 0; k < IPL; ++k) {
        R dx, dy, dz;
        disp(r, pi[k], dx, dy, dz);
        R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
        R ri = rsq(r2);
        R s = (mj * ri) * (ri * ri);
        if (excl) s = (j == ii[k]) ? R(0) : s;
        px[k] = fma(s, dx, px[k]);
        py[k] = fma(s, dy, py[k]);
        pz[k] = fma(s, dz, pz[k]);
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
      if (i < sv.nc) {
        A[i] = G * ((double)hx[k] + (double)lx[k]);
        A[sv.T + i] = G * ((double)hy[k] + (double)ly[k]);
        A[2 * sv.T + i] = G * ((double)hz[k] + (double)lz[k]);
      }
    }
  }
}

template <int MODE>
__device__ __forceinline__ void system_force_pass(const SysView& sv, int kb, int cnt, const JRec<MODE>* rec,
                                                  Part<MODE>* part, Real<MODE> e2, double G, int excl, double* A) {
  switch (cnt) {
    case 1: system_force<MODE, 1>(sv, kb, rec, part, e2, G, excl, A); break;
    case 2: system_force<MODE, 2>(sv, kb, rec, part, e2, G, excl, A); break;
    case 3: system_force<MODE, 3>(sv, kb, rec, part, e2, G, excl, A); break;
    default: system_force<MODE, 4>(sv, kb, rec, part, e2, G, excl, A); break;
  }
}

// All of a lane's i-particles, in passes of at most kPass.
template <int MODE>
__device__ __forceinline__ void system_force_dispatch(const SysView& sv, const JRec<MODE>* rec, Part<MODE>* part,
                                                      Real<MODE> e2, double G, int excl, double* A) {
  for (int kb = 0; kb < sv.ipl; kb += kPass) system_force_pass<MODE>(sv, kb, min(kPass, sv.ipl - kb), rec, part, e2, G, excl, A);
}

// One launch integrates every system of the plan for nsteps KDK steps.
// Particle i of a system is read and written in global memory only by the
// lane that owns it (group 0, lane i % gsz), so the lanes of a workgroup
// exchange positions only through the LDS records.
template <int MODE>
__global__ __launch_bounds__(kEnsBlock) void ensemble_kernel(
    const int64_t* __restrict__ off, const double* __restrict__ epsv, const int* __restrict__ maps,
    const int* __restrict__ wg_off, const int* __restrict__ wg_list, double* __restrict__ x,
    double* __restrict__ v, double* __restrict__ a, const double* __restrict__ m, int64_t total, double dt,
    int64_t nsteps, double G, int acc_valid, int excl) {
  using R = Real<MODE>;
  extern __shared__ __align__(16) unsigned char smem[];
  JRec<MODE>* rec = reinterpret_cast<JRec<MODE>*>(smem);
  const int t = threadIdx.x;
  const double h = 0.5 * dt;

  for (int q = wg_off[blockIdx.x]; q < wg_off[blockIdx.x + 1]; ++q) {
    const int c = wg_list[q];
    const int64_t o = off[c];
    SysView sv;
    sv.nc = (int)(off[c + 1] - o);
    if (sv.nc <= 0) continue;
    sv.T = total;
    sv.ipl = maps[c] & 0xff;
    sv.js = maps[c] >> 8;
    sv.gsz = ((sv.nc + sv.ipl - 1) / sv.ipl + 63) / 64 * 64;
    sv.g = t / sv.gsz;
    sv.l = t - sv.g * sv.gsz;
    const int jc = (sv.nc + sv.js - 1) / sv.js;
    sv.j0 = sv.g < sv.js ? min(sv.nc, sv.g * jc) : sv.nc;
    sv.j1 = sv.g < sv.js ? min(sv.nc, sv.j0 + jc) : sv.nc;
    const R e2 = (R)(epsv[c] * epsv[c]);
    Part<MODE>* part = reinterpret_cast<Part<MODE>*>(smem + align16((size_t)sv.nc * sizeof(JRec<MODE>)));
    double* X = x + o;
    double* V = v + o;
    double* A = a + o;
    const double* M = m + o;
    const bool owner = sv.g == 0;

    if (!acc_valid) {
      if (owner)
        for (int k = 0; k < sv.ipl; ++k) {
          const int i = sv.l + k * sv.gsz;
          if (i < sv.nc) rec[i] = JRec<MODE>::make(X[i], X[total + i], X[2 * total + i], M[i]);
        }
      __syncthreads();
      system_force_dispatch<MODE>(sv, rec, part, e2, G, excl, A);
      __syncthreads();
    }
    for (int64_t s = 0; s < nsteps; ++s) {
      const int nk = s == 0 ? 1 : 2;
      if (owner)
        for (int k = 0; k < sv.ipl; ++k) {
          const int i = sv.l + k * sv.gsz;
          if (i < sv.nc) {
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
      system_force_dispatch<MODE>(sv, rec, part, e2, G, excl, A);
      __syncthreads();
    }
    if (nsteps > 0 && owner)
      for (int k = 0; k < sv.ipl; ++k) {
        const int i = sv.l + k * sv.gsz;
        if (i < sv.nc)
#pragma unroll
          for (int d = 0; d < 3; ++d) V[d * total + i] = fma(h, A[d * total + i], V[d * total + i]);
      }
  }
}

// ------------------------------------------------------------------ plans
struct Plan {
  std::vector<int64_t> off;
  std::vector<double> eps;
  int precision = 0;
  int device = 0;
  int nwg = 0;
  size_t lds = 0;
  int64_t* d_off = nullptr;
  double* d_eps = nullptr;
  int* d_maps = nullptr;
  int* d_wg_off = nullptr;
  int* d_wg_list = nullptr;
};

std::mutex g_plan_mu;
std::vector<Plan*> g_plans;

void free_plan(Plan* p) {
  if (p->d_off) (void)hipFree(p->d_off);
  if (p->d_eps) (void)hipFree(p->d_eps);
  if (p->d_maps) (void)hipFree(p->d_maps);
  if (p->d_wg_off) (void)hipFree(p->d_wg_off);
  if (p->d_wg_list) (void)hipFree(p->d_wg_list);
  delete p;
}

template <int MODE>
int build_plan(int32_t ncl, const int64_t* off, const double* eps, int precision, int device, Plan** out) {
  Plan* p = new Plan();
  p->off.assign(off, off + ncl + 1);
  p->eps.assign(eps, eps + ncl);
  p->precision = precision;
  p->device = device;
  std::vector<int> maps(ncl);
  std::vector<double> cost(ncl);
  size_t lds = 16;
  for (int c = 0; c < ncl; ++c) {
    const int64_t nc = off[c + 1] - off[c];
    if (nc == 0) { maps[c] = 1 | (1 << 8); cost[c] = 0; continue; }
    Map mp;
    if (nc > kEnsBlock * kMaxIpl || !choose_map<MODE>((int)nc, &mp, &cost[c])) {
      delete p;
      return set_error(NBODY_EUNSUPPORTED, "batched: system " + std::to_string(c) + " of " + std::to_string(nc) +
                                               " particles exceeds the persistent kernel's LDS capacity");
    }
    maps[c] = mp.ipl | (mp.js << 8);
    lds = std::max(lds, lds_bytes<MODE>((int)nc, mp));
  }
  // longest-processing-time assignment of systems to workgroups (one per CU)
  const int nwg = std::max(1, std::min<int>(ncl, cu_count(device)));
  std::vector<int> order(ncl);
  for (int c = 0; c < ncl; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int u, int w) { return cost[u] > cost[w]; });
  using Slot = std::pair<double, int>;
  std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
  for (int w = 0; w < nwg; ++w) heap.push({0.0, w});
  std::vector<std::vector<int>> lists(nwg);
  for (int c : order) {
    Slot s = heap.top();
    heap.pop();
    lists[s.second].push_back(c);
    heap.push({s.first + cost[c], s.second});
  }
  std::vector<int> wg_off(nwg + 1, 0), wg_list;
  wg_list.reserve(ncl);
  for (int w = 0; w < nwg; ++w) {
    wg_list.insert(wg_list.end(), lists[w].begin(), lists[w].end());
    wg_off[w + 1] = (int)wg_list.size();
  }
  p->nwg = nwg;
  p->lds = lds;
  bool ok = hipMalloc(&p->d_off, sizeof(int64_t) * (ncl + 1)) == hipSuccess &&
            hipMalloc(&p->d_eps, sizeof(double) * ncl) == hipSuccess &&
            hipMalloc(&p->d_maps, sizeof(int) * ncl) == hipSuccess &&
            hipMalloc(&p->d_wg_off, sizeof(int) * (nwg + 1)) == hipSuccess &&
            hipMalloc(&p->d_wg_list, sizeof(int) * std::max(1, ncl)) == hipSuccess;
  ok = ok && hipMemcpy(p->d_off, off, sizeof(int64_t) * (ncl + 1), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(p->d_eps, eps, sizeof(double) * ncl, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(p->d_maps, maps.data(), sizeof(int) * ncl, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(p->d_wg_off, wg_off.data(), sizeof(int) * (nwg + 1), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(p->d_wg_list, wg_list.data(), sizeof(int) * ncl, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_plan(p);
    return set_error(NBODY_ENOMEM, "batched: plan upload failed");
  }
  *out = p;
  return NBODY_OK;
}

Plan* find_plan(int32_t ncl, const int64_t* off, const double* eps, int precision, int device) {
  for (Plan* p : g_plans) {
    if (p->device != device || p->precision != precision || (int)p->eps.size() != ncl) continue;
    if (std::equal(p->off.begin(), p->off.end(), off) && std::equal(p->eps.begin(), p->eps.end(), eps)) return p;
  }
  return nullptr;
}

template <int MODE>
int launch_plan(const Plan* p, double* x, double* v, double* a, const double* m, int64_t total, double dt,
                int64_t nsteps, double G, bool acc_valid, bool excl, hipStream_t s) {
  NB_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&ensemble_kernel<MODE>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lds));
  ensemble_kernel<MODE><<<p->nwg, kEnsBlock, p->lds, s>>>(p->d_off, p->d_eps, p->d_maps, p->d_wg_off,
                                                          p->d_wg_list, x, v, a, m, total, dt, nsteps, G,
                                                          acc_valid ? 1 : 0, excl ? 1 : 0);
  NB_LAUNCH_CHECK("ensemble_kernel");
  return NBODY_OK;
}

}  // namespace

int run_batched(int32_t ncl, const int64_t* off, const double* eps, double* x, double* v, double* a,
                const double* m, double dt, int64_t nsteps, double G, int precision, bool excl, bool acc_valid,
                hipStream_t s) {
  const int device = current_device();
  std::lock_guard<std::mutex> lk(g_plan_mu);
  Plan* p = find_plan(ncl, off, eps, precision, device);
  if (!p) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return set_error(NBODY_EINVAL, "batched: the plan for this layout must be built by one call outside stream capture");
    int st;
    if (precision == NBODY_FP64) st = build_plan<NBODY_FP64>(ncl, off, eps, precision, device, &p);
    else if (precision == NBODY_FP32C) st = build_plan<NBODY_FP32C>(ncl, off, eps, precision, device, &p);
    else st = build_plan<NBODY_FP32>(ncl, off, eps, precision, device, &p);
    if (st) return st;
    g_plans.push_back(p);
  }
  const int64_t total = off[ncl];
  if (precision == NBODY_FP64)
    return launch_plan<NBODY_FP64>(p, x, v, a, m, total, dt, nsteps, G, acc_valid, excl, s);
  if (precision == NBODY_FP32C)
    return launch_plan<NBODY_FP32C>(p, x, v, a, m, total, dt, nsteps, G, acc_valid, excl, s);
  return launch_plan<NBODY_FP32>(p, x, v, a, m, total, dt, nsteps, G, acc_valid, excl, s);
}

void release_batched_plans() {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  for (Plan* p : g_plans) free_plan(p);
  g_plans.clear();
}

}  // namespace nb
