// O(N) kernels and drivers of libnbody_accel: the kick-drift-kick integrator,
// the fourth- and sixth-order Hermite predictors and correctors, the
// energy/momentum diagnostics and the checkpointed adjoint sweep.  All of this
// is FP64 and bound by HBM bandwidth; the all-pairs work lives in pairs.hip.
#include <mutex>

#include "common.h"

namespace nb {

namespace {

constexpr int kEw = 256;  // threads per block of the elementwise kernels

inline unsigned ew_blocks(int64_t cnt) { return (unsigned)((cnt + kEw - 1) / kEw); }

// v += h a (nkicks times, each rounded separately) then x += dt v.
// nkicks = 2 is the closing half-kick of one step followed by the opening
// half-kick of the next, so one call of S steps equals two calls of S1 + S2.
__global__ void kick_drift_kernel(int64_t n3, double* __restrict__ x, double* __restrict__ v,
                                  const double* __restrict__ a, double h, double dt, int nkicks) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n3) return;
  double ae = a[e];
  double ve = v[e];
  for (int k = 0; k < nkicks; ++k) ve = fma(h, ae, ve);
  v[e] = ve;
  x[e] = fma(dt, ve, x[e]);
}

__global__ void kick_kernel(int64_t n3, double* __restrict__ v, const double* __restrict__ a, double h) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n3) return;
  v[e] = fma(h, a[e], v[e]);
}

__global__ void copy_kernel(int64_t cnt, const double* __restrict__ src, double* __restrict__ dst) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) dst[e] = src[e];
}

__global__ void fill_kernel(int64_t cnt, double* __restrict__ dst, double val) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) dst[e] = val;
}

// Adjoint bookkeeping after one merged VJP at position index p:
//   lx += gxp;  gm += gmp;  if (drift) lv += dt * lx
__global__ void adjoint_update_kernel(int64_t n, double* __restrict__ lx, double* __restrict__ lv,
                                      double* __restrict__ gm, const double* __restrict__ gxp,
                                      const double* __restrict__ gmp, double dt, int drift) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * n) return;
  double l = lx[e] + gxp[e];
  lx[e] = l;
  if (drift) lv[e] = fma(dt, l, lv[e]);
  if (e < n) gm[e] += gmp[e];
}

// Hermite predictor: xp = x + v dt + a dt^2/2 + j dt^3/6, vp = v + a dt + j dt^2/2.
__global__ void hermite_predict_kernel(int64_t n3, const double* __restrict__ x, const double* __restrict__ v,
                                       const double* __restrict__ a, const double* __restrict__ jk, double dt,
                                       double* __restrict__ xp, double* __restrict__ vp) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n3) return;
  const double h2 = 0.5 * dt * dt, h3 = dt * dt * dt / 6.0;
  xp[e] = fma(jk[e], h3, fma(a[e], h2, fma(v[e], dt, x[e])));
  vp[e] = fma(jk[e], h2, fma(a[e], dt, v[e]));
}

// Hermite corrector, in place on (x, v, a, jk) from the evaluation (a1, j1):
//   v1 = v + (a0 + a1) dt/2 + (j0 - j1) dt^2/12
//   x1 = x + (v + v1) dt/2 + (a0 - a1) dt^2/12
__global__ void hermite_correct_kernel(int64_t n3, double* __restrict__ x, double* __restrict__ v,
                                       double* __restrict__ a, double* __restrict__ jk,
                                       const double* __restrict__ a1, const double* __restrict__ j1, double dt) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n3) return;
  const double h = 0.5 * dt, h12 = dt * dt / 12.0;
  const double a0 = a[e], j0 = jk[e], an = a1[e], jn = j1[e], v0 = v[e];
  const double v1 = fma(j0 - jn, h12, fma(a0 + an, h, v0));
  x[e] = fma(a0 - an, h12, fma(v0 + v1, h, x[e]));
  v[e] = v1;
  a[e] = an;
  jk[e] = jn;
}

// Sixth-order Hermite predictor (shared step h, crackle c from the previous step):
//   xp = x + v h + a h^2/2 + j h^3/6 + s h^4/24 + c h^5/120
//   vp = v + a h + j h^2/2 + s h^3/6 + c h^4/24
//   ap = a + j h + s h^2/2 + c h^3/6
__global__ void hermite6_predict_kernel(int64_t n3, const double* __restrict__ x, const double* __restrict__ v,
                                        const double* __restrict__ a, const double* __restrict__ jk,
                                        const double* __restrict__ sn, const double* __restrict__ cr, double h,
                                        double* __restrict__ xp, double* __restrict__ vp, double* __restrict__ ap) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n3) return;
  const double c2 = h * h / 2.0, c3 = h * h * h / 6.0, c4 = h * h * h * h / 24.0, c5 = h * h * h * h * h / 120.0;
  const double ae = a[e], je = jk[e], se = sn[e], ce = cr[e];
  xp[e] = fma(ce, c5, fma(se, c4, fma(je, c3, fma(ae, c2, fma(v[e], h, x[e])))));
  vp[e] = fma(ce, c4, fma(se, c3, fma(je, c2, fma(ae, h, v[e]))));
  ap[e] = fma(ce, c3, fma(se, c2, fma(je, h, ae)));
}

// Sixth-order Hermite corrector, in place on (x, v, a, jk, sn, cr) from the
// evaluation (a1, j1, s1) at the predicted state:
//   v1 = v + (a + a1) h/2 - (j1 - j) h^2/10 + (s + s1) h^3/120
//   x1 = x + (v + v1) h/2 - (a1 - a) h^2/10 + (j + j1) h^3/120
// and the crackle for the next predictor, the third derivative at t = h of the
// quintic through (a, j, s) at both ends: 60 A - 36 B + 9 C with
//   A = (a1 - a - j h - s h^2/2) / h^3,  B = (j1 - j - s h) / h^2,  C = (s1 - s) / h.
__global__ void hermite6_correct_kernel(int64_t n3, double* __restrict__ x, double* __restrict__ v,
                                        double* __restrict__ a, double* __restrict__ jk, double* __restrict__ sn,
                                        double* __restrict__ cr, const double* __restrict__ a1,
                                        const double* __restrict__ j1, const double* __restrict__ s1, double h) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n3) return;
  const double hh = h / 2.0, h10 = h * h / 10.0, h120 = h * h * h / 120.0;
  const double a0 = a[e], j0 = jk[e], s0 = sn[e], an = a1[e], jn = j1[e], snn = s1[e], v0 = v[e];
  const double v1 = fma(s0 + snn, h120, fma(-(jn - j0), h10, fma(a0 + an, hh, v0)));
  x[e] = fma(j0 + jn, h120, fma(-(an - a0), h10, fma(v0 + v1, hh, x[e])));
  v[e] = v1;
  const double A = (an - a0 - j0 * h - s0 * (h * h / 2.0)) / (h * h * h);
  const double B = (jn - j0 - s0 * h) / (h * h);
  const double C = (snn - s0) / h;
  cr[e] = 60.0 * A - 36.0 * B + 9.0 * C;
  a[e] = an;
  jk[e] = jn;
  sn[e] = snn;
}

// ---- deterministic reduction of the diagnostics -----------------------
// Each thread accumulates fixed-stride elements into 9 (hi, lo) TwoSum pairs;
// the block then combines lanes in a fixed tree order.
struct DD { double h, l; };

__device__ __forceinline__ void dd_add(DD& a, double x) {
  double s = a.h + x;
  double bp = s - a.h;
  a.l += (a.h - (s - bp)) + (x - bp);
  a.h = s;
}
__device__ __forceinline__ void dd_add(DD& a, const DD& b) {
  dd_add(a, b.h);
  a.l += b.l;
}

constexpr int kRedBlock = 256;
constexpr int kRedBlocks = 256;
constexpr int kQ = 9;  // K, W, (unused slot for E), Px, Py, Pz, Lx, Ly, Lz

__device__ void block_reduce_store(DD (&acc)[kQ], DD* __restrict__ dst) {
  __shared__ DD sh[kQ][kRedBlock];
  const int t = threadIdx.x;
  for (int q = 0; q < kQ; ++q) sh[q][t] = acc[q];
  __syncthreads();
  for (int w = kRedBlock / 2; w > 0; w >>= 1) {
    if (t < w)
      for (int q = 0; q < kQ; ++q) dd_add(sh[q][t], sh[q][t + w]);
    __syncthreads();
  }
  if (t == 0)
    for (int q = 0; q < kQ; ++q) dst[q] = sh[q][0];
}

__global__ __launch_bounds__(kRedBlock) void energy_partial_kernel(int64_t n, const double* __restrict__ x,
                                                                   const double* __restrict__ v,
                                                                   const double* __restrict__ m,
                                                                   const double* __restrict__ phi, double G,
                                                                   DD* __restrict__ part) {
  DD acc[kQ];
  for (int q = 0; q < kQ; ++q) acc[q] = DD{0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double mi = m[i];
    const double px = x[i], py = x[n + i], pz = x[2 * n + i];
    const double vx = v[i], vy = v[n + i], vz = v[2 * n + i];
    dd_add(acc[0], 0.5 * mi * (vx * vx + vy * vy + vz * vz));
    dd_add(acc[1], -0.5 * G * mi * phi[i]);
    dd_add(acc[3], mi * vx);
    dd_add(acc[4], mi * vy);
    dd_add(acc[5], mi * vz);
    dd_add(acc[6], mi * (py * vz - pz * vy));
    dd_add(acc[7], mi * (pz * vx - px * vz));
    dd_add(acc[8], mi * (px * vy - py * vx));
  }
  block_reduce_store(acc, part + (size_t)blockIdx.x * kQ);
}

__global__ __launch_bounds__(kRedBlock) void energy_final_kernel(int nparts, const DD* __restrict__ part,
                                                                 double* __restrict__ out9) {
  DD acc[kQ];
  for (int q = 0; q < kQ; ++q) acc[q] = DD{0.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += blockDim.x)
    for (int q = 0; q < kQ; ++q) dd_add(acc[q], part[(size_t)b * kQ + q]);
  __shared__ DD res[kQ];
  block_reduce_store(acc, res);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double K = res[0].h + res[0].l;
    const double W = res[1].h + res[1].l;
    out9[0] = K;
    out9[1] = W;
    out9[2] = K + W;
    for (int q = 3; q < kQ; ++q) out9[q] = res[q].h + res[q].l;
  }
}

__global__ void nonfinite_kernel(int64_t cnt, const double* __restrict__ p, int* __restrict__ flag) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt && !isfinite(p[e])) *flag = 1;  // benign race: every writer stores 1
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

}  // namespace

int launch_kick(int64_t n3, double* v, const double* a, double h, hipStream_t s) {
  if (n3 == 0) return NBODY_OK;
  kick_kernel<<<ew_blocks(n3), kEw, 0, s>>>(n3, v, a, h);
  NB_LAUNCH_CHECK("kick_kernel");
  return NBODY_OK;
}

int launch_kick_drift(int64_t n3, double* x, double* v, const double* a, double h, double dt, int nkicks,
                      hipStream_t s) {
  if (n3 == 0) return NBODY_OK;
  kick_drift_kernel<<<ew_blocks(n3), kEw, 0, s>>>(n3, x, v, a, h, dt, nkicks);
  NB_LAUNCH_CHECK("kick_drift_kernel");
  return NBODY_OK;
}

int launch_copy(int64_t cnt, const double* src, double* dst, hipStream_t s) {
  if (cnt == 0) return NBODY_OK;
  copy_kernel<<<ew_blocks(cnt), kEw, 0, s>>>(cnt, src, dst);
  NB_LAUNCH_CHECK("copy_kernel");
  return NBODY_OK;
}

int launch_fill(int64_t cnt, double* dst, double val, hipStream_t s) {
  if (cnt == 0) return NBODY_OK;
  fill_kernel<<<ew_blocks(cnt), kEw, 0, s>>>(cnt, dst, val);
  NB_LAUNCH_CHECK("fill_kernel");
  return NBODY_OK;
}

int launch_energy(int64_t n, const double* x, const double* v, const double* m, double G, double eps,
                  double* out9, hipStream_t s) {
  int st = NBODY_OK;
  const size_t part_bytes = sizeof(DD) * kQ * kRedBlocks;
  char* ws = static_cast<char*>(workspace(current_device(), 1, part_bytes + sizeof(double) * (size_t)(n > 0 ? n : 1), &st));
  if (!ws) return st;
  DD* part = reinterpret_cast<DD*>(ws);
  double* phi = reinterpret_cast<double*>(ws + part_bytes);
  if (n > 0) {
    const int64_t iblocks = (n + kBlock - 1) / kBlock;
    const int64_t want = 4LL * cu_count(current_device());
    int split = (int)std::min<int64_t>(64, std::max<int64_t>(1, (want + iblocks - 1) / iblocks));
    st = launch_potential(n, x, m, eps, 1.0, phi, split, s);
    if (st) return st;
  }
  energy_partial_kernel<<<kRedBlocks, kRedBlock, 0, s>>>(n, x, v, m, phi, G, part);
  NB_LAUNCH_CHECK("energy_partial_kernel");
  energy_final_kernel<<<1, kRedBlock, 0, s>>>(kRedBlocks, part, out9);
  NB_LAUNCH_CHECK("energy_final_kernel");
  return NBODY_OK;
}

int check_finite(const double* p, int64_t cnt, hipStream_t s, bool* all_finite) {
  int st = NBODY_OK;
  int* flag = static_cast<int*>(workspace(current_device(), 3, sizeof(int), &st));
  if (!flag) return st;
  zero_int_kernel<<<1, 1, 0, s>>>(flag);
  NB_LAUNCH_CHECK("zero_int_kernel");
  if (cnt > 0) {
    nonfinite_kernel<<<ew_blocks(cnt), kEw, 0, s>>>(cnt, p, flag);
    NB_LAUNCH_CHECK("nonfinite_kernel");
  }
  int h = 0;
  NB_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  NB_HIP(hipStreamSynchronize(s));
  *all_finite = (h == 0);
  return NBODY_OK;
}

int run_kdk(int64_t n, double* x, double* v, double* a, const double* m, double dt, int64_t nsteps,
            double G, double eps, int precision, bool excl, bool acc_valid, const PairConfig& cfg,
            hipStream_t s, double* traj) {
  const int64_t n3 = 3 * n;
  const double h = 0.5 * dt;
  int st;
  if (!acc_valid) {
    st = launch_accel(n, x, m, a, G, eps, precision, excl, cfg, s);
    if (st) return st;
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    st = launch_kick_drift(n3, x, v, a, h, dt, k == 0 ? 1 : 2, s);
    if (st) return st;
    st = launch_accel(n, x, m, a, G, eps, precision, excl, cfg, s);
    if (st) return st;
    if (traj) {
      st = launch_copy(n3, x, traj + (size_t)(k + 1) * n3, s);
      if (st) return st;
    }
  }
  if (nsteps > 0) return launch_kick(n3, v, a, h, s);
  return NBODY_OK;
}

int run_hermite(int64_t n, double* x, double* v, double* a, double* jk, const double* m, double dt, int64_t nsteps,
                double G, double eps, int precision, bool excl, bool acc_valid, const PairConfig& cfg,
                hipStream_t s) {
  const int64_t n3 = 3 * n;
  int st = NBODY_OK;
  if (!acc_valid && (st = launch_accel_jerk(n, x, v, m, a, jk, G, eps, precision, excl, cfg, s))) return st;
  if (nsteps == 0) return NBODY_OK;
  double* ws = static_cast<double*>(workspace(current_device(), 1, sizeof(double) * 4 * (size_t)n3, &st));
  if (!ws) return st;
  double* xp = ws;
  double* vp = xp + n3;
  double* a1 = vp + n3;
  double* j1 = a1 + n3;
  for (int64_t k = 0; k < nsteps; ++k) {
    hermite_predict_kernel<<<ew_blocks(n3), kEw, 0, s>>>(n3, x, v, a, jk, dt, xp, vp);
    NB_LAUNCH_CHECK("hermite_predict_kernel");
    if ((st = launch_accel_jerk(n, xp, vp, m, a1, j1, G, eps, precision, excl, cfg, s))) return st;
    hermite_correct_kernel<<<ew_blocks(n3), kEw, 0, s>>>(n3, x, v, a, jk, a1, j1, dt);
    NB_LAUNCH_CHECK("hermite_correct_kernel");
  }
  return NBODY_OK;
}

// Start: a, j at (x, v) by Algorithm 3, then a, j, s at (x, v, a) and c = 0.
int run_hermite6(int64_t n, double* x, double* v, double* a, double* jk, double* sn, double* cr, const double* m,
                 double dt, int64_t nsteps, double G, double eps, int precision, bool excl, bool acc_valid,
                 const PairConfig& cfg, hipStream_t s) {
  const int64_t n3 = 3 * n;
  int st = NBODY_OK;
  double* ws = static_cast<double*>(workspace(current_device(), 1, sizeof(double) * 6 * (size_t)n3, &st));
  if (!ws) return st;
  double* xp = ws;
  double* vp = xp + n3;
  double* ap = vp + n3;
  double* a1 = ap + n3;
  double* j1 = a1 + n3;
  double* s1 = j1 + n3;
  if (!acc_valid) {
    if ((st = launch_accel_jerk(n, x, v, m, a1, j1, G, eps, precision, excl, cfg, s))) return st;
    if ((st = launch_accel_jerk_snap(n, x, v, a1, m, a, jk, sn, G, eps, precision, excl, cfg, s))) return st;
    if ((st = launch_fill(n3, cr, 0.0, s))) return st;
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    hermite6_predict_kernel<<<ew_blocks(n3), kEw, 0, s>>>(n3, x, v, a, jk, sn, cr, dt, xp, vp, ap);
    NB_LAUNCH_CHECK("hermite6_predict_kernel");
    if ((st = launch_accel_jerk_snap(n, xp, vp, ap, m, a1, j1, s1, G, eps, precision, excl, cfg, s))) return st;
    hermite6_correct_kernel<<<ew_blocks(n3), kEw, 0, s>>>(n3, x, v, a, jk, sn, cr, a1, j1, s1, dt);
    NB_LAUNCH_CHECK("hermite6_correct_kernel");
  }
  return NBODY_OK;
}

namespace {

// The adjoint sweep's second stream per device (default priority, created on
// first use outside stream capture, kept until nbody_finalize) and its events:
// fork/join with the caller's stream, and per trajectory buffer b the end of
// its recompute (done[b]) and the end of the adjoint steps that read it
// (freed[b]).
struct SweepStream {
  hipStream_t r = nullptr;
  hipEvent_t fork = nullptr, done[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
};
constexpr int kSweepDev = 64;
std::mutex g_sweep_mu;
SweepStream g_sweep[kSweepDev];

void destroy_sweep(SweepStream& S) {
  for (hipEvent_t* e : {&S.fork, &S.done[0], &S.done[1], &S.freed[0], &S.freed[1]})
    if (*e) {
      (void)hipEventDestroy(*e);
      *e = nullptr;
    }
  if (S.r) (void)hipStreamDestroy(S.r);
  S.r = nullptr;
}

// The current device's sweep stream with lk locked for the caller's whole
// sweep, or nullptr (lk unlocked) where there is none and none can be made
// (s capturing before the first use, or a HIP failure): the sweep then runs
// on s alone.
SweepStream* acquire_sweep_stream(hipStream_t s, std::unique_lock<std::mutex>& lk) {
  const int dev = current_device();
  if (dev < 0 || dev >= kSweepDev) return nullptr;
  lk = std::unique_lock<std::mutex>(g_sweep_mu);
  SweepStream& S = g_sweep[dev];
  if (S.r) return &S;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  bool ok = hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone &&
            hipStreamCreateWithFlags(&S.r, hipStreamNonBlocking) == hipSuccess;
  for (hipEvent_t* e : {&S.fork, &S.done[0], &S.done[1], &S.freed[0], &S.freed[1]})
    ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    destroy_sweep(S);
    lk.unlock();
    return nullptr;
  }
  return &S;
}

// Largest system whose sweep overlaps the recompute with the adjoint steps:
// below it one all-pairs launch leaves much of the GPU idle (at N = 16384 an
// FP32C force and a VJP take 0.13 and 0.21 ms alone, 0.26 ms side by side).
constexpr int64_t kSweepOverlapMaxN = 65536;

}  // namespace

void release_sweep_streams() {
  std::lock_guard<std::mutex> lk(g_sweep_mu);
  int prev = 0;
  (void)hipGetDevice(&prev);
  for (int d = 0; d < kSweepDev; ++d)
    if (g_sweep[d].r) {
      (void)hipSetDevice(d);
      (void)hipStreamSynchronize(g_sweep[d].r);
      destroy_sweep(g_sweep[d]);
    }
  (void)hipSetDevice(prev);
}

// Reverse sweep over checkpointed segments; see nbody_traj_grad in nbody.h.
// Segment seg's trajectory is recomputed from its checkpoint into trajectory
// buffer seg % nbuf, then its adjoint steps read it from the last step back.
// With one buffer everything runs on s in that order.  With two (the overlap:
// a second stream r, the recompute's all-pairs scratch in its own workspace
// slot), r recomputes segment seg - 1 while s runs the adjoint steps of seg:
// a recompute waits for the adjoint steps that last read its buffer (freed),
// the adjoint steps of a segment wait for its recompute (done).  Every kernel
// sees the same inputs either way, so the results are bitwise the same.
int run_traj_grad(int64_t n, const double* ckx, const double* ckv, int64_t every, int64_t nsteps,
                  const double* m, double dt, const double* gxT, const double* gvT, double* gx0, double* gv0,
                  double* gm, double G, double eps, int precision, bool excl, const PairConfig& cfg,
                  hipStream_t s) {
  const int64_t n3 = 3 * n;
  const int64_t seglen = std::min<int64_t>(every, std::max<int64_t>(nsteps, 1));
  const int64_t nseg = (nsteps + every - 1) / every;
  std::unique_lock<std::mutex> sweep_lk;
  SweepStream* ss = cfg.sweep == 0 && nseg >= 2 && n <= kSweepOverlapMaxN && cfg.launches == 0 && !cfg.scratch
                        ? acquire_sweep_stream(s, sweep_lk)
                        : nullptr;
  const int nbuf = ss ? 2 : 1;
  // per buffer: the trajectory ((seglen + 1) x 3n) and the state (x, v, a: 3 x 3n)
  const size_t bufd = (size_t)(seglen + 1) * n3 + 3 * (size_t)n3;
  const size_t need = sizeof(double) * (nbuf * bufd + (size_t)n3 + (size_t)n);
  int st = NBODY_OK;
  double* ws = static_cast<double*>(workspace(current_device(), 1, need, &st));
  if (!ws) return st;
  double* gxp = ws + nbuf * bufd;  // 3n
  double* gmp = gxp + n3;          // n
  auto traj_of = [&](int b) { return ws + b * bufd; };
  auto state_of = [&](int b) { return ws + b * bufd + (size_t)(seglen + 1) * n3; };  // xs, vs, acc
  // lambda_x and lambda_v live in the caller's outputs gx0 / gv0.
  double* lx = gx0;
  double* lv = gv0;
  if ((st = launch_copy(n3, gxT, lx, s))) return st;
  if ((st = launch_copy(n3, gvT, lv, s))) return st;
  if ((st = launch_fill(n, gm, 0.0, s))) return st;
  const double h = 0.5 * dt;
  PairConfig rcfg = cfg;
  if (ss) rcfg.ws_slot = kSweepSlot;
  hipStream_t rs = ss ? ss->r : s;

  auto recompute = [&](int64_t seg) -> int {
    const int b = (int)(seg % nbuf);
    const int64_t k0 = seg * every;
    const int64_t L = std::min<int64_t>(nsteps, k0 + every) - k0;
    double* traj = traj_of(b);
    double* xs = state_of(b);
    double* vs = xs + n3;
    double* acc = vs + n3;
    int e;
    if ((e = launch_copy(n3, ckx + (size_t)seg * n3, xs, rs))) return e;
    if ((e = launch_copy(n3, ckv + (size_t)seg * n3, vs, rs))) return e;
    if ((e = launch_copy(n3, xs, traj, rs))) return e;
    return run_kdk(n, xs, vs, acc, m, dt, L, G, eps, precision, excl, false, rcfg, rs, traj);
  };
  auto adjoint_steps = [&](int64_t seg) -> int {
    const double* traj = traj_of((int)(seg % nbuf));
    const int64_t k0 = seg * every;
    const int64_t k1 = std::min<int64_t>(nsteps, k0 + every);
    for (int64_t p = k1; p > k0; --p) {
      // the kicks at x_p: one closing half-kick at the final position, two
      // (closing + opening) at interior positions, merged into one VJP
      const double c = (p == nsteps) ? h : dt;
      const double* xp = traj + (size_t)(p - k0) * n3;
      int e;
      if ((e = launch_vjp(n, xp, m, lv, gxp, gmp, G * c, eps, precision, excl, cfg, s))) return e;
      adjoint_update_kernel<<<ew_blocks(n3), kEw, 0, s>>>(n, lx, lv, gm, gxp, gmp, dt, 1);
      NB_LAUNCH_CHECK("adjoint_update_kernel");
    }
    return NBODY_OK;
  };

  if (!ss) {
    for (int64_t seg = nseg - 1; seg >= 0; --seg) {
      if ((st = recompute(seg))) return st;
      if ((st = adjoint_steps(seg))) return st;
    }
  } else {
    // r starts after what s holds so far (the caller's checkpoints among it)
    NB_HIP(hipEventRecord(ss->fork, s));
    NB_HIP(hipStreamWaitEvent(rs, ss->fork, 0));
    st = recompute(nseg - 1);
    if (!st) st = hip_ok(hipEventRecord(ss->done[(nseg - 1) % 2], rs), "hipEventRecord");
    for (int64_t seg = nseg - 1; seg >= 0 && !st; --seg) {
      if (seg >= 1) {
        const int b = (int)((seg - 1) % 2);
        // buffer b was last read by the adjoint steps of segment seg + 1
        if (seg + 1 <= nseg - 1 && (st = hip_ok(hipStreamWaitEvent(rs, ss->freed[b], 0), "hipStreamWaitEvent")))
          break;
        if ((st = recompute(seg - 1))) break;
        if ((st = hip_ok(hipEventRecord(ss->done[b], rs), "hipEventRecord"))) break;
      }
      const int b = (int)(seg % 2);
      if ((st = hip_ok(hipStreamWaitEvent(s, ss->done[b], 0), "hipStreamWaitEvent"))) break;
      if ((st = adjoint_steps(seg))) break;
      st = hip_ok(hipEventRecord(ss->freed[b], s), "hipEventRecord");
    }
    // join: s continues after all of r's work (also after an error, so that a
    // captured sweep stays one graph)
    const int sj = hip_ok(hipEventRecord(ss->fork, rs), "hipEventRecord");
    const int sw = sj ? sj : hip_ok(hipStreamWaitEvent(s, ss->fork, 0), "hipStreamWaitEvent");
    if (st) return st;
    if (sw) return sw;
  }
  // opening half-kick of step 0 at x_0
  if (nsteps > 0) {
    if ((st = launch_vjp(n, ckx, m, lv, gxp, gmp, G * h, eps, precision, excl, cfg, s))) return st;
    adjoint_update_kernel<<<ew_blocks(n3), kEw, 0, s>>>(n, lx, lv, gm, gxp, gmp, dt, 0);
    NB_LAUNCH_CHECK("adjoint_update_kernel");
  }
  return NBODY_OK;
}

}  // namespace nb
