// C ABI of libnbody_accel (declared in include/nbody.h): argument validation,
// per-device workspace, tile-configuration choice and the autotuner.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace nb {

int run_traj_grad(int64_t n, const double* ckx, const double* ckv, int64_t every, int64_t nsteps,
                  const double* m, double dt, const double* gxT, const double* gvT, double* gx0, double* gv0,
                  double* gm, double G, double eps, int precision, bool excl, const PairConfig& cfg,
                  hipStream_t s);
void release_batched_plans();
void release_stream_plans();
void release_sym_ensemble_plans();
void release_side_streams();
void release_sweep_streams();
bool sym_ensemble_default(int32_t ncl, const int64_t* off);

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

int set_error(int status, const std::string& msg) {
  g_err = msg;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  return set_error(NBODY_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// --------------------------------------------------------------- workspace
namespace {
constexpr int kMaxDev = 64;
constexpr int kSlots = 5;
struct Buf { void* p = nullptr; size_t bytes = 0; };
std::mutex g_ws_mu;
Buf g_ws[kMaxDev][kSlots];
std::atomic<int> g_cus[kMaxDev];  // zero-initialised (static storage)
std::atomic<bool> g_used[kMaxDev];  // devices the library has run on (false initially)
}  // namespace

int current_device() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return 0;
  if (d >= 0 && d < kMaxDev && !g_used[d].load(std::memory_order_relaxed)) g_used[d].store(true, std::memory_order_relaxed);
  return d;
}

// Waits for all work on every device the library has run on (every path that
// enqueues work or keeps state asks current_device() first).
void sync_used_devices() {
  int prev = 0;
  (void)hipGetDevice(&prev);
  for (int d = 0; d < kMaxDev; ++d)
    if (g_used[d].load(std::memory_order_relaxed)) {
      (void)hipSetDevice(d);
      (void)hipDeviceSynchronize();
    }
  (void)hipSetDevice(prev);
}

int cu_count(int device) {
  if (device < 0 || device >= kMaxDev) return 256;
  int c = g_cus[device].load(std::memory_order_relaxed);
  if (c == 0) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c <= 0) c = 256;
    g_cus[device].store(c, std::memory_order_relaxed);
  }
  return c;
}

void* workspace(int device, int slot, size_t bytes, int* status) {
  if (device < 0 || device >= kMaxDev || slot < 0 || slot >= kSlots) {
    *status = set_error(NBODY_EINVAL, "workspace: bad device or slot");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_ws_mu);
  Buf& b = g_ws[device][slot];
  if (b.bytes >= bytes && b.p) return b.p;
  size_t want = std::max<size_t>(bytes + bytes / 4, 1 << 20);
  if (b.p) {
    // the old buffer may still be read by enqueued work
    if (hipDeviceSynchronize() != hipSuccess || hipFree(b.p) != hipSuccess) {
      *status = set_error(NBODY_EHIP, "workspace: releasing the previous buffer failed");
      return nullptr;
    }
    b.p = nullptr;
    b.bytes = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    *status = set_error(NBODY_ENOMEM, "workspace: hipMalloc of " + std::to_string(want) + " bytes failed");
    return nullptr;
  }
  b.p = p;
  b.bytes = want;
  return p;
}

void* pair_scratch(const PairConfig& cfg, size_t bytes, int* status) {
  if (!cfg.scratch) return workspace(current_device(), cfg.ws_slot, bytes, status);
  if (bytes > cfg.scratch_bytes) {
    *status = set_error(NBODY_EINVAL, "the call needs " + std::to_string(bytes) + " bytes of scratch, more than the " +
                                          std::to_string(cfg.scratch_bytes) + " it was given");
    return nullptr;
  }
  return cfg.scratch;
}

void release_workspaces() {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  for (int d = 0; d < kMaxDev; ++d)
    for (int s = 0; s < kSlots; ++s)
      if (g_ws[d][s].p) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(d);
        (void)hipDeviceSynchronize();
        (void)hipFree(g_ws[d][s].p);
        (void)hipSetDevice(prev);
        g_ws[d][s] = Buf{};
      }
}

// ------------------------------------------------------------- configuration
namespace {
thread_local nbody_config t_cfg = {0, 0, 0, 0, 0, 0, 0, 0};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int64_t>, PairConfig> g_tuned;  // (device, precision, n)
}  // namespace

void set_thread_config(const nbody_config& c) { t_cfg = c; }
const nbody_config& thread_config() { return t_cfg; }

void record_tuned(int device, int64_t n, int precision, const PairConfig& c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[std::make_tuple(device, precision, n)] = c;
}

// Default j-split: enough workgroups for about 32 rounds of 4 per CU, so the
// last round's imbalance stays small (the autotuner's choice at N = 2^20 was
// 32768 workgroups of one i per lane), while keeping at least 2 LDS tiles per
// workgroup.
static int auto_split(int64_t n, int ipl, int device) {
  const int64_t iblocks = (n + kBlock * ipl - 1) / (kBlock * ipl);
  const int64_t target = 128LL * cu_count(device);
  // slices of at least two tiles, or of one fold block for small systems whose
  // i-blocks alone cannot fill the chip
  const int64_t smax = std::max<int64_t>(1, n / (n < (int64_t(1) << 14) ? kFold : 2 * kTile));
  int64_t s = (target + iblocks - 1) / iblocks;
  return (int)std::max<int64_t>(1, std::min<int64_t>(s, std::min<int64_t>(smax, 1024)));
}

PairConfig choose_config(int64_t n, int precision, int device) {
  PairConfig c;
  // measured at N = 2^20: one i per lane is fastest for the FP32 pair loops,
  // four for FP64 (whose rsqrt refinement leaves more latency to hide); fewer
  // for smaller FP64 systems so that they still spread over many workgroups
  c.ipl = precision != NBODY_FP64 ? 1 : (n >= (int64_t(1) << 18) ? 4 : (n >= (int64_t(1) << 14) ? 2 : 1));
  const nbody_config& t = t_cfg;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(device, precision, n));
    if (it != g_tuned.end()) c = it->second;
    else {
      c.split = 0;
      c.sym = n >= (precision == NBODY_FP64 ? kSymMinN64 : kSymMinN) ? 1 : 0;
    }
  }
  c.sym_vjp = n >= kSymMinNVjp ? 1 : 0;
  c.sym_vjp64 = n >= kSymMinNVjp64 ? 1 : 0;
  c.sym_jerk = n >= kSymMinNJerk ? 1 : 0;
  c.sym_jerk64 = n >= kSymMinNJerk64 ? 1 : 0;
  c.sym_snap64 = n >= kSymMinNSnap64 ? 1 : 0;
  c.sym_snap = n >= kSymMinNSnap ? 1 : 0;
  if (t.ipl) c.ipl = t.ipl;
  if (t.split) c.split = t.split;
  if (t.pairs) c.sym = c.sym_vjp = c.sym_vjp64 = c.sym_jerk = c.sym_jerk64 = c.sym_snap = c.sym_snap64 = t.pairs == 2 ? 1 : 0;
  c.rescue = t.rescue == 2 ? 0 : 1;
  c.sweep = t.sweep;
  // the symmetric kernels read a set split as a least number of launches (0 =
  // automatic); the ordered kernels that serve the same sizes (acceleration +
  // jerk (+ snap) below their thresholds, the FP64 VJP) keep their own j-split
  c.launches = c.sym || c.sym_vjp || c.sym_vjp64 || c.sym_jerk || c.sym_jerk64 || c.sym_snap || c.sym_snap64 ? t.split : 0;
  if (c.split <= 0) c.split = auto_split(n, c.ipl, device);
  return c;
}

// ------------------------------------------------------------- validation
namespace {

int check_dev_range(const void* p, size_t bytes, const char* name) {
  if (!p) return set_error(NBODY_EINVAL, std::string(name) + " is NULL");
  if (reinterpret_cast<uintptr_t>(p) % 8 != 0)
    return set_error(NBODY_EINVAL, std::string(name) + " is not 8-byte aligned");
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(NBODY_EINVAL, std::string(name) + " is not a HIP device pointer");
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
    return set_error(NBODY_EINVAL, std::string(name) + " is not device memory");
  if (at.device != current_device())
    return set_error(NBODY_EINVAL, std::string(name) + " belongs to another device");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess && base) {
    const char* b = static_cast<const char*>(base);
    const char* q = static_cast<const char*>(p);
    if (q < b || q + bytes > b + size)
      return set_error(NBODY_EINVAL, std::string(name) + " is smaller than the size implied by n");
  } else {
    (void)hipGetLastError();
  }
  return NBODY_OK;
}

constexpr int64_t kMaxN = int64_t(1) << 29;

int check_common(int64_t n, const nbody_params* p, bool need_eps_rule) {
  if (!p) return set_error(NBODY_EINVAL, "params is NULL");
  if (n < 0) return set_error(NBODY_EINVAL, "n < 0");
  if (n > kMaxN) return set_error(NBODY_EINVAL, "n exceeds 2^29");
  if (!std::isfinite(p->G)) return set_error(NBODY_EINVAL, "G is not finite");
  if (!std::isfinite(p->eps) || p->eps < 0) return set_error(NBODY_EINVAL, "eps must be finite and >= 0");
  if (p->precision != NBODY_FP64 && p->precision != NBODY_FP32C && p->precision != NBODY_FP32)
    return set_error(NBODY_EINVAL, "unknown precision");
  if (p->flags & ~uint32_t(NBODY_EXCLUDE_SELF | NBODY_CHECK_FINITE | NBODY_ACC_VALID))
    return set_error(NBODY_EINVAL, "unknown flag bits");
  if (need_eps_rule && p->eps == 0.0 && !(p->flags & NBODY_EXCLUDE_SELF))
    return set_error(NBODY_EINVAL, "eps == 0 requires NBODY_EXCLUDE_SELF");
  return NBODY_OK;
}

#define NB_TRY(expr)          \
  do {                        \
    int nb_s_ = (expr);       \
    if (nb_s_) return nb_s_;  \
  } while (0)

int finish(int st, hipStream_t s, const nbody_params* p, std::initializer_list<std::pair<const double*, int64_t>> outs) {
  if (st) return st;
  if (!(p->flags & NBODY_CHECK_FINITE)) return NBODY_OK;
  for (auto& o : outs) {
    bool ok = true;
    NB_TRY(check_finite(o.first, o.second, s, &ok));
    if (!ok) return set_error(NBODY_ENONFINITE, "output contains NaN or Inf");
  }
  return NBODY_OK;
}

}  // namespace
}  // namespace nb

using namespace nb;

namespace {

// Host-side checks shared by the batched calls; total receives off[ncl].
int check_batched_host(int32_t ncl, const int64_t* off, const double* eps, double dt, int64_t nsteps,
                       const nbody_params* p, int64_t* total) {
  if (!p) return set_error(NBODY_EINVAL, "params is NULL");
  if (ncl < 0) return set_error(NBODY_EINVAL, "ncl < 0");
  *total = 0;
  if (ncl == 0) return NBODY_OK;
  if (!off || !eps) return set_error(NBODY_EINVAL, "off and eps must be host arrays");
  if (!std::isfinite(dt)) return set_error(NBODY_EINVAL, "dt is not finite");
  if (nsteps < 0) return set_error(NBODY_EINVAL, "nsteps < 0");
  if (!std::isfinite(p->G)) return set_error(NBODY_EINVAL, "G is not finite");
  if (p->precision != NBODY_FP64 && p->precision != NBODY_FP32C && p->precision != NBODY_FP32)
    return set_error(NBODY_EINVAL, "unknown precision");
  if (p->flags & ~uint32_t(NBODY_EXCLUDE_SELF | NBODY_CHECK_FINITE | NBODY_ACC_VALID))
    return set_error(NBODY_EINVAL, "unknown flag bits");
  if (off[0] != 0) return set_error(NBODY_EINVAL, "off[0] must be 0");
  for (int32_t c = 0; c < ncl; ++c) {
    if (off[c + 1] < off[c]) return set_error(NBODY_EINVAL, "off must be non-decreasing");
    if (!std::isfinite(eps[c]) || eps[c] < 0) return set_error(NBODY_EINVAL, "eps[c] must be finite and >= 0");
    if (eps[c] == 0.0 && !(p->flags & NBODY_EXCLUDE_SELF))
      return set_error(NBODY_EINVAL, "eps[c] == 0 requires NBODY_EXCLUDE_SELF");
  }
  *total = off[ncl];
  if (*total > kMaxN) return set_error(NBODY_EINVAL, "total particle count exceeds 2^29");
  return NBODY_OK;
}

// Batched configurations chosen by nbody_tune_batched, per (device, precision, layout).
struct TunedBatch {
  int device, precision;
  std::vector<int64_t> off;
  std::vector<double> eps;
  BatchConfig bc;
};
std::mutex g_tb_mu;
std::vector<TunedBatch> g_tuned_batch;

// The thread's forced configuration if it sets any batched field, else the
// tuned one for this layout, else the per-step wave items: their symmetric form
// (mode 4) for FP32C/FP32 layouts whose systems mostly span several blocks of
// 64, else the ordered form (mode 3).
BatchConfig batch_config_for(int32_t ncl, const int64_t* off, const double* eps, int precision, int device) {
  const nbody_config& t = t_cfg;
  BatchConfig bc;
  bc.rescue = t.rescue == 2 ? 0 : 1;
  if (t.bsplit || t.bpass || t.bitem) {
    bc.mode = t.bsplit;
    bc.pass = t.bpass;
    bc.item = t.bitem;
    return bc;
  }
  std::lock_guard<std::mutex> lk(g_tb_mu);
  for (const TunedBatch& e : g_tuned_batch)
    if (e.device == device && e.precision == precision && (int)e.eps.size() == ncl &&
        std::equal(e.off.begin(), e.off.end(), off) && std::equal(e.eps.begin(), e.eps.end(), eps) &&
        e.bc.rescue == bc.rescue)
      return e.bc;
  // the symmetric per-step items where they pay (FP32C and FP32 layouts whose
  // systems mostly span several blocks of 64), else the ordered ones; both
  // carry the FP32C rescue
  const bool sym = precision == NBODY_FP32 || precision == NBODY_FP32C;
  bc.mode = (sym && sym_ensemble_default(ncl, off)) ? 4 : 3;
  return bc;
}

// --------------------------------------------- fixed scratch, no allocation
// The device memory of nbody_accel_noalloc: a file-scope array that the code
// object brings along, one copy on every GPU the library runs on, held until
// the process ends.  On the host `scratch` is only a stand-in for the symbol;
// host code takes each device's address from hipGetSymbolAddress and uses
// that address (kernel arguments, offsets) instead of the name.
constexpr size_t kNoAllocBytes = (size_t)NBODY_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[64];  // per device, looked up on the device's first call

// This device's address of `scratch`, looked up once per device with that
// device current (the caller's current device).
int noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= 64) return set_error(NBODY_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return set_error(NBODY_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return NBODY_OK;
}

}  // namespace

extern "C" {

int nbody_accel_noalloc(int64_t n, const double* x, const double* m, double* a, const nbody_params* p,
                        void* stream) {
  NB_TRY(check_common(n, p, true));
  if (n > NBODY_NOALLOC_MAX_N)
    return set_error(NBODY_EINVAL, "nbody_accel_noalloc: n = " + std::to_string(n) + " exceeds " +
                                       std::to_string((long long)NBODY_NOALLOC_MAX_N) +
                                       ", the largest system its fixed scratch serves (use nbody_accel)");
  if (p->flags & NBODY_CHECK_FINITE)
    return set_error(NBODY_EINVAL, "nbody_accel_noalloc: NBODY_CHECK_FINITE waits for the stream and needs a "
                                   "status buffer; use nbody_accel");
  if (n == 0) return NBODY_OK;
  const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
  NB_TRY(check_dev_range(x, b3, "x"));
  NB_TRY(check_dev_range(m, b1, "m"));
  NB_TRY(check_dev_range(a, b3, "a"));
  if ((const void*)a == (const void*)x || (const void*)a == (const void*)m)
    return set_error(NBODY_EINVAL, "a aliases an input");
  const int dev = current_device();
  void* scr = nullptr;
  NB_TRY(noalloc_scratch(dev, &scr));
  PairConfig cfg = choose_config(n, p->precision, dev);
  cfg.scratch = scr;
  cfg.scratch_bytes = kNoAllocBytes;
  if (!cfg.sym) {
    // the ordered kernels keep 3 n FP64 partial sums per slice of the j-range and,
    // with the FP32C rescue, n FP32 estimate shares per slice and the flagged-row
    // list (n + 64 ints, after 256-byte alignment of the shares)
    const bool resc = p->precision == NBODY_FP32C && cfg.rescue;
    const size_t per = sizeof(double) * 3 * (size_t)n + (resc ? sizeof(float) * (size_t)n : 0);
    const size_t fixed = resc ? sizeof(int) * ((size_t)n + 64) + 256 : 0;
    const int64_t most = std::max<int64_t>(1, (int64_t)((kNoAllocBytes - fixed) / per));
    cfg.split = (int)std::min<int64_t>(cfg.split, most);
  }
  return launch_accel(n, x, m, a, p->G, p->eps, p->precision, (p->flags & NBODY_EXCLUDE_SELF) != 0, cfg,
                      static_cast<hipStream_t>(stream));
}

int nbody_accel(int64_t n, const double* x, const double* m, double* a, const nbody_params* p, void* stream) {
  NB_TRY(check_common(n, p, true));
  if (n == 0) return NBODY_OK;
  const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
  NB_TRY(check_dev_range(x, b3, "x"));
  NB_TRY(check_dev_range(m, b1, "m"));
  NB_TRY(check_dev_range(a, b3, "a"));
  if ((const void*)a == (const void*)x || (const void*)a == (const void*)m)
    return set_error(NBODY_EINVAL, "a aliases an input");
  hipStream_t s = static_cast<hipStream_t>(stream);
  PairConfig cfg = choose_config(n, p->precision, current_device());
  int st = launch_accel(n, x, m, a, p->G, p->eps, p->precision, (p->flags & NBODY_EXCLUDE_SELF) != 0, cfg, s);
  return finish(st, s, p, {{a, 3 * n}});
}

int nbody_step(int64_t n, double* x, double* v, double* a, const double* m, double dt, int64_t nsteps,
               const nbody_params* p, void* stream) {
  NB_TRY(check_common(n, p, true));
  if (!std::isfinite(dt)) return set_error(NBODY_EINVAL, "dt is not finite");
  if (nsteps < 0) return set_error(NBODY_EINVAL, "nsteps < 0");
  if (n == 0) return NBODY_OK;
  const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
  NB_TRY(check_dev_range(x, b3, "x"));
  NB_TRY(check_dev_range(v, b3, "v"));
  NB_TRY(check_dev_range(a, b3, "a"));
  NB_TRY(check_dev_range(m, b1, "m"));
  if (x == v || x == a || v == a) return set_error(NBODY_EINVAL, "x, v and a must be distinct");
  hipStream_t s = static_cast<hipStream_t>(stream);
  PairConfig cfg = choose_config(n, p->precision, current_device());
  int st = run_kdk(n, x, v, a, m, dt, nsteps, p->G, p->eps, p->precision, (p->flags & NBODY_EXCLUDE_SELF) != 0,
                   (p->flags & NBODY_ACC_VALID) != 0, cfg, s, nullptr);
  return finish(st, s, p, {{x, 3 * n}, {v, 3 * n}, {a, 3 * n}});
}

int nbody_energy(int64_t n, const double* x, const double* v, const double* m, const nbody_params* p,
                 double* out9, void* stream) {
  NB_TRY(check_common(n, p, false));
  const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
  if (n > 0) {
    NB_TRY(check_dev_range(x, b3, "x"));
    NB_TRY(check_dev_range(v, b3, "v"));
    NB_TRY(check_dev_range(m, b1, "m"));
  }
  NB_TRY(check_dev_range(out9, 9 * sizeof(double), "out9"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  int st = launch_energy(n, x, v, m, p->G, p->eps, out9, s);
  return finish(st, s, p, {{out9, 9}});
}

int nbody_accel_vjp(int64_t n, const double* x, const double* m, const double* w, double* gx, double* gm,
                    const nbody_params* p, void* stream) {
  NB_TRY(check_common(n, p, true));
  if (n == 0) return NBODY_OK;
  const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
  NB_TRY(check_dev_range(x, b3, "x"));
  NB_TRY(check_dev_range(m, b1, "m"));
  NB_TRY(check_dev_range(w, b3, "w"));
  NB_TRY(check_dev_range(gx, b3, "gx"));
  NB_TRY(check_dev_range(gm, b1, "gm"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  PairConfig cfg = choose_config(n, p->precision, current_device());
  int st = launch_vjp(n, x, m, w, gx, gm, p->G, p->eps, p->precision, (p->flags & NBODY_EXCLUDE_SELF) != 0, cfg, s);
  return finish(st, s, p, {{gx, 3 * n}, {gm, n}});
}

int nbody_traj_grad(int64_t n, const double* ckpt_x, const double* ckpt_v, int64_t every, int64_t nsteps,
                    const double* m, double dt, const double* gxT, const double* gvT, double* gx0, double* gv0,
                    double* gm, const nbody_params* p, void* stream) {
  NB_TRY(check_common(n, p, true));
  if (!std::isfinite(dt)) return set_error(NBODY_EINVAL, "dt is not finite");
  if (nsteps < 0) return set_error(NBODY_EINVAL, "nsteps < 0");
  if (every < 1) return set_error(NBODY_EINVAL, "every < 1");
  if (n == 0) return NBODY_OK;
  const int64_t nck = std::max<int64_t>(1, (nsteps + every - 1) / every);
  const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
  NB_TRY(check_dev_range(ckpt_x, b3 * nck, "ckpt_x"));
  NB_TRY(check_dev_range(ckpt_v, b3 * nck, "ckpt_v"));
  NB_TRY(check_dev_range(m, b1, "m"));
  NB_TRY(check_dev_range(gxT, b3, "gxT"));
  NB_TRY(check_dev_range(gvT, b3, "gvT"));
  NB_TRY(check_dev_range(gx0, b3, "gx0"));
  NB_TRY(check_dev_range(gv0, b3, "gv0"));
  NB_TRY(check_dev_range(gm, b1, "gm"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  PairConfig cfg = choose_config(n, p->precision, current_device());
  int st = run_traj_grad(n, ckpt_x, ckpt_v, every, nsteps, m, dt, gxT, gvT, gx0, gv0, gm, p->G, p->eps,
                         p->precision, (p->flags & NBODY_EXCLUDE_SELF) != 0, cfg, s);
  return finish(st, s, p, {{gx0, 3 * n}, {gv0, 3 * n}, {gm, n}});
}


int nbody_step_batched(int32_t ncl, const int64_t* off, const double* eps, double* x, double* v, double* a,
                       const double* m, double dt, int64_t nsteps, const nbody_params* p, void* stream) {
  int64_t total = 0;
  NB_TRY(check_batched_host(ncl, off, eps, dt, nsteps, p, &total));
  if (total == 0) return NBODY_OK;
  const size_t b3 = sizeof(double) * 3 * (size_t)total, b1 = sizeof(double) * (size_t)total;
  NB_TRY(check_dev_range(x, b3, "x"));
  NB_TRY(check_dev_range(v, b3, "v"));
  NB_TRY(check_dev_range(a, b3, "a"));
  NB_TRY(check_dev_range(m, b1, "m"));
  if (x == v || x == a || v == a) return set_error(NBODY_EINVAL, "x, v and a must be distinct");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const BatchConfig bc = batch_config_for(ncl, off, eps, p->precision, current_device());
  if (p->precision == NBODY_FP32C && t_cfg.rescue == 1 && bc.mode != 3 && bc.mode != 4)
    return set_error(NBODY_EUNSUPPORTED,
                     "batched: the FP32C rescue runs with the per-step items (bsplit 3 or 4) only");
  int st = run_batched(ncl, off, eps, x, v, a, m, dt, nsteps, p->G, p->precision,
                       (p->flags & NBODY_EXCLUDE_SELF) != 0, (p->flags & NBODY_ACC_VALID) != 0, bc, s);
  return finish(st, s, p, {{x, 3 * total}, {v, 3 * total}, {a, 3 * total}});
}

int nbody_tune_batched(int32_t ncl, const int64_t* off, const double* eps, const double* x, const double* v,
                       const double* m, double dt, int64_t nsteps, int32_t allow_cooperative,
                       const nbody_params* p, nbody_config* best) {
  int64_t total = 0;
  NB_TRY(check_batched_host(ncl, off, eps, dt, nsteps, p, &total));
  if (nsteps < 1) return set_error(NBODY_EINVAL, "tune_batched: nsteps must be >= 1");
  if (allow_cooperative < 0 || allow_cooperative > 2)
    return set_error(NBODY_EINVAL, "tune_batched: allow_cooperative must be 0, 1 or 2");
  if (total == 0) return set_error(NBODY_EINVAL, "tune_batched: the ensemble is empty");
  const size_t b3 = sizeof(double) * 3 * (size_t)total, b1 = sizeof(double) * (size_t)total;
  NB_TRY(check_dev_range(x, b3, "x"));
  NB_TRY(check_dev_range(v, b3, "v"));
  NB_TRY(check_dev_range(m, b1, "m"));
  const int dev = current_device();
  const int rescue = t_cfg.rescue == 2 ? 0 : 1;
  std::vector<BatchConfig> cand;
  if (p->precision == NBODY_FP32C && rescue && (allow_cooperative != 2 || t_cfg.rescue == 1)) {
    // only the per-step items carry the FP32C rescue (the single-launch
    // search, allow_cooperative = 2, goes without it unless it was asked for)
    if (allow_cooperative == 2)
      return set_error(NBODY_EUNSUPPORTED, "tune_batched: no single-launch mode carries the FP32C rescue");
    cand.push_back(BatchConfig{3, 0, 64, 1});
    cand.push_back(BatchConfig{4, 0, 0, 1});
  } else {
    for (int pass : {1, 2, 4}) cand.push_back(BatchConfig{0, pass, 0, rescue});
    if (allow_cooperative != 2) {
      cand.push_back(BatchConfig{3, 0, 64, rescue});
      if (p->precision != NBODY_FP64) cand.push_back(BatchConfig{4, 0, 0, rescue});
    }
    if (allow_cooperative) {
      cand.push_back(BatchConfig{1, 0, 0, rescue});
      for (int item : {64, 256, 512, 1024}) cand.push_back(BatchConfig{2, 0, item, rescue});
    }
  }
  double *sx = nullptr, *sv = nullptr, *sa = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    for (double* q : {sx, sv, sa})
      if (q) (void)hipFree(q);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&sx, b3) != hipSuccess || hipMalloc(&sv, b3) != hipSuccess || hipMalloc(&sa, b3) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return set_error(NBODY_ENOMEM, "tune_batched: allocation failed");
  }
  const bool excl = (p->flags & NBODY_EXCLUDE_SELF) != 0;
  float best_ms = 0.0f;
  int best_k = -1;
  for (size_t k = 0; k < cand.size(); ++k) {
    if (hipMemcpy(sx, x, b3, hipMemcpyDeviceToDevice) != hipSuccess ||
        hipMemcpy(sv, v, b3, hipMemcpyDeviceToDevice) != hipSuccess) {
      cleanup();
      return set_error(NBODY_EHIP, "tune_batched: copy failed");
    }
    int st = run_batched(ncl, off, eps, sx, sv, sa, m, dt, 0, p->G, p->precision, excl, false, cand[k], nullptr);
    if (st == NBODY_EUNSUPPORTED) continue;  // e.g. the resident kernel with a system above 4096 particles
    if (st) { cleanup(); return st; }
    // an untimed run of the same length first: a short timed run straight after the copies
    // above mostly measures the GPU coming back to its clock, not the configuration
    st = run_batched(ncl, off, eps, sx, sv, sa, m, dt, nsteps, p->G, p->precision, excl, true, cand[k], nullptr);
    if (st) { cleanup(); return st; }
    (void)hipEventRecord(e0, nullptr);
    st = run_batched(ncl, off, eps, sx, sv, sa, m, dt, nsteps, p->G, p->precision, excl, true, cand[k], nullptr);
    if (st) { cleanup(); return st; }
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess) { cleanup(); return set_error(NBODY_EHIP, "tune_batched: sync failed"); }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    bool finite_ok = true;
    if ((st = check_finite(sx, 3 * total, nullptr, &finite_ok))) { cleanup(); return st; }
    if (finite_ok && (best_k < 0 || ms < best_ms)) {
      best_ms = ms;
      best_k = (int)k;
    }
  }
  cleanup();
  if (best_k < 0) return set_error(NBODY_ENONFINITE, "tune_batched: every configuration produced non-finite state");
  const BatchConfig bc = cand[best_k];
  {
    std::lock_guard<std::mutex> lk(g_tb_mu);
    bool found = false;
    for (TunedBatch& e : g_tuned_batch)
      if (e.device == dev && e.precision == p->precision && (int)e.eps.size() == ncl &&
          std::equal(e.off.begin(), e.off.end(), off) && std::equal(e.eps.begin(), e.eps.end(), eps) &&
          e.bc.rescue == bc.rescue) {
        e.bc = bc;
        found = true;
      }
    if (!found)
      g_tuned_batch.push_back(TunedBatch{dev, p->precision, std::vector<int64_t>(off, off + ncl + 1),
                                         std::vector<double>(eps, eps + ncl), bc});
  }
  if (best) *best = nbody_config{0, 0, bc.mode, bc.pass, bc.item, 0, 0};
  return NBODY_OK;
}

int nbody_accel_jerk(int64_t n, const double* x, const double* v, const double* m, double* a, double* jk,
                     const nbody_params* p, void* stream) {
  NB_TRY(check_common(n, p, true));
  if (n == 0) return NBODY_OK;
  const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
  NB_TRY(check_dev_range(x, b3, "x"));
  NB_TRY(check_dev_range(v, b3, "v"));
  NB_TRY(check_dev_range(m, b1, "m"));
  NB_TRY(check_dev_range(a, b3, "a"));
  NB_TRY(check_dev_range(jk, b3, "jk"));
  if (a == jk || (const double*)a == x || (const double*)a == v || (const double*)jk == x || (const double*)jk == v)
    return set_error(NBODY_EINVAL, "a and jk must be distinct from each other and the inputs");
  hipStream_t s = static_cast<hipStream_t>(stream);
  PairConfig cfg = choose_config(n, p->precision, current_device());
  int st = launch_accel_jerk(n, x, v, m, a, jk, p->G, p->eps, p->precision, (p->flags & NBODY_EXCLUDE_SELF) != 0,
                             cfg, s);
  return finish(st, s, p, {{a, 3 * n}, {jk, 3 * n}});
}

int nbody_potential(int64_t n, const double* x, const double* m, double* phi, const nbody_params* p,
                    void* stream) {
  NB_TRY(check_common(n, p, false));
  if (n == 0) return NBODY_OK;
  const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
  NB_TRY(check_dev_range(x, b3, "x"));
  NB_TRY(check_dev_range(m, b1, "m"));
  NB_TRY(check_dev_range(phi, b1, "phi"));
  if ((const double*)phi == x || (const double*)phi == m) return set_error(NBODY_EINVAL, "phi must not alias x or m");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int split = t_cfg.split ? t_cfg.split : auto_split(n, 1, current_device());
  int st = launch_potential(n, x, m, p->eps, -p->G, phi, split, s);
  return finish(st, s, p, {{phi, n}});
}

int nbody_accel_jerk_snap(int64_t n, const double* x, const double* v, const double* acc, const double* m,
                          double* a, double* jk, double* sn, const nbody_params* p, void* stream) {
  NB_TRY(check_common(n, p, true));
  if (n == 0) return NBODY_OK;
  const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
  NB_TRY(check_dev_range(x, b3, "x"));
  NB_TRY(check_dev_range(v, b3, "v"));
  NB_TRY(check_dev_range(acc, b3, "acc"));
  NB_TRY(check_dev_range(m, b1, "m"));
  NB_TRY(check_dev_range(a, b3, "a"));
  NB_TRY(check_dev_range(jk, b3, "jk"));
  NB_TRY(check_dev_range(sn, b3, "sn"));
  for (const double* o : {(const double*)a, (const double*)jk, (const double*)sn})
    for (const double* q : {x, v, acc, m})
      if (o == q) return set_error(NBODY_EINVAL, "a, jk and sn must be distinct from the inputs");
  if (a == jk || a == sn || jk == sn) return set_error(NBODY_EINVAL, "a, jk and sn must be distinct");
  hipStream_t s = static_cast<hipStream_t>(stream);
  PairConfig cfg = choose_config(n, p->precision, current_device());
  int st = launch_accel_jerk_snap(n, x, v, acc, m, a, jk, sn, p->G, p->eps, p->precision,
                                  (p->flags & NBODY_EXCLUDE_SELF) != 0, cfg, s);
  return finish(st, s, p, {{a, 3 * n}, {jk, 3 * n}, {sn, 3 * n}});
}

int nbody_step_hermite6(int64_t n, double* x, double* v, double* a, double* jk, double* sn, double* cr,
                        const double* m, double dt, int64_t nsteps, const nbody_params* p, void* stream) {
  NB_TRY(check_common(n, p, true));
  if (!std::isfinite(dt) || dt == 0.0) return set_error(NBODY_EINVAL, "dt must be finite and non-zero");
  if (nsteps < 0) return set_error(NBODY_EINVAL, "nsteps < 0");
  if (n == 0) return NBODY_OK;
  const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
  double* arr[6] = {x, v, a, jk, sn, cr};
  const char* names[6] = {"x", "v", "a", "jk", "sn", "cr"};
  for (int k = 0; k < 6; ++k) NB_TRY(check_dev_range(arr[k], b3, names[k]));
  NB_TRY(check_dev_range(m, b1, "m"));
  for (int k = 0; k < 6; ++k)
    for (int l = k + 1; l < 6; ++l)
      if (arr[k] == arr[l]) return set_error(NBODY_EINVAL, "x, v, a, jk, sn and cr must be distinct");
  hipStream_t s = static_cast<hipStream_t>(stream);
  PairConfig cfg = choose_config(n, p->precision, current_device());
  int st = run_hermite6(n, x, v, a, jk, sn, cr, m, dt, nsteps, p->G, p->eps, p->precision,
                        (p->flags & NBODY_EXCLUDE_SELF) != 0, (p->flags & NBODY_ACC_VALID) != 0, cfg, s);
  return finish(st, s, p, {{x, 3 * n}, {v, 3 * n}, {a, 3 * n}, {jk, 3 * n}, {sn, 3 * n}, {cr, 3 * n}});
}

int nbody_step_hermite(int64_t n, double* x, double* v, double* a, double* jk, const double* m, double dt,
                       int64_t nsteps, const nbody_params* p, void* stream) {
  NB_TRY(check_common(n, p, true));
  if (!std::isfinite(dt)) return set_error(NBODY_EINVAL, "dt is not finite");
  if (nsteps < 0) return set_error(NBODY_EINVAL, "nsteps < 0");
  if (n == 0) return NBODY_OK;
  const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
  NB_TRY(check_dev_range(x, b3, "x"));
  NB_TRY(check_dev_range(v, b3, "v"));
  NB_TRY(check_dev_range(a, b3, "a"));
  NB_TRY(check_dev_range(jk, b3, "jk"));
  NB_TRY(check_dev_range(m, b1, "m"));
  if (x == v || x == a || x == jk || v == a || v == jk || a == jk)
    return set_error(NBODY_EINVAL, "x, v, a and jk must be distinct");
  hipStream_t s = static_cast<hipStream_t>(stream);
  PairConfig cfg = choose_config(n, p->precision, current_device());
  int st = run_hermite(n, x, v, a, jk, m, dt, nsteps, p->G, p->eps, p->precision,
                       (p->flags & NBODY_EXCLUDE_SELF) != 0, (p->flags & NBODY_ACC_VALID) != 0, cfg, s);
  return finish(st, s, p, {{x, 3 * n}, {v, 3 * n}, {a, 3 * n}, {jk, 3 * n}});
}

int nbody_set_config(const nbody_config* cfg) {
  if (!cfg) return set_error(NBODY_EINVAL, "cfg is NULL");
  if (cfg->ipl != 0 && cfg->ipl != 1 && cfg->ipl != 2 && cfg->ipl != 4)
    return set_error(NBODY_EINVAL, "ipl must be 0, 1, 2 or 4");
  if (cfg->split < 0 || cfg->split > 1024) return set_error(NBODY_EINVAL, "split must be in 0..1024");
  if (cfg->bsplit < 0 || cfg->bsplit > 4) return set_error(NBODY_EINVAL, "bsplit must be 0 .. 4");
  if (cfg->bpass != 0 && cfg->bpass != 1 && cfg->bpass != 2 && cfg->bpass != 4)
    return set_error(NBODY_EINVAL, "bpass must be 0, 1, 2 or 4");
  if (cfg->bitem != 0 && cfg->bitem != 64 && cfg->bitem != 256 && cfg->bitem != 512 && cfg->bitem != 1024)
    return set_error(NBODY_EINVAL, "bitem must be 0, 64, 256, 512 or 1024");
  if (cfg->pairs < 0 || cfg->pairs > 2) return set_error(NBODY_EINVAL, "pairs must be 0, 1 or 2");
  if (cfg->rescue < 0 || cfg->rescue > 2) return set_error(NBODY_EINVAL, "rescue must be 0, 1 or 2");
  if (cfg->sweep < 0 || cfg->sweep > 1) return set_error(NBODY_EINVAL, "sweep must be 0 or 1");
  set_thread_config(*cfg);
  return NBODY_OK;
}

int nbody_tune(int64_t n, int32_t precision, const char* cache_path, nbody_config* best) {
  if (n <= 0 || n > kMaxN) return set_error(NBODY_EINVAL, "n must be in 1..2^29");
  if (precision != NBODY_FP64 && precision != NBODY_FP32C && precision != NBODY_FP32)
    return set_error(NBODY_EINVAL, "unknown precision");
  const int dev = current_device();
  // synthetic input: a deterministic pseudo-random cloud in the unit cube
  std::vector<double> hx(3 * (size_t)n), hm((size_t)n);
  uint64_t st64 = 0x9E3779B97F4A7C15ull;
  auto next = [&]() {
    st64 = st64 * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(st64 >> 11) * (1.0 / 9007199254740992.0);
  };
  for (auto& v : hx) v = 2.0 * next() - 1.0;
  for (auto& v : hm) v = (0.5 + next()) / (double)n;
  double *dx = nullptr, *dm = nullptr, *da = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (dx) (void)hipFree(dx);
    if (dm) (void)hipFree(dm);
    if (da) (void)hipFree(da);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&dx, hx.size() * 8) != hipSuccess || hipMalloc(&dm, hm.size() * 8) != hipSuccess ||
      hipMalloc(&da, hx.size() * 8) != hipSuccess) {
    cleanup();
    return set_error(NBODY_ENOMEM, "tune: allocation failed");
  }
  if (hipMemcpy(dx, hx.data(), hx.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dm, hm.data(), hm.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
    cleanup();
    return set_error(NBODY_EHIP, "tune: copy failed");
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return set_error(NBODY_EHIP, "tune: event creation failed");
  }
  float best_ms = 1e30f;
  PairConfig bc;
  const int ipls[3] = {1, 2, 4};
  std::vector<std::pair<PairConfig, float>> log;
  for (int ipl : ipls) {
    const int base = auto_split(n, ipl, dev);
    std::vector<int> splits = {base};
    for (int f : {2, 4}) {
      if (base / f >= 1) splits.push_back(base / f);
      if ((int64_t)base * f <= std::max<int64_t>(1, std::min<int64_t>(1024, n / (2 * kTile)))) splits.push_back(base * f);
    }
    std::sort(splits.begin(), splits.end());
    splits.erase(std::unique(splits.begin(), splits.end()), splits.end());
    for (int sp : splits) {
      PairConfig c;
      c.ipl = ipl;
      c.split = sp;
      int st = launch_accel(n, dx, dm, da, 1.0, 0.01, precision, false, c, nullptr);
      if (st) { cleanup(); return st; }
      const int reps = 3;
      (void)hipEventRecord(e0, nullptr);
      for (int r = 0; r < reps; ++r) launch_accel(n, dx, dm, da, 1.0, 0.01, precision, false, c, nullptr);
      (void)hipEventRecord(e1, nullptr);
      if (hipEventSynchronize(e1) != hipSuccess) { cleanup(); return set_error(NBODY_EHIP, "tune: sync failed"); }
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      log.push_back({c, ms});
      if (ms < best_ms) { best_ms = ms; bc = c; }
    }
  }
  {
    // the symmetric kernel (its tiling is fixed)
    PairConfig c;
    c.ipl = 2;
    c.split = 0;
    c.sym = 1;
    int st = launch_accel(n, dx, dm, da, 1.0, 0.01, precision, false, c, nullptr);
    if (st) { cleanup(); return st; }
    const int reps = 3;
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps; ++r) launch_accel(n, dx, dm, da, 1.0, 0.01, precision, false, c, nullptr);
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess) { cleanup(); return set_error(NBODY_EHIP, "tune: sync failed"); }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= reps;
    log.push_back({c, ms});
    if (ms < best_ms) { best_ms = ms; bc = c; }
  }
  cleanup();
  record_tuned(dev, n, precision, bc);
  if (best) *best = nbody_config{bc.ipl, bc.split, 0, 0, 0, bc.sym ? 2 : 1, 0};
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (f) {
      hipDeviceProp_t prop;
      (void)hipGetDeviceProperties(&prop, dev);
      std::fprintf(f, "{\"arch\": \"%s\", \"n\": %lld, \"precision\": %d, \"ipl\": %d, \"split\": %d, \"pairs\": %d, \"ms\": %.6f, \"trials\": [",
                   prop.gcnArchName, (long long)n, precision, bc.ipl, bc.split, bc.sym ? 2 : 1, best_ms);
      for (size_t k = 0; k < log.size(); ++k)
        std::fprintf(f, "%s[%d, %d, %d, %.6f]", k ? ", " : "", log[k].first.ipl, log[k].first.split,
                     log[k].first.sym ? 2 : 1, log[k].second);
      std::fprintf(f, "]}\n");
      std::fclose(f);
    }
  }
  return NBODY_OK;
}

const char* nbody_last_error(void) { return g_err.c_str(); }

int nbody_finalize(void) {
  // nothing enqueued may still read what is released below
  sync_used_devices();
  release_batched_plans();
  release_stream_plans();
  release_sym_ensemble_plans();
  {
    std::lock_guard<std::mutex> lk(g_tb_mu);
    g_tuned_batch.clear();
  }
  release_side_streams();
  release_sweep_streams();
  release_workspaces();
  return NBODY_OK;
}

int nbody_version(void) { return 100; }

}  // extern "C"
