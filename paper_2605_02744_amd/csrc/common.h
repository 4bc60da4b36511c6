// Internal declarations shared by the HIP sources of libnbody_accel.so.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "nbody.h"

namespace nb {

// ---------------------------------------------------------------- errors
// Thread-local message for nbody_last_error(); set_error returns the status.
int set_error(int status, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
inline int hip_ok(hipError_t e, const char* what) { return e == hipSuccess ? NBODY_OK : hip_fail(e, what); }

#define NB_HIP(call)                                        \
  do {                                                      \
    hipError_t nb_e_ = (call);                              \
    if (nb_e_ != hipSuccess) return ::nb::hip_fail(nb_e_, #call); \
  } while (0)

#define NB_LAUNCH_CHECK(what)                                \
  do {                                                       \
    hipError_t nb_e_ = hipGetLastError();                    \
    if (nb_e_ != hipSuccess) return ::nb::hip_fail(nb_e_, what); \
  } while (0)

// ---------------------------------------------------------------- workspace
// Growable scratch allocations, one per (device, slot), never shrunk.  Slots
// keep nested users apart: 0 = per-launch partial sums of the all-pairs
// kernels, 1 = per-call buffers of a driver (energy, adjoint sweep),
// 2 = batched plans, 3 = status flags, 4 = the all-pairs scratch of the
// adjoint sweep's recompute on its second stream (kSweepSlot), which runs
// alongside slot 0's users.  Growing a slot synchronises the device.
constexpr int kSweepSlot = 4;
void* workspace(int device, int slot, size_t bytes, int* status);
void release_workspaces();
int current_device();
int cu_count(int device);

// ---------------------------------------------------------------- constants
constexpr int kBlock = 256;        // threads per workgroup of the all-pairs kernels
constexpr int kTile = 256;         // j-particles staged in LDS per tile
constexpr int kFold = 64;          // j-terms summed in plain FP32/FP64 before a TwoSum fold
constexpr double kFarAway = 1.0e15;  // position of padding j-records (mass 0)
// Sizes from which the symmetric kernels are the default (measured crossovers
// against the ordered kernels): the FP32C/FP32 force from 49152 particles, the
// FP64 force from 8192, the FP32C/FP32 VJP from 12288, the FP64 VJP from 8192,
// the FP32C/FP32 acceleration + jerk from 12288 and the FP64 one from 8192, the
// acceleration + jerk + snap from 8192 in every precision.
constexpr int64_t kSymMinN = 49152;
constexpr int64_t kSymMinN64 = 8192;
constexpr int64_t kSymMinNVjp = 12288;
constexpr int64_t kSymMinNVjp64 = 8192;
constexpr int64_t kSymMinNJerk64 = 8192;
constexpr int64_t kSymMinNSnap64 = 8192;
constexpr int64_t kSymMinNJerk = 12288;
constexpr int64_t kSymMinNSnap = 8192;

// Per-call configuration of the all-pairs kernels.
struct PairConfig {
  int ipl = 1;    // i-particles per lane
  int split = 1;  // j-range split across workgroups (the ordered kernels)
  int sym = 0;      // 1: the symmetric force kernels (each unordered pair once)
  int sym_vjp = 0;  // 1: the symmetric VJP (FP32C/FP32)
  int sym_vjp64 = 0;  // 1: the symmetric FP64 VJP
  int sym_jerk = 0;  // 1: the symmetric acceleration + jerk (FP32C/FP32)
  int sym_jerk64 = 0;  // 1: the symmetric FP64 acceleration + jerk
  int sym_snap64 = 0;  // 1: the symmetric FP64 acceleration + jerk + snap
  int sym_snap = 0;  // 1: the symmetric acceleration + jerk + snap (FP32C/FP32 only)
  int launches = 0;  // symmetric kernels: least number of launches of the half ring (0 = automatic)
  int rescue = 1;  // FP32C force: recompute rows flagged by the error estimate in FP64
  int sweep = 0;   // adjoint sweep: 0 = recompute overlapped on a second stream where allowed, 1 = one stream
  int ws_slot = 0;  // workspace slot of the all-pairs launchers' scratch (kSweepSlot on the sweep's second stream)
  // Device memory the caller lends for this call's partial sums, staged
  // records and slots.  When set, the all-pairs launchers fit their plans into
  // scratch_bytes and never touch the library workspace (no allocation).
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
};

// `bytes` of scratch for one all-pairs launch: cfg.scratch when the caller lent
// memory (NBODY_EINVAL if it is smaller), else workspace slot cfg.ws_slot.
void* pair_scratch(const PairConfig& cfg, size_t bytes, int* status);

PairConfig choose_config(int64_t n, int precision, int device);
void set_thread_config(const nbody_config& c);
const nbody_config& thread_config();
void record_tuned(int device, int64_t n, int precision, const PairConfig& c);

// ---------------------------------------------------------------- launchers
// Accelerations a(x) into `a` (FP64 SoA).  Uses the workspace for j-split
// partial sums.  Returns NBODY_OK or an error status.
int launch_accel(int64_t n, const double* x, const double* m, double* a, double G, double eps,
                 int precision, bool exclude_self, const PairConfig& cfg, hipStream_t s);

// The same accelerations from the symmetric kernel (FP32C or FP32): every
// unordered pair once, applied to both particles; slot sums in the workspace
// (or in cfg.scratch).  cfg.split > 0: at least that many kernel launches over
// the half ring (0 = as few as the scratch bound allows).
int launch_sym_accel(int64_t n, const double* x, const double* m, double* a, double G, double eps, int precision,
                     bool exclude_self, const PairConfig& cfg, hipStream_t s);

// The same accelerations in FP64 from the symmetric FP64 kernel.
int launch_sym_accel64(int64_t n, const double* x, const double* m, double* a, double G, double eps,
                       bool exclude_self, const PairConfig& cfg, hipStream_t s);

// Acceleration and jerk (Algorithm 3) from the symmetric kernel: each
// unordered pair once, both particles' terms (FP32C or FP32; launches as above).
int launch_sym_jerk(int64_t n, const double* x, const double* v, const double* m, double* a, double* jk, double G,
                    double eps, int precision, bool exclude_self, const PairConfig& cfg, hipStream_t s);

// Acceleration, jerk and snap of a sixth-order Hermite evaluation from the
// symmetric kernel (FP32C or FP32; launches as above).
int launch_sym_snap(int64_t n, const double* x, const double* v, const double* acc, const double* m, double* a,
                    double* jk, double* sn, double G, double eps, int precision, bool exclude_self,
                    const PairConfig& cfg, hipStream_t s);

// The same VJP from the symmetric kernel (FP32C or FP32; launches as above).
int launch_sym_vjp(int64_t n, const double* x, const double* m, const double* w, double* gx, double* gm, double G,
                   double eps, int precision, bool exclude_self, const PairConfig& cfg, hipStream_t s);

// Acceleration and jerk in FP64 from the symmetric FP64 kernel (launches as above).
int launch_sym_jerk64(int64_t n, const double* x, const double* v, const double* m, double* a, double* jk, double G,
                      double eps, bool exclude_self, const PairConfig& cfg, hipStream_t s);

// Acceleration, jerk and snap in FP64 from the symmetric FP64 kernel (launches as above).
int launch_sym_snap64(int64_t n, const double* x, const double* v, const double* acc, const double* m, double* a,
                      double* jk, double* sn, double G, double eps, bool exclude_self, const PairConfig& cfg,
                      hipStream_t s);

// The same VJP in FP64 from the symmetric FP64 kernel (launches as above).
int launch_sym_vjp64(int64_t n, const double* x, const double* m, const double* w, double* gx, double* gm, double G,
                     double eps, const PairConfig& cfg, hipStream_t s);

// (da/dx)^T w into gx and (da/dm)^T w into gm.
int launch_vjp(int64_t n, const double* x, const double* m, const double* w, double* gx,
               double* gm, double G, double eps, int precision, bool exclude_self,
               const PairConfig& cfg, hipStream_t s);

// Acceleration, jerk and snap along paths of constant acceleration acc (the
// evaluation of a sixth-order Hermite step) into a, jk and sn (FP64 SoA).
int launch_accel_jerk_snap(int64_t n, const double* x, const double* v, const double* acc, const double* m,
                           double* a, double* jk, double* sn, double G, double eps, int precision, bool excl,
                           const PairConfig& cfg, hipStream_t s);

// Acceleration and jerk (App. A, Algorithm 3) into a and jk (FP64 SoA).
int launch_accel_jerk(int64_t n, const double* x, const double* v, const double* m, double* a, double* jk, double G,
                      double eps, int precision, bool exclude_self, const PairConfig& cfg, hipStream_t s);

// The fourth-order Hermite loop of nbody_step_hermite.
int run_hermite(int64_t n, double* x, double* v, double* a, double* jk, const double* m, double dt, int64_t nsteps,
                double G, double eps, int precision, bool exclude_self, bool acc_valid, const PairConfig& cfg,
                hipStream_t s);

// The sixth-order Hermite loop of nbody_step_hermite6.
int run_hermite6(int64_t n, double* x, double* v, double* a, double* jk, double* sn, double* cr, const double* m,
                 double dt, int64_t nsteps, double G, double eps, int precision, bool exclude_self, bool acc_valid,
                 const PairConfig& cfg, hipStream_t s);

// FP64 rescue of ill-conditioned FP32C rows: flags the rows whose error
// estimate (the sum of nslices float slices of est, stride apart) is too large
// against |a_i| and recomputes them in FP64 in place in a.  list (n ints) and
// count (one int) are scratch; count must be zero when the flag kernel starts
// (the evaluation's first kernel clears it).
int launch_rescue(int64_t n, const double* x, const double* m, double eps, double G, bool excl, const float* est,
                  int nslices, size_t stride, double* a, int* list, int* count, hipStream_t s);

// FP64 rescue of batched FP32C rows: the rcnt[c] rows of system c listed in
// rlist from the system's first particle on (system-local indices, in any
// order), each recomputed in FP64 over its own system and written to a in
// place (x, a: [3][total], m: [total]; d_off: ncl + 1 system offsets, d_eps:
// ncl softenings, all on the device).  Results do not depend on the lists'
// order.
int launch_ens_rescue(int32_t ncl, const int64_t* d_off, const double* d_eps, int64_t total, const double* x,
                      const double* m, double G, bool excl, const int* rcnt, const int* rlist, double* a,
                      hipStream_t s);

// Elementwise KDK pieces over 3n entries.
int launch_kick(int64_t n3, double* v, const double* a, double h, hipStream_t s);
int launch_kick_drift(int64_t n3, double* x, double* v, const double* a, double h, double dt,
                      int nkicks, hipStream_t s);

// scale * phi_i, phi_i = sum_{j != i} m_j (|d|^2 + eps^2)^-1/2 in FP64, into phi[n].
int launch_potential(int64_t n, const double* x, const double* m, double eps, double scale, double* phi,
                     int split, hipStream_t s);

// Configuration of the batched (ensemble) kernels: mode 0 resident systems,
// 1 resident with split systems, 2 streamed items, 3 per-step wave items, 4
// symmetric per-step items; pass = i-particles per lane per pass of mode 0/1
// (0 = automatic); item = most particles per item of mode 2 (0 = automatic).
struct BatchConfig {
  int mode = 0;
  int pass = 0;
  int item = 0;
  int rescue = 1;  // FP32C, modes 3 and 4: rows flagged by the error estimate recomputed in FP64
};


// nsteps KDK steps of every system of the ensemble with the given kernel configuration.
int run_batched(int32_t ncl, const int64_t* off, const double* eps, double* x, double* v, double* a,
                const double* m, double dt, int64_t nsteps, double G, int precision, bool excl,
                bool acc_valid, const BatchConfig& bc, hipStream_t s);

// Energy/momentum diagnostics into out9 (device).
int launch_energy(int64_t n, const double* x, const double* v, const double* m, double G,
                  double eps, double* out9, hipStream_t s);

// Returns true if any of the n doubles at p is NaN/Inf (synchronises s).
int check_finite(const double* p, int64_t n, hipStream_t s, bool* all_finite);

// The KDK integration loop shared by nbody_step and the adjoint's recompute.
// If traj != nullptr, positions after every step are copied to traj[(k+1)*3n].
int run_kdk(int64_t n, double* x, double* v, double* a, const double* m, double dt,
            int64_t nsteps, double G, double eps, int precision, bool exclude_self,
            bool acc_valid, const PairConfig& cfg, hipStream_t s, double* traj);

}  // namespace nb
