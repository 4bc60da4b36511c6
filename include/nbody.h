/*
 * nbody.h -- C ABI of libnbody_accel.so: softened O(N^2) direct-summation
 * gravity on one AMD Instinct MI355X (gfx950), with a kick-drift-kick
 * integrator, energy/momentum diagnostics, a batched ensemble integrator and
 * the adjoint (reverse-mode) of the integrated trajectory.
 *
 * What is computed (paper: "Assessing Performance and Porting Strategies for
 * Gravitational N-Body Simulations on the RISC-V-Based Tenstorrent Wormhole"):
 *   a_i = G * sum_{j != i} m_j (x_j - x_i) / (|x_j - x_i|^2 + eps^2)^(3/2)
 * which is the force of Eq. (1) (Sec. 2.1) divided by m_i, with the softening
 * parameter of App. A entering the squared distance.  The pair arithmetic
 * follows App. A, Algorithm 3 (displacement, squared distance, inverse square
 * root, its cube, weight times cube, accumulate); the weight p_w,j is G m_j.
 * The accelerator computes only the pairwise evaluation and the rest stays in
 * FP64 (Sec. 3.1); here that rest (state update, diagnostics) also stays on
 * the GPU, in FP64.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers (hipMalloc / torch CUDA tensors) on
 *     the current HIP device, owned by the caller, contiguous, 8-byte aligned,
 *     float64.  Vectors are SoA: v[c*n + i] for component c = 0 (x), 1 (y),
 *     2 (z) of particle i; masses m[i].  Pointers marked "host" are ordinary
 *     host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     work is enqueued on it and the call returns without waiting, unless a
 *     function says otherwise.  Outputs are valid once the stream reaches the
 *     enqueued work.
 *   - Arguments are validated before anything is enqueued; on a negative
 *     status nothing was launched and no output was touched (except where a
 *     function says so).  nbody_last_error() then returns a message.
 *   - The library keeps one scratch workspace per device.  It grows on demand
 *     (hipMalloc, which may synchronise the device) and is released by
 *     nbody_finalize().  Calls that share a device share that workspace, so
 *     calls enqueued on different streams of one device must not overlap.
 *   - Results are deterministic: the same inputs and configuration give
 *     bitwise-identical outputs (no floating-point atomics anywhere).
 */
#ifndef NBODY_H
#define NBODY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes returned by every entry point. */
typedef enum {
  NBODY_OK = 0,
  NBODY_EINVAL = -1,       /* bad argument (null pointer, n < 0, eps < 0, ...) */
  NBODY_EHIP = -2,         /* a HIP runtime call or kernel launch failed */
  NBODY_ENOMEM = -3,       /* workspace allocation failed */
  NBODY_ENONFINITE = -4,   /* NBODY_CHECK_FINITE found NaN/Inf in an output */
  NBODY_EUNSUPPORTED = -5  /* valid request the library cannot serve */
} nbody_status;

/* Arithmetic of the pair evaluation.  The particle state, the integrator and
 * the diagnostics are FP64 in every mode. */
typedef enum {
  NBODY_FP64 = 0,   /* all pair arithmetic in FP64 (the plain FP64 path) */
  NBODY_FP32C = 1,  /* FP32 pairs on float-float (hi+lo) positions, so the
                       displacement x_j - x_i keeps FP64-level accuracy;
                       compensated (TwoSum) accumulation of the j-sum */
  NBODY_FP32 = 2    /* FP32 pairs on positions rounded to FP32; same
                       compensated accumulation (faster, less accurate for
                       close pairs far from the origin) */
} nbody_precision;

/* Bits of nbody_params.flags. */
enum {
  NBODY_EXCLUDE_SELF = 1,  /* mask j == i explicitly; required when eps == 0
                              (with eps > 0 the self term is exactly zero) */
  NBODY_CHECK_FINITE = 2,  /* after the call, wait for the stream and return
                              NBODY_ENONFINITE if an output holds NaN/Inf */
  NBODY_ACC_VALID = 4      /* nbody_step / nbody_step_batched: `a` already
                              holds a(x) on entry, skip the initial evaluation */
};

typedef struct nbody_params {
  double G;           /* gravitational constant (Eq. (1)); any finite value */
  double eps;         /* Plummer softening length, >= 0 (App. A) */
  int32_t precision;  /* an nbody_precision value */
  uint32_t flags;     /* OR of the flag bits above */
} nbody_params;

/* Accelerations a (3*n) of particles at x (3*n) with masses m (n).
 * Eq. (1) of Sec. 2.1 divided by m_i, softened as in App. A.
 * From 49152 particles on in FP32C and FP32, from 8192 in FP64 (or as
 * nbody_config.pairs says), each unordered pair is evaluated once and applied
 * to both particles, with sums in a fixed order; this uses a workspace of up
 * to about 4 GiB (staged records and two sets of per-distance sums) and
 * several launches per call: when the half ring takes several launches, each
 * one's per-distance sums are added on a second stream of the library's while
 * the next launch runs, and the caller's stream waits for that stream before
 * the call's last kernel (a captured call records both streams' work).
 * n == 0 is a no-op.  x, m, a must not alias.  Errors: NBODY_EINVAL for null
 * pointers with n > 0, n < 0, n > 2^29, eps < 0, eps == 0 without
 * NBODY_EXCLUDE_SELF, non-finite G, unknown precision; NBODY_ENOMEM if the
 * workspace cannot grow. */
int nbody_accel(int64_t n, const double* x, const double* m, double* a,
                const nbody_params* p, void* stream);

/* For callers that cannot allocate memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The accelerations of
 * nbody_accel (same arguments, same kernels and the same accuracy), with every
 * scratch byte (staged records, partial and per-distance sums) taken from one
 * fixed device array of NBODY_NOALLOC_SCRATCH_BYTES (256 MiB) that the library
 * holds on each GPU it runs on until the process ends.  The call never
 * allocates or frees memory and never synchronises.  The symmetric path fits
 * its half ring into that array, in more launches than nbody_accel uses at the
 * largest sizes (its sums then run in another order: results agree with
 * nbody_accel to the precision's tolerance, not bitwise).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (nothing in it needs to start at zero): calls that overlap on one GPU
 * (on different streams, or from different threads) race and must not be
 * issued.
 * Errors: as nbody_accel; NBODY_EINVAL also for n > NBODY_NOALLOC_MAX_N (2^21)
 * and for NBODY_CHECK_FINITE (which waits for the stream). */
enum { NBODY_NOALLOC_SCRATCH_BYTES = 268435456, NBODY_NOALLOC_MAX_N = 2097152 };
int nbody_accel_noalloc(int64_t n, const double* x, const double* m, double* a, const nbody_params* p,
                        void* stream);

/* nsteps kick-drift-kick leapfrog steps of size dt, in place on x, v, a:
 *   v += dt/2 a(x);  x += dt v;  a = a(x);  v += dt/2 a
 * (the workloads' integrator; the paper's Sec. 2.1 predict-evaluate-correct
 * loop has the same structure of one all-pairs evaluation per step).
 * On entry a must hold a(x) if NBODY_ACC_VALID is set, otherwise it is
 * computed first; on return a = a(x_final), so consecutive calls chain and
 * S steps in one call equal S1 + S2 steps in two calls bitwise.
 * nsteps == 0 only (re)computes a unless NBODY_ACC_VALID is set.
 * Errors: as nbody_accel, plus non-finite dt or nsteps < 0. */
int nbody_step(int64_t n, double* x, double* v, double* a, const double* m, double dt,
               int64_t nsteps, const nbody_params* p, void* stream);

/* Diagnostics of the state (x, v, m), always in FP64, written to the device
 * array out9 = {K, W, E, Px, Py, Pz, Lx, Ly, Lz}:
 *   K = 1/2 sum m_i |v_i|^2,  W = -G sum_{i<j} m_i m_j / sqrt(|d_ij|^2 + eps^2)
 *   (the self pair is always excluded), E = K + W, P = sum m v, L = sum m x x v.
 * These are the energies compared in Sec. 4.1 (Fig. 4) and the conserved
 * quantities of the integrator.  p->precision is ignored.  eps == 0 is
 * allowed (the self pair is excluded by index). */
int nbody_energy(int64_t n, const double* x, const double* v, const double* m,
                 const nbody_params* p, double* out9, void* stream);

/* Per-particle softened potential, always in FP64 (p->precision is not used):
 *   phi_i = -G sum_{j != i} m_j / (|x_j - x_i|^2 + eps^2)^(1/2),
 * the self pair excluded by index (so eps = 0 needs no flag).  With it the
 * specific energy of particle i is |v_i|^2/2 + phi_i: the per-particle energy
 * distribution that Sec. 4.1 (Fig. 4) compares between the accelerated run
 * and the double-precision reference; sum_i m_i phi_i = 2 W of nbody_energy.
 * x: [3][n], m: [n], phi: [n] FP64 device memory, caller-owned; phi must not
 * alias x or m.  Errors: as nbody_accel (NBODY_ENONFINITE with
 * NBODY_CHECK_FINITE). */
int nbody_potential(int64_t n, const double* x, const double* m, double* phi, const nbody_params* p,
                    void* stream);

/* Vector-Jacobian products of the acceleration map at (x, m) with cotangent
 * w (3*n), obtained by differentiating Eq. (1) / m_i term by term:
 *   gx_k = G sum_{j != k} K(d_kj) (m_k w_j - m_j w_k),
 *   gm_k = -G sum_{j != k} s_kj^(-3/2) (d_kj . w_j),
 *   d_kj = x_j - x_k, s = |d|^2 + eps^2, K(d) = s^(-3/2) I - 3 s^(-5/2) d d^T.
 * Outputs gx (3*n) and gm (n) are overwritten.  Pair arithmetic follows
 * p->precision (FP32C/FP32 use FP32 pairs with compensated sums).  From 12288
 * particles in FP32C/FP32 and from 8192 in FP64 (or as nbody_config.pairs
 * says) each unordered pair is evaluated once and serves both particles (the
 * pair term changes sign when k and j swap), with sums in a fixed order; the
 * own pair is then always left out (its term is zero for eps > 0).
 * Errors: as nbody_accel. */
int nbody_accel_vjp(int64_t n, const double* x, const double* m, const double* w,
                    double* gx, double* gm, const nbody_params* p, void* stream);

/* Reverse-mode derivative of `nsteps` KDK steps from (x0, v0) (the map of
 * nbody_step starting without NBODY_ACC_VALID), using checkpoints.  The
 * paper defines no adjoint: this is the exact derivative of the workloads'
 * integrator, built from the pairwise VJP above.
 *   ckpt_x, ckpt_v: [nckpt][3][n] states at steps 0, every, 2*every, ...,
 *                   nckpt = ceil(nsteps / every); checkpoint 0 is (x0, v0).
 *   gxT, gvT:       cotangents of the final positions and velocities (3*n).
 *   gx0, gv0, gm:   outputs, cotangents of x0, v0 (3*n) and m (n).
 * Each segment is recomputed forward from its checkpoint with the same kernels
 * as nbody_step (bitwise the same trajectory), then swept in reverse; the two
 * Jacobian products at each interior position share one cotangent and are
 * merged into one VJP evaluation per step.  Inputs are not modified.
 * The checkpoints may come from a forward pass in another precision than
 * p->precision: with FP64 checkpoints and an FP32C sweep, each segment's
 * FP32C recompute restarts from an FP64 state, and the result is the
 * gradient of the FP64 trajectory to FP32C accuracy.
 * With more than one segment and n <= 65536 (nbody_config.sweep 0) the
 * recompute of the next segment runs on a second stream that the library
 * owns, ordered against `stream` by events and joined back into it before
 * the call returns (a captured call records the fork and the join); it uses
 * a second trajectory buffer and workspace of its own, so the call needs
 * about twice the memory of a one-stream sweep.  The result is bitwise the
 * same either way.
 * Errors: as nbody_step, plus every < 1. */
int nbody_traj_grad(int64_t n, const double* ckpt_x, const double* ckpt_v, int64_t every,
                    int64_t nsteps, const double* m, double dt, const double* gxT,
                    const double* gvT, double* gx0, double* gv0, double* gm,
                    const nbody_params* p, void* stream);

/* Batched ensemble (the workloads' ensemble of independent clusters; the
 * paper defines no such call): ncl independent systems concatenated along the
 * particle axis; system c owns columns [off[c], off[c+1]) of x, v, a (each
 * 3*total, SoA over the whole concatenation, total = off[ncl]) and m (total),
 * and has softening eps[c].  Each system advances nsteps KDK steps exactly as
 * nbody_step would advance it alone (same pair arithmetic, FP64 state).  By
 * default (nbody_config.bsplit and friends all zero, no tuned choice) every
 * step is a few launches over items of 64 particles of all systems: two per
 * step (mode 3: kicks and records, then forces), or three for FP32C/FP32
 * layouts whose systems span several blocks of 64 (mode 4: each unordered
 * pair of a system once, then a fixed-order sum of the far-side terms), and
 * one more with the FP32C rescue (the FP64 rows); the steps of a call may be
 * captured into a HIP graph.  All systems and all
 * steps run inside ONE persistent kernel launch in modes 0-2 (bsplit 0, 1, 2
 * or nbody_tune_batched with allow_cooperative).  off (ncl+1, int64,
 * off[0] == 0, non-decreasing) and eps (ncl) are HOST arrays; the work plan
 * built from them is cached, so a repeated call with the same layout enqueues
 * only the launches.  Systems of up to 2^24 particles are served by modes 2-4;
 * the resident kernel (modes 0 and 1) returns NBODY_EUNSUPPORTED for a system
 * of more than 4096.  In mode 1 the largest systems are split over up to 4
 * workgroups that exchange their positions through global memory every step,
 * and mode 2 synchronises the items of a system every step the same way; if
 * such an exchange ever waits more than about a second (the GPU shared with
 * other work), that system's x, v and a are set to NaN rather than hanging,
 * which NBODY_CHECK_FINITE reports.  p->eps is ignored; p->precision must be
 * NBODY_FP32C, NBODY_FP32 or NBODY_FP64. */
int nbody_step_batched(int32_t ncl, const int64_t* off, const double* eps, double* x,
                       double* v, double* a, const double* m, double dt, int64_t nsteps,
                       const nbody_params* p, void* stream);

/* Accelerations a (3*n) and jerks jk (3*n) of particles at x (3*n) with
 * velocities v (3*n) and masses m (n): App. A, Algorithm 3 in full,
 *   a_i  = G sum_{j != i} m_j r_ij / r^3,
 *   jk_i = G sum_{j != i} m_j [ v_ij - 3 (r_ij . v_ij) r_ij / r^2 ] / r^3,
 * r_ij = x_j - x_i, v_ij = v_j - v_i, r^2 = |r_ij|^2 + eps^2 (the time
 * derivative of the softened acceleration along the motion).  FP32C rounds
 * positions to FP32 and gives the pairs closer than the near-field radius
 * float-float displacements (as nbody_accel), with FP32 velocities.  From
 * 12288 particles in FP32C and FP32 and from 8192 in FP64 (or as
 * nbody_config.pairs says) each
 * unordered pair is evaluated once and applied to both particles (the jerk
 * term, like the acceleration, changes sign when i and j swap), summed in a
 * fixed order, with a workspace of per-distance sums as nbody_accel's.
 * Errors: as nbody_accel; a and jk must be distinct from each other and the
 * inputs. */
int nbody_accel_jerk(int64_t n, const double* x, const double* v, const double* m, double* a, double* jk,
                     const nbody_params* p, void* stream);

/* nsteps fourth-order Hermite predictor-evaluator-corrector steps with a
 * shared step dt (the integrator family of Sec. 2.1: predict positions and
 * velocities from a and its derivative, evaluate acceleration and jerk,
 * correct), in place on x, v, a, jk:
 *   predict  xp = x + v dt + a dt^2/2 + jk dt^3/6,  vp = v + a dt + jk dt^2/2
 *   evaluate (a1, jk1) at (xp, vp)
 *   correct  v' = v + (a + a1) dt/2 + (jk - jk1) dt^2/12,
 *            x' = x + (v + v') dt/2 + (a - a1) dt^2/12.
 * NBODY_ACC_VALID means a and jk already hold the evaluation at (x, v).
 * Errors: as nbody_step. */
int nbody_step_hermite(int64_t n, double* x, double* v, double* a, double* jk, const double* m, double dt,
                       int64_t nsteps, const nbody_params* p, void* stream);

/* Acceleration, jerk and snap of n particles at positions x, velocities v and
 * accelerations acc (all [3][n] SoA), the evaluation of a sixth-order Hermite
 * step (Sec. 2.1; the scheme of Nitadori & Makino 2008 that the paper cites):
 * along paths x_k(t) = x_k + v_k t + acc_k t^2/2, with d = x_j - x_i,
 * w = v_j - v_i, u = acc_j - acc_i, s = |d|^2 + eps^2, t_j = m_j s^-3/2,
 * alpha = (d.w)/s and beta = (w.w + d.u)/s + alpha^2,
 *   a_i  = G sum_j t_j d
 *   jk_i = G sum_j (t_j w - 3 alpha t_j d)            (as Algorithm 3)
 *   sn_i = G sum_j (t_j u - 6 alpha P' - 3 beta t_j d), P' the jerk term.
 * acc is an input: the snap takes the accelerations the particles move with
 * (in a Hermite step, the predicted ones).  Outputs a, jk, sn: [3][n] FP64,
 * caller-owned, distinct from each other and the inputs.  FP32C evaluates
 * pairs with FP32-rounded positions (float-float displacements for the pairs
 * closer than the near-field radius, as nbody_accel) and FP32 velocity and
 * acceleration differences.  From 8192 particles in every precision (or as
 * nbody_config.pairs says) each unordered pair is evaluated once and applied
 * to both particles (every term changes sign when i and j swap), summed in a
 * fixed order.  Errors: as nbody_accel_jerk. */
int nbody_accel_jerk_snap(int64_t n, const double* x, const double* v, const double* acc, const double* m,
                          double* a, double* jk, double* sn, const nbody_params* p, void* stream);

/* nsteps sixth-order Hermite predictor-evaluator-corrector steps with a
 * shared step h = dt (Sec. 2.1), in place on x, v and the state a, jk, sn, cr
 * (acceleration, jerk, snap and crackle, each [3][n] FP64):
 *   predict  xp = x + v h + a h^2/2 + jk h^3/6 + sn h^4/24 + cr h^5/120
 *            vp = v + a h + jk h^2/2 + sn h^3/6 + cr h^4/24
 *            ap = a + jk h + sn h^2/2 + cr h^3/6
 *   evaluate (a1, jk1, sn1) at (xp, vp, ap) with nbody_accel_jerk_snap
 *   correct  v' = v + (a + a1) h/2 - (jk1 - jk) h^2/10 + (sn + sn1) h^3/120
 *            x' = x + (v + v') h/2 - (a1 - a) h^2/10 + (jk + jk1) h^3/120
 *   crackle  cr' = 60 A - 36 B + 9 C, the third derivative at the step's end of
 *            the quintic through (a, jk, sn) at both ends, with
 *            A = (a1 - a - jk h - sn h^2/2)/h^3, B = (jk1 - jk - sn h)/h^2,
 *            C = (sn1 - sn)/h.
 * Without NBODY_ACC_VALID the call first evaluates a, jk at (x, v), then
 * a, jk, sn at (x, v, a), and sets cr = 0; with it, a, jk, sn, cr hold the
 * state a previous call left (so that calls resume bitwise).
 * Errors: as nbody_step, and NBODY_EINVAL for dt = 0 (the crackle divides
 * by the step); the six arrays must be distinct. */
int nbody_step_hermite6(int64_t n, double* x, double* v, double* a, double* jk, double* sn, double* cr,
                        const double* m, double dt, int64_t nsteps, const nbody_params* p, void* stream);

/* Tile configuration of the all-pairs kernels (see nbody_set_config). */
typedef struct nbody_config {
  int32_t ipl;     /* i-particles per lane: 1, 2 or 4 */
  int32_t split;   /* j-range split across workgroups: 0 = automatic, else 1..1024;
                      with the symmetric force kernel (pairs), the least number of
                      launches its half ring of block pairs is cut into */
  int32_t bsplit;  /* batched kernel, used when any of bsplit, bpass, bitem is
                      non-zero (all zero: the tuned choice for the layout, else
                      mode 4 for FP32C and FP32 when the layout's block pairs
                      outnumber its blocks of 64, else mode 3): 0 = one workgroup per system, its records
                      resident in LDS (force it with bpass); 1 = as 0, but systems costlier than
                      the per-CU average split across up to 4 workgroups that
                      exchange positions every step; 2 = streamed: every system cut
                      into items (see bitem) evaluated by 1024-lane workgroups
                      resident for all steps, records streamed through LDS, the
                      items of a system synchronised every step; 3 = the items of
                      64 particles of mode 2, with two launches per step (kicks and
                      drift, then the forces) instead of one persistent launch;
                      4 = as 3, but each unordered pair of a system evaluated once
                      (Eq. 1's antisymmetry: an item's block of 64 meets its own
                      block and half of its system's other blocks, and the terms
                      of the far side are added per particle in FP64 in a fixed
                      order by a third launch per step, and with the FP32C rescue
                      a fourth recomputes the flagged rows); FP32C and FP32 only
                      (FP64 runs mode 3), and layouts whose per-distance sums would
                      exceed 1 GiB (about 3 x sum of N_c^2 / 128 floats) run mode 3.
                      Modes 1 and 2 need every workgroup of the launch resident at
                      once: with another kernel occupying the GPU a bounded wait can
                      expire, and the affected systems then end NaN.  Modes 0 and 3
                      have no such requirement, nor has 4. */
  int32_t bpass;   /* batched kernel: i-particles per lane evaluated together in one
                      pass over a system's records: 0 = automatic (4), or 1, 2, 4 */
  int32_t bitem;   /* streamed batched kernel (bsplit = 2): 64 (or 0 = automatic):
                      items of 64 particles of any system, each evaluated by one
                      wave against the system's whole j-range; or 256, 512, 1024:
                      most particles per item of a system above 256 particles,
                      evaluated by a whole workgroup */
  int32_t pairs;   /* form of the force kernel of nbody_accel and of the KDK
                      steps, of nbody_accel_vjp and the adjoint sweep, of
                      nbody_accel_jerk, nbody_accel_jerk_snap and the Hermite
                      steps:
                      0 = automatic (the tuned choice for (n, precision),
                      else symmetric from 49152 particles on in FP32C/FP32
                      and from 8192 in FP64 for the force, from 12288 in
                      FP32C/FP32 and 8192 in FP64 for the VJP and for
                      acceleration + jerk, from 8192 in every precision for
                      acceleration + jerk + snap),
                      1 = ordered: every ordered pair evaluated for its i;
                      2 = symmetric: every unordered pair evaluated once and
                      applied to both particles (a_j gets the opposite of i's
                      term scaled by m_i / m_j), results summed in a fixed order
                      (reproducible), at the cost of a workspace of about
                      4 GiB for large n and, in FP32C/FP32, an FP32 sum of up
                      to 512 terms per j before the FP64 sums */
  int32_t rescue;  /* FP32C force of nbody_accel, nbody_accel_noalloc, the
                      KDK steps of nbody_step and of the adjoint's recompute,
                      and of nbody_step_batched with the per-step items of 64
                      (modes 3 and 4): 0 = automatic (on where the kernels
                      carry it), 1 = on (batched modes 0-2 then return
                      NBODY_EUNSUPPORTED), 2 = off.  On: while summing, the
                      kernels estimate each row's FP32 rounding error (per
                      block of terms summed in FP32: the magnitude of the
                      block's partial sum, weighted by the distance of its
                      closest pair left in rounded positions; blocks combined
                      as independent errors), and rows whose estimate exceeds
                      4e-6 |a_i| (rows whose terms cancel strongly) are
                      recomputed in FP64; this keeps such rows inside the 1e-5
                      FP32C bound at the cost of one FP64 row evaluation each
                      (0.12 % of the rows of the 2^20 two-component model). */
  int32_t sweep;   /* reverse sweep of nbody_traj_grad: 0 = automatic (with more
                      than one segment, n <= 65536 and the symmetric kernels'
                      launches left automatic, the trajectory of the next
                      segment is recomputed on a second stream of the library,
                      with its own workspace, while the caller's stream runs
                      the adjoint steps of the current one: at such sizes
                      neither fills the GPU alone), 1 = everything on the
                      caller's stream.  Both give bitwise the same result. */
} nbody_config;

/* Force a tile configuration for subsequent calls on this thread (all zeros
 * restores the automatic choice); like the tuners, a tool of this library,
 * not a call the paper defines.  A batched plan is built with the bsplit
 * value in force when its layout is first seen.  Errors: NBODY_EINVAL for
 * values outside the lists above. */
int nbody_set_config(const nbody_config* cfg);

/* Autotuner (a tool of this library; the paper defines no tuner): for a
 * system of n particles and the given precision, time every supported tile
 * configuration of the force kernel with HIP events on a synthetic input
 * (synchronous; allocates and frees its own buffers) and record the fastest
 * in the library's per-device table, which automatic selection then uses for
 * that (n, precision).  The choice is per (n, precision) because the fastest
 * tiling depends on both, hence those arguments.  If cache_path is non-NULL
 * the table is also appended there as one JSON object per line.  best (host,
 * may be NULL) receives the chosen configuration. */
int nbody_tune(int64_t n, int32_t precision, const char* cache_path, nbody_config* best);

/* Autotuner of the batched kernels (a tool of this library, like
 * nbody_tune) for one ensemble layout (off, eps as in
 * nbody_step_batched, precision and flags from p): times every candidate
 * configuration for nsteps (>= 1) KDK steps, after an untimed run of nsteps
 * steps, from the state (x, v, m), on the
 * library's own copies (the caller's arrays are only read), and keeps the
 * fastest whose state stays finite.  Candidates: the resident kernel with 1, 2
 * or 4 i-particles per lane per pass, the per-step items of 64 (mode 3) and,
 * for FP32C and FP32, their symmetric form (mode 4); with allow_cooperative != 0 also the
 * split mode and the streamed kernel with items of 64, 256, 512 or 1024 particles
 * (the modes that need every workgroup of a launch resident at once). allow_cooperative = 2 keeps
 * to the single-launch modes 0, 1 and 2 (all steps in one persistent launch).
 * FP32C with the rescue on (nbody_config.rescue 0 or 1) has two candidates, the
 * per-step items of 64 (modes 3 and 4), the batched forms that carry it; the
 * single-launch search (allow_cooperative = 2) then goes without the rescue,
 * or returns NBODY_EUNSUPPORTED if the rescue was asked for explicitly.  The
 * choice is recorded for this (device, precision, rescue, layout): later
 * nbody_step_batched calls on the same layout use it whenever the thread has
 * not forced a batched configuration with nbody_set_config.  best (may be
 * NULL) receives it as bsplit/bpass/bitem.  Candidates that cannot serve the
 * layout (the resident kernel with a system above 4096 particles) are skipped.
 * Synchronous; allocates and frees
 * its own buffers and builds (and caches) one plan per candidate.  Errors: as
 * nbody_step_batched; NBODY_EINVAL for allow_cooperative outside 0..2;
 * NBODY_ENONFINITE if no candidate stayed finite. */
int nbody_tune_batched(int32_t ncl, const int64_t* off, const double* eps, const double* x, const double* v,
                       const double* m, double dt, int64_t nsteps, int32_t allow_cooperative,
                       const nbody_params* p, nbody_config* best);

/* Message describing the last non-OK status returned on this thread. */
const char* nbody_last_error(void);

/* Waits for the work of every device the library has run on, then releases
 * its per-device workspaces, batched plans and batched tuned choices and its
 * own second streams.  Later calls build again what they need (results are
 * bitwise as before).  Not to be called while another thread is inside the
 * library. */
int nbody_finalize(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int nbody_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
