// Definitions shared by the symmetric all-pairs kernels (sym_pairs.hip: the
// FP32C/FP32 acceleration; sym_fp64.hip: the FP64 acceleration; sym_vjp.hip:
// the vector-Jacobian product): block and tile
// sizes, the in-row rotation, the kernel arguments, the half ring of block
// pairs and the slot sums.  Each unordered pair {i, j} is evaluated once and
// its term applied to both particles; the layout is described in sym_pairs.hip.
#pragma once

#include <mutex>

#include "pair_math.h"

namespace nb {
namespace {

constexpr int kSL = 256;            // lanes per workgroup
constexpr int kSI = 2 * kSL;        // particles per I-block / J-block
constexpr int kST = 64;             // j-particles per LDS tile
constexpr int kSR = 16;             // lanes per row = records per sub-block
constexpr int kSTiles = kSI / kST;  // tiles per J-block
constexpr int kSW = kSL / 64;       // waves per workgroup
constexpr int kDiagG = 4;          // lane groups of the block-diagonal kernels, each over kSI / kDiagG of the j
// Workgroups per block of the block-diagonal kernels (each over a slice of the
// j, the slices summed by the slot-sum kernel): several where the blocks are
// too few to fill the chip (eight below 64 blocks, 32768 particles, so that
// those sizes still launch about one workgroup per CU), one where the slices'
// extra sums would only cost memory.
constexpr int kDiagMaxSlices = 8;
inline int diag_slices(int nb) { return nb < 64 ? kDiagMaxSlices : nb < 256 ? 4 : 1; }
static_assert(kSI % (kDiagMaxSlices * kDiagG * 16) == 0, "each diagonal lane group takes whole runs of 16 j");

// v rotated within each row of 16 lanes: lane r gets the value of lane (r - K) mod 16.
template <int K>
__device__ __forceinline__ float row_ror(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x120 + K, 0xF, 0xF, true));
}

// Workgroups go to the chip's 8 XCDs round-robin (workgroup id mod 8), and
// each XCD has its own L2.  This logical index gives each XCD runs of
// kXCDRun consecutive indices (the runs dealt to the XCDs in turn), so that
// the workgroups of neighbouring I-blocks, which read the same J-blocks one
// ring distance apart, share an L2, while every XCD still gets a share of the
// whole grid (whole-grid ranges per XCD leave the XCDs unevenly loaded where
// the half ring ends).  A bijection on [0, grid): the tail past the last whole
// round of runs keeps its index.
constexpr int kXCDs = 8;
constexpr int kXCDRun = 16;
__device__ __forceinline__ int xcd_local_index(int bid, int grid) {
  const int whole = grid / (kXCDs * kXCDRun) * (kXCDs * kXCDRun);
  if (bid >= whole) return bid;
  const int x = bid % kXCDs, k = bid / kXCDs;
  return ((k / kXCDRun) * kXCDs + x) * kXCDRun + k % kXCDRun;
}

// Orders a wave's LDS accesses around a rewrite by other lanes (LDS
// instructions of one wave execute in order; this keeps the compiler from
// moving, merging or dropping reads and writes across the point, which it may
// otherwise do because to it different lanes are different threads).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct SymArgs {
  const double* x;  // [3][n]
  const double* m;  // [n]
  int n;
  int nb;           // blocks of kSI particles
  int npad;         // nb * kSI
  int dmax;         // largest ring distance
  int half;         // nb even: distance dmax only for g < nb / 2
  int d_lo;         // first distance of this chunk
  int T;            // tiles per workgroup (kSTiles per ring distance)
  int nparts;       // workgroups per I-block in this chunk
  double eps;
  float fx;         // repair-radius factor max(kNearX, kNearN n^-1/3)
  const float4* rhi;  // [npad] staged j-records: (x, y, z, m) rounded to FP32
  const float4* rlo;  // [npad] (x, y, z) lo parts and the repair radius^2 (-1 for padding)
  const double* w;  // [3][n] cotangent (VJP) or velocities (acceleration + jerk (+ snap))
  const float4* rw; // [npad] staged cotangents or velocities
  const double* u;  // [3][n] accelerations the particles move with (acceleration + jerk + snap)
  const float4* ru; // [npad] staged accelerations
  float* pj;        // [D][C][npad] j-side tile sums of the chunk's distances (C = 3; 4 for the VJP, 6 for a + jerk, 9 with snap)
  double* pi;       // [nparts][C][npad] i-side sums of the chunk's workgroups
  float* pe;        // [nparts][npad] i-side error estimates of the chunk's workgroups (FP32C force), or null
  float* pw;        // [D][npad] j-side error estimates of the chunk's distances (FP32C force), or null
};

// Largest valid distance + 1 for I-block g.
__device__ __forceinline__ int ring_end(const SymArgs& A, int g) {
  return (A.half && g >= A.nb / 2) ? A.dmax : A.dmax + 1;
}

// Squared repair radius (the near-field rule of the ordered kernel, with its
// n-dependent factor f given): a pair closer than max(f |x|_inf, kNearEps eps)
// to the particle at (xa, ya, za) gets float-float displacements.
__device__ __forceinline__ float sym_rc2(double xa, double ya, double za, double eps, float f) {
  const float dc = fmaxf(f * (float)fmax(fabs(xa), fmax(fabs(ya), fabs(za))), kNearEps * (float)eps);
  return dc * dc + (float)(eps * eps);
}

using lds_ptr = __attribute__((address_space(3))) void*;

// Adds the chunk's slots into the outputs (component c < 3 at out[c n + p],
// 3 <= c < 6 at outm[(c - 3) n + p], c >= 6 at outs[(c - 6) n + p]): the j-side tile sums of distances d_lo .. d_lo + D - 1
// that were evaluated (slots of type S: float, or double for the FP64 kernel),
// then the i-side sums of the chunk's workgroups; the first chunk starts from
// the distance-0 sums pd, the last applies G.  One thread per (particle,
// component), fixed order.  Only the largest distance can be missing for some
// blocks (the opposite block of an even ring, visited from the lower half only).
// With eo (FP32C force only; the thread of component 0 does it): the error
// estimate of the rescue in eo[npad], the far side's shares pw of the chunk's
// distances and the workgroups' i-side shares pe added to what earlier chunks
// left, or to the block-diagonal shares ed in the first chunk.  The
// block-diagonal sums come in pds slices (pd[pds][C][npad], ed[pds][npad]),
// added in slice order.
template <int C, typename S>
__global__ void sym_reduce_kernel(int n, int npad, int nb, int dmax, int half, int d_lo, int D, int nparts,
                                  const S* __restrict__ pj, const double* __restrict__ pi,
                                  const double* __restrict__ pd, double* __restrict__ out, double* __restrict__ outm,
                                  double G, int first, int last, const float* __restrict__ pe = nullptr,
                                  const float* __restrict__ pw = nullptr, const float* __restrict__ ed = nullptr,
                                  float* __restrict__ eo = nullptr, int pds = 1, double* __restrict__ outs = nullptr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (p >= n) return;
  double* o = c < 3 ? out + (size_t)c * n + p : c < 6 ? outm + (size_t)(c - 3) * n + p : outs + (size_t)(c - 6) * n + p;
  const int J = p / kSI;
  double acc = first ? 0.0 : *o;
  if (first)
    for (int k = 0; k < pds; ++k) acc += pd[((size_t)k * C + c) * npad + p];
  const bool est = eo && c == 0;
  float ea = 0.f;
  if (est) {
    if (first)
      for (int k = 0; k < pds; ++k) ea += ed[(size_t)k * npad + p];
    else
      ea = eo[p];
  }
  const int send = min(D, dmax - d_lo + 1);  // slots of this chunk within the ring
  // the last slot of the ring is dropped where its block pair was not evaluated
  const bool drop_last = half && d_lo + send - 1 == dmax && ((J - dmax) % nb + nb) % nb >= nb / 2;
  const int sn = drop_last ? send - 1 : send;
  const S* q = pj + (size_t)c * npad + p;
  const size_t stride = (size_t)C * npad;
  int s = 0;
  for (; s + 4 <= sn; s += 4) {
    const S v0 = q[s * stride], v1 = q[(s + 1) * stride], v2 = q[(s + 2) * stride], v3 = q[(s + 3) * stride];
    acc += (double)v0;
    acc += (double)v1;
    acc += (double)v2;
    acc += (double)v3;
  }
  for (; s < sn; ++s) acc += (double)q[s * stride];
  const double* qi = pi + (size_t)c * npad + p;
  const size_t pstride = (size_t)C * npad;
  int k = 0;
  for (; k + 4 <= nparts; k += 4) {
    const double v0 = qi[k * pstride], v1 = qi[(k + 1) * pstride], v2 = qi[(k + 2) * pstride],
                 v3 = qi[(k + 3) * pstride];
    acc += v0;
    acc += v1;
    acc += v2;
    acc += v3;
  }
  for (; k < nparts; ++k) acc += qi[k * pstride];
  if (est) {
    for (int d = 0; d < sn; ++d) ea += pw[(size_t)d * npad + p];
    for (int k = 0; k < nparts; ++k) ea += pe[(size_t)k * npad + p];
    eo[p] = ea;
  }
  *o = last ? G * acc : acc;
}

}  // namespace

// A second stream per device for the symmetric evaluations: their
// block-diagonal kernel and their slot sums run on it while the caller's
// stream runs the half ring's pair kernels (the slot sums stream HBM, the pair
// kernels are bound by VALU issue), ordered by events.  Created on first use
// outside stream capture (a captured call then records the fork and the join
// into the graph) and kept until nbody_finalize.
struct SideStream {
  hipStream_t side = nullptr;
  hipEvent_t stage = nullptr, pair[2] = {nullptr, nullptr}, red[2] = {nullptr, nullptr}, join = nullptr;
};

// The current device's side stream, with lk (the side streams' mutex, which
// keeps one call's records and waits together) locked; or nullptr, lk
// unlocked, where there is none: the caller then runs on its own stream.
SideStream* acquire_side_stream(hipStream_t s, std::unique_lock<std::mutex>& lk);

// The launches of one symmetric evaluation after its staging kernel on s:
// diag(stream) launches the block-diagonal kernel, pair(c, b) the pair kernel
// of half-ring chunk c on s, writing slot set b = c % nbuf, and sum(c, b,
// stream) that chunk's slot sum.  Without a side stream everything runs on s
// in that order.  With one, the diagonal kernel waits for the staging and the
// slot sums run after it on the side stream, each after its pair kernel; a
// pair kernel that reuses a slot set waits for the slot sum that last read
// it, and s waits for the last slot sum before it goes on.
template <class Diag, class Pair, class Sum>
int run_sym_chunks(SideStream* side, hipStream_t s, int nchunks, int nbuf, Diag diag, Pair pair, Sum sum) {
  auto ok = [](hipError_t e, const char* what) { return e == hipSuccess ? NBODY_OK : hip_fail(e, what); };
  int st = NBODY_OK;
  const hipStream_t rs = side ? side->side : s;
  if (side && ((st = ok(hipEventRecord(side->stage, s), "hipEventRecord")) ||
               (st = ok(hipStreamWaitEvent(rs, side->stage, 0), "hipStreamWaitEvent"))))
    return st;
  if ((st = diag(rs))) return st;
  for (int c = 0; c < nchunks; ++c) {
    const int b = c % nbuf;
    if (side && c >= nbuf && (st = ok(hipStreamWaitEvent(s, side->red[b], 0), "hipStreamWaitEvent"))) return st;
    if ((st = pair(c, b))) return st;
    if (side && ((st = ok(hipEventRecord(side->pair[b], s), "hipEventRecord")) ||
                 (st = ok(hipStreamWaitEvent(rs, side->pair[b], 0), "hipStreamWaitEvent"))))
      return st;
    if ((st = sum(c, b, rs))) return st;
    if (side && (st = ok(hipEventRecord(side->red[b], rs), "hipEventRecord"))) return st;
  }
  if (side && ((st = ok(hipEventRecord(side->join, rs), "hipEventRecord")) ||
               (st = ok(hipStreamWaitEvent(s, side->join, 0), "hipStreamWaitEvent"))))
    return st;
  return NBODY_OK;
}

// Chunking of the half ring for n particles, with slot_bytes bytes of j-side
// sums (sum_bytes of them the sums themselves, the rest error estimates) per
// particle and distance, part_bytes of i-side sums per particle and workgroup
// of a block, and fixed_bytes per particle of staged records and
// block-diagonal sums: tiles per workgroup (T: whole distances of kSTiles
// tiles, or for small rings a part of one) and distances per launch (D), the
// sum slots of a launch kept near 1 GiB and the whole layout within budget
// bytes; launches > 0 asks for at least that many launches.  Returns the bytes
// the layout needs, which exceed budget only if one distance per launch does
// not fit.
inline size_t sym_plan(int64_t n, int launches, int slot_bytes, int sum_bytes, int part_bytes, int fixed_bytes,
                       size_t budget, int* nb_out, int* T_out, int* D_out) {
  const int nb = (int)((n + kSI - 1) / kSI);
  const int dmax = nb / 2;
  const int64_t npad = (int64_t)nb * kSI;
  int64_t dcap = std::max<int64_t>(1, (int64_t(1) << 30) / (sum_bytes * npad));
  if (launches > 0) dcap = std::min<int64_t>(dcap, std::max(1, (dmax + launches - 1) / launches));
  int d0 = (int)std::max<int64_t>(1, std::min<int64_t>(dmax, dcap));
  int T = kSTiles, D = 1;
  size_t need = 0;
  for (;;) {
    // whole distances per workgroup (at most 16), as many as still leave
    // `want` workgroups per launch (several rounds of 6-7 per CU); one while
    // that leaves ~4096; below that 2 or 4 tiles each.  A launch that covers
    // the whole half ring (small rings) wants ~8192: 8192 workgroups of one or
    // four distances beat 4096 of two or eight by 2-3 % at 65536 and 131072
    // particles, while halving the tiles of one distance to reach 8192 lost
    // 0.3-1.2 % at 49152, and fewer, longer workgroups lost more; the chunked
    // launches of large rings keep ~4096 (16 distances per workgroup at 2^20)
    const int64_t bp = (int64_t)nb * d0;  // block pairs of whole distances
    const int64_t want = d0 == dmax ? 8192 : 4096;
    if (bp >= want) {
      const int L = (int)std::min<int64_t>(std::min(16, d0), bp / want);
      T = L * kSTiles;
      D = (d0 + L - 1) / L * L;
    } else if (bp >= 4096) {
      T = kSTiles;
      D = d0;
    } else {
      T = bp * kSTiles / 4096 >= 4 ? 4 : 2;
      D = d0;
    }
    need = (size_t)npad * ((size_t)fixed_bytes + (size_t)D * slot_bytes + (size_t)(D * kSTiles / T) * part_bytes);
    if (need <= budget || d0 == 1) break;
    d0 = std::max(1, d0 - std::max(1, d0 / 8));
  }
  *nb_out = nb;
  *T_out = T;
  *D_out = D;
  return need;
}

}  // namespace nb
