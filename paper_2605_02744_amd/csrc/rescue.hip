// Rescue of ill-conditioned rows of the FP32C force.
//
// An FP32C row a_i is a sum of FP32 pair terms, each carrying a relative
// rounding error of a few u (u = 2^-24): the inverse square root, its cube,
// the weight and the products, and, for pairs outside the near-field radius,
// the rounding of both positions to FP32, which moves the displacement by up
// to about u (|x_i| + |x_j|).  Where the terms of a row cancel (|a_i| much
// smaller than the sum of their magnitudes, e.g. particles near the centre of
// a cluster) those errors are large relative to |a_i|; the largest come from
// strong pairs just outside the near-field radius, whose terms keep the
// rounding of both positions.  The pair kernels keep a cheap estimate of each
// row's error: for every block of terms they sum in FP32 (64 terms of the
// row's own j-loop, or, for the far side of the symmetric kernels, one slot of
// up to 512 terms) they add the square of the block's partial sum |P_b|,
// weighted by 1 + kEstNear |x_i|_inf / d_b, d_b the smallest softened distance
// of a pair of that block that was not repaired with float-float
// displacements (for a far-side slot, a lower bound of it: the smallest such
// distance among all pairs of the tile of 64 j the slot belongs to):
//   E_i = sum_b ((1 + kEstNear |x_i| / d_b) |P_b|)^2 .
// The rounding error of a block's sum grows like the magnitude of its partial
// sum both when one term dominates the block and when its terms have random
// directions (both the sum and the error then grow like the square root of the
// number of terms), the distance factor prices the position rounding of the
// block's closest pair, and the errors of different blocks (different j,
// different roundings) add like independent variables, hence the root of the
// sum of squares.  A row is recomputed in FP64 when
//   kEstC u |G| sqrt(E_i) > kRescueTol |a_i| .
// kEstC and kRescueTol were set against measured errors: over half a million
// rows of Plummer spheres (512 to 2^20 particles, softenings down to
// 6.25e-4) and the two-component model, the estimate exceeded the actual
// error of FP32C (without rescue, against FP64) by 4 to 10 at the median and
// the row left unflagged with the largest error stayed at 2.7e-6, against 4e-5
// for the largest error without rescue.  With the far side's per-tile bound,
// 610 000 rows of Plummer spheres (4096 to 262144 particles, softenings
// 6.25e-4 to 1e-3, symmetric kernel) left 2.3e-6 as the largest unflagged
// error with 0.86 % of the rows recomputed; 0.12 % of the rows of the 2^20
// two-component model are.  The estimate misses cancellation that is
// systematic inside one block of consecutive indices (terms of a block that
// cancel each other more than random directions do).
//
// Here, for the force of one system: the flagged rows go to a list (an atomic
// counter, one add per wave, orders them, which does not change any result:
// every row is recomputed on its own, in a fixed order) and a grid-stride
// kernel recomputes them in FP64.  The count of flagged rows is cleared by the
// first kernel of the evaluation (its block 0, thread 0), so that the flag
// kernel starts from zero without a launch of its own.  The batched wave items
// (ensemble_stream.hip) flag their rows in the force kernel, where each wave
// holds whole rows, into per-system lists that their own rescue kernel reads.
#include "pair_math.h"

namespace nb {
namespace {

constexpr int64_t kRSmall = 131072;  // systems up to this size take one row per workgroup pass

// One thread per particle: sums the nslices slices of the estimate (stride
// apart) and appends the row to the list if scale * sqrt(E_i) > |a_i|.  A
// wave reserves the places of all its flagged rows with one atomic add.
__global__ void flag_rows_kernel(int n, const float* __restrict__ est, int nslices, size_t stride,
                                 const double* __restrict__ a, double scale, int* __restrict__ list,
                                 int* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool flag = false;
  if (i < n) {
    float e = 0.f;
    for (int k = 0; k < nslices; ++k) e += est[(size_t)k * stride + i];
    const double ax = a[i], ay = a[n + i], az = a[2 * n + i];
    const double an = sqrt(ax * ax + ay * ay + az * az);
    flag = sqrt((double)e) * scale > an;
  }
  const unsigned long long mask = __ballot(flag);
  if (mask == 0) return;
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == __ffsll((long long)mask) - 1) base = atomicAdd(count, __popcll(mask));
  base = __shfl(base, __ffsll((long long)mask) - 1, 64);
  if (flag) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = i;
}

// Recomputes the listed rows of a = G sum_j m_j d / (|d|^2 + eps^2)^(3/2) in
// FP64: each pass takes R rows of the list (8 for large systems, where each j
// record then serves eight rows; 1 for small ones, where the few flagged rows
// should run side by side), the B lanes split the j-range (lane t takes
// j = t, t + B, ...), loading U records ahead of the arithmetic (the records
// come from L2 or HBM, and few waves are resident when few rows are flagged),
// and the lane sums are added in a fixed order: a butterfly inside each wave,
// then the wave sums in wave order.
template <int R, int B, int U>
__global__ __launch_bounds__(B) void rescue_rows_kernel(int n, const double* __restrict__ x,
                                                        const double* __restrict__ m, double eps, double G,
                                                        int excl, const int* __restrict__ list,
                                                        const int* __restrict__ count, double* __restrict__ a) {
  constexpr int W = B / 64;
  __shared__ double red[3][R][W];
  const int t = threadIdx.x;
  const int wave = t / 64, lane = t % 64;
  const int cnt = *count;
  const double e2 = eps * eps;
  for (int r0 = blockIdx.x * R; r0 < cnt; r0 += gridDim.x * R) {
    int row[R];
    double xi[R], yi[R], zi[R], sx[R], sy[R], sz[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      row[k] = r0 + k < cnt ? list[r0 + k] : -1;
      const int i = row[k] < 0 ? 0 : row[k];
      xi[k] = x[i];
      yi[k] = x[n + i];
      zi[k] = x[2 * n + i];
      sx[k] = sy[k] = sz[k] = 0.0;
    }
    for (int j0 = t; j0 < n; j0 += U * B) {
      // U records per lane, all loaded before any is used; past n: far away
      // and massless, so they add exact zeros
      double xj[U], yj[U], zj[U], mj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * B;
        const bool in = j < n;
        xj[u] = in ? x[j] : 1.0e30;
        yj[u] = in ? x[n + j] : 1.0e30;
        zj[u] = in ? x[2 * n + j] : 1.0e30;
        mj[u] = in ? m[j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * B;
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const double dx = xj[u] - xi[k], dy = yj[u] - yi[k], dz = zj[u] - zi[k];
          const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
          const double ri = rsqrt64(r2);
          double s = (mj[u] * ri) * (ri * ri);
          if (excl && j == row[k]) s = 0.0;
          sx[k] = fma(s, dx, sx[k]);
          sy[k] = fma(s, dy, sy[k]);
          sz[k] = fma(s, dz, sz[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      for (int off = 32; off > 0; off >>= 1) {
        sx[k] += __shfl_xor(sx[k], off, 64);
        sy[k] += __shfl_xor(sy[k], off, 64);
        sz[k] += __shfl_xor(sz[k], off, 64);
      }
      if (lane == 0) {
        red[0][k][wave] = sx[k];
        red[1][k][wave] = sy[k];
        red[2][k][wave] = sz[k];
      }
    }
    __syncthreads();
    if (t < R && row[t] >= 0) {
      const int i = row[t];
      double v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v[c] = red[c][t][0];
#pragma unroll
        for (int w = 1; w < W; ++w) v[c] += red[c][t][w];
      }
      a[i] = G * v[0];
      a[n + i] = G * v[1];
      a[2 * n + i] = G * v[2];
    }
    __syncthreads();
  }
}

// Launch shapes of the rescue, small systems (one row per pass) and large ones
// (eight rows per pass): lanes per workgroup and records loaded ahead.
constexpr int kRBSmall = 512, kRUSmall = 8;
constexpr int kRBLarge = 1024, kRULarge = 4;

}  // namespace

int launch_rescue(int64_t n, const double* x, const double* m, double eps, double G, bool excl, const float* est,
                  int nslices, size_t stride, double* a, int* list, int* count, hipStream_t s) {
  if (n == 0) return NBODY_OK;
  const double scale = kRescueScale * std::fabs(G);
  flag_rows_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>((int)n, est, nslices, stride, a, scale, list, count);
  NB_LAUNCH_CHECK("flag_rows_kernel");
  const int cus = cu_count(current_device());
  // about as many workgroups as are resident at once; each strides over the list
  if (n <= kRSmall) {
    const unsigned grid = (unsigned)std::min<int64_t>(n, (2048 / kRBSmall) * (int64_t)cus);
    rescue_rows_kernel<1, kRBSmall, kRUSmall><<<grid, kRBSmall, 0, s>>>((int)n, x, m, eps, G, excl ? 1 : 0, list,
                                                                        count, a);
  } else {
    const unsigned grid = (unsigned)std::min<int64_t>((n + 7) / 8, (2048 / kRBLarge) * (int64_t)cus);
    rescue_rows_kernel<8, kRBLarge, kRULarge><<<grid, kRBLarge, 0, s>>>((int)n, x, m, eps, G, excl ? 1 : 0, list,
                                                                        count, a);
  }
  NB_LAUNCH_CHECK("rescue_rows_kernel");
  return NBODY_OK;
}

}  // namespace nb
