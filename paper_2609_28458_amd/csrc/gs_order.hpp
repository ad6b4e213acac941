// Longest-first queue order built on the device.
//
// The persistent grid hands trajectories out in queue order; when costs are
// very uneven the makespan is set by the trajectories that start last, so the
// queue should start with the longest ones (the idle cost of eq:cost moves to
// the end of the launch, where short trajectories fill it).  Here each
// trajectory gets a predicted cost key, and a counting sort over 65,536
// buckets of the key range puts the largest keys first:
//   1. clear the histogram and the key range,
//   2. key of every trajectory, and the range of the finite keys (one
//      64-bit atomic min/max per wavefront on order-preserving integer
//      images of the keys),
//   3. bucket of every key (descending; non-finite keys in the last bucket)
//      and the bucket histogram,
//   4. exclusive prefix sum of the histogram in one workgroup,
//   5. scatter: each trajectory takes the next slot of its bucket.
// Within a bucket the order is whatever the atomics give; the solution of
// every trajectory is independent of where it runs, so results do not depend
// on it.  All five steps are kernels (no memset), so the build can be
// captured in a graph with the solve.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gs {
namespace order {

constexpr int kBuckets = 65536;
constexpr int kScanThreads = 1024;

struct Ws {
  double* key;                 // [n]
  uint32_t* bucket;            // [n]
  uint32_t* hist;              // [kBuckets]; after the scan: next free slot per bucket
  unsigned long long* range;   // [2]: order-preserving images of min and max key
};

// Order-preserving map of a double to an unsigned 64-bit integer (and back).
__device__ __forceinline__ unsigned long long ord_bits(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ord(unsigned long long u) {
  const unsigned long long b = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
  return __longlong_as_double((long long)b);
}

__global__ void clear_kernel(Ws w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kBuckets) w.hist[i] = 0u;
  if (i == 0) {
    w.range[0] = ~0ull;  // min
    w.range[1] = 0ull;   // max
  }
}

// Inputs of the built-in cost models (a plain copy of the solve arguments).
struct CostIn {
  int64_t n;
  int32_t loghalo;        // the dynamical-time model of the logarithmic halo
  double inv_nu;          // 1 / order of the pair
  const double* y0;       // [d][n]
  const double* theta;    // [p][theta_stride]
  int64_t theta_stride;
  const double* t0;
  const double* t1;
  int64_t t_stride;
  const double* rtol;
  int64_t tol_stride;
  const double* cost;     // [n] caller's costs, or null for the built-in model
};

// Predicted cost key of trajectory i.  A caller's cost is used as given.
// Built in: the number of dynamical times in the span times rtol^(-1/nu) (a
// pair of order nu takes about rtol^(-1/nu) steps per dynamical time), as a
// logarithm.  For orbits in the logarithmic halo (eq:loghalo) the dynamical
// time is (rc + r_E) / v0 with r_E the in-plane radius at which the
// potential equals the orbit's energy (eq:st-scales); otherwise the span
// itself stands in for the number of dynamical times.
__device__ __forceinline__ double cost_key(const CostIn& c, int64_t i) {
  if (c.cost) return c.cost[i];
  const double span = c.t1[c.t_stride ? i : 0] - c.t0[c.t_stride ? i : 0];
  const double rtol = c.rtol[c.tol_stride ? i : 0];
  double lk = log(span) - c.inv_nu * log(rtol);
  if (c.loghalo) {
    auto th = [&](int j) { return c.theta_stride ? c.theta[j * c.theta_stride + i] : c.theta[j]; };
    const double v0 = th(0), q = th(1), rc = th(2);
    auto y = [&](int k) { return c.y0[(int64_t)k * c.n + i]; };
    const double Dn = rc * rc + y(0) * y(0) + y(1) * y(1) + y(2) * y(2) / (q * q);
    const double E = 0.5 * (y(3) * y(3) + y(4) * y(4) + y(5) * y(5)) + 0.5 * v0 * v0 * log(Dn);
    const double rE2 = exp(2.0 * E / (v0 * v0)) - rc * rc;
    const double rE = sqrt(rE2 > 0.0 ? rE2 : 0.0);
    lk += log(v0) - log(rc + rE);
  }
  return lk;
}

__global__ void __launch_bounds__(256) key_kernel(CostIn c, Ws w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double k = 0.0;
  bool fin = false;
  if (i < c.n) {
    k = cost_key(c, i);
    w.key[i] = k;
    fin = (k - k) == 0.0;
  }
  unsigned long long lo = fin ? ord_bits(k) : ~0ull;
  unsigned long long hi = fin ? ord_bits(k) : 0ull;
  // wavefront min / max, then one atomic per wavefront
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long olo = __shfl_xor(lo, off);
    const unsigned long long ohi = __shfl_xor(hi, off);
    lo = olo < lo ? olo : lo;
    hi = ohi > hi ? ohi : hi;
  }
  if ((threadIdx.x & 63) == 0 && lo != ~0ull) {
    atomicMin(w.range, lo);
    atomicMax(w.range + 1, hi);
  }
}

__global__ void __launch_bounds__(256) bucket_kernel(int64_t n, Ws w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double k = w.key[i];
  uint32_t b = kBuckets - 1;
  if ((k - k) == 0.0) {
    const double lo = from_ord(w.range[0]), hi = from_ord(w.range[1]);
    // largest key first: bucket 0 holds the top of the range
    const double x = hi > lo ? (hi - k) / (hi - lo) * (double)(kBuckets - 2) : 0.0;
    b = (uint32_t)(x < 0.0 ? 0.0 : (x > (double)(kBuckets - 2) ? (double)(kBuckets - 2) : x));
  }
  w.bucket[i] = b;
  atomicAdd(w.hist + b, 1u);
}

// Exclusive prefix sum of the histogram in place, one workgroup of
// kScanThreads threads, each owning kBuckets / kScanThreads buckets.
__global__ void __launch_bounds__(kScanThreads) scan_kernel(Ws w) {
  constexpr int per = kBuckets / kScanThreads;
  __shared__ uint32_t part[kScanThreads];
  const int t = threadIdx.x;
  uint32_t* h = w.hist + t * per;
  uint32_t sum = 0;
  for (int j = 0; j < per; ++j) sum += h[j];
  part[t] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - sum;  // exclusive
  for (int j = 0; j < per; ++j) {
    const uint32_t c = h[j];
    h[j] = run;
    run += c;
  }
}

__global__ void __launch_bounds__(256) scatter_kernel(int64_t n, Ws w, int64_t* order) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t pos = atomicAdd(w.hist + w.bucket[i], 1u);
  order[pos] = i;
}

}  // namespace order
}  // namespace gs
