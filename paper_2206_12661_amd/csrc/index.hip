// Plan-time index work by sorting: the reduced focal grid (Sec. 2: one
// sample row or column per distinct focus coordinate), the gather index of
// every focus into it, the duplicate-focus test and the focus order of the
// scatter's compressed rows.  A stable least-significant-digit radix sort of
// 64-bit keys (8-bit digits) carries each focus number along; every result
// follows from the sorted order, so the work is O(n) per digit pass instead
// of comparing all pairs.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gswmtp_internal.h"

namespace gswmtp {
namespace {

constexpr int kSortChunk = 2048;   // keys per workgroup in a digit pass
constexpr int kSortThreads = 256;  // one thread per digit value

// -0.0 and +0.0 are one coordinate.
__device__ __forceinline__ double canon_d(double x) { return x == 0.0 ? 0.0 : x; }

// IEEE bits of a finite double mapped so that unsigned order is numeric
// order: negative values flip every bit, the others set the sign bit.
__device__ __forceinline__ uint64_t order_bits(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(canon_d(x));
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void k_keys_of(const double *c, const int *val, int n, uint64_t *key, int *val_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int i = val ? val[p] : p;
  key[p] = order_bits(c[i]);
  if (val_out) val_out[p] = i;
}

// Digit counts of one chunk: hist[digit * nblk + chunk] (digit-major, so
// one exclusive scan gives every chunk's first output position per digit).
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t *key, int n, int shift,
                                                             int nblk, int *hist) {
  __shared__ int cnt[256];
  const int t = threadIdx.x, b = blockIdx.x;
  cnt[t] = 0;
  __syncthreads();
  const int lo = b * kSortChunk, hi = min(n, lo + kSortChunk);
  for (int i = lo + t; i < hi; i += kSortThreads)
    atomicAdd(&cnt[(int)((key[i] >> shift) & 255u)], 1);
  __syncthreads();
  hist[t * nblk + b] = cnt[t];
}

// Exclusive scan of m <= 256 * 128 counts in place (one workgroup).
__global__ __launch_bounds__(1024) void k_radix_scan(int *hist, int m) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (m + 1023) / 1024;
  const int lo = min(t * per, m), hi = min(lo + per, m);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += hist[i];
  part[t] = s;
  __syncthreads();
  for (int w = 1; w < 1024; w <<= 1) {   // inclusive Hillis-Steele scan
    const int v = t >= w ? part[t - w] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int i = lo; i < hi; ++i) {
    const int v = hist[i];
    hist[i] = run;
    run += v;
  }
}

// Stable scatter of one chunk, 256 keys at a time in order.  Within a wave
// the lanes holding the same digit are found with eight ballots (one per
// digit bit); a key's place is its chunk's scanned offset for the digit, plus
// the keys with that digit in earlier tiles, earlier waves of the tile and
// lower lanes of its wave - so equal digits keep their input order.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t *kin,
                                                                const int *vin, int n, int shift,
                                                                int nblk, const int *hist,
                                                                uint64_t *kout, int *vout) {
  constexpr int kWaves = kSortThreads / 64;
  __shared__ int off[256];
  __shared__ int wcnt[kWaves][256];
  const int t = threadIdx.x, b = blockIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int lo = b * kSortChunk, cnt = min(kSortChunk, n - lo);
  off[t] = hist[t * nblk + b];
  for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int base = 0; base < cnt; base += kSortThreads) {
    const int i = base + t;
    const bool valid = i < cnt;
    const uint64_t k = valid ? kin[lo + i] : 0ull;
    const int v = valid ? vin[lo + i] : 0;
    const uint32_t d = (uint32_t)((k >> shift) & 255u);
    unsigned long long peers = __ballot(valid);
    for (int bit = 0; bit < 8; ++bit) {
      const bool set = (d >> bit) & 1u;
      const unsigned long long m = __ballot(set);
      peers &= set ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = off[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    int tot = 0;
    for (int w = 0; w < kWaves; ++w) {
      tot += wcnt[w][t];
      wcnt[w][t] = 0;
    }
    off[t] += tot;
    __syncthreads();
  }
}

// Group heads of the (coordinate, z) order: head[p] = 1 when position p
// starts a new distinct pair.
__global__ void k_heads(const double *c, const double *z, const int *val, int n, int *head) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int h = 1;
  if (p > 0) {
    const int i = val[p], m = val[p - 1];
    h = (canon_d(c[i]) != canon_d(c[m]) || canon_d(z[i]) != canon_d(z[m])) ? 1 : 0;
  }
  head[p] = h;
}

// rank[p] = (number of heads at positions <= p) - 1; *count = number of heads.
// One workgroup; n <= 262144.
__global__ __launch_bounds__(1024) void k_head_rank(const int *head, int n, int *rank,
                                                    int *count) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = min(t * per, n), hi = min(lo + per, n);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += head[i];
  part[t] = s;
  __syncthreads();
  for (int w = 1; w < 1024; w <<= 1) {
    const int v = t >= w ? part[t - w] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int i = lo; i < hi; ++i) {
    run += head[i];
    rank[i] = run - 1;
  }
  if (t == 1023) *count = part[1023];
}

// Gather index of every focus and the sorted distinct pairs.
__global__ void k_assign(const double *c, const double *z, const int *val, const int *head,
                         const int *rank, int n, int *idx, double *uniq, double *uniq_z) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int i = val[p], r = rank[p];
  idx[i] = r;
  if (head[p]) {
    uniq[r] = canon_d(c[i]);
    uniq_z[r] = canon_d(z[i]);
  }
}

// (hi, lo) index pairs as one key (each index < 2^18).
__global__ void k_pair_keys(const int *hi, const int *lo, int n, uint64_t *key, int *val) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  key[p] = ((uint64_t)(uint32_t)hi[p] << 18) | (uint64_t)(uint32_t)lo[p];
  val[p] = p;
}

__global__ void k_adjacent_equal(const uint64_t *key, int n, int *flag) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > 0 && p < n && key[p] == key[p - 1]) atomicOr(flag, 1);
}

__global__ void k_copy_int(const int *a, int n, int *out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) out[p] = a[p];
}

dim3 grid_of(int n) { return dim3((unsigned)((n + 255) / 256)); }

// Stable sort of (key, val) by the low `bits` bits of key, ping-ponging
// between the two buffers of sc; returns the index (0 or 1) of the buffer
// that holds the result.
int radix_sort(IndexScratch &sc, int cur, int n, int bits, hipStream_t s) {
  const int nblk = (n + kSortChunk - 1) / kSortChunk;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, s, sc.key[cur], n,
                       shift, nblk, sc.hist);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, s, sc.hist, 256 * nblk);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortThreads), 0, s, sc.key[cur],
                       sc.val[cur], n, shift, nblk, sc.hist, sc.key[cur ^ 1], sc.val[cur ^ 1]);
    cur ^= 1;
  }
  return cur;
}

}  // namespace

size_t index_hist_ints(int n) { return 256 * (size_t)((n + kSortChunk - 1) / kSortChunk); }

hipError_t unique_pairs(const double *c, const double *z, bool has_z, int n, IndexScratch sc,
                        int *idx, double *uniq, double *uniq_z, int *count, hipStream_t s) {
  if (n < 1 || n > kMaxFoci) return hipErrorInvalidValue;
  const dim3 g = grid_of(n);
  int cur = 0;
  if (has_z) {   // by z first, then (stably) by the coordinate
    hipLaunchKernelGGL(k_keys_of, g, dim3(256), 0, s, z, nullptr, n, sc.key[0], sc.val[0]);
    cur = radix_sort(sc, 0, n, 64, s);
    hipLaunchKernelGGL(k_keys_of, g, dim3(256), 0, s, c, sc.val[cur], n, sc.key[cur],
                       nullptr);
  } else {
    hipLaunchKernelGGL(k_keys_of, g, dim3(256), 0, s, c, nullptr, n, sc.key[0], sc.val[0]);
  }
  cur = radix_sort(sc, cur, n, 64, s);
  hipLaunchKernelGGL(k_heads, g, dim3(256), 0, s, c, z, sc.val[cur], n, sc.head);
  hipLaunchKernelGGL(k_head_rank, dim3(1), dim3(1024), 0, s, sc.head, n, sc.rank, count);
  hipLaunchKernelGGL(k_assign, g, dim3(256), 0, s, c, z, sc.val[cur], sc.head, sc.rank, n, idx,
                     uniq, uniq_z);
  return hipGetLastError();
}

hipError_t pair_order(const int *hi, const int *lo, int n, IndexScratch sc, int *order,
                      int *dup, hipStream_t s) {
  if (n < 1 || n > kMaxFoci) return hipErrorInvalidValue;
  const dim3 g = grid_of(n);
  hipLaunchKernelGGL(k_pair_keys, g, dim3(256), 0, s, hi, lo, n, sc.key[0], sc.val[0]);
  const int cur = radix_sort(sc, 0, n, 36, s);
  if (dup) hipLaunchKernelGGL(k_adjacent_equal, g, dim3(256), 0, s, sc.key[cur], n, dup);
  if (order) hipLaunchKernelGGL(k_copy_int, g, dim3(256), 0, s, sc.val[cur], n, order);
  return hipGetLastError();
}

}  // namespace gswmtp
