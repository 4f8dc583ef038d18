// q2x_bucket.hip -- grouping of elements by leaf box (stable LSD radix sort of
// the box ids) and the box start table.
//
// The recursion kernel needs the elements of one box contiguous (the paper's
// element-to-box rule, Sec. 2 after Eq. (5), makes every element belong to
// exactly one box).  Keys are box ids in [0, B]; ids outside [0, B) are mapped
// to B ("invalid", sorted last and never used).  Each pass sorts 8 key bits:
//   1. hist    : per chunk of kChunk elements, a 256-bin digit histogram,
//                stored digit-major (hist[d * n_chunks + chunk]);
//   2. scan    : exclusive prefix sum over that table (one workgroup);
//   3. scatter : every element moves to scan[d][chunk] + its rank among the
//                earlier elements of its chunk with the same digit.  Ranks come
//                from wavefront ballots (match on the 8 digit bits) plus a
//                per-digit running count across the waves of the chunk, taken
//                in element order -- so the sort is stable and deterministic.
// A final pass writes box_start[b] = first sorted position of box b.
#include "q2x_internal.hpp"

namespace q2x {

constexpr int kBins = 256;
constexpr int kSortThreads = 256;
constexpr int kItems = 4;
constexpr int kChunk = kSortThreads * kItems;  // 1024 elements per workgroup

__device__ __forceinline__ int32_t clamp_key(int32_t k, int64_t nb) {
  return (k < 0 || k >= nb) ? (int32_t)nb : k;
}

// Pass histogram. first_pass: read raw elem_box (map invalid ids to B and
// count them in the status block).
__global__ __launch_bounds__(kSortThreads) void radix_hist(const int32_t* __restrict__ keys, int64_t n, int shift,
                                                          int first_pass, int64_t nb, int32_t* __restrict__ hist,
                                                          int64_t n_chunks, Status* status) {
  __shared__ int32_t h[kBins];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = base + j * kSortThreads + t;
    if (i < n) {
      int32_t k = keys[i];
      if (first_pass) {
        const int32_t kc = clamp_key(k, nb);
        bad += (k < 0 || k >= nb);
        k = kc;
      }
      atomicAdd(&h[(k >> shift) & (kBins - 1)], 1);
    }
  }
  __syncthreads();
  hist[(int64_t)t * n_chunks + blockIdx.x] = h[t];
  if (first_pass) {
    const uint64_t m = __ballot(bad != 0);
    if (m) {
      int cnt = bad;
      for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off);
      if ((t & 63) == 0) {
        atomicAdd(&status->n_skipped, (unsigned long long)cnt);
        atomicOr(&status->flags, (uint32_t)Q2X_FLAG_BAD_BOX);
      }
    }
  }
}

// Exclusive scan of n int32 values in place, one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void scan_exclusive(int32_t* __restrict__ v, int64_t n) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t lo = t * per, hi = min<int64_t>(n, lo + per);
  int32_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += v[i];
  part[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t x = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += x;
    __syncthreads();
  }
  int32_t run = (t == 0) ? 0 : part[t - 1];
  for (int64_t i = lo; i < hi; ++i) {
    const int32_t x = v[i];
    v[i] = run;
    run += x;
  }
}

// Stable scatter of one pass.  vals_in == nullptr means identity (element index).
__global__ __launch_bounds__(kSortThreads) void radix_scatter(const int32_t* __restrict__ keys_in,
                                                             const int32_t* __restrict__ vals_in, int64_t n, int shift,
                                                             int first_pass, int64_t nb,
                                                             const int32_t* __restrict__ scanned, int64_t n_chunks,
                                                             int32_t* __restrict__ keys_out,
                                                             int32_t* __restrict__ vals_out) {
  __shared__ int32_t gbase[kBins];
  __shared__ int32_t running[kBins];
  __shared__ int32_t wcnt[kSortThreads / 64][kBins];
  __shared__ int32_t woff[kSortThreads / 64][kBins];
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int lane = t & 63;
  gbase[t] = scanned[(int64_t)t * n_chunks + blockIdx.x];
  running[t] = 0;
#pragma unroll
  for (int k = 0; k < kSortThreads / 64; ++k) wcnt[k][t] = 0;
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = base + j * kSortThreads + t;
    const bool valid = i < n;
    int32_t key = 0, val = 0, d = 0, rank = 0;
    if (valid) {
      key = keys_in[i];
      if (first_pass) key = clamp_key(key, nb);
      val = vals_in ? vals_in[i] : (int32_t)i;
      d = (key >> shift) & (kBins - 1);
    }
    // peers: lanes of this wave with the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(valid && bit);
      peers &= bit ? m : ~m;
    }
    if (valid) {
      rank = __popcll(peers & lt_mask);
      if (rank == 0) wcnt[w][d] = __popcll(peers);
    }
    __syncthreads();
    {
      int32_t r = running[t];
#pragma unroll
      for (int k = 0; k < kSortThreads / 64; ++k) {
        woff[k][t] = r;
        r += wcnt[k][t];
        wcnt[k][t] = 0;
      }
      running[t] = r;
    }
    __syncthreads();
    if (valid) {
      const int64_t pos = (int64_t)gbase[d] + woff[w][d] + rank;
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
  }
}

// box_start[b] = first sorted position whose key >= b, for b in [0, B];
// keys outside [0, B) count as -1 (before everything) or B (after).  With
// check_sorted, a decreasing neighbour pair sets Q2X_FLAG_NOT_SORTED.
__global__ void box_bounds(const int32_t* __restrict__ keys, int64_t n, int64_t nb, int32_t* __restrict__ box_start,
                           int check_sorted, Status* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  auto ck = [&](int64_t j) -> int64_t {
    const int32_t k = keys[j];
    return (k < 0) ? -1 : (k >= nb ? nb : k);
  };
  const int64_t k = (i < n) ? ck(i) : nb;
  const int64_t kp = (i == 0) ? -1 : ck(i - 1);
  if (check_sorted) {
    // presorted input: count ids outside [0, B) here (the sort does it otherwise)
    const bool bad = (i < n) && (keys[i] < 0 || keys[i] >= nb);
    const uint64_t m = __ballot(bad);
    if (m && (threadIdx.x & 63) == __ffsll((unsigned long long)m) - 1) {
      atomicAdd(&status->n_skipped, (unsigned long long)__popcll(m));
      atomicOr(&status->flags, (uint32_t)Q2X_FLAG_BAD_BOX);
    }
    if (i > 0 && i < n && kp > k) atomicOr(&status->flags, (uint32_t)Q2X_FLAG_NOT_SORTED);
  }
  for (int64_t b = kp + 1; b <= k; ++b) box_start[b] = (int32_t)i;
}

// Zero a small device region (status block) with a kernel so that callers may
// capture the whole sequence in a HIP graph.
__global__ void zero_words(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

int radix_passes(int64_t n_boxes) {
  int bits = 1;
  while (bits < 31 && (((int64_t)1 << bits) <= n_boxes)) ++bits;  // keys in [0, n_boxes]
  return (bits + 7) / 8;
}

size_t bucket_scratch_bytes(int64_t n, int64_t nb) {
  const int64_t n_chunks = (n + kChunk - 1) / kChunk;
  (void)nb;
  return (size_t)(4 * n + (int64_t)kBins * (n_chunks > 0 ? n_chunks : 1)) * sizeof(int32_t);
}

// Sort elem_box -> (keys, perm); writes box_start.  Returns the buffers that
// hold the final keys and permutation.
hipError_t bucket_elements(const int32_t* elem_box, int64_t n, int64_t nb, int32_t* scratch, int32_t* box_start,
                           Status* status, hipStream_t s, const int32_t** keys_out, const int32_t** perm_out) {
  const int64_t n_chunks = (n + kChunk - 1) / kChunk;
  int32_t* ka = scratch;
  int32_t* va = ka + n;
  int32_t* kb = va + n;
  int32_t* vb = kb + n;
  int32_t* hist = vb + n;
  const int passes = radix_passes(nb);
  const int32_t* kin = elem_box;
  const int32_t* vin = nullptr;
  int32_t* ko = ka;
  int32_t* vo = va;
  if (n > 0) {
    for (int ps = 0; ps < passes; ++ps) {
      const int shift = 8 * ps;
      const int first = (ps == 0);
      hipLaunchKernelGGL(radix_hist, dim3((unsigned)n_chunks), dim3(kSortThreads), 0, s, kin, n, shift, first, nb,
                         hist, n_chunks, status);
      hipLaunchKernelGGL(scan_exclusive, dim3(1), dim3(1024), 0, s, hist, (int64_t)kBins * n_chunks);
      hipLaunchKernelGGL(radix_scatter, dim3((unsigned)n_chunks), dim3(kSortThreads), 0, s, kin, vin, n, shift,
                         first, nb, hist, n_chunks, ko, vo);
      kin = ko;
      vin = vo;
      ko = (ko == ka) ? kb : ka;
      vo = (vo == va) ? vb : va;
    }
  }
  const unsigned nbl = (unsigned)((n + 1 + 255) / 256);
  hipLaunchKernelGGL(box_bounds, dim3(nbl), dim3(256), 0, s, n > 0 ? kin : elem_box, n, nb, box_start, 0, status);
  *keys_out = n > 0 ? kin : elem_box;
  *perm_out = vin;
  return hipGetLastError();
}

hipError_t presorted_bounds(const int32_t* elem_box, int64_t n, int64_t nb, int32_t* box_start, Status* status,
                            hipStream_t s) {
  const unsigned nbl = (unsigned)((n + 1 + 255) / 256);
  hipLaunchKernelGGL(box_bounds, dim3(nbl), dim3(256), 0, s, elem_box, n, nb, box_start, 1, status);
  return hipGetLastError();
}

__global__ void copy_i32(int32_t* __restrict__ d, const int32_t* __restrict__ s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

hipError_t copy_words(int32_t* dst, const int32_t* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t clear_status(Status* st, hipStream_t s) {
  hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(st),
                     (int64_t)(sizeof(Status) / 4));
  return hipGetLastError();
}

}  // namespace q2x
