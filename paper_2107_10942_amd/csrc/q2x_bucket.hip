// q2x_bucket.hip -- grouping of elements by leaf box (stable LSD radix sort of
// the box ids).
//
// The recursion kernel needs the elements of one box contiguous (the paper's
// element-to-box rule, Sec. 2 after Eq. (5), makes every element belong to
// exactly one box).  Keys are box ids in [0, B]; ids outside [0, B) are mapped
// to B ("invalid", sorted last, counted, never used).  Each pass sorts 8 key
// bits with three kernels:
//   1. hist    : per chunk of kChunk elements, a 256-bin digit histogram,
//                stored digit-major (hist[d * n_chunks + chunk]);
//   2. rowscan : one workgroup per digit scans its row over the chunks
//                (exclusive, in place) and stores the row total;
//                (With at most kRawRowChunks chunks there is no row scan:
//                every scatter workgroup sums the raw rows it needs itself.)
//   3. scatter : every element moves to base[d] + row[d][chunk] + its rank
//                among the earlier elements of its chunk with the same digit
//                (base = exclusive scan of the 256 row totals, redone in LDS
//                by every workgroup).  Ranks come from wavefront ballots (match
//                on the 8 digit bits) plus a per-digit running count across the
//                waves of the chunk, taken in element order -- so the sort is
//                stable and deterministic.
// With few boxes (B + 1 <= 1024 bins) and up to 2^17 elements one pass of a
// counting sort on the whole (clamped) key replaces the 8-bit passes, with the
// same three steps: per chunk of 2048 elements a histogram over all B + 1 bins
// (in LDS), the same row scan, and a scatter that ranks equal keys with
// wavefront ballots (match on all key bits) and a per-bin running position
// advanced wave by wave in element order.  Same stable order, three kernels
// instead of up to six.  (With more bins the scatter's bin scan and its
// wave-serial steps cost more than the second radix pass saves: measured
// slower at 6,617 boxes and 81,920 elements.)
// The box start table is written by the tile kernel (it reads every sorted key
// and its predecessor anyway); box_bounds is used by the standalone entry point.
#include "q2x_internal.hpp"

namespace q2x {

constexpr int kBins = 256;
constexpr int kSortThreads = 256;
constexpr int kItems = 4;
constexpr int kChunk = kSortThreads * kItems;  // 1024 elements per workgroup
// up to this many chunks, the scatter sums the raw chunk histograms itself
// (each of its threads reads one digit's row) instead of a row-scan kernel
constexpr int64_t kRawRowChunks = 128;

__device__ __forceinline__ int32_t clamp_key(int32_t k, int64_t nb) {
  return (k < 0 || k >= nb) ? (int32_t)nb : k;
}

// Pass histogram.  first_pass: read raw elem_box (invalid ids -> B) and clear
// the status block (workgroup 0; nothing else touches it in this kernel).
__global__ __launch_bounds__(kSortThreads) void radix_hist(const int32_t* __restrict__ keys, int64_t n, int shift,
                                                          int first_pass, int64_t nb, int32_t* __restrict__ hist,
                                                          int64_t n_chunks, Status* status) {
  __shared__ int32_t h[kBins];
  const int t = threadIdx.x;
  if (first_pass && blockIdx.x == 0 && t < (int)(sizeof(Status) / 4)) reinterpret_cast<uint32_t*>(status)[t] = 0u;
  h[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kChunk;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = base + j * kSortThreads + t;
    if (i < n) {
      int32_t k = keys[i];
      if (first_pass) k = clamp_key(k, nb);
      atomicAdd(&h[(k >> shift) & (kBins - 1)], 1);
    }
  }
  __syncthreads();
  hist[(int64_t)t * n_chunks + blockIdx.x] = h[t];
}

// Block-wide exclusive scan of one value per thread (256 threads); returns the
// exclusive prefix and writes the block total to *total.
__device__ __forceinline__ int32_t block_scan_256(int32_t v, int32_t* sh, int32_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kSortThreads; off <<= 1) {
    const int32_t x = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  const int32_t incl = sh[t];
  if (total) *total = sh[kSortThreads - 1];
  __syncthreads();
  return incl - v;
}

// One workgroup per digit: exclusive scan of hist[d][0..n_chunks) in place,
// row total to totals[d].
__global__ __launch_bounds__(kSortThreads) void radix_rowscan(int32_t* __restrict__ hist, int64_t n_chunks,
                                                             int32_t* __restrict__ totals) {
  __shared__ int32_t sh[kSortThreads];
  __shared__ int32_t tot;
  int32_t* row = hist + (int64_t)blockIdx.x * n_chunks;
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < n_chunks; b0 += kSortThreads) {
    const int64_t i = b0 + threadIdx.x;
    const int32_t v = (i < n_chunks) ? row[i] : 0;
    const int32_t ex = block_scan_256(v, sh, &tot);
    if (i < n_chunks) row[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Stable scatter of one pass.  vals_in == nullptr means identity (element
// index).  first_pass: count ids outside [0, B) in the status block.
__global__ __launch_bounds__(kSortThreads) void radix_scatter(const int32_t* __restrict__ keys_in,
                                                             const int32_t* __restrict__ vals_in, int64_t n, int shift,
                                                             int first_pass, int64_t nb,
                                                             const int32_t* __restrict__ rows,
                                                             const int32_t* __restrict__ totals, int64_t n_chunks,
                                                             int32_t* __restrict__ keys_out,
                                                             int32_t* __restrict__ vals_out, Status* status,
                                                             int raw_rows) {
  __shared__ int32_t gbase[kBins];
  __shared__ int32_t running[kBins];
  __shared__ int32_t wcnt[kSortThreads / 64][kBins];
  __shared__ int32_t woff[kSortThreads / 64][kBins];
  __shared__ int32_t sh[kSortThreads];
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int lane = t & 63;
  if (raw_rows) {
    // rows holds the raw chunk histograms (no row scan ran): thread t sums its
    // digit's row, before this chunk and in total
    const int32_t* row = rows + (int64_t)t * n_chunks;
    const int64_t me = blockIdx.x;
    int32_t before = 0, total = 0;
#pragma unroll 8
    for (int64_t c = 0; c < n_chunks; ++c) {
      const int32_t v = row[c];
      total += v;
      before += (c < me) ? v : 0;
    }
    const int32_t dbase = block_scan_256(total, sh, nullptr);
    gbase[t] = dbase + before;
  } else {
    const int32_t dbase = block_scan_256(totals[t], sh, nullptr);
    gbase[t] = dbase + rows[(int64_t)t * n_chunks + blockIdx.x];
  }
  running[t] = 0;
#pragma unroll
  for (int k = 0; k < kSortThreads / 64; ++k) wcnt[k][t] = 0;
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  int bad = 0;
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = base + j * kSortThreads + t;
    const bool valid = i < n;
    int32_t key = 0, val = 0, d = 0, rank = 0;
    if (valid) {
      key = keys_in[i];
      if (first_pass) {
        bad += (key < 0 || key >= nb);
        key = clamp_key(key, nb);
      }
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
  if (first_pass) {
    const uint64_t m = __ballot(bad != 0);
    if (m) {
      int cnt = bad;
      for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off);
      if (lane == 0) {
        atomicAdd(&status->n_skipped, (unsigned long long)cnt);
        atomicOr(&status->flags, (uint32_t)Q2X_FLAG_BAD_BOX);
      }
    }
  }
}

// ---- one-pass counting sort (few boxes)
constexpr int kCsThreads = 1024;
constexpr int kCsSub = 2;                      // sub-rounds of kCsThreads elements per chunk
constexpr int kCsChunk = kCsThreads * kCsSub;  // 2048 elements per workgroup
constexpr int kCsMaxBins = 1024;               // box ids 0..B-1 and the invalid bin B
constexpr int64_t kCsMaxN = (int64_t)1 << 17;

bool counting_sort_applies(int64_t n, int64_t nb) { return nb + 1 <= kCsMaxBins && n <= kCsMaxN; }

// Chunk histogram over all bins; workgroup 0 also clears the status block.
__global__ __launch_bounds__(kCsThreads) void cs_hist(const int32_t* __restrict__ keys, int64_t n, int64_t nb,
                                                     int32_t* __restrict__ counts, int64_t n_chunks,
                                                     Status* status) {
  __shared__ int32_t h[kCsMaxBins];
  const int t = threadIdx.x;
  const int nbins = (int)nb + 1;
  if (blockIdx.x == 0 && t < (int)(sizeof(Status) / 4)) reinterpret_cast<uint32_t*>(status)[t] = 0u;
  for (int i = t; i < nbins; i += kCsThreads) h[i] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kCsChunk;
#pragma unroll
  for (int j = 0; j < kCsSub; ++j) {
    const int64_t i = base + j * kCsThreads + t;
    if (i < n) atomicAdd(&h[clamp_key(keys[i], nb)], 1);
  }
  __syncthreads();
  for (int i = t; i < nbins; i += kCsThreads) counts[(int64_t)i * n_chunks + blockIdx.x] = h[i];
}

// Stable scatter: element i of the chunk goes to (start of its bin) + (number
// of earlier elements of the chunk in the bin), the latter from the wavefront
// match of all nbits key bits and the bin's running position, which the
// waves advance one after the other.  Ids outside [0, B) are counted.
__global__ __launch_bounds__(kCsThreads) void cs_scatter(const int32_t* __restrict__ keys, int64_t n, int64_t nb,
                                                        int nbits, const int32_t* __restrict__ rows,
                                                        const int32_t* __restrict__ totals, int64_t n_chunks,
                                                        int32_t* __restrict__ keys_out,
                                                        int32_t* __restrict__ vals_out, Status* status) {
  __shared__ int32_t pos_of[kCsMaxBins];  // next output position of each bin for this chunk
  __shared__ int32_t sh[kCsThreads];
  __shared__ int32_t carry;
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int nbins = (int)nb + 1;
  // pos_of[b] = (exclusive scan of the bin totals)[b] + (this chunk's row offset of b)
  if (t == 0) carry = 0;
  for (int b0 = 0; b0 < nbins; b0 += kCsThreads) {
    const int b = b0 + t;
    const int32_t v = (b < nbins) ? totals[b] : 0;
    __syncthreads();
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kCsThreads; off <<= 1) {
      const int32_t x = (t >= off) ? sh[t - off] : 0;
      __syncthreads();
      sh[t] += x;
      __syncthreads();
    }
    if (b < nbins) pos_of[b] = carry + sh[t] - v + rows[(int64_t)b * n_chunks + blockIdx.x];
    __syncthreads();
    if (t == kCsThreads - 1) carry += sh[t];
  }
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t cbase = (int64_t)blockIdx.x * kCsChunk;
  int bad = 0;
  for (int j = 0; j < kCsSub; ++j) {
    const int64_t i = cbase + j * kCsThreads + t;
    const bool valid = i < n;
    int32_t key = 0;
    if (valid) {
      const int32_t k0 = keys[i];
      bad += (k0 < 0 || k0 >= nb);
      key = clamp_key(k0, nb);
    }
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (key >> b) & 1;
      const uint64_t m = __ballot(valid && bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & lt_mask);
    const int cnt = __popcll(peers);
    for (int ww = 0; ww < kCsThreads / 64; ++ww) {
      if (w == ww && valid) {
        const int32_t start = pos_of[key];  // every lane reads before the leaders advance
        keys_out[start + rank] = key;
        vals_out[start + rank] = (int32_t)i;
        if (rank == 0) pos_of[key] = start + cnt;
      }
      __syncthreads();
    }
  }
  const uint64_t m = __ballot(bad != 0);
  if (m) {
    int c = bad;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
    if (lane == 0) {
      atomicAdd(&status->n_skipped, (unsigned long long)c);
      atomicOr(&status->flags, (uint32_t)Q2X_FLAG_BAD_BOX);
    }
  }
}

// box_start[b] = first sorted position whose key >= b, for b in [0, B];
// keys outside [0, B) count as -1 (before everything) or B (after).  With
// `order_check`, a decrease of the (clamped) keys sets Q2X_FLAG_NOT_SORTED.
__global__ void box_bounds(const int32_t* __restrict__ keys, int64_t n, int64_t nb, int32_t* __restrict__ box_start,
                           Status* order_check) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  auto ck = [&](int64_t j) -> int64_t {
    const int32_t k = keys[j];
    return (k < 0) ? -1 : (k >= nb ? nb : k);
  };
  const int64_t k = (i < n) ? ck(i) : nb;
  const int64_t kp = (i == 0) ? -1 : ck(i - 1);
  if (order_check && kp > k) atomicOr(&order_check->flags, (uint32_t)Q2X_FLAG_NOT_SORTED);
  for (int64_t b = kp + 1; b <= k; ++b) box_start[b] = (int32_t)i;
}

// Zero a small device region (status block) with a kernel, not a memset, so
// that callers may capture the whole call sequence in a HIP graph.
__global__ void zero_words(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void copy_i32(int32_t* __restrict__ d, const int32_t* __restrict__ s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

int radix_passes(int64_t n_boxes) {
  int bits = 1;
  while (bits < 31 && (((int64_t)1 << bits) <= n_boxes)) ++bits;  // keys in [0, n_boxes]
  return (bits + 7) / 8;
}

size_t bucket_scratch_bytes(int64_t n, int64_t nb) {
  const int64_t n_chunks = (n + kChunk - 1) / kChunk;
  int64_t words = 4 * n + (int64_t)kBins * (n_chunks > 0 ? n_chunks : 1) + kBins;
  if (counting_sort_applies(n, nb)) {
    const int64_t cs_chunks = (n + kCsChunk - 1) / kCsChunk;
    const int64_t cs = 2 * n + (nb + 1) * (cs_chunks > 0 ? cs_chunks : 1) + (nb + 1);
    if (cs > words) words = cs;
  }
  return (size_t)words * sizeof(int32_t);
}

// Sort elem_box -> (keys, perm); the first kernel also clears the status
// block.  n must be > 0.  Returns the buffers that hold the final keys and
// permutation.
hipError_t bucket_elements(const int32_t* elem_box, int64_t n, int64_t nb, int32_t* scratch, Status* status,
                           hipStream_t s, const int32_t** keys_out, const int32_t** perm_out) {
  if (counting_sort_applies(n, nb)) {
    const int64_t cs_chunks = (n + kCsChunk - 1) / kCsChunk;
    int32_t* ko = scratch;
    int32_t* vo = ko + n;
    int32_t* counts = vo + n;
    int32_t* tot = counts + (nb + 1) * cs_chunks;
    int nbits = 1;
    while (nbits < 31 && ((int64_t)1 << nbits) <= nb) ++nbits;  // keys in [0, nb]
    hipLaunchKernelGGL(cs_hist, dim3((unsigned)cs_chunks), dim3(kCsThreads), 0, s, elem_box, n, nb, counts,
                       cs_chunks, status);
    hipLaunchKernelGGL(radix_rowscan, dim3((unsigned)(nb + 1)), dim3(kSortThreads), 0, s, counts, cs_chunks, tot);
    hipLaunchKernelGGL(cs_scatter, dim3((unsigned)cs_chunks), dim3(kCsThreads), 0, s, elem_box, n, nb, nbits, counts,
                       tot, cs_chunks, ko, vo, status);
    *keys_out = ko;
    *perm_out = vo;
    return hipGetLastError();
  }
  const int64_t n_chunks = (n + kChunk - 1) / kChunk;
  int32_t* ka = scratch;
  int32_t* va = ka + n;
  int32_t* kb = va + n;
  int32_t* vb = kb + n;
  int32_t* hist = vb + n;
  int32_t* totals = hist + (int64_t)kBins * n_chunks;
  const int passes = radix_passes(nb);
  const int32_t* kin = elem_box;
  const int32_t* vin = nullptr;
  int32_t* ko = ka;
  int32_t* vo = va;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = 8 * ps;
    const int first = (ps == 0);
    hipLaunchKernelGGL(radix_hist, dim3((unsigned)n_chunks), dim3(kSortThreads), 0, s, kin, n, shift, first, nb, hist,
                       n_chunks, status);
    // few chunks: every scatter workgroup sums the raw rows itself (one
    // kernel less per pass); many chunks: the row scan runs once
    const int raw = (n_chunks <= kRawRowChunks) ? 1 : 0;
    if (!raw) hipLaunchKernelGGL(radix_rowscan, dim3(kBins), dim3(kSortThreads), 0, s, hist, n_chunks, totals);
    hipLaunchKernelGGL(radix_scatter, dim3((unsigned)n_chunks), dim3(kSortThreads), 0, s, kin, vin, n, shift, first,
                       nb, hist, totals, n_chunks, ko, vo, status, raw);
    kin = ko;
    vin = vo;
    ko = (ko == ka) ? kb : ka;
    vo = (vo == va) ? vb : va;
  }
  *keys_out = kin;
  *perm_out = vin;
  return hipGetLastError();
}

hipError_t launch_box_bounds(const int32_t* keys, int64_t n, int64_t nb, int32_t* box_start, hipStream_t s,
                             Status* order_check) {
  const unsigned nbl = (unsigned)((n + 1 + 255) / 256);
  hipLaunchKernelGGL(box_bounds, dim3(nbl), dim3(256), 0, s, keys, n, nb, box_start, order_check);
  return hipGetLastError();
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
