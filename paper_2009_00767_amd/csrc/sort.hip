// sort.hip -- binning of particles into leaves (Section 2.1 items 1-4) and a
// stable counting sort of the particles by the Morton key of their leaf.
//
// After the sort, the particles of every box at every level form one contiguous
// range (Morton order nests the boxes of all levels), which is what lets the
// per-level passes stream the particles without any shift between levels.
//
// The sort is a least-significant-digit radix sort with 8-bit digits over
// tiles of kRadixTile keys, three kernels per pass:
//   k_rs_hist    per-tile digit counts in LDS (integer atomics only; the
//                first pass's come with the binning, k_bin),
//   k_scan_rows  exclusive scan of each digit's row of the digit-major count
//                table (one workgroup per digit) and the digit totals,
//   k_rs_scatter stable ranking inside a tile with wave ballots (64-wide match
//                masks) into LDS in digit order, then coalesced runs out to the
//                digits' global ranges.
// It is deterministic: equal keys keep their input order.
#include "device_common.h"

namespace sffmm {



// Leaf key of particle i; bad: the position lies outside the box or is NaN.
template <int D>
__device__ __forceinline__ uint32_t bin_key(const double* __restrict__ pos, int64_t i,
                                            const LevelTable& lt, bool& bad) {
  const int64_t nl = (int64_t)1 << lt.L;
  uint32_t c[3] = {0, 0, 0};
  bad = false;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double x = pos[D * i + d];
    const double o = lt.origin[d];
    if (!(x >= o && x <= o + lt.side)) {
      bad = true;
      continue;
    }
    // leaf coordinate: min(floor((x - o) * (2^L / S)), 2^L - 1), in FP64
    const double t = floor(__dmul_rn(__dsub_rn(x, o), lt.leaf_scale));
    int64_t li = (int64_t)t;
    if (li > nl - 1) li = nl - 1;
    c[d] = (uint32_t)li;
  }
  if (D == 2) return spread2(c[0]) | (spread2(c[1]) << 1);
  return spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
}

// FP32 leaf-local record of particle i in the leaf of `key` (FP32 modes): the
// offsets x - (origin + s_L (i + 1/2)) evaluated in FP64 and rounded once, and
// the charge; the leaf-centre differences used later are exact in FP32.  In 2D
// the fourth component carries the leaf's column and row as bits (column in
// the low 16), which the moments read instead of decoding the Morton key.
template <int D>
__device__ __forceinline__ float4 leaf_record(const double* __restrict__ pos,
                                              const double* __restrict__ q, int64_t i,
                                              uint32_t key, const double* origin, double sL) {
  float4 r;
  if (D == 2) {
    const uint32_t ix = compact2(key), iy = compact2(key >> 1);
    r.x = (float)(pos[2 * i] - (origin[0] + sL * ((double)ix + 0.5)));
    r.y = (float)(pos[2 * i + 1] - (origin[1] + sL * ((double)iy + 0.5)));
    r.z = (float)q[i];
    r.w = __uint_as_float(ix | (iy << 16));
  } else {
    const uint32_t ix = compact3(key), iy = compact3(key >> 1), iz = compact3(key >> 2);
    r.x = (float)(pos[3 * i] - (origin[0] + sL * ((double)ix + 0.5)));
    r.y = (float)(pos[3 * i + 1] - (origin[1] + sL * ((double)iy + 0.5)));
    r.z = (float)(pos[3 * i + 2] - (origin[2] + sL * ((double)iz + 0.5)));
    r.w = (float)q[i];
  }
  return r;
}

// Keys and identity values of one radix tile per workgroup, the tile's
// histogram of the first 8-bit digit (the first radix pass's counts), and in
// the FP32 modes (rec != NULL) each particle's leaf-local record in input order,
// which the radix passes then carry to sorted order.
template <int D>
__global__ __launch_bounds__(256) void k_bin(const double* __restrict__ pos, int64_t n, LevelTable lt,
                                             uint32_t* __restrict__ keys,
                                             int32_t* __restrict__ vals, int32_t* flag,
                                             int32_t tag, int32_t* __restrict__ hist,
                                             int64_t ntiles, int hshift,
                                             const double* __restrict__ q,
                                             float4* __restrict__ rec) {
  __shared__ int32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
  for (int r = 0; r < kRadixTile / 256; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    if (i < n) {
      bool bad;
      const uint32_t key = bin_key<D>(pos, i, lt, bad);
      if (bad) flag[0] = tag;  // every writer stores the same value
      keys[i] = key;
      vals[i] = (int32_t)i;
      if (rec) rec[i] = leaf_record<D>(pos, q, i, key, lt.origin, lt.s[lt.L]);
      atomicAdd(&cnt[(key >> hshift) & 255u], 1);
    }
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

void launch_bin(int dim, const double* pos, int64_t n, const LevelTable& lt, uint32_t* keys,
                int32_t* vals, int32_t* flag, int32_t tag, int32_t* hist, hipStream_t st,
                const double* q, float4* rec, int hist_shift) {
  const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  if (dim == 2)
    hipLaunchKernelGGL(k_bin<2>, dim3(ntiles), dim3(256), 0, st, pos, n, lt, keys, vals, flag,
                       tag, hist, ntiles, hist_shift, q, rec);
  else
    hipLaunchKernelGGL(k_bin<3>, dim3(ntiles), dim3(256), 0, st, pos, n, lt, keys, vals, flag,
                       tag, hist, ntiles, hist_shift, q, rec);
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
}

// ---------------------------------------------------------------------------
// Radix passes.
// ---------------------------------------------------------------------------
constexpr int kScatterThreads = 512;  // 8 waves: four rounds of a tile

// Exclusive scan of one value per thread over an NT-thread workgroup; *total
// receives the sum.  wt: NT / 64 ints of LDS.
template <int NT>
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t* wt, int32_t* total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t o = __shfl_up(x, d, 64);
    if (lane >= d) x += o;
  }
  if (lane == 63) wt[wave] = x;
  __syncthreads();
  int32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w < wave) before += wt[w];
    all += wt[w];
  }
  *total = all;
  __syncthreads();
  return before + x - v;
}

// Per-tile digit counts of keys >> shift, digit-major: hist[d * ntiles + tile].
__global__ __launch_bounds__(256) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                 int shift, int32_t* __restrict__ hist,
                                                 int64_t ntiles) {
  __shared__ int32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
  for (int r = 0; r < kRadixTile / 256; ++r) {
    const int64_t e = base + r * 256 + threadIdx.x;
    if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Workgroup d: exclusive scan, in place, of row d (the count of digit d in
// every tile) and tot[d] = the row's sum.
__global__ __launch_bounds__(256) void k_scan_rows(int32_t* __restrict__ hist, int64_t ntiles,
                                                   int32_t* __restrict__ tot) {
  __shared__ int32_t wt[4];
  int32_t* row = hist + (int64_t)blockIdx.x * ntiles;
  constexpr int kPer = 8;
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < ntiles; c0 += 256 * kPer) {
    const int64_t b = c0 + (int64_t)threadIdx.x * kPer;
    int32_t x[kPer];
    int32_t v = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      x[i] = b + i < ntiles ? row[b + i] : 0;
      v += x[i];
    }
    int32_t chunk;
    int32_t run = carry + block_exclusive_scan<256>(v, wt, &chunk);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      if (b + i < ntiles) row[b + i] = run;
      run += x[i];
    }
    carry += chunk;
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// 64-bit mask of the lanes whose valid digit equals this lane's (eight ballots).
__device__ __forceinline__ uint64_t digit_match(uint32_t d, bool valid) {
  uint64_t mk = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const bool on = (d >> bit) & 1u;
    const uint64_t bb = __ballot(on);
    mk &= on ? bb : ~bb;
  }
  return mk;
}

// Adds the wave's valid digits to row[0..255]: one atomic per distinct digit
// (clustered keys repeat digits, and 64 atomics on one address serialise).
__device__ __forceinline__ void count_digits(int32_t* row, uint32_t d, bool valid) {
  const uint64_t mk = digit_match(d, valid);
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  if (valid && __popcll(mk & lt_mask) == 0) atomicAdd(&row[d], __popcll(mk));
}

// Stable scatter of one tile.  Elements are ranked in input order: inside a
// wave the rank among equal digits comes from a 64-bit match mask built from
// eight ballots.  Each element goes to LDS at its place in the tile sorted by
// digit; the tile's digit runs are then written out with consecutive threads
// on consecutive destinations.
__global__ __launch_bounds__(kScatterThreads) void k_rs_scatter(
    const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    int32_t* __restrict__ vout, int64_t n, int shift, const int32_t* __restrict__ scanned,
    const int32_t* __restrict__ tot, int64_t ntiles, const float4* __restrict__ pin,
    float4* __restrict__ pout) {
  constexpr int NW = kScatterThreads / 64;
  extern __shared__ float4 srec[];  // kRadixTile records when pin is given
  __shared__ uint32_t skey[kRadixTile];
  __shared__ int32_t sval[kRadixTile];
  __shared__ int32_t gbase[256];    // destination of digit d's first element of this tile
  __shared__ int32_t loff[256];     // digit d's first place in the tile sorted by digit
  __shared__ int32_t wcnt[NW][256];
  __shared__ int32_t wt[NW];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t tile = blockIdx.x, tile0 = tile * kRadixTile;
  const int m = (int)(n - tile0 < kRadixTile ? n - tile0 : kRadixTile);
  {
    int32_t here = 0, cnt = 0, dt = 0;
    if (t < 256) {
      here = scanned[(int64_t)t * ntiles + tile];
      cnt = (tile + 1 < ntiles ? scanned[(int64_t)t * ntiles + tile + 1] : tot[t]) - here;
      dt = tot[t];
    }
    int32_t s1, s2;
    const int32_t lo = block_exclusive_scan<kScatterThreads>(cnt, wt, &s1);
    const int32_t gb = block_exclusive_scan<kScatterThreads>(dt, wt, &s2);
    if (t < 256) {
      loff[t] = lo;
      gbase[t] = gb + here;
    }
  }
  // Wave w ranks the contiguous piece [w PW, (w + 1) PW) of the tile: one count
  // of each wave's digits, one scan across the waves, then every wave places
  // its piece 64 keys at a time with no further barrier (its running digit
  // offsets in LDS, read and advanced in program order).
  constexpr int PW = kRadixTile / NW, CH = PW / 64;
  if (t < 256)
#pragma unroll
    for (int w = 0; w < NW; ++w) wcnt[w][t] = 0;
  const int p0 = wave * PW;
  uint32_t kk[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int e = p0 + 64 * c + lane;
    kk[c] = e < m ? kin[tile0 + e] : 0u;
  }
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t mks[CH];  // each chunk's match masks, kept for the ranking
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const bool valid = p0 + 64 * c + lane < m;
    const uint32_t d = (kk[c] >> shift) & 255u;
    mks[c] = digit_match(d, valid);
    // one atomic per distinct digit of the chunk (repeated digits do not serialise)
    if (valid && __popcll(mks[c] & lt_mask) == 0) atomicAdd(&wcnt[wave][d], __popcll(mks[c]));
  }
  __syncthreads();
  if (t < 256) {  // per digit: each wave's first place in the tile sorted by digit
    int32_t o = loff[t];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int32_t c = wcnt[w][t];
      wcnt[w][t] = o;
      o += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    if (p0 + 64 * c >= m) break;  // wave-uniform
    const int e = p0 + 64 * c + lane;
    const bool valid = e < m;
    const uint32_t d = (kk[c] >> shift) & 255u;
    const uint64_t mk = mks[c];
    const int rank = __popcll(mk & lt_mask);
    const int32_t base = valid ? wcnt[wave][d] : 0;
    if (valid && rank == 0) wcnt[wave][d] = base + __popcll(mk);  // after every lane's read
    const int lp = base + rank;
    if (valid && (unsigned)lp < (unsigned)m) {
      skey[lp] = kk[c];
      sval[lp] = vin[tile0 + e];
      if (pin) srec[lp] = pin[tile0 + e];
    }
  }
  __syncthreads();
  for (int i = t; i < m; i += kScatterThreads) {
    const uint32_t key = skey[i];
    const uint32_t d = (key >> shift) & 255u;
    const int32_t dst = gbase[d] + (i - loff[d]);
    if ((uint64_t)(uint32_t)dst >= (uint64_t)n) continue;  // only if the counts were inconsistent
    kout[dst] = key;
    vout[dst] = sval[i];
    if (pin) pout[dst] = srec[i];
  }
}

size_t radix_hist_entries(int64_t maxn) {
  const int64_t ntiles = (maxn + kRadixTile - 1) / kRadixTile;
  return (size_t)(256 * (ntiles > 0 ? ntiles : 1));
}

int radix_sort(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n,
               int bits, int32_t* hist, int32_t* tot, hipStream_t st, bool first_hist_done,
               float4* recs, float4* recs_alt) {
  const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  const int passes = bits <= 0 ? 0 : (bits + 7) / 8;
  if (passes == 0 || n <= 0) return 0;
  uint32_t* ki = keys;
  int32_t* vi = vals;
  uint32_t* ko = keys_alt;
  int32_t* vo = vals_alt;
  float4* pi = recs;
  float4* po = recs_alt;
  const size_t lds = recs ? sizeof(float4) * kRadixTile : 0;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = 8 * ps;
    if (ps > 0 || !first_hist_done)
      hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(256), 0, st, ki, n, shift, hist, ntiles);
    hipLaunchKernelGGL(k_scan_rows, dim3(256), dim3(256), 0, st, hist, ntiles, tot);
    hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(kScatterThreads), lds, st, ki, vi, ko, vo,
                       n, shift, hist, tot, ntiles, pi, po);
    std::swap(ki, ko);
    std::swap(vi, vo);
    std::swap(pi, po);
  }
  return passes & 1;
}

// ---------------------------------------------------------------------------
// Keys of 9..16 bits: two digits.  The first pass scatters by the high digit
// (key >> 8; the binning counted it), which leaves each high digit's elements
// in one contiguous bucket, in input order; then each bucket is sorted stably
// by the low 8 bits and the leaf offsets of its 256 keys are written from the
// same counts, which replaces the second pass's count, scan and scatter and
// the leaf-offset search.  Two launches share the buckets.  The first has one
// workgroup per bucket: a bucket that fits the LDS stage is placed there at
// its final order and written out in one coalesced sweep; for a larger one
// (clustered inputs) it counts the digits of each of the bucket's
// kBucketSplit parts into a table.  In the second, the kBucketSplit
// workgroups of such a bucket each place one part, their digit offsets taken
// from the table, straight to the final places (the workgroups of the other
// buckets leave at once).  Inside a workgroup every wave takes a contiguous
// piece: after one count of each wave's digits and one scan, the waves rank
// and place their pieces 64 keys at a time with no further barrier (a wave's
// running digit offsets in LDS, read and advanced in program order).
constexpr int kBucketCap = 5120;  // elements of a bucket the LDS stage holds
constexpr int kBucketSplit = 8;   // parts of a bucket beyond the stage

// First place and size of bucket b from the digit totals (every thread of the
// workgroup calls it; one block scan).
template <int NT>
__device__ __forceinline__ void bucket_range(const int32_t* __restrict__ tot, int64_t n, int b,
                                             int32_t* wt, int64_t* s_b0, int32_t* s_m) {
  const int t = threadIdx.x;
  int32_t all;
  const int32_t ex = block_exclusive_scan<NT>(t < 256 ? tot[t] : 0, wt, &all);
  if (t == b) {
    *s_b0 = ex;
    const int64_t m = tot[t];
    *s_m = (int32_t)(ex + m <= n ? m : (n > ex ? n - ex : 0));  // (only if the counts were inconsistent)
  }
  __syncthreads();
}

// Part s of a bucket of m elements: [s per, min(m, (s + 1) per)).
__device__ __forceinline__ int bucket_part_size(int m) {
  return (m + kBucketSplit - 1) / kBucketSplit;
}

template <int NT, bool STAGED>
__global__ __launch_bounds__(NT) void k_bucket_sort(
    const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin,
    const float4* __restrict__ pin, uint32_t* __restrict__ kout, int32_t* __restrict__ vout,
    float4* __restrict__ pout, int64_t n, const int32_t* __restrict__ tot,
    int32_t* __restrict__ leaf_start, int64_t nleaf, int32_t* __restrict__ parts) {
  static_assert(NT >= 256, "one thread per digit");
  constexpr int NW = NT / 64;
  // chunks of 64 keys a wave holds at once: a staged bucket's whole piece, so
  // that its keys, values and records are loaded once, up front
  constexpr int G = STAGED ? (kBucketCap / NW + 63) / 64 : 4;
  extern __shared__ __align__(16) unsigned char bsmem[];  // STAGED: keys, values [, records]
  __shared__ int32_t wcnt[NW][256];
  __shared__ int32_t pre[256], all_cnt[256];
  __shared__ int32_t wt[NW];
  __shared__ int64_t s_b0;
  __shared__ int32_t s_m;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int b = STAGED ? (int)blockIdx.x : (int)blockIdx.x / kBucketSplit;
  const int part = STAGED ? 0 : (int)blockIdx.x % kBucketSplit;
  bucket_range<NT>(tot, n, b, wt, &s_b0, &s_m);
  const int64_t b0 = s_b0;
  const int m = s_m;
  const bool fits = m <= kBucketCap;
  if (!STAGED && fits) return;  // sorted by the first launch (workgroup-uniform)
  const int per = bucket_part_size(m);
  if (STAGED && !fits) {
    // count the digits of each part of this bucket into parts[b][s][256]
    for (int s = 0; s < kBucketSplit; ++s) {
      if (t < 256) all_cnt[t] = 0;
      __syncthreads();
      const int plo = min(m, s * per), phi = min(m, plo + per);
      for (int g0 = plo + wave * 64 * G; g0 < phi; g0 += NT * G) {
        uint32_t k2[G];
#pragma unroll
        for (int c = 0; c < G; ++c) {
          const int e = g0 + 64 * c + lane;
          k2[c] = e < phi ? kin[b0 + e] : 0u;
        }
#pragma unroll
        for (int c = 0; c < G; ++c)
          if (g0 + 64 * c < phi) count_digits(all_cnt, k2[c] & 255u, g0 + 64 * c + lane < phi);
      }
      __syncthreads();
      if (t < 256) parts[((int64_t)b * kBucketSplit + s) * 256 + t] = all_cnt[t];
    }
    return;
  }
  const int lo = STAGED ? 0 : min(m, part * per), hi = STAGED ? m : min(m, lo + per);
  const int wper = (hi - lo + NW - 1) / NW;  // STAGED: at most 64 G
  const int wlo = min(hi, lo + wave * wper), whi = min(hi, wlo + wper);  // this wave's piece
  if (t < 256) {
#pragma unroll
    for (int w = 0; w < NW; ++w) wcnt[w][t] = 0;
    if (STAGED) {
      pre[t] = 0;
    } else {
      // the bucket's digit counts and those of the parts before this one
      int32_t a = 0, p = 0;
      for (int s = 0; s < kBucketSplit; ++s) {
        const int32_t c = parts[((int64_t)b * kBucketSplit + s) * 256 + t];
        a += c;
        if (s < part) p += c;
      }
      all_cnt[t] = a;
      pre[t] = p;
    }
  }
  uint32_t kk[G];
  int32_t vv[G];
  float4 rr[G];
  if (STAGED) {
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const int e = wlo + 64 * c + lane;
      const bool ok = e < whi;
      kk[c] = ok ? kin[b0 + e] : 0u;
      vv[c] = ok ? vin[b0 + e] : 0;
      if (pin) rr[c] = ok ? pin[b0 + e] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  __syncthreads();
  // digit counts of each wave's piece
  if (STAGED) {
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (wlo + 64 * c + lane < whi) atomicAdd(&wcnt[wave][kk[c] & 255u], 1);
  } else {
    for (int g0 = wlo; g0 < whi; g0 += 64 * G) {
#pragma unroll
      for (int c = 0; c < G; ++c) {
        const int e = g0 + 64 * c + lane;
        kk[c] = e < whi ? kin[b0 + e] : 0u;
      }
#pragma unroll
      for (int c = 0; c < G; ++c)
        if (g0 + 64 * c < whi) count_digits(wcnt[wave], kk[c] & 255u, g0 + 64 * c + lane < whi);
    }
  }
  __syncthreads();
  {
    int32_t c = 0;
    if (t < 256) {
      if (STAGED) {
#pragma unroll
        for (int w = 0; w < NW; ++w) c += wcnt[w][t];
      } else {
        c = all_cnt[t];
      }
    }
    int32_t all;
    const int32_t ex = block_exclusive_scan<NT>(c, wt, &all);
    if (t < 256) {
      const int64_t leaf = ((int64_t)b << 8) | t;
      if (part == 0 && leaf < nleaf) leaf_start[leaf] = (int32_t)(b0 + ex);
      // each wave's first place for digit t inside the bucket
      int32_t o = ex + pre[t];
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const int32_t k = wcnt[w][t];
        wcnt[w][t] = o;
        o += k;
      }
    }
    if (b == 0 && part == 0 && t == 0) leaf_start[nleaf] = (int32_t)n;
  }
  __syncthreads();
  uint32_t* skey = reinterpret_cast<uint32_t*>(bsmem);
  int32_t* sval = reinterpret_cast<int32_t*>(skey + kBucketCap);
  float4* srec = reinterpret_cast<float4*>(sval + kBucketCap);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int g0 = wlo; g0 < whi; g0 += 64 * G) {  // wave-uniform (STAGED: once)
    if (!STAGED) {
#pragma unroll
      for (int c = 0; c < G; ++c) {
        const int e = g0 + 64 * c + lane;
        const bool ok = e < whi;
        kk[c] = ok ? kin[b0 + e] : 0u;
        vv[c] = ok ? vin[b0 + e] : 0;
        if (pin) rr[c] = ok ? pin[b0 + e] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int c = 0; c < G; ++c) {
      if (g0 + 64 * c >= whi) break;  // wave-uniform
      const bool valid = g0 + 64 * c + lane < whi;
      const uint32_t d = kk[c] & 255u;
      const uint64_t mk = digit_match(d, valid);
      const int rank = __popcll(mk & lt_mask);
      const int32_t base = valid ? wcnt[wave][d] : 0;
      if (valid && rank == 0) wcnt[wave][d] = base + __popcll(mk);  // after every lane's read
      const int lp = base + rank;
      if (valid && (unsigned)lp < (unsigned)m) {
        if (STAGED) {
          skey[lp] = kk[c];
          sval[lp] = vv[c];
          if (pin) srec[lp] = rr[c];
        } else {
          kout[b0 + lp] = kk[c];
          vout[b0 + lp] = vv[c];
          if (pin) pout[b0 + lp] = rr[c];
        }
      }
    }
  }
  if (STAGED) {
    __syncthreads();
    for (int i = t; i < m; i += NT) {
      kout[b0 + i] = skey[i];
      vout[b0 + i] = sval[i];
      if (pin) pout[b0 + i] = srec[i];
    }
  }
}

bool radix_two_digit(int64_t n, int bits) {
  if (bits <= 8 || bits > 16 || n <= 0) return false;
  const int64_t buckets = (int64_t)1 << (bits - 8);
  return n <= buckets * (kBucketCap * 9 / 10);  // the mean bucket well inside the stage
}

size_t radix_two_digit_parts() { return (size_t)256 * kBucketSplit * 256; }

void radix_sort_two_digit(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt,
                          int64_t n, int bits, int32_t* hist, int32_t* tot, int32_t* leaf_start,
                          int64_t nleaf, int32_t* parts, hipStream_t st, float4* recs,
                          float4* recs_alt) {
  const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  const size_t lds = recs ? sizeof(float4) * kRadixTile : 0;
  hipLaunchKernelGGL(k_scan_rows, dim3(256), dim3(256), 0, st, hist, ntiles, tot);
  hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(kScatterThreads), lds, st, keys, vals,
                     keys_alt, vals_alt, n, 8, hist, tot, ntiles, recs, recs_alt);
  const size_t blds = (size_t)kBucketCap * (sizeof(uint32_t) + sizeof(int32_t) +
                                            (recs ? sizeof(float4) : 0));
  if (blds > 65536)
    (void)hipFuncSetAttribute((const void*)k_bucket_sort<1024, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)blds);
  const unsigned buckets = 1u << (bits - 8);
  hipLaunchKernelGGL((k_bucket_sort<1024, true>), dim3(buckets), dim3(1024), blds, st, keys_alt,
                     vals_alt, recs_alt, keys, vals, recs, n, tot, leaf_start, nleaf, parts);
  hipLaunchKernelGGL((k_bucket_sort<512, false>), dim3(buckets * kBucketSplit), dim3(512), 0, st,
                     keys_alt, vals_alt, recs_alt, keys, vals, recs, n, tot, leaf_start, nleaf,
                     parts);
}

// leaf_start[l] = lower_bound(sorted_keys, l), l = 0..nleaf.  (A binary
// search per leaf: its cost does not depend on how the particles cluster,
// unlike a scan over key boundaries, which serialises the long runs of empty
// leaves of clustered inputs.)
__global__ void k_leaf_bounds(const uint32_t* __restrict__ keys, int64_t n, int64_t nleaf,
                              int32_t* __restrict__ leaf_start) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l > nleaf) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] < l)
      lo = mid + 1;
    else
      hi = mid;
  }
  leaf_start[l] = (int32_t)lo;
}

void launch_leaf_bounds(const uint32_t* sorted_keys, int64_t n, int64_t nleaf, int32_t* leaf_start,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_leaf_bounds, dim3((nleaf + 1 + 255) / 256), dim3(256), 0, st, sorted_keys,
                     n, nleaf, leaf_start);
}

template <int D>
__global__ __launch_bounds__(256) void k_gather_f64(const double* __restrict__ pos,
                                                    const double* __restrict__ q,
                                                    const int32_t* __restrict__ perm, int64_t n,
                                                    double* __restrict__ xs, double* __restrict__ ys,
                                                    double* __restrict__ zs,
                                                    double* __restrict__ qs,
                                                    const BatchIo* __restrict__ io) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (io) {
    pos = io->pos;
    q = io->q;
  }
  const int64_t i = perm[j];
  xs[j] = pos[D * i];
  ys[j] = pos[D * i + 1];
  if (D == 3) zs[j] = pos[D * i + 2];
  qs[j] = q[i];
}

void launch_gather_f64(int dim, const double* pos, const double* q, const int32_t* perm, int64_t n,
                       double* xs, double* ys, double* zs, double* qs, hipStream_t st,
                       const BatchIo* io) {
  const int64_t blocks = (n + 255) / 256;
  if (dim == 2)
    hipLaunchKernelGGL(k_gather_f64<2>, dim3(blocks), dim3(256), 0, st, pos, q, perm, n, xs, ys,
                       zs, qs, io);
  else
    hipLaunchKernelGGL(k_gather_f64<3>, dim3(blocks), dim3(256), 0, st, pos, q, perm, n, xs, ys,
                       zs, qs, io);
}



}  // namespace sffmm

namespace sffmm {

// Batched 2D binning, one radix tile per workgroup (as k_bin).  Particle i
// belongs to system s with sys_off[s] <= i < sys_off[s+1]; info[2s] = rank of s
// in (depth, index) order, info[2s+1] = its depth L_s.  The sort key puts the
// rank above a Morton code scaled to depth lmax (the deepest system), so one
// sort groups particles by depth, then system, then leaf.  The leaf
// coordinate uses the same FP64 expression as a single system.  The tile's
// first system comes from one binary search; each thread then walks forward
// (systems hold many particles, so rarely more than one step).  Also writes the
// tile's histogram of the first radix digit.
__global__ __launch_bounds__(256) void k_bin_batched(const double* __restrict__ pos, int64_t n,
                                                     const int64_t* __restrict__ sys_off, int nsys,
                                                     const int32_t* __restrict__ info, double ox,
                                                     double oy, double side, int lmax,
                                                     uint32_t* __restrict__ keys,
                                                     int32_t* __restrict__ vals, int32_t* flag,
                                                     int32_t tag, const double* __restrict__ q,
                                                     float4* __restrict__ rec,
                                                     int32_t* __restrict__ hist, int64_t ntiles,
                                                     const BatchIo* __restrict__ io) {
  __shared__ int32_t cnt[256];
  __shared__ int s_first;
  if (io) {
    pos = io->pos;
    q = io->q;
  }
  const int64_t tile0 = (int64_t)blockIdx.x * kRadixTile;
  cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    int lo = 0, hi = nsys - 1;  // last s with sys_off[s] <= tile0
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sys_off[mid] <= tile0)
        lo = mid;
      else
        hi = mid - 1;
    }
    s_first = lo;
  }
  __syncthreads();
  int s = s_first;
  const double o[2] = {ox, oy};
  for (int r = 0; r < kRadixTile / 256; ++r) {
    const int64_t i = tile0 + r * 256 + threadIdx.x;
    if (i >= n) break;
    while (s + 1 < nsys && sys_off[s + 1] <= i) ++s;
    const int L = info[2 * s + 1];
    const int64_t nl = (int64_t)1 << L;
    const double scale = (double)nl / side;
    uint32_t c[2] = {0, 0};
    bool bad = false;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const double x = pos[2 * i + d];
      if (!(x >= o[d] && x <= o[d] + side)) {
        bad = true;
        continue;
      }
      int64_t li = (int64_t)floor(__dmul_rn(__dsub_rn(x, o[d]), scale));
      if (li > nl - 1) li = nl - 1;
      c[d] = (uint32_t)li;
    }
    if (bad) flag[0] = tag;  // every writer stores the same value
    const uint32_t m = spread2(c[0]) | (spread2(c[1]) << 1);
    const uint32_t key = ((uint32_t)info[2 * s] << (2 * lmax)) | (m << (2 * (lmax - L)));
    keys[i] = key;
    vals[i] = (int32_t)i;
    if (rec) rec[i] = leaf_record<2>(pos, q, i, m, o, side / (double)nl);
    atomicAdd(&cnt[key & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

void launch_bin_batched(const double* pos, int64_t n, const int64_t* sys_off, int nsys,
                        const int32_t* info, const LevelTable& lt, int lmax, uint32_t* keys,
                        int32_t* vals, int32_t* flag, int32_t tag, int32_t* hist,
                        hipStream_t st, const double* q, float4* rec, const BatchIo* io) {
  if (n <= 0) return;
  const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  hipLaunchKernelGGL(k_bin_batched, dim3((unsigned)ntiles), dim3(256), 0, st, pos, n, sys_off,
                     nsys, info, lt.origin[0], lt.origin[1], lt.side, lmax, keys, vals, flag, tag,
                     q, rec, hist, ntiles, io);
}

// Start of a batched replay: the caller's buffer addresses into the record the
// graph's kernels read, and the caller's device system tables checked against
// the prepared shape (the graph runs the prepared tables; a caller table that
// differs is an argument error, reported through flag[2]).
__global__ __launch_bounds__(1024) void k_batch_begin(BatchIo* __restrict__ io,
                                                      const double* pos, const double* q,
                                                      double* pot, double* field,
                                                      const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ levels,
                                                      const int64_t* __restrict__ prep_off,
                                                      const int32_t* __restrict__ prep_info,
                                                      int nsys, int lmax, int32_t* flag,
                                                      int32_t tag) {
  __shared__ int bad;
  if (threadIdx.x == 0) {
    io->pos = pos;
    io->q = q;
    io->pot = pot;
    io->field = field;
    bad = 0;
  }
  __syncthreads();
  bool b = false;
  for (int s = threadIdx.x; s <= nsys; s += blockDim.x) {
    b = b || off[s] != prep_off[s];
    if (s < nsys) {
      int L;
      if (levels) {
        L = levels[s];
      } else {  // clamp(round(log4(n_s / 16)), 2, lmax), as the host rule
        const double ns = (double)(off[s + 1] - off[s]);
        L = ns > 0 ? (int)lround(log(ns / 16.0) / log(4.0)) : 2;
        L = min(max(L, 2), lmax);
      }
      b = b || L != prep_info[2 * s + 1];
    }
  }
  if (b) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) flag[2] = bad ? tag : 0;
}

void launch_batch_begin(BatchIo* io, const double* pos, const double* q, double* pot,
                        double* field, const int64_t* off, const int32_t* levels,
                        const int64_t* prep_off, const int32_t* prep_info, int nsys, int lmax,
                        int32_t* flag, int32_t tag, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(1024), 0, st, io, pos, q, pot, field, off,
                     levels, prep_off, prep_info, nsys, lmax, flag, tag);
}

// Rewrites the sorted batched keys of one depth group (ranks r0.., depth L) as
// stacked keys ((rank - r0) << 2L) | Morton at depth L.
__global__ void k_rekey(uint32_t* __restrict__ keys, int64_t n, int r0, int L, int lmax) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint32_t k = keys[j];
  const uint32_t rank = k >> (2 * lmax);
  const uint32_t m = (k & ((2 * lmax >= 32) ? 0xFFFFFFFFu : ((1u << (2 * lmax)) - 1u))) >> (2 * (lmax - L));
  keys[j] = ((rank - (uint32_t)r0) << (2 * L)) | m;
}

void launch_rekey(uint32_t* keys, int64_t n, int r0, int L, int lmax, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_rekey, dim3((n + 255) / 256), dim3(256), 0, st, keys, n, r0, L, lmax);
}

}  // namespace sffmm
