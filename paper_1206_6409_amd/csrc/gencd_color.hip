// Greedy partial distance-2 colouring of the column conflict graph
// (section 4.1: columns conflict when they share a row), computed on the GPU
// and identical to the sequential greedy colouring.
//
// The sequential greedy visits columns in priority order (decreasing nnz,
// ties by index) and gives each the smallest colour not used by an earlier
// column sharing a row.  A column's colour depends only on the colours of its
// earlier neighbours, so columns can be coloured in rounds (Jones-Plassmann
// by priority): a column is ready once all its earlier neighbours are
// coloured.  Readiness is tracked with a counter per column holding the
// number of (row, earlier column) pairs still uncoloured:
//   * CSR rows are sorted by column priority, so the earlier neighbours of a
//     column in a row are the prefix of that row before it; the counter
//     starts at the sum of these prefix lengths;
//   * when a column is coloured it decrements, in each of its rows, every
//     later column of the row; a counter reaching zero puts the column in the
//     next round's frontier.
// Each frontier column takes the mex of the colours in its row prefixes.
// A small frontier (the heavy columns come first and form long chains of
// single-column rounds) spreads its row prefixes over the whole grid, into
// a bitmap per frontier column in global memory; a large one takes one
// workgroup per column with the bitmap in LDS.
#include <vector>

#include "gencd_common.hpp"
#include "gencd_kernels.hpp"

namespace gencd {

constexpr int kMexWords = 8192;  // LDS bitmap: 262144 colours
constexpr int kFlatMax = 64;     // frontiers up to this size use the spread mex
// Lanes that share one CSC entry's row prefix (mex) or row suffix
// (readiness counts): a row holds ~30 entries on the Lasso workload, so one
// or two rounds of loads instead of a serial walk.
constexpr int kSG = 16;

struct ColorWs {
  uint32_t *keys_a, *keys_b;  // [max(k, nnz)] radix sort keys
  int32_t *vals_a, *vals_b;   // [max(k, nnz)] radix sort values
  int32_t *order;             // [k] column at each priority rank
  int32_t *rank;              // [k] priority rank of each column
  int32_t *roff;              // [k+1] first slot of each rank's entries in the rank-ordered list
  int32_t *erank;             // [nnz] priority rank of the column of each CSC entry
  int32_t *row_ptr;           // [n+1]
  int32_t *rank_at;           // [nnz] CSR slot -> column rank
  int32_t *pos_in_row;        // [nnz] CSC entry -> position in its CSR row
  int32_t *count;             // [k]
  int32_t *front_a, *front_b; // [k]
  int32_t *fcnt;              // [k+1] frontier nnz counts, then offsets
  int32_t *foff;              // [k+1]
  int32_t *scan_part;
  int32_t *rhist, *roffs;     // [radix_hist_len(max(k, nnz))] radix digit counts, offsets
  int32_t *ctl;               // [8] frontier sizes (0, 4: by round parity), max colour
                              // snapshot (1), error flag (2), max colour (3), coloured (5)
  uint32_t *gbits;            // [kFlatMax][kMexWords] colour bitmaps of a small frontier
                              // (all zero between rounds)
};

static size_t color_layout(int64_t n, int64_t k, int64_t nnz, void *base, ColorWs *w) {
  const size_t al = 256;
  size_t off = 0;
  char *b = static_cast<char *>(base);
  auto take = [&](size_t bytes) -> void * {
    off = (off + al - 1) / al * al;
    void *p = b ? b + off : nullptr;
    off += bytes > 0 ? bytes : 1;
    return p;
  };
  const int64_t m = k > nnz ? k : nnz;
  ColorWs c{};
  c.keys_a = static_cast<uint32_t *>(take(sizeof(uint32_t) * m));
  c.keys_b = static_cast<uint32_t *>(take(sizeof(uint32_t) * m));
  c.vals_a = static_cast<int32_t *>(take(sizeof(int32_t) * m));
  c.vals_b = static_cast<int32_t *>(take(sizeof(int32_t) * m));
  c.order = static_cast<int32_t *>(take(sizeof(int32_t) * k));
  c.rank = static_cast<int32_t *>(take(sizeof(int32_t) * k));
  c.roff = static_cast<int32_t *>(take(sizeof(int32_t) * (k + 1)));
  c.erank = static_cast<int32_t *>(take(sizeof(int32_t) * nnz));
  c.row_ptr = static_cast<int32_t *>(take(sizeof(int32_t) * (n + 1)));
  c.rank_at = static_cast<int32_t *>(take(sizeof(int32_t) * nnz));
  c.pos_in_row = static_cast<int32_t *>(take(sizeof(int32_t) * nnz));
  c.count = static_cast<int32_t *>(take(sizeof(int32_t) * k));
  c.front_a = static_cast<int32_t *>(take(sizeof(int32_t) * k));
  c.front_b = static_cast<int32_t *>(take(sizeof(int32_t) * k));
  const int64_t mn = m > n ? m : n;
  c.fcnt = static_cast<int32_t *>(take(sizeof(int32_t) * (mn + 1)));
  c.foff = static_cast<int32_t *>(take(sizeof(int32_t) * (k + 1)));
  const int64_t rl = radix_hist_len(m);
  const int64_t scan_len = mn + 1 > rl ? mn + 1 : rl;
  c.scan_part = static_cast<int32_t *>(take(sizeof(int32_t) * scan_partials_for(scan_len)));
  c.rhist = static_cast<int32_t *>(take(sizeof(int32_t) * rl));
  c.roffs = static_cast<int32_t *>(take(sizeof(int32_t) * rl));
  c.ctl = static_cast<int32_t *>(take(sizeof(int32_t) * 8));
  c.gbits = static_cast<uint32_t *>(take(sizeof(uint32_t) * kFlatMax * kMexWords));
  if (w) *w = c;
  return off + al;
}

// priority key n - nnz_j: a stable sort of the columns (natural order) by it
// gives decreasing nnz, ties by index
__global__ __launch_bounds__(kBlock) void k_prio_keys(const int64_t *col_ptr, int64_t k, int64_t n,
                                                       uint32_t *keys, int32_t *vals) {
  for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < k;
       j += int64_t(gridDim.x) * kBlock) {
    int64_t m = col_ptr[j + 1] - col_ptr[j];
    keys[j] = uint32_t(n - m);
    vals[j] = int32_t(j);
  }
}

// rank of every column and the nnz of the column at every rank
__global__ __launch_bounds__(kBlock) void k_rank_of(const int32_t *order, int64_t k,
                                                     const int64_t *col_ptr, int32_t *rank,
                                                     int32_t *rnnz) {
  for (int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x; r < k;
       r += int64_t(gridDim.x) * kBlock) {
    const int32_t j = order[r];
    rank[j] = int32_t(r);
    rnnz[r] = int32_t(col_ptr[j + 1] - col_ptr[j]);
  }
}

// One wave per rank: the CSC entries listed column by column in priority
// order (sort key: the entry's row, value: the entry), the rank of every
// entry's column, and the row histogram.  A stable sort of this list by row
// leaves each row's entries in priority order.
__global__ __launch_bounds__(kBlock) void k_csr_list(const int64_t *col_ptr, const int32_t *row_idx,
                                                      int64_t k, const int32_t *order,
                                                      const int32_t *roff, uint32_t *keys,
                                                      int32_t *vals, int32_t *erank, int32_t *hist) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wid = (int64_t(blockIdx.x) * kBlock + threadIdx.x) / kWave;
  const int64_t nw = int64_t(gridDim.x) * kBlock / kWave;
  for (int64_t r = wid; r < k; r += nw) {
    const int32_t j = order[r];
    const int64_t e0 = col_ptr[j], e1 = col_ptr[j + 1];
    const int64_t p0 = roff[r];
    for (int64_t e = e0 + lane; e < e1; e += kWave) {
      const int32_t row = row_idx[e];
      keys[p0 + (e - e0)] = uint32_t(row);
      vals[p0 + (e - e0)] = int32_t(e);
      erank[e] = int32_t(r);
      atomicAdd(&hist[row], 1);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_csr_fill(const uint32_t *rows, const int32_t *ents,
                                                      int64_t nnz, const int32_t *row_ptr,
                                                      const int32_t *erank, int32_t *rank_at,
                                                      int32_t *pos_in_row) {
  for (int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x; q < nnz;
       q += int64_t(gridDim.x) * kBlock) {
    const int32_t row = int32_t(rows[q]);
    const int32_t e = ents[q];
    rank_at[q] = erank[e];
    pos_in_row[e] = int32_t(q) - row_ptr[row];
  }
}

// counter = number of (row, earlier column) pairs; frontier = columns with 0
__global__ __launch_bounds__(kBlock) void k_init_count(const int64_t *col_ptr, int64_t k,
                                                        const int32_t *pos_in_row, int32_t *count,
                                                        int32_t *color, int32_t *front,
                                                        int32_t *ctl) {
  // An empty column has no neighbours: the greedy order gives it colour 0
  // (the mex of nothing) whenever it is visited, so it is coloured here and
  // counted once per workgroup instead of joining the first frontier, where
  // the many empty columns would queue on one counter.
  __shared__ int32_t nempty;
  if (threadIdx.x == 0) nempty = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wid = (int64_t(blockIdx.x) * kBlock + threadIdx.x) / kWave;
  const int64_t nw = int64_t(gridDim.x) * kBlock / kWave;
  for (int64_t j = wid; j < k; j += nw) {
    const int64_t e0 = col_ptr[j], e1 = col_ptr[j + 1];
    int32_t s = 0;
    for (int64_t e = e0 + lane; e < e1; e += kWave) s += pos_in_row[e];
    s = group_sum<kWave>(s);
    if (lane == 0) {
      count[j] = s;
      if (e1 == e0) {
        color[j] = 0;
        atomicAdd(&nempty, 1);
      } else {
        color[j] = -1;
        if (s == 0) front[atomicAdd(&ctl[0], 1)] = int32_t(j);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && nempty > 0) {
    atomicAdd(&ctl[5], nempty);  // coloured columns
    atomicMax(&ctl[3], 0);       // largest colour so far
  }
}

// colour of each frontier column: mex of the colours in its row prefixes
// (one workgroup per frontier column, LDS bitmap of the colours so far)
__device__ void mex_blocks(int64_t vb, int64_t nvb, uint32_t *bits, int32_t &best,
                           const int32_t *Fp, const int64_t *col_ptr, const int32_t *row_idx,
                           const int32_t *front, const int32_t *row_ptr, const int32_t *rank_at,
                           const int32_t *pos_in_row, const int32_t *order, int32_t *color,
                           int32_t *ctl) {
  const int32_t F = *Fp;
  if (F <= kFlatMax) return;  // k_mex_flat / k_mex_pick take small frontiers
  const int32_t maxc = ctl[1];  // largest colour so far (-1 initially)
  int32_t words = (maxc + 2 + 31) / 32;
  if (words > kMexWords) words = kMexWords;
  for (int64_t f = vb; f < F; f += nvb) {
    const int32_t j = front[f];
    for (int32_t u = threadIdx.x; u < words; u += kBlock) bits[u] = 0u;
    if (threadIdx.x == 0) best = INT32_MAX;
    __syncthreads();
    const int sub = int(threadIdx.x) / kSG, l = int(threadIdx.x) % kSG;
    for (int64_t e = col_ptr[j] + sub; e < col_ptr[j + 1]; e += kBlock / kSG) {
      const int32_t r = row_idx[e];
      const int32_t a = row_ptr[r], b = a + pos_in_row[e];
      for (int32_t q = a + l; q < b; q += kSG) {
        const int32_t c = color[order[rank_at[q]]];
        if (c >= 0 && c < kMexWords * 32) atomicOr(&bits[c >> 5], 1u << (c & 31));
      }
    }
    __syncthreads();
    int32_t mine = INT32_MAX;
    for (int32_t u = threadIdx.x; u < words; u += kBlock) {
      const uint32_t free_bits = ~bits[u];
      if (free_bits) {
        mine = u * 32 + __ffs(int(free_bits)) - 1;
        break;
      }
    }
    if (mine != INT32_MAX) atomicMin(&best, mine);
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t c = best == INT32_MAX ? words * 32 : best;
      if (c >= kMexWords * 32) {
        atomicOr(&ctl[2], 1);
        c = kMexWords * 32 - 1;
      }
      color[j] = c;
      atomicMax(&ctl[3], c);
    }
    __syncthreads();
  }
}

// Small frontier, first pass: the frontier's CSC entries, in order, are cut
// into one contiguous chunk per workgroup.  A workgroup marks the colours of
// its entries' row prefixes in an LDS bitmap, column by column of its
// chunk, and ORs each nonzero word into that column's global bitmap (one
// global atomic per word and workgroup: the heavy columns' prefixes would
// otherwise pile millions of atomics onto a few words).
__device__ void mex_flat_blocks(int64_t vb, int64_t nvb, uint32_t *bits, const int32_t *Fp,
                                const int32_t *foff, const int32_t *front, const int64_t *col_ptr,
                                const int32_t *row_idx, const int32_t *row_ptr,
                                const int32_t *rank_at, const int32_t *pos_in_row,
                                const int32_t *order, const int32_t *color, const int32_t *ctl,
                                uint32_t *gbits) {
  const int32_t F = *Fp;
  if (F > kFlatMax || F == 0) return;
  const int32_t total = foff[F];
  const int32_t maxc = ctl[1];
  int32_t words = (maxc + 2 + 31) / 32;
  if (words > kMexWords) words = kMexWords;
  const int32_t chunk = int32_t((int64_t(total) + nvb - 1) / nvb);
  int32_t t0 = int32_t(vb * chunk);
  const int32_t t1 = int32_t(std::min<int64_t>(int64_t(t0) + chunk, total));
  if (t0 >= t1) return;
  int32_t f = 0, hi = F;  // last f with foff[f] <= t0
  while (hi - f > 1) {
    const int32_t mid = (f + hi) >> 1;
    if (foff[mid] <= t0) f = mid; else hi = mid;
  }
  while (t0 < t1) {
    const int32_t fe = std::min(t1, foff[f + 1]);
    for (int32_t u = threadIdx.x; u < words; u += kBlock) bits[u] = 0u;
    __syncthreads();
    const int64_t cbeg = col_ptr[front[f]] - foff[f];
    const int sub = int(threadIdx.x) / kSG, l = int(threadIdx.x) % kSG;
    for (int32_t t = t0 + sub; t < fe; t += kBlock / kSG) {
      const int64_t e = cbeg + t;
      const int32_t r = row_idx[e];
      const int32_t a = row_ptr[r], b = a + pos_in_row[e];
      for (int32_t q = a + l; q < b; q += kSG) {
        const int32_t c = color[order[rank_at[q]]];
        if (c >= 0 && c < words * 32) atomicOr(&bits[c >> 5], 1u << (c & 31));
      }
    }
    __syncthreads();
    uint32_t *g = gbits + int64_t(f) * kMexWords;
    for (int32_t u = threadIdx.x; u < words; u += kBlock)
      if (bits[u]) atomicOr(&g[u], bits[u]);
    __syncthreads();
    t0 = fe;
    ++f;
  }
}

// Small frontier, second pass: one workgroup per frontier column takes the
// lowest clear bit of its bitmap, then clears the words it read.  The last
// workgroup to finish (by a ticket) also ends the round: the snapshot of
// the largest colour for the next round's mex, the running count of
// coloured columns, and a zero count for the round after next (`fc`, this
// round's frontier counter, read by no later kernel of the round).
__global__ __launch_bounds__(kBlock) void k_mex_pick(int32_t *Fp, const int32_t *front,
                                                      int32_t *color, int32_t *ctl,
                                                      uint32_t *gbits) {
  __shared__ int32_t best;
  const int32_t F = *Fp;
  const int32_t maxc = ctl[1];
  int32_t words = (maxc + 2 + 31) / 32;
  if (words > kMexWords) words = kMexWords;
  for (int32_t f = blockIdx.x; F <= kFlatMax && f < F; f += gridDim.x) {
    uint32_t *bits = gbits + int64_t(f) * kMexWords;
    if (threadIdx.x == 0) best = INT32_MAX;
    __syncthreads();
    int32_t mine = INT32_MAX;
    for (int32_t u = threadIdx.x; u < words; u += kBlock) {
      const uint32_t free_bits = ~bits[u];
      if (free_bits) {
        mine = u * 32 + __ffs(int(free_bits)) - 1;
        break;
      }
    }
    if (mine != INT32_MAX) atomicMin(&best, mine);
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t c = best == INT32_MAX ? words * 32 : best;
      if (c >= kMexWords * 32) {
        atomicOr(&ctl[2], 1);
        c = kMexWords * 32 - 1;
      }
      color[front[f]] = c;
      atomicMax(&ctl[3], c);
    }
    for (int32_t u = threadIdx.x; u < words; u += kBlock) bits[u] = 0u;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&ctl[6], 1) == int32_t(gridDim.x) - 1) {  // every other workgroup is done
      ctl[6] = 0;
      ctl[1] = atomicAdd(&ctl[3], 0);
      ctl[5] += F;
      *Fp = 0;
    }
  }
}

// Offsets of the frontier columns' entries, foff[0..F] (exclusive scan of
// their nonzero counts), in three passes that read F from the device and
// touch only the frontier: tile sums, scan of the tile sums, apply.
constexpr int kFItems = 8;
constexpr int kFTile = kBlock * kFItems;

__device__ __forceinline__ int32_t front_block_scan(int32_t v, int32_t &total) {
  __shared__ int32_t wsum[kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t t = __shfl_up(x, off, kWave);
    if (lane >= off) x += t;
  }
  if (lane == kWave - 1) wsum[wid] = x;
  __syncthreads();
  int32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    if (w < wid) pre += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  total = tot;
  return pre + x - v;
}

__device__ __forceinline__ int32_t front_len(const int32_t *front, const int64_t *col_ptr,
                                             int64_t f, int32_t F) {
  if (f >= F) return 0;
  const int32_t j = front[f];
  return int32_t(col_ptr[j + 1] - col_ptr[j]);
}

__global__ __launch_bounds__(kBlock) void k_fscan_tiles(const int32_t *Fp, const int32_t *front,
                                                         const int64_t *col_ptr, int32_t *part) {
  const int32_t F = *Fp;
  if (int64_t(blockIdx.x) * kFTile >= F) return;  // past the frontier (uniform per workgroup)
  const int64_t base = int64_t(blockIdx.x) * kFTile + int64_t(threadIdx.x) * kFItems;
  int32_t sum = 0;
#pragma unroll
  for (int u = 0; u < kFItems; ++u) sum += front_len(front, col_ptr, base + u, F);
  int32_t tot;
  front_block_scan(sum, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_fscan_part(const int32_t *Fp, int32_t *part) {
  const int64_t np = (int64_t(*Fp) + kFTile - 1) / kFTile;
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < np; b0 += kBlock) {
    const int64_t i = b0 + threadIdx.x;
    const int32_t v = i < np ? part[i] : 0;
    int32_t tot;
    const int32_t ex = front_block_scan(v, tot);
    if (i < np) part[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[np] = carry;
}

__global__ __launch_bounds__(kBlock) void k_fscan_apply(const int32_t *Fp, const int32_t *front,
                                                         const int64_t *col_ptr,
                                                         const int32_t *part, int32_t *foff) {
  const int32_t F = *Fp;
  const int64_t np = (int64_t(F) + kFTile - 1) / kFTile;
  if (blockIdx.x == 0 && threadIdx.x == 0) foff[F] = part[np];
  if (int64_t(blockIdx.x) >= np) return;
  const int64_t base = int64_t(blockIdx.x) * kFTile + int64_t(threadIdx.x) * kFItems;
  int32_t v[kFItems];
  int32_t sum = 0;
#pragma unroll
  for (int u = 0; u < kFItems; ++u) {
    v[u] = front_len(front, col_ptr, base + u, F);
    sum += v[u];
  }
  int32_t tot;
  int32_t ex = front_block_scan(sum, tot) + part[blockIdx.x];
#pragma unroll
  for (int u = 0; u < kFItems; ++u) {
    if (base + u < F) foff[base + u] = ex;
    ex += v[u];
  }
}

// Flattened over the frontier's CSC entries: decrement later row neighbours.
// A heavy column's rows share later columns many times over, so each
// workgroup first sums its decrements per column in an LDS hash table and
// applies one atomic per distinct column (a column whose slot is not found
// within kProbe probes is decremented directly).  The atomic that takes a
// count to zero puts the column in the next frontier.
constexpr int kHash = 2048;
constexpr int kProbe = 8;
__device__ void decrement_blocks(int64_t vb, int64_t nvb, int32_t *hkey, int32_t *hcnt,
                                 const int32_t *Fp, const int64_t *col_ptr, const int32_t *row_idx,
                                 const int32_t *front, const int32_t *foff, const int32_t *row_ptr,
                                 const int32_t *rank_at, const int32_t *pos_in_row,
                                 const int32_t *order, int32_t *count, int32_t *next,
                                 int32_t *next_cnt) {
  const int32_t F = *Fp;
  const int32_t total = foff[F];
  constexpr int EPB = kBlock / kSG;  // entries per workgroup and pass
  if (vb * EPB >= total) return;  // no entries for this workgroup
  for (int32_t u = threadIdx.x; u < kHash; u += kBlock) {
    hkey[u] = -1;
    hcnt[u] = 0;
  }
  __syncthreads();
  const int sub = int(threadIdx.x) / kSG, l = int(threadIdx.x) % kSG;
  for (int64_t t = vb * EPB + sub; t < total; t += nvb * EPB) {
    int32_t lo = 0, hi = F;  // find f with foff[f] <= t < foff[f+1]
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (foff[mid] <= t) lo = mid; else hi = mid;
    }
    const int32_t j = front[lo];
    const int64_t e = col_ptr[j] + (t - foff[lo]);
    const int32_t r = row_idx[e];
    const int32_t b = row_ptr[r + 1];
    for (int32_t q = row_ptr[r] + pos_in_row[e] + 1 + l; q < b; q += kSG) {
      const int32_t j2 = order[rank_at[q]];
      uint32_t h = (uint32_t(j2) * 2654435761u) & (kHash - 1);
      bool done = false;
      for (int p = 0; p < kProbe && !done; ++p, h = (h + 1) & (kHash - 1)) {
        const int32_t prev = atomicCAS(&hkey[h], -1, j2);
        if (prev == -1 || prev == j2) {
          atomicAdd(&hcnt[h], 1);
          done = true;
        }
      }
      if (!done && atomicSub(&count[j2], 1) == 1) next[atomicAdd(next_cnt, 1)] = j2;
    }
  }
  __syncthreads();
  for (int32_t u = threadIdx.x; u < kHash; u += kBlock) {
    const int32_t key = hkey[u];
    if (key >= 0) {
      const int32_t c = hcnt[u];
      if (atomicSub(&count[key], c) == c) next[atomicAdd(next_cnt, 1)] = key;
    }
  }
}

// One launch per round for the three independent jobs of the frontier:
// workgroups [0, gm) colour a large frontier one column per workgroup,
// [gm, gm + gf) spread a small frontier's entries (k_mex_pick finishes it),
// and the rest update the readiness counts.  Colouring reads only colours
// of earlier rounds and the counts are not read by it, so the jobs do not
// depend on each other.  The LDS buffer serves the role a workgroup takes.
__global__ __launch_bounds__(kBlock) void k_round_work(
    const int32_t *Fp, const int64_t *col_ptr, const int32_t *row_idx, const int32_t *front,
    const int32_t *foff, const int32_t *row_ptr, const int32_t *rank_at, const int32_t *pos_in_row,
    const int32_t *order, int32_t *color, int32_t *ctl, uint32_t *gbits, int32_t *count,
    int32_t *next, int32_t *next_cnt, int32_t gm, int32_t gf) {
  __shared__ uint32_t lds[kMexWords];  // mex bitmap, or the decrement hash (2 x kHash ints)
  __shared__ int32_t best;
  static_assert(2 * kHash <= kMexWords, "hash table fits the bitmap buffer");
  const int64_t b = blockIdx.x;
  if (b < gm) {
    mex_blocks(b, gm, lds, best, Fp, col_ptr, row_idx, front, row_ptr, rank_at, pos_in_row,
               order, color, ctl);
  } else if (b < gm + gf) {
    mex_flat_blocks(b - gm, gf, lds, Fp, foff, front, col_ptr, row_idx, row_ptr, rank_at,
                    pos_in_row, order, color, ctl, gbits);
  } else {
    int32_t *h = reinterpret_cast<int32_t *>(lds);
    decrement_blocks(b - gm - gf, int64_t(gridDim.x) - gm - gf, h, h + kHash, Fp, col_ptr,
                     row_idx, front, foff, row_ptr, rank_at, pos_in_row, order, count, next,
                     next_cnt);
  }
}


static unsigned g1(int64_t m, unsigned cap = 4096) {
  int64_t b = (m + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return unsigned(b);
}

int color_run(const gencd_csc *X, int32_t *color, int32_t *num_colors, void *ws_base,
              size_t ws_bytes, hipStream_t s) {
  const int64_t n = X->n, k = X->k, nnz = X->nnz;
  size_t need = color_layout(n, k, nnz, nullptr, nullptr);
  if (!ws_base || ws_bytes < need) return GENCD_ERR_WORKSPACE;
  char *base = static_cast<char *>(ws_base);
  size_t mis = reinterpret_cast<uintptr_t>(base) % 256;
  if (mis) base += 256 - mis;
  ColorWs w{};
  color_layout(n, k, nnz, base, &w);
  int st;
  // priority order: decreasing nnz, ties by index
  hipLaunchKernelGGL(k_prio_keys, dim3(g1(k)), dim3(kBlock), 0, s, X->col_ptr, k, n, w.keys_a,
                     w.vals_a);
  int ob = 0;
  st = radix_sort_pairs(w.keys_a, w.vals_a, w.keys_b, w.vals_b, k, bits_for(uint64_t(n)), w.rhist,
                        w.roffs, w.scan_part, s, &ob);
  if (st) return st;
  st = copy_i32(w.order, ob ? w.vals_b : w.vals_a, k, s);
  if (st) return st;
  hipLaunchKernelGGL(k_rank_of, dim3(g1(k)), dim3(kBlock), 0, s, w.order, k, X->col_ptr, w.rank,
                     w.fcnt);
  st = scan_exclusive(w.fcnt, w.roff, k, w.scan_part, s);
  if (st) return st;
  // CSR with every row's entries in priority order
  st = fill_i32(w.fcnt, n + 1, 0, s);
  if (st) return st;
  hipLaunchKernelGGL(k_csr_list, dim3(g1(k * kWave, 8192)), dim3(kBlock), 0, s, X->col_ptr,
                     X->row_idx, k, w.order, w.roff, w.keys_a, w.vals_a, w.erank, w.fcnt);
  st = scan_exclusive(w.fcnt, w.row_ptr, n, w.scan_part, s);
  if (st) return st;
  if (nnz > 0) {
    st = radix_sort_pairs(w.keys_a, w.vals_a, w.keys_b, w.vals_b, nnz, bits_for(uint64_t(n - 1)),
                          w.rhist, w.roffs, w.scan_part, s, &ob);
    if (st) return st;
    hipLaunchKernelGGL(k_csr_fill, dim3(g1(nnz)), dim3(kBlock), 0, s, ob ? w.keys_b : w.keys_a,
                       ob ? w.vals_b : w.vals_a, nnz, w.row_ptr, w.erank, w.rank_at, w.pos_in_row);
  }
  st = fill_i32(w.ctl, 8, 0, s);
  if (st) return st;
  st = fill_i32(reinterpret_cast<int32_t *>(w.gbits), int64_t(kFlatMax) * kMexWords, 0, s);
  if (st) return st;
  // ctl[1] = largest colour so far, start at -1
  st = fill_i32(w.ctl + 1, 1, -1, s);
  if (st) return st;
  st = fill_i32(w.ctl + 3, 1, -1, s);
  if (st) return st;
  hipLaunchKernelGGL(k_init_count, dim3(g1(k * kWave, 8192)), dim3(kBlock), 0, s, X->col_ptr, k,
                     w.pos_in_row, w.count, color, w.front_a, w.ctl);
  GENCD_HIP(hipGetLastError());
  // Rounds run without the host: every kernel reads the frontier size from
  // the device (counters by round parity); the host looks at the counters
  // once per kRoundsPerSync rounds.  Rounds past the last frontier find an
  // empty one and do nothing.
  constexpr int kRoundsPerSync = 32;
  // workgroups of the three jobs of k_round_work (they stride over their
  // work; on the Lasso workload 2-8x larger grids were slower, as most
  // rounds are small and every workgroup is dispatched)
  constexpr int32_t kMexGrid = 512, kFlatGrid = 256, kDecGrid = 1024;
  int32_t *cur = w.front_a, *nxt = w.front_b;
  int32_t ctl_host[8];
  int64_t round = 0;
  for (;;) {
    for (int r = 0; r < kRoundsPerSync; ++r, ++round) {
      int32_t *fc = w.ctl + ((round & 1) ? 4 : 0), *fn = w.ctl + ((round & 1) ? 0 : 4);
      const unsigned ft = unsigned((k + kFTile - 1) / kFTile);  // tiles of the largest frontier
      hipLaunchKernelGGL(k_fscan_tiles, dim3(ft), dim3(kBlock), 0, s, fc, cur, X->col_ptr,
                         w.scan_part);
      hipLaunchKernelGGL(k_fscan_part, dim3(1), dim3(kBlock), 0, s, fc, w.scan_part);
      hipLaunchKernelGGL(k_fscan_apply, dim3(ft), dim3(kBlock), 0, s, fc, cur, X->col_ptr,
                         w.scan_part, w.foff);
      // the frontier's colours (one of the two forms, by its size) and the
      // readiness counts in one launch; then the small form's pick, which
      // also ends the round
      hipLaunchKernelGGL(k_round_work, dim3(kMexGrid + kFlatGrid + kDecGrid), dim3(kBlock), 0, s,
                         fc, X->col_ptr, X->row_idx, cur, w.foff, w.row_ptr, w.rank_at,
                         w.pos_in_row, w.order, color, w.ctl, w.gbits, w.count, nxt, fn,
                         kMexGrid, kFlatGrid);
      hipLaunchKernelGGL(k_mex_pick, dim3(kFlatMax), dim3(kBlock), 0, s, fc, cur, color, w.ctl,
                         w.gbits);
      int32_t *t = cur;
      cur = nxt;
      nxt = t;
    }
    GENCD_HIP(hipGetLastError());
    GENCD_HIP(hipMemcpyAsync(ctl_host, w.ctl, sizeof(ctl_host), hipMemcpyDeviceToHost, s));
    GENCD_HIP(hipStreamSynchronize(s));
    if (ctl_host[2]) return GENCD_ERR_UNSUPPORTED;  // more colours than the bitmap holds
    if (ctl_host[5] > k) return GENCD_ERR_HIP;      // cannot happen for a valid CSC
    if (ctl_host[(round & 1) ? 4 : 0] == 0) break;
    if (round > k + kRoundsPerSync) return GENCD_ERR_HIP;
  }
  if (ctl_host[5] != k) return GENCD_ERR_HIP;
  *num_colors = ctl_host[3] + 1;
  return GENCD_OK;
}

size_t color_workspace(int64_t n, int64_t k, int64_t nnz) {
  return color_layout(n, k, nnz, nullptr, nullptr) + 256;
}

// ---------------------------------------------------------------------------
// Balanced colouring: every class above `cap` live columns is split into
// ceil(size / cap) near-equal parts, members in column order (rank r of a
// class of size s with p parts goes to part floor(r p / s)).  A stable sort
// of the live columns by colour gives each member its rank.
// ---------------------------------------------------------------------------
struct BalanceWs {
  uint32_t *keys_a, *keys_b;  // [k]
  int32_t *vals_a, *vals_b;   // [k]
  int32_t *size, *first, *parts, *off;  // [C+1]
  int32_t *rhist, *roffs;     // [radix_hist_len(k)]
  int32_t *scan_part;
};

static size_t balance_layout(int64_t k, int64_t C, void *base, BalanceWs *w) {
  const size_t al = 256;
  size_t off = 0;
  char *b = static_cast<char *>(base);
  auto take = [&](size_t bytes) -> void * {
    off = (off + al - 1) / al * al;
    void *p = b ? b + off : nullptr;
    off += bytes > 0 ? bytes : 1;
    return p;
  };
  BalanceWs c{};
  c.keys_a = static_cast<uint32_t *>(take(sizeof(uint32_t) * k));
  c.keys_b = static_cast<uint32_t *>(take(sizeof(uint32_t) * k));
  c.vals_a = static_cast<int32_t *>(take(sizeof(int32_t) * k));
  c.vals_b = static_cast<int32_t *>(take(sizeof(int32_t) * k));
  c.size = static_cast<int32_t *>(take(sizeof(int32_t) * (C + 1)));
  c.first = static_cast<int32_t *>(take(sizeof(int32_t) * (C + 1)));
  c.parts = static_cast<int32_t *>(take(sizeof(int32_t) * (C + 1)));
  c.off = static_cast<int32_t *>(take(sizeof(int32_t) * (C + 1)));
  const int64_t rl = radix_hist_len(k);
  c.rhist = static_cast<int32_t *>(take(sizeof(int32_t) * rl));
  c.roffs = static_cast<int32_t *>(take(sizeof(int32_t) * rl));
  c.scan_part = static_cast<int32_t *>(take(sizeof(int32_t) * scan_partials_for(rl)));
  if (w) *w = c;
  return off + al;
}

// keys: colour of live columns, C for empty ones (sorted last); class sizes
__global__ __launch_bounds__(kBlock) void k_bal_keys(const int64_t *col_ptr, int64_t k,
                                                      const int32_t *color, int32_t C,
                                                      uint32_t *keys, int32_t *vals, int32_t *size,
                                                      int32_t *bad) {
  for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < k;
       j += int64_t(gridDim.x) * kBlock) {
    const int32_t c = color[j];
    if (c < 0 || c >= C) {
      atomicOr(bad, 1);
      keys[j] = uint32_t(C);
    } else if (col_ptr[j + 1] > col_ptr[j]) {
      keys[j] = uint32_t(c);
      atomicAdd(&size[c], 1);
    } else {
      keys[j] = uint32_t(C);
    }
    vals[j] = int32_t(j);
  }
}

__global__ __launch_bounds__(kBlock) void k_bal_assign(const int64_t *col_ptr, int64_t k,
                                                        const int32_t *color, const uint32_t *keys,
                                                        const int32_t *vals, const int32_t *size,
                                                        const int32_t *first, const int32_t *parts,
                                                        const int32_t *off, int32_t C,
                                                        int32_t *out) {
  for (int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x; t < k;
       t += int64_t(gridDim.x) * kBlock) {
    const int32_t j = vals[t];
    const uint32_t c = keys[t];
    if (c < uint32_t(C)) {
      const int64_t r = t - off[c];  // rank of j in its class, column order
      out[j] = int32_t(first[c] + r * parts[c] / size[c]);
    } else {
      const int32_t c0 = color[j];
      out[j] = (c0 >= 0 && c0 < C) ? first[c0] : 0;
    }
  }
}

int balance_run(const gencd_csc *X, const int32_t *color, int32_t C, int64_t cap, int32_t *out,
                int32_t *num_out, void *ws_base, size_t ws_bytes, hipStream_t s) {
  const int64_t k = X->k;
  size_t need = balance_layout(k, C, nullptr, nullptr);
  if (!ws_base || ws_bytes < need) return GENCD_ERR_WORKSPACE;
  char *base = static_cast<char *>(ws_base);
  size_t mis = reinterpret_cast<uintptr_t>(base) % 256;
  if (mis) base += 256 - mis;
  BalanceWs w{};
  balance_layout(k, C, base, &w);
  int st = fill_i32(w.size, C + 1, 0, s);
  if (st) return st;
  hipLaunchKernelGGL(k_bal_keys, dim3(g1(k)), dim3(kBlock), 0, s, X->col_ptr, k, color, C, w.keys_a,
                     w.vals_a, w.size, w.size + C);
  GENCD_HIP(hipGetLastError());
  // stable by colour (key C: empty columns, last), so each class keeps column order
  int ob = 0;
  st = radix_sort_pairs(w.keys_a, w.vals_a, w.keys_b, w.vals_b, k, bits_for(uint64_t(C)), w.rhist,
                        w.roffs, w.scan_part, s, &ob);
  if (st) return st;
  // parts and numbering on the host (C + 1 counters)
  std::vector<int32_t> size(size_t(C) + 1), first(size_t(C) + 1), parts(size_t(C) + 1),
      off(size_t(C) + 1);
  GENCD_HIP(hipMemcpyAsync(size.data(), w.size, sizeof(int32_t) * (size_t(C) + 1),
                           hipMemcpyDeviceToHost, s));
  GENCD_HIP(hipStreamSynchronize(s));
  if (size[size_t(C)]) return GENCD_ERR_INVALID_ARG;  // a colour outside [0, C)
  int64_t kl = 0;
  for (int32_t c = 0; c < C; ++c) kl += size[size_t(c)];
  if (cap <= 0) cap = (kl + C - 1) / C;
  if (cap < 1) cap = 1;
  int64_t total = 0, o = 0;
  for (int32_t c = 0; c < C; ++c) {
    const int64_t sz = size[size_t(c)];
    const int64_t pc = sz > cap ? (sz + cap - 1) / cap : 1;
    parts[size_t(c)] = int32_t(pc);
    first[size_t(c)] = int32_t(total);
    off[size_t(c)] = int32_t(o);
    total += pc;
    o += sz;
  }
  if (total >= INT32_MAX) return GENCD_ERR_UNSUPPORTED;
  GENCD_HIP(hipMemcpyAsync(w.first, first.data(), sizeof(int32_t) * size_t(C), hipMemcpyHostToDevice, s));
  GENCD_HIP(hipMemcpyAsync(w.parts, parts.data(), sizeof(int32_t) * size_t(C), hipMemcpyHostToDevice, s));
  GENCD_HIP(hipMemcpyAsync(w.off, off.data(), sizeof(int32_t) * size_t(C), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_bal_assign, dim3(g1(k)), dim3(kBlock), 0, s, X->col_ptr, k, color,
                     ob ? w.keys_b : w.keys_a, ob ? w.vals_b : w.vals_a, w.size, w.first, w.parts,
                     w.off, C, out);
  GENCD_HIP(hipGetLastError());
  GENCD_HIP(hipStreamSynchronize(s));  // the host vectors above must outlive the copies
  *num_out = int32_t(total);
  return GENCD_OK;
}

}  // namespace gencd

extern "C" {

int gencd_color_workspace_bytes(const gencd_csc *X, size_t *out_bytes) {
  if (!X || !out_bytes || X->n <= 0 || X->k <= 0 || X->nnz < 0) return GENCD_ERR_INVALID_ARG;
  if (X->n > INT32_MAX || X->k >= INT32_MAX || X->nnz >= INT32_MAX) return GENCD_ERR_UNSUPPORTED;
  *out_bytes = gencd::color_workspace(X->n, X->k, X->nnz);
  return GENCD_OK;
}

int gencd_balance_workspace_bytes(const gencd_csc *X, int32_t num_colors, size_t *out_bytes) {
  if (!X || !out_bytes || X->k <= 0 || num_colors <= 0) return GENCD_ERR_INVALID_ARG;
  if (X->k >= INT32_MAX) return GENCD_ERR_UNSUPPORTED;
  *out_bytes = gencd::balance_layout(X->k, num_colors, nullptr, nullptr) + 256;
  return GENCD_OK;
}

int gencd_balance_colors(const gencd_csc *X, const int32_t *color, int32_t num_colors,
                         int64_t cap, int32_t *balanced, int32_t *num_balanced, void *ws,
                         size_t ws_bytes, hipStream_t stream) {
  if (!X || !color || !balanced || !num_balanced || X->k <= 0 || !X->col_ptr || num_colors <= 0)
    return GENCD_ERR_INVALID_ARG;
  if (X->k >= INT32_MAX) return GENCD_ERR_UNSUPPORTED;
  (void)hipGetLastError();
  return gencd::balance_run(X, color, num_colors, cap, balanced, num_balanced, ws, ws_bytes,
                            stream);
}

int gencd_color(const gencd_csc *X, int32_t *color, int32_t *num_colors, void *ws, size_t ws_bytes,
                hipStream_t stream) {
  if (!X || !color || !num_colors || X->n <= 0 || X->k <= 0 || X->nnz < 0 || !X->col_ptr ||
      (X->nnz > 0 && !X->row_idx))
    return GENCD_ERR_INVALID_ARG;
  if (X->n > INT32_MAX || X->k >= INT32_MAX || X->nnz >= INT32_MAX) return GENCD_ERR_UNSUPPORTED;
  (void)hipGetLastError();  // launch checks below must not see an earlier error
  return gencd::color_run(X, color, num_colors, ws, ws_bytes, stream);
}

}  // extern "C"
