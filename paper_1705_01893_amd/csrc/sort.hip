// Device-side construction of the deterministic binning structures (gfx950).
//
// Binning P^T y (the projection TOD -> map of Section 2.1) runs one workgroup per pixel
// tile over that tile's samples, cut into sub-batches of at most kSubBatch samples and
// kMaxSegs time-contiguous segments, each sub-batch also listed in pixel-sorted order.
// Everything here builds those lists from the device pointing, in a fixed order, so the
// plan never copies the pointing to the host:
//
//   k_sort_stats    per slab of samples: on-map count, mean step of the scan (for the tile
//                   shape), validation of pixel indices and angles;
//   k_sort_count    per slab: run starts (a run is a maximal time-contiguous stretch of
//                   on-map samples inside one tile and one chunk), in total and per tile;
//   k_sort_runs     per slab: every run's start, end and chunk, written at its place in
//                   the tile-major, time-ordered run list;
//   k_sort_batches  per tile: the greedy cut of its runs into sub-batches and segments
//                   (count mode, then write mode at the scanned offsets);
//   k_sort_pixels   per tile: each sub-batch's stage positions sorted by local pixel
//                   (stable: equal pixels keep time order), with the angles in that order.
//
// A slab is a contiguous range of samples walked by one thread in time order, so every
// count is an integer and every list position follows from prefix sums: the result does
// not depend on scheduling.  With composite pointing the walks run over the 2 N_s pointing
// entries (the first components, then the second ones), each a "sample" of its own here.  The scratch array at the end serves the allocation-free
// workspace query.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"

namespace mm {

namespace {

__device__ __forceinline__ int chunk_of(const int64_t* __restrict__ off, int nchunk, int64_t j) {
  int lo = 0, hi = nchunk;  // off[lo] <= j < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= j)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// the pixel of pointing entry j: first components below na, second ones from there
struct PixSrc {
  const int32_t* a;
  const int32_t* b;
  int64_t na;
};
__device__ __forceinline__ int32_t pix_at(const PixSrc& q, int64_t j) { return j < q.na ? q.a[j] : q.b[j - q.na]; }
template <typename E>
__device__ __forceinline__ E psi_at(const void* a, const void* b, int64_t na, int64_t j) {
  return j < na ? ((const E*)a)[j] : ((const E*)b)[j - na];
}
inline PixSrc pix_src(const SlabWalk& w) { return PixSrc{w.pix, w.pix_b, w.ns_a}; }

__device__ __forceinline__ int tile_of(int32_t p, const TileGeom& g) {
  const uint32_t y = (uint32_t)p / (uint32_t)g.nxm, x = (uint32_t)p - y * (uint32_t)g.nxm;
  return (int)((y / (uint32_t)g.th) * (uint32_t)g.ntx + x / (uint32_t)g.tw);
}

}  // namespace

__global__ void k_sort_clear(unsigned long long* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Scan statistics, on-map count and validation.  The statistics follow every fourth pair of
// consecutive samples inside a chunk (j - off_c = 1 mod 4) whose two pixels are on the map and
// at most 16 pixels apart in x and in y (scan-line turnarounds left out).
__global__ __launch_bounds__(256) void k_sort_stats(PixSrc pix, const int64_t* __restrict__ off,
                                                    int nchunk, int64_t ns, int64_t slab, int64_t nslabs,
                                                    int64_t npix, int64_t nxm, const void* __restrict__ psi,
                                                    const void* __restrict__ psi_b, int psi_kind, int64_t table_len,
                                                    SortCounters* ctr) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  unsigned long long sx = 0, sy = 0, nst = 0, non = 0;
  unsigned int flags = 0;
  if (s < nslabs) {
    const int64_t j0 = s * slab;
    const int64_t j1 = j0 + slab < ns ? j0 + slab : ns;
    if (j0 < ns) {
      int c = chunk_of(off, nchunk, j0);
      int64_t cbeg = off[c], cend = off[c + 1];
      for (int64_t j = j0; j < j1; ++j) {
        if (j == cend) {
          ++c;
          cbeg = cend;
          cend = off[c + 1];
        }
        const int32_t p = pix_at(pix, j);
        if ((int64_t)p >= npix) flags |= 1u;
        non += p >= 0 ? 1ull : 0ull;
        if (j > cbeg && ((j - cbeg) & 3) == 1 && p >= 0) {
          const int32_t a = pix_at(pix, j - 1);
          if (a >= 0 && (int64_t)a < npix && (int64_t)p < npix) {
            const int64_t ax = a % nxm, ay = a / nxm, bx = p % nxm, by = p / nxm;
            const int64_t dx = ax > bx ? ax - bx : bx - ax, dy = ay > by ? ay - by : by - ay;
            if (dx <= 16 && dy <= 16) {
              sx += (unsigned long long)dx;
              sy += (unsigned long long)dy;
              ++nst;
            }
          }
        }
        if (psi_kind == 1) {
          const double v = psi_at<double>(psi, psi_b, pix.na, j);
          if (!(fabs(v) < kMaxAngle)) flags |= 2u;
        } else if (psi_kind == 2) {
          const float v = psi_at<float>(psi, psi_b, pix.na, j);
          if (!(fabs((double)v) < kMaxAngle)) flags |= 2u;
        } else if (psi_kind == 3) {
          if ((int64_t)psi_at<uint16_t>(psi, psi_b, pix.na, j) >= table_len) flags |= 4u;
        }
      }
    }
  }
  // one atomic per wave and counter
  for (int d = 32; d > 0; d >>= 1) {
    sx += __shfl_down(sx, d);
    sy += __shfl_down(sy, d);
    nst += __shfl_down(nst, d);
    non += __shfl_down(non, d);
    flags |= (unsigned int)__shfl_down((int)flags, d);
  }
  if ((threadIdx.x & 63) == 0) {
    if (sx) atomicAdd(&ctr->sx, sx);
    if (sy) atomicAdd(&ctr->sy, sy);
    if (nst) atomicAdd(&ctr->nst, nst);
    if (non) atomicAdd(&ctr->non, non);
    if (flags) atomicOr(&ctr->flags, flags);
  }
}

// Run starts.  Sample j starts a run when it is on the map and its tile differs from that of
// sample j - 1 (off the map, or the previous chunk's last sample, count as no tile).  With
// `starts` (row s of an nslabs x ntiles matrix) the starts are also counted per tile.
__global__ __launch_bounds__(256) void k_sort_count(PixSrc pix, const int64_t* __restrict__ off,
                                                    int nchunk, int64_t ns, int64_t slab, int64_t nslabs, TileGeom g,
                                                    SortCounters* ctr, int64_t* __restrict__ starts) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  unsigned long long nr = 0;
  if (s < nslabs) {
    const int64_t j0 = s * slab;
    const int64_t j1 = j0 + slab < ns ? j0 + slab : ns;
    if (j0 < ns) {
      int c = chunk_of(off, nchunk, j0);
      int64_t cend = off[c + 1];
      int prev_t = -1;
      if (j0 > off[c]) {
        const int32_t p = pix_at(pix, j0 - 1);
        prev_t = p >= 0 ? tile_of(p, g) : -1;
      }
      int64_t* row = starts ? starts + s * (int64_t)g.ntiles : nullptr;
      int run_t = -1;
      int64_t run_n = 0;
      for (int64_t j = j0; j < j1; ++j) {
        if (j == cend) {
          ++c;
          cend = off[c + 1];
          prev_t = -1;
        }
        const int32_t p = pix_at(pix, j);
        const int t = p >= 0 ? tile_of(p, g) : -1;
        if (t >= 0 && t != prev_t) {
          ++nr;
          if (row) {
            if (t != run_t) {
              if (run_t >= 0) row[run_t] += run_n;
              run_t = t;
              run_n = 0;
            }
            ++run_n;
          }
        }
        prev_t = t;
      }
      if (row && run_t >= 0) row[run_t] += run_n;
    }
  }
  for (int d = 32; d > 0; d >>= 1) nr += __shfl_down(nr, d);
  if ((threadIdx.x & 63) == 0 && nr) atomicAdd(&ctr->nruns, nr);
}

// Per tile: exclusive prefix of the per-slab start counts down the slabs (in place), and the
// tile's total.
__global__ void k_sort_slab_prefix(int64_t* __restrict__ starts, int64_t nslabs, int ntiles,
                                   int64_t* __restrict__ tile_total) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  int64_t run = 0;
  for (int64_t s = 0; s < nslabs; ++s) {
    int64_t* q = starts + s * (int64_t)ntiles + t;
    const int64_t v = *q;
    *q = run;
    run += v;
  }
  tile_total[t] = run;
}

// Exclusive prefix sum of n int64 values by one workgroup of 1024 threads; the total goes to
// *total when it is not null.
__global__ __launch_bounds__(1024) void k_scan_i64(const int64_t* __restrict__ in, int64_t* __restrict__ out,
                                                   int64_t n, int64_t* total) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t carry_s;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < n ? in[i] : 0;
    int64_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int64_t before = carry_s;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (i < n) out[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry_s = before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry_s;
}

// The run list: run r of tile t (in time order) sits at runbase[t] + r.  `cur` holds, for row s,
// the number of tile-t runs that start before slab s (k_sort_slab_prefix); the slab's thread
// advances it as it meets run starts.  A run's end (one past its last sample) is written by the
// slab holding its last sample, at the slot of the tile's latest run.
__global__ __launch_bounds__(256) void k_sort_runs(PixSrc pix, const int64_t* __restrict__ off,
                                                   int nchunk, int64_t ns, int64_t slab, int64_t nslabs, TileGeom g,
                                                   int64_t* __restrict__ cur, const int64_t* __restrict__ runbase,
                                                   int64_t* __restrict__ rstart, int64_t* __restrict__ rend,
                                                   int32_t* __restrict__ rchunk) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nslabs) return;
  const int64_t j0 = s * slab;
  if (j0 >= ns) return;
  const int64_t j1 = j0 + slab < ns ? j0 + slab : ns;
  int64_t* row = cur + s * (int64_t)g.ntiles;
  int c = chunk_of(off, nchunk, j0);
  int64_t cend = off[c + 1];
  int prev_t = -1;
  if (j0 > off[c]) {
    const int32_t p = pix_at(pix, j0 - 1);
    prev_t = p >= 0 ? tile_of(p, g) : -1;
  }
  // row[ct] cached in a register while the walk stays in one tile
  int ct = -1;
  int64_t cv = 0;
  auto slot_of = [&](int t) -> int64_t& {
    if (t != ct) {
      if (ct >= 0) row[ct] = cv;
      ct = t;
      cv = row[t];
    }
    return cv;
  };
  for (int64_t j = j0; j < j1; ++j) {
    if (j == cend) {
      if (prev_t >= 0 && j > j0) rend[runbase[prev_t] + slot_of(prev_t) - 1] = j;
      ++c;
      cend = off[c + 1];
      prev_t = -1;
    }
    const int32_t p = pix_at(pix, j);
    const int t = p >= 0 ? tile_of(p, g) : -1;
    if (prev_t >= 0 && t != prev_t && j > j0) rend[runbase[prev_t] + slot_of(prev_t) - 1] = j;
    if (t >= 0 && t != prev_t) {
      int64_t& k = slot_of(t);
      const int64_t r = runbase[t] + k;
      ++k;
      rstart[r] = j;
      rchunk[r] = c;
    }
    prev_t = t;
  }
  // the run holding sample j1 - 1 ends at j1 unless sample j1 continues it
  if (prev_t >= 0) {
    bool ends = true;
    if (j1 < ns && j1 != cend) {
      const int32_t p = pix_at(pix, j1);
      ends = !(p >= 0 && tile_of(p, g) == prev_t);
    }
    if (ends) rend[runbase[prev_t] + slot_of(prev_t) - 1] = j1;
  }
  if (ct >= 0) row[ct] = cv;
}

// Greedy cut of one tile's runs (time order) into sub-batches: a sub-batch closes when it holds
// kSubBatch samples or when the next segment would be its (kMaxSegs + 1)-th.  A segment is the
// part of a run inside one sub-batch.  Count mode (write == 0) gives each tile's sub-batch,
// segment and padded sorted-entry counts; write mode writes the records at the scanned offsets
// (and flags an overflow of the reserved sizes instead of writing past them).  Runs come in entry
// order, so a sub-batch's first-component entries (below ns_a) precede its second-component ones;
// SubBatch::na counts the former.
__global__ __launch_bounds__(256) void k_sort_batches(int write, TileGeom g, int64_t nym, int64_t ns_a,
                                                      const int64_t* __restrict__ runbase,
                                                      const int64_t* __restrict__ rstart,
                                                      const int64_t* __restrict__ rend,
                                                      const int32_t* __restrict__ rchunk, int64_t* __restrict__ nsb,
                                                      int64_t* __restrict__ nseg, int64_t* __restrict__ nsort,
                                                      const int64_t* __restrict__ sbbase,
                                                      const int64_t* __restrict__ segbase,
                                                      const int64_t* __restrict__ sortbase, Tile* __restrict__ tiles,
                                                      SubBatch* __restrict__ sbs, Segment* __restrict__ segs,
                                                      int64_t cap_sb, int64_t cap_seg, int64_t cap_sort,
                                                      SortCounters* ctr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.ntiles) return;
  const int64_t r0 = runbase[t], r1 = runbase[t + 1];
  int64_t sb = write ? sbbase[t] : 0, sg = write ? segbase[t] : 0, so = write ? sortbase[t] : 0;
  const int64_t sb0 = sb;
  bool open = false, bad = false;
  int cnt = 0, ns_ = 0, cnt_a = 0;
  SubBatch cur = {};
  auto close = [&]() {
    if (write) {
      cur.seg_end = (int32_t)sg;
      cur.count = cnt;
      cur.na = cnt_a;
      if (sb < cap_sb) sbs[sb] = cur; else bad = true;
    }
    ++sb;
    so += (cnt + kSortAlign - 1) / kSortAlign * kSortAlign;
    open = false;
  };
  for (int64_t r = r0; r < r1 && !bad; ++r) {
    int64_t j = rstart[r];
    const int64_t e = rend[r];
    const int32_t ch = rchunk[r];
    while (j < e) {
      if (open && ns_ == kMaxSegs) close();
      if (!open) {
        open = true;
        cur.sorted_begin = so;
        cur.seg_begin = (int32_t)sg;
        cnt = 0;
        cnt_a = 0;
        ns_ = 0;
      }
      const int64_t take = (e - j) < (int64_t)(kSubBatch - cnt) ? (e - j) : (int64_t)(kSubBatch - cnt);
      if (write) {
        if (sg < cap_seg) {
          Segment q;
          q.start = j;
          q.pos = cnt;
          q.chunk = ch;
          segs[sg] = q;
        } else {
          bad = true;
        }
      }
      ++sg;
      ++ns_;
      cnt += (int)take;
      if (j < ns_a) cnt_a += (int)take;
      j += take;
      if (cnt == kSubBatch) close();
    }
  }
  if (open) close();
  if (write) {
    if (so > cap_sort) bad = true;
    if (bad) {
      atomicOr(&ctr->flags, 8u);
      return;
    }
    Tile tl;
    const int ty = t / g.ntx, tx = t - ty * g.ntx;
    tl.x0 = tx * g.tw;
    tl.y0 = ty * g.th;
    tl.tw = (g.nxm - tl.x0) < g.tw ? (int)(g.nxm - tl.x0) : g.tw;
    tl.th = (nym - tl.y0) < g.th ? (int)(nym - tl.y0) : g.th;
    tl.sb_begin = (int32_t)sb0;
    tl.sb_end = (int32_t)sb;
    tiles[t] = tl;
  } else {
    nsb[t] = sb;
    nseg[t] = sg;
    nsort[t] = so;
  }
}

// One workgroup per tile: for each of its sub-batches, the stage positions q (0 .. count-1, the
// sub-batch's samples in time order) sorted by the key (local pixel, q), i.e. by pixel with time
// order kept; perm = q, lp = local pixel, psi_sorted = the sample's stored angle.  The entries
// past count up to the next multiple of kSortAlign are zero.
constexpr int kSortBlock = 256;
__global__ __launch_bounds__(kSortBlock) void k_sort_pixels(PixSrc pix, const void* __restrict__ psi,
                                                            const void* __restrict__ psi_b, int psi_esz, TileGeom g,
                                                            const Tile* __restrict__ tiles,
                                                            const SubBatch* __restrict__ sbs,
                                                            const Segment* __restrict__ segs,
                                                            uint16_t* __restrict__ perm, uint16_t* __restrict__ lp,
                                                            uint8_t* __restrict__ psi_sorted,
                                                            uint32_t* __restrict__ packed, int lp_bits,
                                                            uint16_t* __restrict__ lp_stage,
                                                            uint8_t* __restrict__ psi_stage) {
  __shared__ uint32_t key[kSubBatch];
  __shared__ int64_t jq[kSubBatch];
  __shared__ int64_t sstart[kMaxSegs];
  __shared__ int32_t spos[kMaxSegs];
  for (int t = blockIdx.x; t < g.ntiles; t += gridDim.x) {
    const Tile tl = tiles[t];
    for (int b = tl.sb_begin; b < tl.sb_end; ++b) {
      const SubBatch S = sbs[b];
      const int nseg = S.seg_end - S.seg_begin, cnt = S.count;
      for (int i = threadIdx.x; i < nseg; i += kSortBlock) {
        const Segment q = segs[S.seg_begin + i];
        sstart[i] = q.start;
        spos[i] = q.pos;
      }
      __syncthreads();
      int n2 = 1;
      while (n2 < cnt) n2 <<= 1;
      for (int q = threadIdx.x; q < n2; q += kSortBlock) {
        if (q < cnt) {
          int lo = 0, hi = nseg;  // spos[lo] <= q < spos[hi]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (spos[mid] <= q)
              lo = mid;
            else
              hi = mid;
          }
          const int64_t j = sstart[lo] + (q - spos[lo]);
          const int32_t p = pix_at(pix, j);
          const int y = p / (int)g.nxm, x = p - y * (int)g.nxm;
          const int l = (y - tl.y0) * tl.tw + (x - tl.x0);
          key[q] = ((uint32_t)l << 12) | (uint32_t)q;
          jq[q] = j;
        } else {
          key[q] = 0xffffffffu;
        }
      }
      if (lp_stage) {
        // stage order (the padding past count left as it is: never read)
        for (int q = threadIdx.x; q < cnt; q += kSortBlock) {
          const int64_t j = jq[q];
          lp_stage[S.sorted_begin + q] = (uint16_t)(key[q] >> 12);
          if (psi_esz) {
            uint8_t* dst = psi_stage + (S.sorted_begin + q) * psi_esz;
            if (psi_esz == 8)
              *(uint64_t*)dst = psi_at<uint64_t>(psi, psi_b, pix.na, j);
            else if (psi_esz == 4)
              *(uint32_t*)dst = psi_at<uint32_t>(psi, psi_b, pix.na, j);
            else
              *(uint16_t*)dst = psi_at<uint16_t>(psi, psi_b, pix.na, j);
          }
        }
      }
      __syncthreads();
      // bitonic sort of the n2 keys (ascending)
      for (int k = 2; k <= n2; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
          for (int i = threadIdx.x; i < n2; i += kSortBlock) {
            const int ix = i ^ jj;
            if (ix > i) {
              const uint32_t a = key[i], c = key[ix];
              const bool up = (i & k) == 0;
              if ((a > c) == up) {
                key[i] = c;
                key[ix] = a;
              }
            }
          }
          __syncthreads();
        }
      }
      const int padded = (cnt + kSortAlign - 1) / kSortAlign * kSortAlign;
      const int64_t base = S.sorted_begin;
      for (int i = threadIdx.x; i < padded; i += kSortBlock) {
        uint16_t q = 0, l = 0;
        if (i < cnt) {
          const uint32_t k = key[i];
          q = (uint16_t)(k & 0xfffu);
          l = (uint16_t)(k >> 12);
        }
        if (packed) {
          // the key already holds the stage position and the local pixel; the angle index above
          packed[base + i] = i < cnt ? key[i] | ((uint32_t)psi_at<uint16_t>(psi, psi_b, pix.na, jq[q]) << (12 + lp_bits))
                                     : 0u;
          continue;
        }
        perm[base + i] = q;
        lp[base + i] = l;
        if (psi_esz) {
          uint8_t* dst = psi_sorted + (base + i) * psi_esz;
          if (psi_esz == 8) {
            *(uint64_t*)dst = i < cnt ? psi_at<uint64_t>(psi, psi_b, pix.na, jq[q]) : 0ull;
          } else if (psi_esz == 4) {
            *(uint32_t*)dst = i < cnt ? psi_at<uint32_t>(psi, psi_b, pix.na, jq[q]) : 0u;
          } else {
            *(uint16_t*)dst = i < cnt ? psi_at<uint16_t>(psi, psi_b, pix.na, jq[q]) : (uint16_t)0;
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------------------
// launchers

static inline int slab_grid(int64_t nslabs) { return (int)((nslabs + 255) / 256); }

hipError_t launch_sort_clear(SortCounters* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_clear, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned long long*>(ctr),
                     (int)(sizeof(SortCounters) / sizeof(unsigned long long)));
  return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_sort_stats(const SlabWalk& w, int64_t npix, int64_t nxm, const void* psi, const void* psi_b,
                             int psi_kind, int64_t table_len, SortCounters* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_stats, dim3(slab_grid(w.nslabs)), dim3(256), 0, s, pix_src(w), w.off, w.nchunk, w.ns,
                     w.slab, w.nslabs, npix, nxm, psi, psi_b, psi_kind, table_len, ctr);
  return hipGetLastError();
}

hipError_t launch_sort_count(const SlabWalk& w, const TileGeom& g, SortCounters* ctr, int64_t* starts, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_count, dim3(slab_grid(w.nslabs)), dim3(256), 0, s, pix_src(w), w.off, w.nchunk, w.ns,
                     w.slab, w.nslabs, g, ctr, starts);
  return hipGetLastError();
}

hipError_t launch_sort_lists(const SlabWalk& w, const TileGeom& g, int64_t nym, const SortTemp& T, const SortOut& O,
                             SortCounters* ctr, hipStream_t s) {
  const int tb = (g.ntiles + 255) / 256;
  hipLaunchKernelGGL(k_sort_slab_prefix, dim3(tb), dim3(256), 0, s, T.starts, w.nslabs, g.ntiles, T.tile_runs);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, T.tile_runs, T.runbase, (int64_t)g.ntiles,
                     T.runbase + g.ntiles);
  hipLaunchKernelGGL(k_sort_runs, dim3(slab_grid(w.nslabs)), dim3(256), 0, s, pix_src(w), w.off, w.nchunk, w.ns,
                     w.slab, w.nslabs, g, T.starts, T.runbase, T.rstart, T.rend, T.rchunk);
  hipLaunchKernelGGL(k_sort_batches, dim3(tb), dim3(256), 0, s, 0, g, nym, w.ns_a, T.runbase, T.rstart, T.rend, T.rchunk,
                     T.nsb, T.nseg, T.nsort, (const int64_t*)nullptr, (const int64_t*)nullptr,
                     (const int64_t*)nullptr, (Tile*)nullptr, (SubBatch*)nullptr, (Segment*)nullptr, (int64_t)0,
                     (int64_t)0, (int64_t)0, ctr);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, T.nsb, T.sbbase, (int64_t)g.ntiles, O.totals + 0);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, T.nseg, T.segbase, (int64_t)g.ntiles, O.totals + 1);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, T.nsort, T.sortbase, (int64_t)g.ntiles, O.totals + 2);
  hipLaunchKernelGGL(k_sort_batches, dim3(tb), dim3(256), 0, s, 1, g, nym, w.ns_a, T.runbase, T.rstart, T.rend,
                     T.rchunk, (int64_t*)nullptr, (int64_t*)nullptr, (int64_t*)nullptr, T.sbbase, T.segbase, T.sortbase,
                     O.tiles, O.sbs, O.segs, O.cap_sb, O.cap_seg, O.cap_sort, ctr);
  return hipGetLastError();
}

hipError_t launch_sort_pixels(const SlabWalk& w, const void* psi, const void* psi_b, int psi_esz, const TileGeom& g,
                              const SortOut& O, hipStream_t s) {
  const int grid = g.ntiles < 65536 ? g.ntiles : 65536;
  hipLaunchKernelGGL(k_sort_pixels, dim3(grid > 0 ? grid : 1), dim3(kSortBlock), 0, s, pix_src(w), psi, psi_b,
                     psi_esz, g, O.tiles, O.sbs, O.segs, O.perm, O.lp, O.psi_sorted, O.packed, O.lp_bits, O.lp_stage,
                     O.psi_stage);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// The fixed device array of the allocation-free workspace query: the chunk table and the
// counters of the analysis passes.  Each device gets its own copy; its address is looked up
// once per device (with that device current) and kept.

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

void* static_scratch(int device, hipError_t* err) {
  static std::mutex mu;
  static void* ptrs[kMaxDevices] = {};
  *err = hipSuccess;
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      *err = e;
      return nullptr;
    }
    ptrs[device] = p;
  }
  return ptrs[device];
}

}  // namespace mm
