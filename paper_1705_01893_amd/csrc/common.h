// Shared host/device definitions of libmm (messenger-field mapmaking on gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mm {

constexpr int kBlock = 512;        // threads per workgroup of the column passes (A, C) and reductions
constexpr int kBlockB = 256;       // threads per workgroup of the row pass (B) and the gradient row pass
constexpr double kMaxAngle = 1.0e5;  // |psi| bound (radians) of the stored polarization angles
constexpr int kBinBlock = 256;     // threads per workgroup of the binning pass
constexpr int kWaves = kBinBlock / 64;
constexpr int kMaxStages = 24;     // radix stages of one sub-transform
constexpr int kSubBatch = 4096;    // samples staged in LDS per binning step (<= 65536: uint16 indices)
constexpr int kMaxTilePix = 512;   // pixels per binning tile by default (LDS accumulators)
constexpr int kMaxTilePixAsked = 1024;  // the largest tile a descriptor may ask for

// complex elements per thread in the LDS transforms (tile capacity = kBlock * ept = 64 KB)
template <typename T> struct Ept;
template <> struct Ept<float> { static constexpr int v = 16; };
template <> struct Ept<double> { static constexpr int v = 8; };

// Column tiles of the column passes.  Element i of column b sits at i * cb + b (interleaved,
// every stage a workgroup-wide step), or, in the wave-local layout the inverse column pass takes
// for eligible classes, at b * Lc + pad8(i): every wave then transforms its own cb / (kBlock / 64)
// columns alone.
// pad8(i) = i + i / 8, and Lc >= pad8(M2 - 1) + 1 is an odd multiple of q = max(G / cb, 1) so
// that the b-fastest global<->LDS copies (G = 256 / sizeof(complex) lanes per bank sweep: G / cb
// rows of cb columns) fall in distinct banks.  Eligible: cb >= kBlock / 64 and a padded tile
// within kMaxColTileBytes.
constexpr int kColWaves = kBlock / 64;
// LDS bound of a padded column tile: two workgroups per CU (160 KB)
constexpr int kMaxColTileBytes = 81920;
__host__ __device__ inline int pad8(int i) { return i + (i >> 3); }
__host__ __device__ inline int wave_col_stride(int M2, int cb, int csz) {
  const int G = 256 / csz;
  const int q = cb < G ? G / cb : 1;
  int L = (pad8(M2 - 1) + q) / q;  // in units of q
  if ((L & 1) == 0) ++L;
  return L * q;
}
__host__ __device__ inline bool wave_cols(int M2, int cb, int csz) {
  return cb >= kColWaves && cb * wave_col_stride(M2, cb, csz) * csz <= kMaxColTileBytes;
}
// complex values of LDS a column tile takes (wave: the plan runs the wave-local layout)
__host__ __device__ inline int col_tile_elems(int M2, int cb, int csz, bool wave) {
  return wave ? cb * wave_col_stride(M2, cb, csz) : cb * M2;
}

// Radices of the transform stages.  A stage holds ceil(Ept / R) butterflies of R complex values
// per lane; the composite radices (two-level DFTs) are kept where that and their twiddles fit
// the 128-VGPR budgets of the transform passes.
__host__ __device__ constexpr bool radix_ok(int R, bool f64) {
  return R == 2 || R == 3 || R == 4 || R == 5 || R == 8 || R == 9 ||
         (!f64 && (R == 16 || R == 20 || R == 25));
}

template <typename T> struct Cx;
template <> struct Cx<float> { using t = float2; };
template <> struct Cx<double> { using t = double2; };
template <typename T> using cx = typename Cx<T>::t;

// Per-chunk parameters.  A chunk of n real samples is transformed as M = n/2
// complex points split M = M1 * M2 (M2-point column transforms, M1-point rows).
struct DevChunk {
  int64_t off;        // first sample of the chunk
  int32_t n, M, M1, M2;
  int32_t cls;        // transform class (shared by chunks of equal M)
  int32_t cb;         // columns per column-pass item (a power of two)
  int32_t lgb;        // log2 cb
  int32_t pad0;
  double df;          // frequency step f_s / n
  double sigma2;      // white level sigma^2
  double fknee, alpha;
  double tau, inv_tau;
  double nbar0;       // sigma^2 - tau (N-bar = nbar0 + sigma^2 (f/fknee)^alpha)
  int64_t spec_off;   // offset of this chunk's M+1 power-law values in DevPlan::spec (FP64 form)
  double inv_M;       // 1 / M
  double lg0;         // log2(df / fknee): the power law at bin k is sigma^2 2^(alpha (log2 k + lg0))
  int64_t xoff;       // complex offset of the chunk in the transform work buffers (16-aligned)
};

constexpr int kWorkAlign = 16;  // complex values: chunk bases in the work buffers sit on 128-byte lines

// Per-length transform data: radix schedules and twiddle-table offsets.
struct DevClass {
  int32_t M, M1, M2;
  int32_t nr1, nr2;   // number of radix stages for the M1 and M2 transforms
  int32_t lb;         // two-level split of the omega_{2M} table: q = (hi << lb) + rem
  int64_t tw1, tw2;   // offsets of omega_{M1}^q, omega_{M2}^q tables (complex entries)
  int64_t twlo, twhi; // offsets of omega_{2M}^rem and omega_{2M}^(hi << lb)
  int8_t rad1[kMaxStages];
  int8_t rad2[kMaxStages];
};

struct ItemAC { int32_t chunk, j1; };            // column block starting at column j1
// rows ra, rb (rb == ra: one row); rc > 0: a second pair of rows rc, M2 - rc in the same item
// (the row pass's items when four rows fit its tile; the gradient row pass never has one)
struct ItemB { int32_t chunk, ra, rb, rc; };

// Deterministic binning structures.  Samples on the map are grouped by pixel
// tile, each tile's samples (in time order) are cut into sub-batches of at most
// kSubBatch samples, and each sub-batch is described by its time-contiguous
// segments (staged into LDS) plus the per-sample order sorted by local pixel.
struct Tile {
  int32_t sb_begin, sb_end;  // sub-batch range
  int32_t x0, y0, tw, th;    // pixel rectangle (map row length DevPlan::nxm)
};
struct SubBatch {
  int64_t sorted_begin;      // offset into perm / lp / psi_sorted
  int32_t seg_begin, seg_end;  // at most kMaxSegs segments
  int32_t count;             // samples in the sub-batch
  int32_t na;                // stage positions below na hold first-component entries (composite
                             // pointing: those of the second follow them); count otherwise
};
constexpr int kMaxSegs = 512;  // segments per sub-batch (LDS segment table)
constexpr int kSortAlign = 16;  // alignment (elements) of each sub-batch in the pixel-sorted arrays
constexpr int kPerLane = 16;    // consecutive pixel-sorted samples one lane accumulates
// Composite pointing (two entries per sample) runs over 2 N_s pointing entries: entry v < N_s is
// sample v's first component, entry N_s + j its second; chunk c + nchunk holds the second
// components of chunk c.  Segments, runs and sub-batches are cut over that entry order.
struct Segment {             // 16 bytes: read by both walks of the binning pass every iteration
  int64_t start;             // first pointing entry (the sample index for a single beam)
  int32_t pos;               // position of the first sample in the LDS stage
  int32_t chunk;             // chunk of the entries (nchunk + c: second components of chunk c)
};

struct DevPlan {
  int32_t ncomp, psi_kind, precision;
  int32_t all_pow2;          // every chunk length is a power of two (radix 8/4/2 transforms)
  int32_t max_tile_pix;      // pixels of the largest binning tile (LDS accumulators)
  int32_t col_wave;          // inverse column pass: wave-local classes 0 none, 1 all, 2 some, 3 all (register transforms)
  int64_t npix, nxm;         // pixels, map row length used by the tiles
  int64_t nsamp;
  int32_t nchunk, ntiles;
  const DevChunk* chunks;
  const DevClass* classes;
  const double2* tw64;
  const float2* tw32;
  const int32_t* pix;
  const void* psi;           // caller's angles (time order)
  const double2* psi_cs64;   // (cos 2psi, sin 2psi) per table entry (MM_PSI_U16), float64
  const float2* psi_cs32;    // same, float32
  const double2* sc_tab;     // (cos, sin)(k pi / 512), k < 1024, for the FP64 angle weights
  const Tile* tiles;
  const SubBatch* sbs;
  const Segment* segs;
  const uint16_t* perm;      // sorted order -> stage position
  const uint16_t* lp;        // sorted order -> local pixel
  const void* psi_sorted;    // angles in sorted order (type psi_kind)
  // the pixel-sorted entries packed into 32 bits, in place of perm, lp and psi_sorted, when a
  // 16-bit angle index fits beside them: stage position (12 bits) | local pixel << 12 | angle
  // index << (12 + pk_lp_bits); else null
  const uint32_t* packed;
  int32_t pk_lp_bits;
  const uint16_t* lp_stage;  // local pixels and angles in stage order (time order within each
  const void* psi_stage;     // sub-batch's segments), for the projection walk; null without P m
  const double* spec;        // FP64 form: sigma^2 (f_k / fknee)^alpha per chunk bin (f_0 -> f_1)
  const double* winv;        // [nw][npix], nw = 1 or 6 (00 01 02 11 12 22)
  const uint8_t* solvable;   // [npix]
  double2* mapi;             // I/Q/U map interleaved, [npix][2] = (I, Q), (U, 0): one line per gather
                             // (gather access with ncomp = 3; null otherwise)
  const double* md;          // m_d(lambda) of the map-sized form (EPI_MAPSIZED launches only)
  // composite pointing P = wa P_A + wb P_B (0 / 1, 0 for a single beam): the projection buffer
  // holds P_A m and P_B m (times their weights) in two halves, pmb_off complex values apart
  int32_t composite;
  int32_t pad1;
  double wa, wb;
  int64_t pmb_off;
  // gap filling (SRC_GAP launches only): the filled data d_0 and the gap flags, time order
  const void* gap_d0;
  const uint8_t* gaps;
};

// ---------------------------------------------------------------------------------------------
// device-side construction of the binning structures (sort.hip)

// Pixel tiles: rectangles of tw x th pixels over a map of rows of nxm pixels, ntx per tile row.
struct TileGeom {
  int32_t nxm, tw, th, ntx, ntiles;
};
// Counters of the analysis passes (integers: independent of scheduling).
struct SortCounters {
  unsigned long long sx, sy, nst;  // summed |dx|, |dy| of the sampled steps, number of steps
  unsigned long long non;          // on-map samples
  unsigned long long nruns;        // runs (time-contiguous stretches inside one tile and chunk)
  unsigned int flags;              // 1 pixel >= npix, 2 angle not finite or too large,
                                   // 4 angle index beyond the table, 8 reserved sizes exceeded
  unsigned int pad;
};
// The pointing entries cut into slabs walked in order, one thread per slab.  Entry v reads
// pix[v] below ns_a and pix_b[v - ns_a] from there (composite pointing: ns = 2 ns_a, and the
// chunk table lists the second components' chunks after the first ones).
struct SlabWalk {
  const int32_t* pix;
  const int32_t* pix_b;  // null for a single beam (ns == ns_a)
  const int64_t* off;    // device chunk table, nchunk + 1 entries
  int32_t nchunk;
  int64_t ns, ns_a, slab, nslabs;
};
// Plan-time temporaries of the sort.
struct SortTemp {
  int64_t* starts;      // [nslabs][ntiles]
  int64_t* tile_runs;   // [ntiles]
  int64_t* runbase;     // [ntiles + 1]
  int64_t* rstart;      // [nruns]
  int64_t* rend;        // [nruns]
  int32_t* rchunk;      // [nruns]
  int64_t *nsb, *nseg, *nsort, *sbbase, *segbase, *sortbase;  // [ntiles] each
};
// What the sort leaves in the plan.
struct SortOut {
  Tile* tiles;
  SubBatch* sbs;
  Segment* segs;
  uint16_t* perm;
  uint16_t* lp;
  uint8_t* psi_sorted;
  uint32_t* packed;     // the packed entries in place of the three above (or null)
  int lp_bits;
  uint16_t* lp_stage;   // the same local pixels and angles in stage order (projecting plans; else null)
  uint8_t* psi_stage;
  int64_t cap_sb, cap_seg, cap_sort;
  int64_t* totals;      // [3]: sub-batches, segments, sorted entries
};

constexpr int kMaxDevices = 64;
// bytes of the fixed device array used by the allocation-free workspace query
constexpr size_t kStaticScratchBytes = size_t(1) << 20;

hipError_t launch_sort_clear(SortCounters* ctr, hipStream_t s);
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s);
hipError_t launch_sort_stats(const SlabWalk& w, int64_t npix, int64_t nxm, const void* psi, const void* psi_b,
                             int psi_kind, int64_t table_len, SortCounters* ctr, hipStream_t s);
hipError_t launch_sort_count(const SlabWalk& w, const TileGeom& g, SortCounters* ctr, int64_t* starts,
                             hipStream_t s);
hipError_t launch_sort_lists(const SlabWalk& w, const TileGeom& g, int64_t nym, const SortTemp& T, const SortOut& O,
                             SortCounters* ctr, hipStream_t s);
hipError_t launch_sort_pixels(const SlabWalk& w, const void* psi, const void* psi_b, int psi_esz, const TileGeom& g,
                              const SortOut& O, hipStream_t s);
// address of the fixed scratch array on `device` (which must be current); looked up once per device
void* static_scratch(int device, hipError_t* err);

// pass-A sources
// pass-A sources: gather P m directly, or read a TOD-sized buffer holding P m written in
// pixel-tile order (by the binning epilogue or the projection kernel)
// SRC_GAP: t_0 - t_1 of gap filling, t_1 = d outside the gaps and d_0 inside (t_0 from the
// buffer argument, d_0 and the flags from DevPlan)
enum { SRC_D_MINUS_PM = 0, SRC_PM = 1, SRC_D = 2, SRC_D_MINUS_PMBUF = 3, SRC_PMBUF = 4, SRC_GAP = 5 };
// pass-B operations (bit set)
enum {
  B_CHI2 = 1,         // accumulate chi^2(., chi2_lambda) partials
  B_FILTER = 2,       // multiply by a gain, inverse-transform and write back
};
// GAIN_GAPFILL: eps / (eps + N-bar_0) with eps = sigma^2 - tau (the d_0 update of gap filling);
// GAIN_MESSENGER_PL: the messenger gain with N-bar = the power-law part alone (N-bar_0 there)
enum { GAIN_MESSENGER = 0, GAIN_NINV = 1, GAIN_LIFT = 2, GAIN_GAPFILL = 3, GAIN_MESSENGER_PL = 4 };
// binning sources / epilogues
enum { BSRC_WORK = 0, BSRC_DATA_OVER_TAU = 1, BSRC_PLAN = 2 };
// EPI_MAPSIZED: m_out = m_d + m_in - W^-1 b (DevPlan::md), the map-sized form of an iteration
enum { EPI_WRITE_B = 0, EPI_UPDATE = 1, EPI_REPLACE = 2, EPI_PLAN = 3, EPI_MAPSIZED = 4 };

// ---------------------------------------------------------------------------------------------
// kernel launchers (kernels.hip)

hipError_t launch_pass_a(const DevPlan& P, const ItemAC* items, int nitems, const void* d, const double* m,
                         int src, void* work, size_t lds_bytes, hipStream_t s, const void* pmbuf = nullptr);
hipError_t launch_pass_b(const DevPlan& P, const ItemB* items, int nitems, void* work, int ops, int gain,
                         double lam, double chi2_lam, double* chi2_part, size_t lds_bytes, hipStream_t s,
                         double* modes = nullptr);
// one chunk's per-mode chi^2 terms (k = 0 .. M) summed in log-spaced bins: out [nbins][2] (sum, modes)
hipError_t launch_modes_bin(const double* modes, int64_t M, int per_octave, int nbins, double* out, hipStream_t s);
hipError_t launch_pass_c(const DevPlan& P, const ItemAC* items, int nitems, void* work, size_t lds_bytes,
                         hipStream_t s);
hipError_t launch_bin(const DevPlan& P, int bsrc, const void* src, int epi, const double* m_in, double* out,
                      double* w_out, int32_t* hits_out, hipStream_t s, void* pm_out = nullptr);
hipError_t launch_interleave(const DevPlan& P, const double* m, hipStream_t s);
// LDS bytes the binning kernels of a plan take per workgroup (tiles of tile_pix pixels)
size_t binning_lds_bytes(int ncomp, int precision, int tile_pix);
// binning by FP64 atomics (the measured alternative): b += P^T src over all samples (b zeroed by
// the caller), then the per-pixel update of the binning epilogue from b
hipError_t launch_bin_atomic(const DevPlan& P, int bsrc, const void* src, double* b, int64_t max_n, hipStream_t s);
hipError_t launch_update(const DevPlan& P, int epi, const double* m_in, const double* b, double* out, hipStream_t s);
// the filtered TOD of the work buffer (chunk bases at xoff) copied to time order
hipError_t launch_unshift(const DevPlan& P, const void* work, void* out, hipStream_t s);
hipError_t launch_project(const DevPlan& P, const double* m, void* pm_out, hipStream_t s);
// gap filling's time-domain steps (time-order TOD buffers; y of the work buffer at chunk bases xoff):
// d_0 = d outside the gaps and 0 inside, t_0 = d_0; then d_0 = t_1 + y; then t_0 = P m + tau y
hipError_t launch_gap_init(const DevPlan& P, const void* d, const uint8_t* gaps, void* d0, void* t0, hipStream_t s);
hipError_t launch_gap_d0(const DevPlan& P, const void* d, const uint8_t* gaps, const void* work, void* d0,
                         hipStream_t s);
hipError_t launch_gap_t0(const DevPlan& P, const void* pm, const void* work, void* t0, hipStream_t s);
hipError_t launch_spectrum(const DevPlan& P, double* spec, hipStream_t s);
hipError_t launch_grad(const DevPlan& P, const ItemB* items, int nitems, const int32_t* chunk_item_begin,
                       const void* Xr, const void* Xz, double* part, double* out, size_t lds, hipStream_t s);
hipError_t launch_chi2_reduce(const int32_t* chunk_item_begin, const double* part, int nchunk, double* per_chunk,
                              double* total, hipStream_t s);
// map-space vector kernels for CG and helpers
hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
hipError_t launch_copy_bytes(void* dst, const void* src, int64_t nbytes, hipStream_t s);
hipError_t launch_dot_partials(const double* a, const double* b, int64_t n, double* part, int nblk, hipStream_t s);
hipError_t launch_reduce(const double* part, int n, double* out, hipStream_t s);
hipError_t launch_winv_apply(const DevPlan& P, const double* x, double* y, hipStream_t s);
hipError_t launch_cg_update_xr(const DevPlan& P, double* x, double* r, double* z, const double* p,
                               const double* q, const double* rz, const double* pq, double* part, int nblk,
                               hipStream_t s);
hipError_t launch_cg_update_p(double* p, const double* z, const double* rz_new, const double* rz_old, int64_t n,
                              hipStream_t s);
hipError_t launch_cg_chi2(const double* chi2_0, const double* xb, const double* xr, double* out, hipStream_t s);
hipError_t launch_sub(double* out, const double* a, const double* b, int64_t n, hipStream_t s);
int dot_blocks(int64_t n);

}  // namespace mm
