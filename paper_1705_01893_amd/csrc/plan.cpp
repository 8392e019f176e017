// Plan construction for libmm: validation, transform splits, twiddle tables, work lists, the
// device-side pixel-tile sort that makes binning deterministic, and the layout of every device
// buffer inside the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "mm.h"
#include "plan.h"

namespace mm {

thread_local std::string g_last_error;

mm_status fail(mm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

namespace {

bool five_smooth(int64_t x) {
  if (x < 1) return false;
  for (int p : {2, 3, 5})
    while (x % p == 0) x /= p;
  return x == 1;
}

size_t psi_elem_size(int kind) {
  switch (kind) {
    case MM_PSI_F64: return 8;
    case MM_PSI_F32: return 4;
    case MM_PSI_U16: return 2;
    default: return 0;
  }
}

bool noise_ok(double sg, double fk, double al, const double* tau, int64_t c, std::string& why) {
  if (!(sg > 0) || !(fk > 0) || !std::isfinite(al) || !std::isfinite(sg) || !std::isfinite(fk)) {
    why = "chunk " + std::to_string(c) + ": invalid noise parameters";
    return false;
  }
  if (tau && (!(tau[c] > 0) || tau[c] > sg * sg * (1 + 1e-12))) {
    why = "chunk " + std::to_string(c) + ": tau must satisfy 0 < tau <= sigma^2";
    return false;
  }
  return true;
}

mm_status validate(const mm_plan_desc* desc) {
  if (!desc) return fail(MM_E_ARG, "null descriptor");
  const mm_plan_desc& D = *desc;
  if (D.ncomp != 1 && D.ncomp != 3) return fail(MM_E_ARG, "ncomp must be 1 or 3");
  if (D.precision != MM_FP64 && D.precision != MM_MIXED) return fail(MM_E_ARG, "unknown precision");
  if (D.npix <= 0 || D.npix > (int64_t)INT32_MAX) return fail(MM_E_ARG, "npix out of range");
  if (D.nx < 0 || (D.nx > 0 && D.npix % D.nx != 0)) return fail(MM_E_ARG, "nx must divide npix");
  if (D.nchunk <= 0 || D.nchunk > (int64_t)INT32_MAX - 1) return fail(MM_E_ARG, "nchunk out of range");
  if (!D.chunk_off || !D.fsample || !D.sigma || !D.fknee || !D.alpha || !D.pix)
    return fail(MM_E_ARG, "missing chunk table, noise parameters or pointing");
  if (D.ncomp == 3) {
    if (!D.psi || (D.psi_kind != MM_PSI_F64 && D.psi_kind != MM_PSI_F32 && D.psi_kind != MM_PSI_U16))
      return fail(MM_E_ARG, "I/Q/U maps need polarization angles");
    if (D.psi_kind == MM_PSI_U16 && (!D.psi_table || D.psi_table_len <= 0 || D.psi_table_len > 65536))
      return fail(MM_E_ARG, "uint16 angle indices need a host angle table of 1..65536 entries");
  }
  if (D.map_access != MM_MAP_AUTO && D.map_access != MM_MAP_GATHER && D.map_access != MM_MAP_PROJECTED)
    return fail(MM_E_ARG, "unknown map_access");
  const bool pick_mode = D.tune >= MM_TUNE_PICK0 && D.tune < MM_TUNE_PICK0 + 4096;
  if (D.tune != MM_TUNE_MEASURE && D.tune != MM_TUNE_STATIC && !pick_mode) return fail(MM_E_ARG, "unknown tune mode");
  if (D.binning != MM_BIN_SORTED && D.binning != MM_BIN_ATOMIC) return fail(MM_E_ARG, "unknown binning mode");
  if (D.with_adjoint != 0 && D.with_adjoint != 1) return fail(MM_E_ARG, "with_adjoint must be 0 or 1");
  if (D.tile_pixels != 0 && (D.tile_pixels < 16 || D.tile_pixels > kMaxTilePixAsked))
    return fail(MM_E_ARG, "tile_pixels must be 0 (automatic) or 16.." + std::to_string(kMaxTilePixAsked));
  if (D.with_gapfill != 0 && D.with_gapfill != 1) return fail(MM_E_ARG, "with_gapfill must be 0 or 1");
  if (D.with_gapfill && D.pix_b) return fail(MM_E_ARG, "gap filling needs single-beam pointing");
  if (D.with_gapfill && D.map_access == MM_MAP_GATHER)
    return fail(MM_E_ARG, "gap filling reads P m from the projection buffer (map_access AUTO or PROJECTED)");
  if (D.pix_b) {
    if (D.ncomp == 3 && !D.psi_b) return fail(MM_E_ARG, "composite I/Q/U pointing needs the second angles (psi_b)");
    if (!std::isfinite(D.weight_a) || !std::isfinite(D.weight_b))
      return fail(MM_E_ARG, "composite pointing weights must be finite");
    if (D.map_access == MM_MAP_GATHER)
      return fail(MM_E_ARG, "composite pointing reads P m from the projection buffer (map_access AUTO or PROJECTED)");
    if (D.binning != MM_BIN_SORTED) return fail(MM_E_ARG, "composite pointing needs sorted binning");
  }
  if (D.chunk_off[0] != 0) return fail(MM_E_ARG, "chunk_off[0] must be 0");
  std::string why;
  for (int64_t c = 0; c < D.nchunk; ++c) {
    const int64_t n = D.chunk_off[c + 1] - D.chunk_off[c];
    if (n <= 0) return fail(MM_E_ARG, "chunk offsets must increase");
    if (n % 2 != 0 || n < 2) return fail(MM_E_LEN, "chunk " + std::to_string(c) + ": length must be even");
    if (!five_smooth(n / 2))
      return fail(MM_E_LEN, "chunk " + std::to_string(c) + ": half length must factor into 2, 3 and 5");
    if (n / 2 > (1 << 24)) return fail(MM_E_LEN, "chunk " + std::to_string(c) + ": too long");
    if (!(D.fsample[c] > 0) || !std::isfinite(D.fsample[c]))
      return fail(MM_E_ARG, "chunk " + std::to_string(c) + ": invalid sample rate");
    if (!noise_ok(D.sigma[c], D.fknee[c], D.alpha[c], D.tau, c, why)) return fail(MM_E_ARG, why);
  }
  if (D.ncomp == 3 && D.psi_kind == MM_PSI_U16)
    for (int64_t i = 0; i < D.psi_table_len; ++i)
      if (!(std::fabs(2.0 * (double)D.psi_table[i]) < 2.0 * kMaxAngle))
        return fail(MM_E_ARG, "angle table entry is not finite or too large");
  return MM_OK;
}

// What the workspace size depends on: the chunk lengths (transform tables), the tiles, and two
// counts the device analysis takes from the pointing (on-map samples and runs).
struct ClassInfo {
  int64_t M = 0;
  std::vector<Layout> cands;
  int64_t nchunks = 0;
  size_t ac = 0, b = 0, g = 0, tw = 0;  // largest per-chunk item counts and twiddles over the candidates
};

struct Prep {
  bool f64 = true;
  size_t tsz = 8, pes = 0;
  int64_t ns = 0, nchunk = 0, mapn = 0;
  // pointing entries and their chunks: N_s and nchunk, doubled with composite pointing
  bool composite = false;
  int64_t nent = 0, nchunk_ent = 0;
  int nw = 1;
  std::vector<int32_t> chunk_class;
  std::vector<ClassInfo> classes;
  int64_t xwork = 0, spec_total = 0;
  size_t capAC = 0, capB = 0, capG = 0, capTW = 0;
  size_t tune_bytes = 0;
  int tune_streams = 1;  // TOD-sized streams pass A reads (what the tuner's timing reads)
  bool pm_mode = false, adjoint = false, bin_atomic = false, mapi = false, gapfill = false;
  // tiles and counts
  int64_t nxm = 0, nym = 0, tw = 0, th = 0, ntx = 0, nty = 0, ntiles = 0;
  int64_t non = 0, nruns = 0;
  int64_t nslabs = 1, slab = 1;
  int64_t cap_sb = 0, cap_seg = 0, cap_sort = 0;
  // sorted entries packed into 32 bits (16-bit angle indices that fit beside the stage position
  // and the local pixel), with lp_bits bits of local pixel
  bool pack = false;
  int lp_bits = 0;
};

void prep_transforms(const mm_plan_desc& D, Prep& P) {
  P.f64 = D.precision == MM_FP64;
  P.tsz = P.f64 ? 8 : 4;
  P.pes = D.ncomp == 3 ? psi_elem_size(D.psi_kind) : 0;
  P.nchunk = D.nchunk;
  P.ns = D.chunk_off[D.nchunk];
  P.composite = D.pix_b != nullptr;
  P.nent = P.composite ? 2 * P.ns : P.ns;
  P.nchunk_ent = P.composite ? 2 * P.nchunk : P.nchunk;
  P.mapn = (int64_t)D.ncomp * D.npix;
  P.nw = D.ncomp == 1 ? 1 : 6;
  P.chunk_class.resize(D.nchunk);
  for (int64_t c = 0; c < D.nchunk; ++c) {
    const int64_t M = (D.chunk_off[c + 1] - D.chunk_off[c]) / 2;
    int cls = -1;
    for (size_t i = 0; i < P.classes.size(); ++i)
      if (P.classes[i].M == M) cls = (int)i;
    if (cls < 0) {
      ClassInfo ci;
      ci.M = M;
      ci.cands = layout_candidates(M, P.f64);
      for (const Layout& L : ci.cands) {
        DevChunk ch;
        std::memset(&ch, 0, sizeof(ch));
        ch.M1 = (int32_t)L.M1;
        ch.M2 = (int32_t)L.M2;
        ch.cb = L.cb;
        std::vector<ItemAC> a;
        std::vector<ItemB> b, g;
        append_col_items(0, ch, a);
        append_row_items(0, ch, b, row_fuse(L.M1, P.f64));
        append_row_items(0, ch, g, false);
        std::vector<double2> tw;
        DevClass k;
        make_class(M, L, tw, k);
        ci.ac = std::max(ci.ac, a.size());
        ci.b = std::max(ci.b, b.size());
        ci.g = std::max(ci.g, g.size());
        ci.tw = std::max(ci.tw, tw.size());
      }
      cls = (int)P.classes.size();
      P.classes.push_back(ci);
    }
    P.chunk_class[c] = cls;
    ClassInfo& ci = P.classes[cls];
    ci.nchunks += 1;
    P.capAC += ci.ac;
    P.capB += ci.b;
    P.capG += ci.g;
    P.xwork += (M + kWorkAlign - 1) / kWorkAlign * kWorkAlign;
    P.spec_total += M + 1;
  }
  P.adjoint = D.with_adjoint != 0;
  P.bin_atomic = D.binning == MM_BIN_ATOMIC;
  // maps larger than the L2 of one XCD (4 MB) are gathered badly by the strided column pass:
  // then P m is produced in pixel-tile order instead
  P.gapfill = D.with_gapfill != 0;
  P.pm_mode = D.map_access == MM_MAP_PROJECTED || P.composite || P.gapfill ||
              (D.map_access == MM_MAP_AUTO && P.mapn * (int64_t)sizeof(double) > ((int64_t)4 << 20));
  P.mapi = !P.pm_mode && D.ncomp == 3;
  P.tune_streams = !P.pm_mode ? 1 : (P.composite ? 3 : 2);
  for (const ClassInfo& ci : P.classes) {
    P.capTW += ci.tw;
    if (D.tune == MM_TUNE_MEASURE)
      P.tune_bytes = std::max(P.tune_bytes, tune_scratch_bytes(ci.M, P.f64, ci.cands, P.tune_streams));
  }
}

// Tile shape: about `target` pixels, tw a power of two, shaped by the scan.  A sample moving
// (mx, my) pixels per step stays about 1 / (mx / tw + my / th) steps in a tile, so the shape
// that maximises it gives the longest time-contiguous segments (fewer, longer HBM runs for the
// staging reads and the P m writes).  mx, my: mean steps between consecutive on-map samples of
// a chunk, from the analysis counters.
void tile_shape(const mm_plan_desc& D, const SortCounters& c, Prep& P) {
  P.nxm = D.nx > 0 ? D.nx : D.npix;
  P.nym = D.npix / P.nxm;
  const int64_t target = D.tile_pixels > 0 ? std::min<int64_t>(D.tile_pixels, D.npix)
                                           : std::max<int64_t>(16, std::min<int64_t>(kMaxTilePix, D.npix / 2048));
  double mx = c.nst ? (double)c.sx / (double)c.nst : 1.0;
  double my = c.nst ? (double)c.sy / (double)c.nst : 1.0;
  if (mx + my <= 0.0) mx = my = 1.0;
  int64_t tw = 1, th = target;
  double best = -1.0;
  for (int64_t w = 1; w <= std::min<int64_t>(target, P.nxm); w *= 2) {
    const int64_t h = std::min<int64_t>(P.nym, std::max<int64_t>(1, target / w));
    const double visit = 1.0 / (mx / (double)w + my / (double)h);
    if (visit > best * 1.000001) {
      best = visit;
      tw = w;
      th = h;
    }
  }
  if (P.nym == 1) {
    tw = target;
    th = 1;
  }
  P.tw = std::min(tw, P.nxm);
  P.th = std::min(th, P.nym);
  P.ntx = (P.nxm + P.tw - 1) / P.tw;
  P.nty = (P.nym + P.th - 1) / P.th;
  P.ntiles = P.ntx * P.nty;
}

TileGeom geom(const Prep& P) {
  TileGeom g;
  g.nxm = (int32_t)P.nxm;
  g.tw = (int32_t)P.tw;
  g.th = (int32_t)P.th;
  g.ntx = (int32_t)P.ntx;
  g.ntiles = (int32_t)P.ntiles;
  return g;
}

constexpr int64_t kFineSlab = int64_t(1) << 14;       // samples per thread of the analysis walks
constexpr int64_t kSlabMatrix = int64_t(1) << 25;     // entries of the per-slab, per-tile run counts

// Bytes of the analysis header at the start of the workspace: the device chunk table of the
// pointing entries (nchunk_ent + 1 offsets) and the counters (with the sort's totals).
size_t header_bytes(int64_t nchunk_ent) {
  Arena a;
  a.take((size_t)(nchunk_ent + 1) * sizeof(int64_t));
  a.take(256);
  return a.used;
}

// The chunk table of the pointing entries: the caller's, followed for composite pointing by the
// same chunks shifted by N_s (the second components).
std::vector<int64_t> entry_chunk_table(const mm_plan_desc& D, const Prep& P) {
  std::vector<int64_t> off(D.chunk_off, D.chunk_off + D.nchunk + 1);
  if (P.composite)
    for (int64_t c = 1; c <= D.nchunk; ++c) off.push_back(P.ns + D.chunk_off[c]);
  return off;
}

SlabWalk entry_walk(const mm_plan_desc& D, const Prep& P, const int64_t* doff) {
  SlabWalk w;
  w.pix = D.pix;
  w.pix_b = P.composite ? D.pix_b : nullptr;
  w.off = doff;
  w.nchunk = (int32_t)P.nchunk_ent;
  w.ns = P.nent;
  w.ns_a = P.ns;
  w.slab = kFineSlab;
  w.nslabs = (P.nent + kFineSlab - 1) / kFineSlab;
  return w;
}

// Analysis passes over the device pointing: validation, scan statistics (tile shape), on-map
// samples and runs.  doff / dctr: device chunk table and counters.  Waits for the stream.
mm_status analyse(const mm_plan_desc& D, Prep& P, int64_t* doff, SortCounters* dctr, hipStream_t s) {
  const std::vector<int64_t> off = entry_chunk_table(D, P);
  if (hipMemcpyAsync(doff, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(MM_E_HIP, "chunk table upload failed");
  const SlabWalk w = entry_walk(D, P, doff);
  hipError_t e = launch_sort_clear(dctr, s);
  if (e == hipSuccess)
    e = launch_sort_stats(w, D.npix, D.nx > 0 ? D.nx : D.npix, D.ncomp == 3 ? D.psi : nullptr,
                          D.ncomp == 3 && P.composite ? D.psi_b : nullptr, D.ncomp == 3 ? D.psi_kind : 0,
                          D.psi_table_len, dctr, s);
  SortCounters c;
  if (e == hipSuccess) e = hipMemcpyAsync(&c, dctr, sizeof(c), hipMemcpyDeviceToHost, s);
  // waited on in every case: the host chunk table must outlive its upload
  const hipError_t es = hipStreamSynchronize(s);
  if (e == hipSuccess) e = es;
  if (e != hipSuccess)
    return fail(MM_E_HIP, std::string("pointing analysis failed (are pix and psi device pointers?): ") +
                              hipGetErrorString(e));
  if (c.flags & 1u) return fail(MM_E_ARG, "a pixel index lies beyond the map");
  if (c.flags & 2u) return fail(MM_E_ARG, "an angle is not finite or has |psi| >= 1e5");
  if (c.flags & 4u) return fail(MM_E_ARG, "an angle index lies beyond the angle table");
  tile_shape(D, c, P);
  if (P.ntiles > (int64_t)INT32_MAX) return fail(MM_E_ARG, "too many pixel tiles");
  // a sorted entry's stage position takes 12 bits and its local pixel lp_bits: a 16-bit angle
  // index of a table of at most 2^(20 - lp_bits) entries fits beside them in one 32-bit word
  P.lp_bits = 1;
  while (((int64_t)1 << P.lp_bits) < P.tw * P.th) ++P.lp_bits;
  P.pack = D.ncomp == 3 && D.psi_kind == MM_PSI_U16 && P.lp_bits <= 16 &&
           D.psi_table_len <= ((int64_t)1 << (20 - P.lp_bits));
  {
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return fail(MM_E_HIP, "device LDS query failed");
    const size_t need = binning_lds_bytes(D.ncomp, D.precision, (int)(P.tw * P.th));
    if (need > (size_t)lds_max)
      return fail(MM_E_ARG, "binning tiles of " + std::to_string(P.tw * P.th) + " pixels need " + std::to_string(need) +
                                " bytes of LDS per workgroup; the device allows " + std::to_string(lds_max));
  }
  e = launch_sort_count(w, geom(P), dctr, nullptr, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&c, dctr, sizeof(c), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(MM_E_HIP, std::string("run count failed: ") + hipGetErrorString(e));
  P.non = (int64_t)c.non;
  P.nruns = (int64_t)c.nruns;
  // Reserved sizes.  A sub-batch closes when it holds kSubBatch samples (at most non / kSubBatch
  // of them) or kMaxSegs segments; a segment is a run or, after a full sub-batch, the rest of a
  // run, so there are at most nruns + non / kSubBatch segments and sub-batches closed on segments
  // number at most that over kMaxSegs; each tile adds one unfinished sub-batch.  The sorted
  // entries of a sub-batch are padded to kSortAlign.
  const int64_t full = P.non / kSubBatch;
  P.cap_seg = P.nruns + full + 1;
  P.cap_sb = full + P.cap_seg / kMaxSegs + P.ntiles + 1;
  P.cap_sort = P.non + (int64_t)(kSortAlign - 1) * P.cap_sb + kSortAlign;
  if (P.cap_seg > (int64_t)INT32_MAX || P.cap_sb > (int64_t)INT32_MAX)
    return fail(MM_E_ARG, "the pointing has too many time-contiguous segments per tile");
  // slabs of the run-list walk: enough threads, within the per-slab, per-tile count budget
  const int64_t want = std::max<int64_t>(1, (P.nent + kFineSlab - 1) / kFineSlab);
  P.nslabs = std::max<int64_t>(1, std::min<int64_t>(want, kSlabMatrix / std::max<int64_t>(1, P.ntiles)));
  P.slab = (P.nent + P.nslabs - 1) / P.nslabs;
  return MM_OK;
}

// Every device buffer of a plan, in workspace order.  With a measuring arena only the size
// comes out.
struct Bufs {
  int64_t* off = nullptr;
  SortCounters* ctr = nullptr;
  DevChunk* chunks = nullptr;
  DevClass* classes = nullptr;
  double2* tw64 = nullptr;
  float2* tw32 = nullptr;
  double2* sc = nullptr;
  double2* cs64 = nullptr;
  float2* cs32 = nullptr;
  ItemAC* itemsAC = nullptr;
  ItemB* itemsB = nullptr;
  int32_t* cib = nullptr;
  ItemB* itemsG = nullptr;
  int32_t* cigb = nullptr;
  Tile* tiles = nullptr;
  SubBatch* sbs = nullptr;
  Segment* segs = nullptr;
  uint16_t* perm = nullptr;
  uint16_t* lp = nullptr;
  uint8_t* psis = nullptr;
  uint32_t* packed = nullptr;  // in place of perm, lp and psis when the plan packs its entries
  uint16_t* lpq = nullptr;  // stage-order copies for the projection walk (projecting plans)
  uint8_t* psiq = nullptr;
  double* winv = nullptr;
  uint8_t* sol = nullptr;
  int32_t* hits = nullptr;
  double* spec = nullptr;
  double* chi2part = nullptr;
  double* scal = nullptr;
  double* part = nullptr;
  double* maps[kScratchMaps] = {};
  double2* mapi = nullptr;
  double* batom = nullptr;
  double* hist = nullptr;
  void* work = nullptr;
  void* pm = nullptr;
  void* work2 = nullptr;
  void* gd0 = nullptr;
  void* gt0 = nullptr;
  char* transient = nullptr;
  size_t transient_bytes = 0;
  SortTemp T = {};
};

template <typename X>
bool take(Arena& a, size_t n, X** out) {
  void* p = a.take(n * sizeof(X));
  *out = (X*)p;
  return p != nullptr;
}

bool carve_sort_temp(Arena& a, const Prep& P, SortTemp& T) {
  const size_t nt = (size_t)P.ntiles;
  return take(a, (size_t)P.nslabs * nt, &T.starts) && take(a, nt, &T.tile_runs) && take(a, nt + 1, &T.runbase) &&
         take(a, (size_t)P.nruns, &T.rstart) && take(a, (size_t)P.nruns, &T.rend) &&
         take(a, (size_t)P.nruns, &T.rchunk) && take(a, nt, &T.nsb) && take(a, nt, &T.nseg) && take(a, nt, &T.nsort) &&
         take(a, nt, &T.sbbase) && take(a, nt, &T.segbase) && take(a, nt, &T.sortbase);
}

bool carve(Arena& a, const mm_plan_desc& D, const Prep& P, Bufs& B) {
  const int64_t npix = D.npix;
  bool ok = take(a, (size_t)P.nchunk_ent + 1, &B.off);
  void* c = a.take(256);
  B.ctr = (SortCounters*)c;
  ok = ok && c && take(a, (size_t)P.nchunk, &B.chunks) && take(a, P.classes.size(), &B.classes) &&
       take(a, P.capTW, &B.tw64) && take(a, P.capTW, &B.tw32) && take(a, 1024, &B.sc);
  if (ok && D.ncomp == 3 && D.psi_kind == MM_PSI_U16)
    ok = take(a, (size_t)D.psi_table_len, &B.cs64) && take(a, (size_t)D.psi_table_len, &B.cs32);
  ok = ok && take(a, P.capAC, &B.itemsAC) && take(a, P.capB, &B.itemsB) && take(a, (size_t)P.nchunk + 1, &B.cib) &&
       take(a, P.capG, &B.itemsG) && take(a, (size_t)P.nchunk + 1, &B.cigb);
  ok = ok && take(a, (size_t)P.ntiles, &B.tiles) && take(a, (size_t)P.cap_sb, &B.sbs) &&
       take(a, (size_t)P.cap_seg, &B.segs);
  if (ok && P.pack) {
    // the packed entries take the start of the space the three unpacked arrays would take, so
    // that the buffers after them keep their offsets (measured: the binning and projection
    // passes of the 1024 x 2^22 workload ran 1.5 ms slower each with the later buffers moved down
    // by the 2 bytes per entry packing saves)
    uint16_t* rest = nullptr;
    ok = take(a, (size_t)P.cap_sort, &B.packed) && take(a, (size_t)P.cap_sort, &rest);
  } else {
    ok = ok && take(a, (size_t)P.cap_sort, &B.perm) && take(a, (size_t)P.cap_sort, &B.lp);
    if (ok && P.pes) ok = take(a, (size_t)P.cap_sort * P.pes, &B.psis);
  }
  if (ok && P.pm_mode) ok = take(a, (size_t)P.cap_sort, &B.lpq);
  if (ok && P.pm_mode && P.pes) ok = take(a, (size_t)P.cap_sort * P.pes, &B.psiq);
  ok = ok && take(a, (size_t)P.nw * npix, &B.winv) && take(a, (size_t)npix, &B.sol) && take(a, (size_t)npix, &B.hits);
  if (ok && P.f64) ok = take(a, (size_t)P.spec_total, &B.spec);
  ok = ok && take(a, std::max<size_t>(P.capB, 3 * P.capG), &B.chi2part) && take(a, 64, &B.scal) &&
       take(a, 1024, &B.part);
  for (int i = 0; ok && i < kScratchMaps; ++i) ok = take(a, (size_t)P.mapn, &B.maps[i]);
  if (ok && P.mapi) ok = take(a, (size_t)npix * 2, &B.mapi);
  if (ok && P.bin_atomic) ok = take(a, (size_t)P.mapn, &B.batom);
  ok = ok && take(a, (size_t)kCgHistCap, &B.hist);
  if (!ok) return false;
  // TOD-sized buffers; the plan-time temporaries (sort lists, tuner scratch) overlay them
  const size_t tod0 = (a.used + 255) / 256 * 256;
  char* w = nullptr;
  ok = take(a, (size_t)(2 * P.xwork) * P.tsz, &w);
  B.work = w;
  if (ok && P.pm_mode) ok = take(a, (size_t)P.nent * P.tsz, (char**)&B.pm);
  if (ok && P.adjoint) ok = take(a, (size_t)(2 * P.xwork) * P.tsz, (char**)&B.work2);
  if (ok && P.gapfill)
    ok = take(a, (size_t)P.ns * P.tsz, (char**)&B.gd0) && take(a, (size_t)P.ns * P.tsz, (char**)&B.gt0);
  if (!ok) return false;
  const size_t tod_bytes = a.used - tod0;
  Arena m;
  SortTemp dummy;
  carve_sort_temp(m, P, dummy);
  const size_t trans = std::max(std::max(tod_bytes, m.used), P.tune_bytes);
  if (trans > tod_bytes && !a.take(trans - tod_bytes)) return false;
  B.transient_bytes = trans;
  if (a.base) {
    B.transient = a.base + tod0;
    Arena t;
    t.base = B.transient;
    t.cap = trans;
    if (!carve_sort_temp(t, P, B.T)) return false;
  }
  return true;
}

// noise spectrum table (FP64 form), hit counts, weight blocks P^T T^-1 P, their inverses and the
// solvable mask; waits for the stream
mm_status plan_precompute(mm_plan_s* pl, hipStream_t s) {
  DevPlan& P = pl->dp;
  if (P.spec) {
    hipError_t es = launch_spectrum(P, (double*)P.spec, s);
    if (es != hipSuccess) return fail(MM_E_HIP, std::string("spectrum kernel launch: ") + hipGetErrorString(es));
  }
  hipError_t e = launch_bin(P, BSRC_PLAN, nullptr, EPI_PLAN, nullptr, (double*)pl->d_solvable, pl->d_winv,
                            pl->d_hits, s);
  if (e != hipSuccess) return fail(MM_E_HIP, std::string("plan kernel launch: ") + hipGetErrorString(e));
  std::vector<uint8_t> sol(pl->npix);
  if (hipMemcpyAsync(sol.data(), pl->d_solvable, pl->npix, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(MM_E_HIP, std::string("plan precompute failed: ") + hipGetErrorString(hipGetLastError()));
  int64_t nsol = 0;
  for (int64_t i = 0; i < pl->npix; ++i) nsol += sol[i];
  pl->nsolvable = nsol;
  return MM_OK;
}

template <typename X>
mm_status upload(const std::vector<X>& v, X* dst, size_t cap, hipStream_t s) {
  if (v.size() > cap) return fail(MM_E_ARG, "internal: a plan table outgrew its reserved size");
  if (v.empty()) return MM_OK;
  if (hipMemcpyAsync(dst, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(MM_E_HIP, "host to device copy failed");
  return MM_OK;
}

}  // namespace

mm_status plan_set_noise(mm_plan_s* pl, const double* sigma, const double* fknee, const double* alpha,
                         const double* tau, hipStream_t s) {
  if (!sigma || !fknee || !alpha) return fail(MM_E_ARG, "missing noise parameters");
  std::string why;
  for (int64_t c = 0; c < pl->nchunk; ++c)
    if (!noise_ok(sigma[c], fknee[c], alpha[c], tau, c, why)) return fail(MM_E_ARG, why);
  for (int64_t c = 0; c < pl->nchunk; ++c) {
    pl->sigma[c] = sigma[c];
    pl->fknee[c] = fknee[c];
    pl->alpha[c] = alpha[c];
    pl->tau[c] = tau ? tau[c] : sigma[c] * sigma[c];
    DevChunk& ch = pl->chunks_host[c];
    ch.sigma2 = sigma[c] * sigma[c];
    ch.fknee = fknee[c];
    ch.alpha = alpha[c];
    ch.tau = pl->tau[c];
    ch.inv_tau = 1.0 / ch.tau;
    ch.nbar0 = ch.sigma2 - ch.tau;
    ch.lg0 = std::log2(ch.df / ch.fknee);
  }
  if (hipMemcpyAsync(pl->d_chunks, pl->chunks_host.data(), pl->chunks_host.size() * sizeof(DevChunk),
                     hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(MM_E_HIP, "chunk table upload failed");
  mm_status st = plan_precompute(pl, s);
  if (st != MM_OK) return st;
  if (pl->nsolvable == 0) return fail(MM_E_SINGULAR, "no pixel has a solvable weight block");
  return MM_OK;
}

mm_status workspace_query(const mm_plan_desc* desc, hipStream_t s, void* scratch, size_t scratch_bytes,
                          size_t* bytes) {
  if (!bytes) return fail(MM_E_ARG, "null output");
  mm_status st = validate(desc);
  if (st != MM_OK) return st;
  const mm_plan_desc& D = *desc;
  Prep P;
  prep_transforms(D, P);
  const size_t hb = header_bytes(P.nchunk_ent);
  void* own = nullptr;
  if (!scratch) {
    if (hipMalloc(&own, hb) != hipSuccess) return fail(MM_E_NOMEM, "device allocation failed (analysis counters)");
    scratch = own;
  } else if (hb > scratch_bytes) {
    return fail(MM_E_ARG, "the fixed scratch of " + std::to_string(scratch_bytes) +
                              " bytes holds a chunk table of at most " +
                              std::to_string((scratch_bytes - 256) / sizeof(int64_t) - 1) +
                              " entries; this description needs " + std::to_string(P.nchunk_ent) +
                              " (twice the chunks with composite pointing)");
  }
  Arena h;
  h.base = (char*)scratch;
  h.cap = hb;
  int64_t* doff = (int64_t*)h.take((size_t)(P.nchunk_ent + 1) * sizeof(int64_t));
  SortCounters* dctr = (SortCounters*)h.take(256);
  st = analyse(D, P, doff, dctr, s);
  if (own) (void)hipFree(own);
  if (st != MM_OK) return st;
  Arena m;
  Bufs B;
  carve(m, D, P, B);
  *bytes = m.used;
  return MM_OK;
}

mm_status build_plan(const mm_plan_desc* desc, void* ws, size_t ws_bytes, hipStream_t s, mm_plan_s** out) {
  if (!out) return fail(MM_E_ARG, "null output");
  mm_status st = validate(desc);
  if (st != MM_OK) return st;
  const mm_plan_desc& D = *desc;
  if (!ws) return fail(MM_E_ARG, "null workspace");
  if ((uintptr_t)ws % 256 != 0) return fail(MM_E_ARG, "the workspace must be 256-byte aligned");
  Prep P;
  prep_transforms(D, P);
  const int64_t ns = P.ns;

  auto* pl = new mm_plan_s();
  std::unique_ptr<mm_plan_s, void (*)(mm_plan_s*)> guard(pl, [](mm_plan_s* p) { destroy_plan(p); });
  pl->ncomp = D.ncomp;
  pl->precision = D.precision;
  pl->psi_kind = D.ncomp == 3 ? D.psi_kind : MM_PSI_NONE;
  pl->npix = D.npix;
  pl->nx = D.nx;
  pl->nchunk = D.nchunk;
  pl->ns = ns;
  pl->off.assign(D.chunk_off, D.chunk_off + D.nchunk + 1);
  pl->sigma.assign(D.sigma, D.sigma + D.nchunk);
  pl->tau.resize(D.nchunk);
  pl->fsample.assign(D.fsample, D.fsample + D.nchunk);
  pl->fknee.assign(D.fknee, D.fknee + D.nchunk);
  pl->alpha.assign(D.alpha, D.alpha + D.nchunk);
  for (int64_t c = 0; c < D.nchunk; ++c) pl->tau[c] = D.tau ? D.tau[c] : D.sigma[c] * D.sigma[c];
  pl->ws = ws;
  pl->ws_bytes = ws_bytes;

  // ---- analysis of the pointing in the workspace's header, then the full layout
  if (header_bytes(P.nchunk_ent) > ws_bytes)
    return fail(MM_E_NOMEM, "the workspace is smaller than mm_plan_workspace_bytes reports");
  {
    Arena h;
    h.base = (char*)ws;
    h.cap = ws_bytes;
    int64_t* doff = (int64_t*)h.take((size_t)(P.nchunk_ent + 1) * sizeof(int64_t));
    SortCounters* dctr = (SortCounters*)h.take(256);
    if ((st = analyse(D, P, doff, dctr, s)) != MM_OK) return st;
  }
  Bufs B;
  {
    Arena m;
    Bufs tmp;
    carve(m, D, P, tmp);
    if (m.used > ws_bytes)
      return fail(MM_E_NOMEM, "the workspace holds " + std::to_string(ws_bytes) + " bytes; this plan needs " +
                                  std::to_string(m.used) + " (mm_plan_workspace_bytes)");
    Arena a;
    a.base = (char*)ws;
    a.cap = ws_bytes;
    if (!carve(a, D, P, B)) return fail(MM_E_NOMEM, "workspace layout failed");
    pl->ws_used = a.used;
  }
  const TileGeom g = geom(P);
  pl->ntiles = P.ntiles;
  pl->tile_w = (int32_t)P.tw;
  pl->tile_h = (int32_t)P.th;

  // ---- binning structures, sorted on the device
  SortOut O;
  O.tiles = B.tiles;
  O.sbs = B.sbs;
  O.segs = B.segs;
  O.perm = B.perm;
  O.lp = B.lp;
  O.psi_sorted = B.psis;
  O.packed = B.packed;
  O.lp_bits = P.lp_bits;
  O.lp_stage = B.lpq;
  O.psi_stage = B.psiq;
  O.cap_sb = P.cap_sb;
  O.cap_seg = P.cap_seg;
  O.cap_sort = P.cap_sort;
  O.totals = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(B.ctr) + 128);
  {
    SlabWalk w = entry_walk(D, P, B.off);
    w.slab = P.slab;
    w.nslabs = P.nslabs;
    hipError_t e = launch_fill_i64(B.T.starts, P.nslabs * P.ntiles, 0, s);
    if (e == hipSuccess) e = launch_sort_clear(B.ctr, s);
    if (e == hipSuccess) e = launch_sort_count(w, g, B.ctr, B.T.starts, s);
    if (e == hipSuccess) e = launch_sort_lists(w, g, P.nym, B.T, O, B.ctr, s);
    struct {
      SortCounters c;
      int64_t pad[10];
      int64_t totals[3];
    } hb;
    static_assert(sizeof(SortCounters) + 10 * sizeof(int64_t) == 128, "counter block layout");
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, B.ctr, sizeof(hb), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(MM_E_HIP, std::string("pixel-tile sort failed: ") + hipGetErrorString(e));
    if ((hb.c.flags & 8u) || (int64_t)hb.c.nruns != P.nruns || hb.totals[0] > P.cap_sb ||
        hb.totals[1] > P.cap_seg || hb.totals[2] > P.cap_sort)
      return fail(MM_E_ARG, "internal: the pixel-tile sort exceeded its reserved sizes");
    pl->nsbs = hb.totals[0];
    pl->nsegs = hb.totals[1];
    pl->nsorted = hb.totals[2];
    e = launch_sort_pixels(w, D.ncomp == 3 ? D.psi : nullptr, D.ncomp == 3 && P.composite ? D.psi_b : nullptr,
                           (int)P.pes, g, O, s);
    if (e != hipSuccess) return fail(MM_E_HIP, std::string("pixel sort launch: ") + hipGetErrorString(e));
  }

  // ---- transform classes (the tuner times candidates in the temporaries' space), tables
  const bool f64 = P.f64;
  const size_t csz = f64 ? sizeof(double2) : sizeof(float2);
  std::vector<double2> tw;
  std::vector<DevClass> classes;
  std::vector<int> class_cb;
  size_t lds_ac = 0, lds_b = 0, lds_g = 0;
  for (const ClassInfo& ci : P.classes) {
    if (ci.cands.empty()) return fail(MM_E_LEN, "a chunk length has no transform split that fits the LDS budget");
    int pick = 0;
    if (D.tune == MM_TUNE_MEASURE)
      pick = tune_layout(ci.M, f64, ci.cands, P.tune_streams, s, B.transient, B.transient_bytes);
    else if (D.tune >= MM_TUNE_PICK0)
      pick = std::min<int>(D.tune - MM_TUNE_PICK0, (int)ci.cands.size() - 1);
    const Layout& L = ci.cands[pick];
    DevClass k;
    make_class(ci.M, L, tw, k);
    classes.push_back(k);
    class_cb.push_back(L.cb);
    pl->class_layout.push_back(pick);
    pl->class_ncand.push_back((int32_t)ci.cands.size());
    lds_b = std::max(lds_b, (size_t)((row_fuse(L.M1, f64) ? 4 : 2) * L.M1) * csz);
    lds_g = std::max(lds_g, (size_t)(4 * L.M1) * csz);  // rows of r and of P z
  }
  std::vector<DevChunk> chunks(D.nchunk);
  int64_t spec_total = 0, xwork = 0;
  for (int64_t c = 0; c < D.nchunk; ++c) {
    const int64_t n = D.chunk_off[c + 1] - D.chunk_off[c];
    const int cls = P.chunk_class[c];
    const DevClass& k = classes[cls];
    DevChunk& ch = chunks[c];
    std::memset(&ch, 0, sizeof(ch));
    ch.off = D.chunk_off[c];
    ch.n = (int32_t)n;
    ch.M = k.M;
    ch.M1 = k.M1;
    ch.M2 = k.M2;
    ch.cls = cls;
    ch.cb = (int32_t)class_cb[cls];
    ch.lgb = 0;
    while ((1 << (ch.lgb + 1)) <= ch.cb) ++ch.lgb;
    ch.df = D.fsample[c] / (double)n;
    ch.sigma2 = D.sigma[c] * D.sigma[c];
    ch.fknee = D.fknee[c];
    ch.alpha = D.alpha[c];
    ch.tau = pl->tau[c];
    ch.inv_tau = 1.0 / pl->tau[c];
    ch.nbar0 = ch.sigma2 - ch.tau;
    ch.spec_off = spec_total;
    ch.inv_M = 1.0 / (double)ch.M;
    ch.lg0 = std::log2(ch.df / ch.fknee);
    ch.xoff = xwork;
    xwork += (ch.M + kWorkAlign - 1) / kWorkAlign * kWorkAlign;
    spec_total += ch.M + 1;
    pl->chunk_item_begin.push_back((int32_t)pl->itemsB.size());
    pl->chunk_itemG_begin.push_back((int32_t)pl->itemsG.size());
    append_col_items((int32_t)c, ch, pl->itemsAC);
    append_row_items((int32_t)c, ch, pl->itemsB, row_fuse(ch.M1, f64));
    append_row_items((int32_t)c, ch, pl->itemsG, false);
  }
  pl->chunk_item_begin.push_back((int32_t)pl->itemsB.size());
  pl->chunk_itemG_begin.push_back((int32_t)pl->itemsG.size());
  bool all_pow2 = true;
  for (const DevClass& k : classes)
    for (int i = 0; i < k.nr1 + k.nr2; ++i) {
      const int r = i < k.nr1 ? k.rad1[i] : k.rad2[i - k.nr1];
      if (r != 2 && r != 4 && r != 8) all_pow2 = false;
    }
  // the inverse column pass takes the wave-local layout for every eligible class, except in
  // FP64 power-of-two plans (their inlined workgroup-wide stages measured faster)
  const bool wave_ok = !(f64 && all_pow2);
  size_t lds_c = 0;
  int nwave = 0;
  for (size_t i = 0; i < classes.size(); ++i) {
    const bool wl = wave_ok && wave_cols(classes[i].M2, class_cb[i], (int)csz);
    nwave += wl ? 1 : 0;
    lds_ac = std::max(lds_ac, (size_t)col_tile_elems(classes[i].M2, class_cb[i], (int)csz, false) * csz);
    lds_c = std::max(lds_c, (size_t)col_tile_elems(classes[i].M2, class_cb[i], (int)csz, wl) * csz);
  }
  pl->nwork = 2 * xwork;
  pl->lds_ac = lds_ac;
  pl->lds_c = lds_c;
  pl->lds_b = lds_b;
  pl->lds_g = lds_g;
  if (lds_c > (size_t)kMaxColTileBytes || lds_b + (kBlockB / 64) * sizeof(double) > 65536)
    return fail(MM_E_LEN, "transform tiles exceed the LDS budget");
  {
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return fail(MM_E_HIP, "device LDS query failed");
    if (lds_c > (size_t)lds_max)
      return fail(MM_E_LEN, "column tiles of " + std::to_string(lds_c) + " bytes exceed the device's " +
                                std::to_string(lds_max) + " bytes of LDS per workgroup");
  }
  std::vector<float2> tw32(tw.size());
  for (size_t i = 0; i < tw.size(); ++i) tw32[i] = make_float2((float)tw[i].x, (float)tw[i].y);
  std::vector<double2> sc(1024);
  for (int k = 0; k < 1024; ++k) {
    const double a = M_PI * (double)k / 512.0;
    sc[k] = make_double2(std::cos(a), std::sin(a));
  }
  std::vector<double2> cs64;
  std::vector<float2> cs32;
  if (pl->psi_kind == MM_PSI_U16) {
    cs64.resize(D.psi_table_len);
    cs32.resize(D.psi_table_len);
    for (int64_t i = 0; i < D.psi_table_len; ++i) {
      const double a = 2.0 * (double)D.psi_table[i];
      cs64[i] = make_double2(std::cos(a), std::sin(a));
      cs32[i] = make_float2((float)cs64[i].x, (float)cs64[i].y);
    }
  }
  // the tuner's last use of the temporaries is ordered before these copies and the clears below
  if ((st = upload(chunks, B.chunks, (size_t)D.nchunk, s)) != MM_OK) return st;
  if ((st = upload(classes, B.classes, P.classes.size(), s)) != MM_OK) return st;
  if ((st = upload(tw, B.tw64, P.capTW, s)) != MM_OK) return st;
  if ((st = upload(tw32, B.tw32, P.capTW, s)) != MM_OK) return st;
  if ((st = upload(sc, B.sc, 1024, s)) != MM_OK) return st;
  if (pl->psi_kind == MM_PSI_U16) {
    if ((st = upload(cs64, B.cs64, cs64.size(), s)) != MM_OK) return st;
    if ((st = upload(cs32, B.cs32, cs32.size(), s)) != MM_OK) return st;
  }
  if ((st = upload(pl->itemsAC, B.itemsAC, P.capAC, s)) != MM_OK) return st;
  if ((st = upload(pl->itemsB, B.itemsB, P.capB, s)) != MM_OK) return st;
  if ((st = upload(pl->chunk_item_begin, B.cib, (size_t)D.nchunk + 1, s)) != MM_OK) return st;
  if ((st = upload(pl->itemsG, B.itemsG, P.capG, s)) != MM_OK) return st;
  if ((st = upload(pl->chunk_itemG_begin, B.cigb, (size_t)D.nchunk + 1, s)) != MM_OK) return st;
  pl->chunks_host = chunks;
  pl->d_chunks = B.chunks;
  pl->d_itemsAC = B.itemsAC;
  pl->d_itemsB = B.itemsB;
  pl->d_chunk_item_begin = B.cib;
  pl->d_itemsG = B.itemsG;
  pl->d_chunk_itemG_begin = B.cigb;

  DevPlan& Pd = pl->dp;
  std::memset(&Pd, 0, sizeof(Pd));
  Pd.ncomp = D.ncomp;
  Pd.all_pow2 = all_pow2 ? 1 : 0;
  Pd.max_tile_pix = (int32_t)(P.tw * P.th);
  // every class a 1024-point FP32 column per wave: the register-transform variant
  bool reg_cols = !f64 && !classes.empty() && nwave == (int)classes.size();
  for (size_t i = 0; i < classes.size(); ++i) reg_cols = reg_cols && classes[i].M2 == 1024 && class_cb[i] == kColWaves;
  Pd.col_wave = reg_cols ? 3 : (nwave == 0 ? 0 : (nwave == (int)classes.size() ? 1 : 2));
  Pd.psi_kind = pl->psi_kind;
  Pd.precision = D.precision;
  Pd.npix = D.npix;
  Pd.nxm = P.nxm;
  Pd.nsamp = ns;
  Pd.nchunk = (int32_t)D.nchunk;
  Pd.ntiles = (int32_t)P.ntiles;
  Pd.pix = D.pix;
  Pd.psi = D.psi;
  Pd.chunks = B.chunks;
  Pd.classes = B.classes;
  Pd.tw64 = B.tw64;
  Pd.tw32 = B.tw32;
  Pd.sc_tab = B.sc;
  Pd.psi_cs64 = B.cs64;
  Pd.psi_cs32 = B.cs32;
  Pd.tiles = B.tiles;
  Pd.sbs = B.sbs;
  Pd.segs = B.segs;
  Pd.perm = B.perm;
  Pd.lp = B.lp;
  Pd.psi_sorted = B.psis;
  Pd.packed = B.packed;
  Pd.pk_lp_bits = P.lp_bits;
  Pd.lp_stage = B.lpq;
  Pd.psi_stage = B.psiq;
  Pd.spec = B.spec;
  Pd.winv = B.winv;
  Pd.solvable = B.sol;
  Pd.mapi = B.mapi;
  Pd.composite = P.composite ? 1 : 0;
  Pd.wa = P.composite ? D.weight_a : 1.0;
  Pd.wb = P.composite ? D.weight_b : 0.0;
  Pd.pmb_off = P.composite ? ns / 2 : 0;
  pl->composite = P.composite;
  pl->d_winv = B.winv;
  pl->d_solvable = B.sol;
  pl->d_hits = B.hits;
  pl->d_work = B.work;
  pl->d_work2 = B.work2;
  pl->d_gd0 = B.gd0;
  pl->d_gt0 = B.gt0;
  pl->d_chi2_part = B.chi2part;
  pl->d_scal = B.scal;
  pl->d_part = B.part;
  for (int i = 0; i < kScratchMaps; ++i) pl->d_map[i] = B.maps[i];
  pl->d_hist = B.hist;
  pl->pm_mode = P.pm_mode ? 1 : 0;
  pl->d_pm = B.pm;
  pl->bin_atomic = P.bin_atomic;
  pl->d_batom = B.batom;
  for (int64_t c = 0; c < D.nchunk; ++c) pl->max_n = std::max<int64_t>(pl->max_n, D.chunk_off[c + 1] - D.chunk_off[c]);
  if (pl->pm_mode) {  // off-map entries: P m = 0 (the buffer held plan-time temporaries)
    if (launch_fill_i64((int64_t*)pl->d_pm, (int64_t)((size_t)P.nent * P.tsz / sizeof(int64_t)), 0, s) != hipSuccess)
      return fail(MM_E_HIP, "clearing the projection buffer failed");
  }
  if ((st = plan_precompute(pl, s)) != MM_OK) return st;
  if (pl->nsolvable == 0) return fail(MM_E_SINGULAR, "no pixel has a solvable weight block");
  if (hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(MM_E_HIP, "stream creation failed");
  *out = guard.release();
  return MM_OK;
}

void destroy_plan(mm_plan_s* pl) {
  if (!pl) return;
  // the workspace goes back to the caller: no kernel of this plan may still use it
  (void)hipDeviceSynchronize();
  if (pl->solve_exec) (void)hipGraphExecDestroy(pl->solve_exec);
  if (pl->solve_done) (void)hipEventDestroy(pl->solve_done);
  for (auto& r : pl->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : pl->ev_pool) (void)hipEventDestroy(e);
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  delete pl;
}

}  // namespace mm
