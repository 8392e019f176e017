// Internal plan object of libmm.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "mm.h"

namespace mm {

constexpr int kScratchMaps = 6;
constexpr int64_t kCgHistCap = 16384;  // CG history entries a plan holds for callers that give none

// Bump allocation of 256-byte-aligned pieces from a byte range; with a null base it only
// measures (cap unlimited), which is how the workspace size is computed.
struct Arena {
  char* base = nullptr;
  size_t cap = ~size_t(0);
  size_t used = 0;
  void* take(size_t bytes) {
    const size_t a = (used + 255) / 256 * 256;
    if (a > cap || bytes > cap - a) return nullptr;
    used = a + bytes;
    return base ? (void*)(base + a) : (void*)(uintptr_t)(a + 256);  // non-null when measuring
  }
};

extern thread_local std::string g_last_error;
mm_status fail(mm_status s, const std::string& msg);

}  // namespace mm

struct mm_plan_s {
  int32_t ncomp = 0, precision = 0, psi_kind = 0;
  int64_t npix = 0, nx = 0, nchunk = 0, ns = 0;
  std::vector<int64_t> off;
  std::vector<double> fsample, sigma, fknee, alpha, tau;
  // work lists
  std::vector<mm::ItemAC> itemsAC;
  std::vector<mm::ItemB> itemsB;           // row pass (two row pairs per item where they fit)
  std::vector<int32_t> chunk_item_begin;   // first row-pass item of each chunk, and the end
  std::vector<mm::ItemB> itemsG;           // gradient row pass (one row pair per item)
  std::vector<int32_t> chunk_itemG_begin;
  std::vector<mm::DevChunk> chunks_host;  // kept for noise-parameter updates
  size_t lds_ac = 0, lds_c = 0, lds_b = 0, lds_g = 0;  // dynamic LDS: column passes A, C; row passes
  std::vector<int32_t> class_layout;      // per transform class: chosen candidate index
  std::vector<int32_t> class_ncand;       // per transform class: number of candidates
  int64_t ntiles = 0, nsegs = 0, nsbs = 0, nsorted = 0;
  int32_t tile_w = 0, tile_h = 0;
  // device: every buffer lies in the caller's workspace
  mm::DevPlan dp;
  void* ws = nullptr;
  size_t ws_bytes = 0, ws_used = 0;
  mm::ItemAC* d_itemsAC = nullptr;
  mm::ItemB* d_itemsB = nullptr;
  int32_t* d_chunk_item_begin = nullptr;
  mm::ItemB* d_itemsG = nullptr;
  int32_t* d_chunk_itemG_begin = nullptr;
  double* d_winv = nullptr;
  uint8_t* d_solvable = nullptr;
  int32_t* d_hits = nullptr;
  void* d_work = nullptr;     // transform work buffer: 2 * xoff_c + (sample - off_c) holds chunk c
  int64_t nwork = 0;          // its length in reals (>= ns: chunk bases padded to 128-byte lines)
  double* d_chi2_part = nullptr;
  double* d_scal = nullptr;
  double* d_part = nullptr;
  double* d_map[mm::kScratchMaps] = {};
  void* d_work2 = nullptr;    // second TOD-sized buffer (gradients, map right-hand sides); null
                              // unless the plan was built with_adjoint
  // P m in time order, written in pixel-tile order (large maps: the column pass reads it instead
  // of gathering the map)
  int pm_mode = 0;
  bool composite = false;  // P = P_A + P_B (second pointing component given)
  void* d_gd0 = nullptr;   // gap filling: the fields d_0 and t_0 (TOD-sized, time order)
  void* d_gt0 = nullptr;
  void* d_pm = nullptr;
  // binning by FP64 atomics (measured alternative): binned vector, longest chunk
  bool bin_atomic = false;
  double* d_batom = nullptr;
  int64_t max_n = 0;
  mm::DevChunk* d_chunks = nullptr;
  double* d_hist = nullptr;  // CG r^T z history when the caller gives none (kCgHistCap entries)
  int64_t nsolvable = 0;
  hipStream_t cap_stream = nullptr;
  std::vector<double> solve_key;        // arguments of the last captured solve (replayed when equal)
  hipGraphExec_t solve_exec = nullptr;  // the one cached solve graph
  hipEvent_t solve_done = nullptr;      // recorded after each launch of solve_exec
  // per-pass timing (measurement only)
  bool timing = false;
  bool capturing = false;
  std::vector<hipEvent_t> ev_pool;
  struct Rec {
    int pass;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
};

namespace mm {

// One way to run the length-2M real transform of a chunk: split M = M1 * M2, cb columns per
// column item, radix schedules of the row (M1) and column (M2) transforms.
struct Layout {
  int64_t M1 = 0, M2 = 0;
  int cb = 0;
  std::vector<int8_t> r1, r2;
};

constexpr int64_t kTuneMinM = int64_t(1) << 14;     // shorter chunks take the static rule
constexpr int64_t kTuneElements = int64_t(1) << 23;  // complex values per timed launch
constexpr size_t kTuneMaxCandidates = 6;
constexpr int kTuneReps = 5;  // timed runs per candidate (best kept)

int tile_cap_ac(bool f64);  // complex values per column item (pass A, C tile)
int tile_cap_b(bool f64);   // complex values per row item (pass B tile)
// layouts that fit the passes' tiles, best first by the static rule
std::vector<Layout> layout_candidates(int64_t M, bool f64);
// radix schedules and twiddle offsets of layout L (twiddles appended to tw)
void make_class(int64_t M, const Layout& L, std::vector<double2>& tw, DevClass& k);
// column items and row-pair items of chunk c
// whether the row pass holds two row pairs (four rows of length M1) per item
bool row_fuse(int M1, bool f64);
void append_col_items(int32_t c, const DevChunk& ch, std::vector<ItemAC>& itemsAC);
void append_row_items(int32_t c, const DevChunk& ch, std::vector<ItemB>& itemsB, bool fuse);
// whether a length with ncand candidates is timed, and the device scratch the timing takes.
// a_streams: the TOD-sized streams the plan's column pass A reads (1: d, its gathers aside;
// 2: d and P m; 3: d and the two halves of a composite plan's P m), which the timing reads too
bool tune_wanted(int64_t M, size_t ncand);
size_t tune_scratch_bytes(int64_t M, bool f64, const std::vector<Layout>& cands, int a_streams);
// index of the fastest candidate, timed on the GPU in the given scratch (0 for short chunks or
// on any failure); cached per process by (M, precision, a_streams)
int tune_layout(int64_t M, bool f64, const std::vector<Layout>& cands, int a_streams, hipStream_t s, void* scratch,
                size_t scratch_bytes);

// device bytes a plan of this description needs; `scratch` (device, scratch_bytes) serves the
// analysis passes, or null to have them allocate their own
mm_status workspace_query(const mm_plan_desc* desc, hipStream_t s, void* scratch, size_t scratch_bytes,
                          size_t* bytes);
mm_status build_plan(const mm_plan_desc* desc, void* ws, size_t ws_bytes, hipStream_t s, mm_plan_s** out);
void destroy_plan(mm_plan_s* pl);
mm_status plan_set_noise(mm_plan_s* pl, const double* sigma, const double* fknee, const double* alpha,
                         const double* tau, hipStream_t s);
}  // namespace mm
