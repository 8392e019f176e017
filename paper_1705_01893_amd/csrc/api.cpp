// C entry points of libmm (declared in include/mm.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mm.h"
#include "plan.h"

using namespace mm;

namespace {

#define MM_TRY_HIP(expr)                                                                           \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return fail(MM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define MM_TRY(expr)               \
  do {                             \
    mm_status s_ = (expr);         \
    if (s_ != MM_OK) return s_;    \
  } while (0)

inline hipStream_t S(mm_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

int64_t mapn(const mm_plan_s* pl) { return (int64_t)pl->ncomp * pl->npix; }

hipEvent_t take_event(mm_plan_s* pl) {
  if (!pl->ev_pool.empty()) {
    hipEvent_t e = pl->ev_pool.back();
    pl->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// run one launch, bracketed by events when timing is on (never inside a graph capture)
template <typename F>
hipError_t timed(mm_plan_s* pl, int pass, hipStream_t s, F&& launch) {
  if (!pl->timing || pl->capturing) return launch();
  hipEvent_t a = take_event(pl), b = take_event(pl);
  if (!a || !b) {
    if (a) pl->ev_pool.push_back(a);
    if (b) pl->ev_pool.push_back(b);
    return hipErrorOutOfMemory;
  }
  hipError_t e = hipEventRecord(a, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, s);
  pl->recs.push_back({pass, a, b});
  return e;
}

// binning by atomics: zero the binned vector (a fill kernel, also under graph capture), add every
// sample, then the per-pixel update
hipError_t bin_atomic_update(mm_plan_s* pl, int bsrc, const void* src, int epi, const double* m_in, double* m_out,
                             hipStream_t s) {
  hipError_t e = launch_fill(pl->d_batom, mapn(pl), 0.0, s);
  if (e == hipSuccess) e = launch_bin_atomic(pl->dp, bsrc, src, pl->d_batom, pl->max_n, s);
  if (e == hipSuccess) e = launch_update(pl->dp, epi, m_in, pl->d_batom, m_out, s);
  return e;
}

// r = src(d, m) -> filtered y in the work buffer (passes A, B, C).  Returns with the
// chi^2 partials in d_chi2_part when ops includes B_CHI2.
// pass A of a sweep: r = src(d, m) column-transformed into the work buffer
mm_status sweep_pass_a(mm_plan_s* pl, const void* d, const double* m, int src, hipStream_t s, bool map_current) {
  // large maps: P m comes from the projection buffer (projected here unless it already holds P m);
  // otherwise I/Q/U maps are gathered from their interleaved copy (made here unless current)
  // atomic binning writes no P m for the next sweep
  if (pl->bin_atomic && pl->pm_mode) map_current = false;
  if (pl->pm_mode && (src == SRC_D_MINUS_PM || src == SRC_PM)) {
    if (!map_current) MM_TRY_HIP(timed(pl, 4, s, [&] { return launch_project(pl->dp, m, pl->d_pm, s); }));
    src = (src == SRC_PM) ? SRC_PMBUF : SRC_D_MINUS_PMBUF;
  } else if (pl->dp.mapi && (src == SRC_D_MINUS_PM || src == SRC_PM) && !map_current) {
    MM_TRY_HIP(launch_interleave(pl->dp, m, s));
  }
  MM_TRY_HIP(timed(pl, 0, s, [&] {
    return launch_pass_a(pl->dp, pl->d_itemsAC, (int)pl->itemsAC.size(), d, m, src, pl->d_work, pl->lds_ac, s,
                         pl->d_pm);
  }));
  return MM_OK;
}

mm_status sweep_filter(mm_plan_s* pl, const void* d, const double* m, int src, int ops, int gain, double lam,
                       double chi2_lam, hipStream_t s, bool map_current = false) {
  MM_TRY(sweep_pass_a(pl, d, m, src, s, map_current));
  MM_TRY_HIP(timed(pl, 1, s, [&] {
    return launch_pass_b(pl->dp, pl->d_itemsB, (int)pl->itemsB.size(), pl->d_work, ops, gain, lam, chi2_lam,
                         pl->d_chi2_part, pl->lds_b, s);
  }));
  if (ops & B_FILTER)
    MM_TRY_HIP(timed(pl, 2, s, [&] {
      return launch_pass_c(pl->dp, pl->d_itemsAC, (int)pl->itemsAC.size(), pl->d_work, pl->lds_c, s);
    }));
  return MM_OK;
}

// chi^2(m, lam) of d - P m into *total (device) and optionally per chunk (device)
mm_status chi2_device(mm_plan_s* pl, const void* d, const double* m, double lam, double* total, double* per_chunk,
                      hipStream_t s, bool map_current = false) {
  MM_TRY(sweep_filter(pl, d, m, SRC_D_MINUS_PM, B_CHI2, GAIN_NINV, 1.0, lam, s, map_current));
  MM_TRY_HIP(launch_chi2_reduce(pl->d_chunk_item_begin, pl->d_chi2_part, (int)pl->nchunk, per_chunk, total, s));
  return MM_OK;
}

// one messenger iteration m_out = m_in + W^-1 P^T G_lambda (d - P m_in); chi2(m_in) into chi2_dev if non-null
// chained: the map-derived copy the sweeps read (P m, or the interleaved map) already belongs to
// m_in: the previous iteration's binning epilogue wrote it
mm_status iterate(mm_plan_s* pl, const void* d, double lam, const double* m_in, double* m_out, double* chi2_dev,
                  hipStream_t s, bool chained = false) {
  // single beam: at lambda = inf the step is the binned map W^-1 P^T T^-1 d whatever m_in is (the
  // filter is T^-1); composite pointing keeps the general step there (F(inf) != 0), with gain 1/tau
  if (std::isinf(lam) && !pl->composite) {
    if (chi2_dev) MM_TRY(chi2_device(pl, d, m_in, 1.0, chi2_dev, nullptr, s, chained));
    MM_TRY_HIP(timed(pl, 3, s, [&] {
      if (pl->bin_atomic) return bin_atomic_update(pl, BSRC_DATA_OVER_TAU, d, EPI_REPLACE, m_in, m_out, s);
      return launch_bin(pl->dp, BSRC_DATA_OVER_TAU, d, EPI_REPLACE, m_in, m_out, nullptr, nullptr, s, pl->d_pm);
    }));
    return MM_OK;
  }
  const int ops = B_FILTER | (chi2_dev ? B_CHI2 : 0);
  MM_TRY(sweep_filter(pl, d, m_in, SRC_D_MINUS_PM, ops, GAIN_MESSENGER, lam, 1.0, s, chained));
  MM_TRY_HIP(timed(pl, 3, s, [&] {
    if (pl->bin_atomic) return bin_atomic_update(pl, BSRC_WORK, pl->d_work, EPI_UPDATE, m_in, m_out, s);
    return launch_bin(pl->dp, BSRC_WORK, pl->d_work, EPI_UPDATE, m_in, m_out, nullptr, nullptr, s, pl->d_pm);
  }));
  if (chi2_dev)
    MM_TRY_HIP(launch_chi2_reduce(pl->d_chunk_item_begin, pl->d_chi2_part, (int)pl->nchunk, nullptr, chi2_dev, s));
  return MM_OK;
}

// out = P^T G P x (x != null) or P^T G d
mm_status apply_op(mm_plan_s* pl, int gain, double lam, const double* x, const void* d, double* out, hipStream_t s) {
  MM_TRY(sweep_filter(pl, x ? nullptr : d, x, x ? SRC_PM : SRC_D, B_FILTER, gain, lam, 1.0, s));
  MM_TRY_HIP(timed(pl, 3, s, [&] {
    if (pl->bin_atomic) {
      hipError_t e = launch_fill(out, mapn(pl), 0.0, s);
      return e != hipSuccess ? e : launch_bin_atomic(pl->dp, BSRC_WORK, pl->d_work, out, pl->max_n, s);
    }
    return launch_bin(pl->dp, BSRC_WORK, pl->d_work, EPI_WRITE_B, nullptr, out, nullptr, nullptr, s);
  }));
  return MM_OK;
}

mm_status dot(mm_plan_s* pl, const double* a, const double* b, double* out, hipStream_t s) {
  const int64_t n = mapn(pl);
  const int nb = dot_blocks(n);
  MM_TRY_HIP(launch_dot_partials(a, b, n, pl->d_part, nb, s));
  MM_TRY_HIP(launch_reduce(pl->d_part, nb, out, s));
  return MM_OK;
}

// out = N T^-1 P W^-1 g in time order (the lifted right-hand side of an adjoint solve); needs
// W = P^T T^-1 P, which composite pointing (W_AB) does not have
mm_status lift(mm_plan_s* pl, const double* g, void* out, hipStream_t s) {
  if (pl->composite) return fail(MM_E_ARG, "the lifted right-hand side needs single-beam pointing");
  double* u = pl->d_map[5];
  MM_TRY_HIP(launch_winv_apply(pl->dp, g, u, s));
  MM_TRY(sweep_filter(pl, nullptr, u, SRC_PM, B_FILTER, GAIN_LIFT, 1.0, 1.0, s));
  MM_TRY_HIP(launch_unshift(pl->dp, pl->d_work, out, s));
  return MM_OK;
}

bool valid_lambda(double lam) { return std::isinf(lam) ? lam > 0 : (lam >= 1.0 && std::isfinite(lam)); }

// the schedule as one lambda per iteration (lambda = inf first when asked)
mm_status expand_schedule(const mm_schedule* sched, std::vector<double>& lams) {
  if (sched->nlevel < 0 || (sched->nlevel > 0 && (!sched->lambda || !sched->iters)))
    return fail(MM_E_ARG, "invalid schedule");
  if (sched->first_inf) lams.push_back(INFINITY);
  for (int l = 0; l < sched->nlevel; ++l) {
    if (sched->iters[l] < 0 || !valid_lambda(sched->lambda[l])) return fail(MM_E_ARG, "invalid schedule level");
    for (int i = 0; i < sched->iters[l]; ++i) lams.push_back(sched->lambda[l]);
  }
  return MM_OK;
}

// Run a solve body on `stream`: captured into the plan's one cached HIP graph (replayed when the
// key, i.e. the buffers and the schedule, equals the previous call's), or directly when per-pass
// timing is on (events between the passes cannot be recorded inside a capture).
template <typename F>
mm_status run_graph(mm_plan_s* plan, const std::vector<double>& key, mm_stream_t stream, F&& body) {
  // per-pass timing records events between the passes: run on the caller's stream, uncaptured
  if (plan->timing) return body(S(stream));
  if (plan->solve_exec && key == plan->solve_key) {
    MM_TRY_HIP(hipGraphLaunch(plan->solve_exec, S(stream)));
    MM_TRY_HIP(hipEventRecord(plan->solve_done, S(stream)));
    return MM_OK;
  }
  hipStream_t cs = plan->cap_stream;
  MM_TRY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  plan->capturing = true;
  mm_status st = body(cs);
  plan->capturing = false;
  hipGraph_t graph = nullptr;
  hipError_t ee = hipStreamEndCapture(cs, &graph);
  if (st != MM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ee != hipSuccess) return fail(MM_E_HIP, std::string("graph capture: ") + hipGetErrorString(ee));
  hipGraphExec_t exec = nullptr;
  ee = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ee != hipSuccess) return fail(MM_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ee));
  // one cached solve graph: the previous one is destroyed once its last launch has completed
  if (plan->solve_exec) {
    (void)hipEventSynchronize(plan->solve_done);
    (void)hipGraphExecDestroy(plan->solve_exec);
    plan->solve_exec = nullptr;
    plan->solve_key.clear();
  }
  if (!plan->solve_done && (ee = hipEventCreateWithFlags(&plan->solve_done, hipEventDisableTiming)) != hipSuccess) {
    plan->solve_done = nullptr;
    (void)hipGraphExecDestroy(exec);
    return fail(MM_E_HIP, std::string("event create: ") + hipGetErrorString(ee));
  }
  plan->solve_exec = exec;  // owned by the plan from here on; replayed only once the key is set
  ee = hipGraphLaunch(exec, S(stream));
  if (ee == hipSuccess) ee = hipEventRecord(plan->solve_done, S(stream));
  if (ee != hipSuccess) return fail(MM_E_HIP, std::string("graph launch: ") + hipGetErrorString(ee));
  plan->solve_key = key;
  return MM_OK;
}


}  // namespace

extern "C" {

const char* mm_status_str(mm_status s) {
  switch (s) {
    case MM_OK: return "ok";
    case MM_E_ARG: return "invalid argument";
    case MM_E_LEN: return "unsupported chunk length";
    case MM_E_NOMEM: return "out of memory";
    case MM_E_HIP: return "HIP runtime error";
    case MM_E_SINGULAR: return "no solvable pixel";
    case MM_E_NONFINITE: return "non-finite chi^2";
  }
  return "unknown status";
}

const char* mm_last_error(void) { return g_last_error.c_str(); }

mm_status mm_set_timing(mm_plan_t plan, int32_t enable) {
  if (!plan) return fail(MM_E_ARG, "null plan");
  plan->timing = enable != 0;
  return MM_OK;
}

mm_status mm_get_timing(mm_plan_t plan, double* ms, int64_t* launches) {
  if (!plan || !ms || !launches) return fail(MM_E_ARG, "null argument");
  for (int i = 0; i < 5; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  mm_status st = MM_OK;
  for (auto& r : plan->recs) {
    float t = 0.f;
    if (st == MM_OK) {
      hipError_t e = hipEventSynchronize(r.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
      if (e != hipSuccess) st = fail(MM_E_HIP, std::string("timing events: ") + hipGetErrorString(e));
    }
    if (r.pass >= 0 && r.pass < 5) {
      ms[r.pass] += t;
      launches[r.pass] += 1;
    }
    plan->ev_pool.push_back(r.a);
    plan->ev_pool.push_back(r.b);
  }
  plan->recs.clear();
  return st;
}

mm_status mm_plan_workspace_bytes(const mm_plan_desc* desc, mm_stream_t stream, size_t* bytes) {
  g_last_error.clear();
  return workspace_query(desc, S(stream), nullptr, 0, bytes);
}

mm_status mm_plan_workspace_bytes_noalloc(const mm_plan_desc* desc, mm_stream_t stream, size_t* bytes) {
  g_last_error.clear();
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  void* scratch = e == hipSuccess ? static_scratch(dev, &e) : nullptr;
  if (!scratch) return fail(MM_E_HIP, std::string("fixed scratch lookup: ") + hipGetErrorString(e));
  return workspace_query(desc, S(stream), scratch, kStaticScratchBytes, bytes);
}

mm_status mm_plan(const mm_plan_desc* desc, void* workspace, size_t workspace_bytes, mm_stream_t stream,
                  mm_plan_t* out) {
  g_last_error.clear();
  return build_plan(desc, workspace, workspace_bytes, S(stream), out);
}

mm_status mm_plan_destroy(mm_plan_t plan) {
  if (!plan) return fail(MM_E_ARG, "null plan");
  destroy_plan(plan);
  return MM_OK;
}

mm_status mm_plan_binning_stats(mm_plan_t plan, int64_t* out) {
  if (!plan || !out) return fail(MM_E_ARG, "null argument");
  out[0] = plan->ntiles;
  out[1] = plan->tile_w;
  out[2] = plan->tile_h;
  out[3] = plan->nsbs;
  out[4] = plan->nsegs;
  out[5] = plan->nsorted;
  out[6] = (int64_t)plan->ws_used;
  return MM_OK;
}

mm_status mm_plan_map_access(mm_plan_t plan, int32_t* access) {
  if (!plan || !access) return fail(MM_E_ARG, "null argument");
  *access = plan->pm_mode ? MM_MAP_PROJECTED : MM_MAP_GATHER;
  return MM_OK;
}

mm_status mm_plan_chunk_layout(mm_plan_t plan, int64_t chunk, int64_t* M1, int64_t* M2, int32_t* cb,
                               int32_t* pick, int32_t* ncand) {
  if (!plan || !M1 || !M2 || !cb || !pick || !ncand) return fail(MM_E_ARG, "null argument");
  if (chunk < 0 || chunk >= plan->nchunk) return fail(MM_E_ARG, "chunk index out of range");
  const DevChunk& ch = plan->chunks_host[chunk];
  *M1 = ch.M1;
  *M2 = ch.M2;
  *cb = ch.cb;
  *pick = plan->class_layout[ch.cls];
  *ncand = plan->class_ncand[ch.cls];
  return MM_OK;
}

mm_status mm_plan_hits(mm_plan_t plan, int32_t* hits_dev, mm_stream_t stream) {
  if (!plan || !hits_dev) return fail(MM_E_ARG, "null argument");
  MM_TRY_HIP(launch_copy_bytes(hits_dev, plan->d_hits, plan->npix * (int64_t)sizeof(int32_t), S(stream)));
  return MM_OK;
}

mm_status mm_plan_solvable(mm_plan_t plan, uint8_t* mask_dev, mm_stream_t stream) {
  if (!plan || !mask_dev) return fail(MM_E_ARG, "null argument");
  MM_TRY_HIP(launch_copy_bytes(mask_dev, plan->d_solvable, plan->npix, S(stream)));
  return MM_OK;
}

mm_status mm_plan_nsolvable(mm_plan_t plan, int64_t* count) {
  if (!plan || !count) return fail(MM_E_ARG, "null argument");
  *count = plan->nsolvable;
  return MM_OK;
}

mm_status mm_messenger_iter(mm_plan_t plan, const void* d, double lambda, const double* m_in, double* m_out,
                            double* chi2_dev, mm_stream_t stream) {
  if (!plan || !d || !m_in || !m_out) return fail(MM_E_ARG, "null argument");
  if (!valid_lambda(lambda)) return fail(MM_E_ARG, "lambda must be >= 1 or +inf");
  return iterate(plan, d, lambda, m_in, m_out, chi2_dev, S(stream));
}

mm_status mm_cooling_levels(mm_plan_t plan, int32_t nlevel, double lambda_max, double* out) {
  if (!plan || !out || nlevel <= 0) return fail(MM_E_ARG, "invalid argument");
  double lmax = lambda_max;
  if (!(lmax > 0)) {
    // lambda tau reaches the largest noise power: the clamped DC bin, N(f_1) (the spectrum
    // falls with frequency for negative slopes; the largest of both ends covers the rest)
    lmax = 1.0;
    for (int64_t c = 0; c < plan->nchunk; ++c) {
      const double n = (double)(plan->off[c + 1] - plan->off[c]);
      const double s2 = plan->sigma[c] * plan->sigma[c];
      const double f1 = plan->fsample[c] / n, fn = 0.5 * plan->fsample[c];
      const double N1 = s2 * (1.0 + std::pow(f1 / plan->fknee[c], plan->alpha[c]));
      const double Nn = s2 * (1.0 + std::pow(fn / plan->fknee[c], plan->alpha[c]));
      lmax = std::max(lmax, std::max(N1, Nn) / plan->tau[c]);
    }
  }
  if (lmax < 1.0) return fail(MM_E_ARG, "lambda_max must be >= 1");
  for (int l = 0; l < nlevel; ++l)
    out[l] = (nlevel == 1) ? 1.0 : std::pow(lmax, (double)(nlevel - 1 - l) / (double)(nlevel - 1));
  out[nlevel - 1] = 1.0;
  return MM_OK;
}

mm_status mm_solve(mm_plan_t plan, const void* d, const double* rhs_map, const mm_schedule* sched, const double* m0,
                   double* m_out, double* chi2_hist_dev, mm_stream_t stream) {
  if (!plan || !sched || !m_out) return fail(MM_E_ARG, "null argument");
  if ((d == nullptr) == (rhs_map == nullptr)) return fail(MM_E_ARG, "give exactly one of d and rhs_map");
  if (rhs_map && !plan->d_work2) return fail(MM_E_ARG, "a map right-hand side needs a plan built with_adjoint");
  if (rhs_map && plan->composite) return fail(MM_E_ARG, "a map right-hand side needs single-beam pointing");
  std::vector<double> lams;
  MM_TRY(expand_schedule(sched, lams));
  const int64_t n = mapn(plan);
  // with a map right-hand side g the data are the lifted TOD N T^-1 P W^-1 g (second TOD buffer)
  const void* dd = rhs_map ? plan->d_work2 : d;
  auto body = [&](hipStream_t cs) -> mm_status {
    if (rhs_map) MM_TRY(lift(plan, rhs_map, plan->d_work2, cs));
    // start map into m_out (fill kernel, no memset nodes in the graph)
    if (m0) {
      if (m0 != m_out) MM_TRY_HIP(launch_copy(m_out, m0, n, cs));
    } else {
      MM_TRY_HIP(launch_fill(m_out, n, 0.0, cs));
    }
    // iterate in place: every pass reads the map before the binning epilogue rewrites it
    const size_t nit = lams.size();
    for (size_t i = 0; i < nit; ++i)
      MM_TRY(iterate(plan, dd, lams[i], m_out, m_out, chi2_hist_dev ? chi2_hist_dev + i : nullptr, cs, i > 0));
    if (chi2_hist_dev) MM_TRY(chi2_device(plan, dd, m_out, 1.0, chi2_hist_dev + nit, nullptr, cs, nit > 0));
    return MM_OK;
  };
  std::vector<double> key = {0.0, (double)(uintptr_t)d, (double)(uintptr_t)rhs_map, (double)(uintptr_t)m0,
                             (double)(uintptr_t)m_out, (double)(uintptr_t)chi2_hist_dev};
  key.insert(key.end(), lams.begin(), lams.end());
  return run_graph(plan, key, stream, body);
}

mm_status mm_solve_mapsized(mm_plan_t plan, const void* d, const mm_schedule* sched, const double* m0,
                            double* m_out, mm_stream_t stream) {
  if (!plan || !d || !sched || !m_out) return fail(MM_E_ARG, "null argument");
  std::vector<double> lams;
  MM_TRY(expand_schedule(sched, lams));
  const int64_t n = mapn(plan);
  double* md = plan->d_map[3];
  double* b = plan->d_map[4];
  auto body = [&](hipStream_t cs) -> mm_status {
    if (m0) {
      if (m0 != m_out) MM_TRY_HIP(launch_copy(m_out, m0, n, cs));
    } else {
      MM_TRY_HIP(launch_fill(m_out, n, 0.0, cs));
    }
    DevPlan P = plan->dp;
    P.md = md;
    const size_t nit = lams.size();
    for (size_t i = 0; i < nit; ++i) {
      const double lam = lams[i];
      if (std::isinf(lam)) {  // m_d(inf) + F(inf) m: the residual-form step at lambda = inf
        MM_TRY(iterate(plan, d, lam, m_out, m_out, nullptr, cs, i > 0));
        continue;
      }
      if (i == 0 || lams[i - 1] != lam) {
        // a new level: m_d(lambda) = W^-1 P^T (lambda^-1 N-bar + T)^-1 d, the one sweep of the level
        // that reads the data (it leaves the map-derived P m / interleaved copy untouched)
        MM_TRY(apply_op(plan, GAIN_MESSENGER, lam, nullptr, d, b, cs));
        MM_TRY_HIP(launch_winv_apply(plan->dp, b, md, cs));
      }
      // m <- m_d + F(lambda) m = m_d + m - W^-1 P^T (lambda^-1 N-bar + T)^-1 P m
      MM_TRY(sweep_filter(plan, nullptr, m_out, SRC_PM, B_FILTER, GAIN_MESSENGER, lam, 1.0, cs, i > 0));
      MM_TRY_HIP(timed(plan, 3, cs, [&] {
        if (plan->bin_atomic) {
          hipError_t e = launch_fill(plan->d_batom, n, 0.0, cs);
          if (e == hipSuccess) e = launch_bin_atomic(P, BSRC_WORK, plan->d_work, plan->d_batom, plan->max_n, cs);
          return e != hipSuccess ? e : launch_update(P, EPI_MAPSIZED, m_out, plan->d_batom, m_out, cs);
        }
        return launch_bin(P, BSRC_WORK, plan->d_work, EPI_MAPSIZED, m_out, m_out, nullptr, nullptr, cs, plan->d_pm);
      }));
    }
    return MM_OK;
  };
  std::vector<double> key = {1.0, (double)(uintptr_t)d, (double)(uintptr_t)m0, (double)(uintptr_t)m_out};
  key.insert(key.end(), lams.begin(), lams.end());
  return run_graph(plan, key, stream, body);
}

mm_status mm_solve_gapfill(mm_plan_t plan, const void* d, const uint8_t* gaps, const mm_schedule* sched,
                           const double* m0, double* m_out, void* d0_out, mm_stream_t stream) {
  if (!plan || !d || !gaps || !sched || !m_out) return fail(MM_E_ARG, "null argument");
  if (!plan->d_gd0) return fail(MM_E_ARG, "gap filling needs a plan built with_gapfill");
  for (int64_t c = 0; c < plan->nchunk; ++c)
    if (!(plan->tau[c] < plan->sigma[c] * plan->sigma[c]))
      return fail(MM_E_ARG, "gap filling needs tau_c < sigma_c^2 (eps_c = sigma_c^2 - tau_c > 0), chunk " +
                                std::to_string(c));
  std::vector<double> lams;
  MM_TRY(expand_schedule(sched, lams));
  hipStream_t s = S(stream);
  const int64_t n = mapn(plan);
  if (m0) {
    if (m0 != m_out) MM_TRY_HIP(launch_copy(m_out, m0, n, s));
  } else {
    MM_TRY_HIP(launch_fill(m_out, n, 0.0, s));
  }
  DevPlan P = plan->dp;
  P.gap_d0 = plan->d_gd0;
  P.gaps = gaps;
  MM_TRY_HIP(launch_gap_init(P, d, gaps, plan->d_gd0, plan->d_gt0, s));
  for (size_t i = 0; i < lams.size(); ++i) {
    // d_0 = t_1 + A (t_0 - t_1)
    MM_TRY_HIP(timed(plan, 0, s, [&] {
      return launch_pass_a(P, plan->d_itemsAC, (int)plan->itemsAC.size(), d, nullptr, SRC_GAP, plan->d_work,
                           plan->lds_ac, s, plan->d_gt0);
    }));
    MM_TRY_HIP(timed(plan, 1, s, [&] {
      return launch_pass_b(P, plan->d_itemsB, (int)plan->itemsB.size(), plan->d_work, B_FILTER, GAIN_GAPFILL, 1.0,
                           1.0, plan->d_chi2_part, plan->lds_b, s);
    }));
    MM_TRY_HIP(timed(plan, 2, s, [&] {
      return launch_pass_c(P, plan->d_itemsAC, (int)plan->itemsAC.size(), plan->d_work, plan->lds_c, s);
    }));
    MM_TRY_HIP(launch_gap_d0(P, d, gaps, plan->d_work, plan->d_gd0, s));
    // t_0 = P m + tau (lambda^-1 N-bar_0 + T_0)^-1 (d_0 - P m), then m = W^-1 P^T T_0^-1 t_0 (the
    // binning pass updates m by W^-1 P^T of the filtered residual and writes P m of the result)
    MM_TRY(sweep_filter(plan, plan->d_gd0, m_out, SRC_D_MINUS_PM, B_FILTER, GAIN_MESSENGER_PL, lams[i], 1.0, s,
                        i > 0));
    MM_TRY_HIP(launch_gap_t0(P, plan->d_pm, plan->d_work, plan->d_gt0, s));
    MM_TRY_HIP(timed(plan, 3, s, [&] {
      return launch_bin(plan->dp, BSRC_WORK, plan->d_work, EPI_UPDATE, m_out, m_out, nullptr, nullptr, s,
                        plan->d_pm);
    }));
  }
  if (d0_out) MM_TRY_HIP(launch_copy_bytes(d0_out, plan->d_gd0, plan->ns * (int64_t)(plan->precision ? 4 : 8), s));
  return MM_OK;
}

mm_status mm_chi2(mm_plan_t plan, const void* d, const double* m, double lambda, double* chi2_host,
                  double* per_chunk_dev, mm_stream_t stream) {
  if (!plan || !d || !m || !chi2_host) return fail(MM_E_ARG, "null argument");
  if (!(lambda >= 1.0) || !std::isfinite(lambda)) return fail(MM_E_ARG, "lambda must be finite and >= 1");
  hipStream_t s = S(stream);
  MM_TRY(chi2_device(plan, d, m, lambda, plan->d_scal, per_chunk_dev, s));
  double v = 0;
  MM_TRY_HIP(hipMemcpyAsync(&v, plan->d_scal, sizeof(double), hipMemcpyDeviceToHost, s));
  MM_TRY_HIP(hipStreamSynchronize(s));
  if (!std::isfinite(v)) return fail(MM_E_NONFINITE, "chi^2 is not finite");
  *chi2_host = v;
  return MM_OK;
}

mm_status mm_chi2_modes(mm_plan_t plan, const void* d, const double* m, double lambda, int32_t nsel,
                        const int64_t* chunks, int32_t per_octave, double* modes_dev, double* bins_dev, int32_t nbins,
                        mm_stream_t stream) {
  if (!plan || !d || !m || !chunks || !modes_dev || !bins_dev) return fail(MM_E_ARG, "null argument");
  if (nsel < 1) return fail(MM_E_ARG, "no chunk listed");
  if (per_octave < 1 || per_octave > 64) return fail(MM_E_ARG, "per_octave must be 1..64");
  if (!(lambda >= 1.0) || !std::isfinite(lambda)) return fail(MM_E_ARG, "lambda must be finite and >= 1");
  int64_t maxM = 1;
  for (int32_t i = 0; i < nsel; ++i) {
    if (chunks[i] < 0 || chunks[i] >= plan->nchunk) return fail(MM_E_ARG, "chunk index out of range");
    maxM = std::max<int64_t>(maxM, (plan->off[chunks[i] + 1] - plan->off[chunks[i]]) / 2);
  }
  int lg = 0;
  while ((int64_t(2) << lg) <= maxM) ++lg;  // floor(log2 maxM)
  const int need = 1 + per_octave * (lg + 1);
  if (nbins != need) return fail(MM_E_ARG, "nbins must be " + std::to_string(need) + " for these chunks");
  hipStream_t s = S(stream);
  MM_TRY(sweep_pass_a(plan, d, m, SRC_D_MINUS_PM, s, false));
  int64_t off = 0;
  for (int32_t i = 0; i < nsel; ++i) {
    const int64_t c = chunks[i];
    const int64_t M = (plan->off[c + 1] - plan->off[c]) / 2;
    const int b0 = plan->chunk_item_begin[c], b1 = plan->chunk_item_begin[c + 1];
    MM_TRY_HIP(launch_pass_b(plan->dp, plan->d_itemsB + b0, b1 - b0, plan->d_work, B_CHI2, GAIN_NINV, 1.0, lambda,
                             plan->d_chi2_part, plan->lds_b, s, modes_dev + off));
    MM_TRY_HIP(launch_modes_bin(modes_dev + off, M, per_octave, nbins, bins_dev + 2 * (int64_t)nbins * i, s));
    off += M + 1;
  }
  return MM_OK;
}

mm_status mm_apply(mm_plan_t plan, int32_t which, double lambda, const double* x, const void* d, double* out,
                   mm_stream_t stream) {
  if (!plan || !out || ((x == nullptr) == (d == nullptr))) return fail(MM_E_ARG, "exactly one of x and d");
  if (which != 0 && which != 1) return fail(MM_E_ARG, "which must be 0 (N^-1) or 1 (messenger filter)");
  if (which == 1 && (!(lambda >= 1.0) || !std::isfinite(lambda))) return fail(MM_E_ARG, "lambda must be >= 1");
  return apply_op(plan, which == 0 ? GAIN_NINV : GAIN_MESSENGER, lambda, x, d, out, S(stream));
}

mm_status mm_lift_rhs(mm_plan_t plan, const double* g, void* out, mm_stream_t stream) {
  if (!plan || !g || !out) return fail(MM_E_ARG, "null argument");
  return lift(plan, g, out, S(stream));
}

mm_status mm_plan_set_noise(mm_plan_t plan, const double* sigma, const double* fknee, const double* alpha,
                            const double* tau, mm_stream_t stream) {
  if (!plan) return fail(MM_E_ARG, "null plan");
  return plan_set_noise(plan, sigma, fknee, alpha, tau, S(stream));
}

mm_status mm_tod_apply(mm_plan_t plan, int32_t which, double lambda, const double* x, void* out,
                       mm_stream_t stream) {
  if (!plan || !x || !out) return fail(MM_E_ARG, "null argument");
  if (which < 0 || which > 2) return fail(MM_E_ARG, "which must be 0, 1 or 2");
  if (which == 1 && (!(lambda >= 1.0) || !std::isfinite(lambda))) return fail(MM_E_ARG, "lambda must be >= 1");
  if (which == 2 && plan->composite) return fail(MM_E_ARG, "the lifting filter needs single-beam pointing");
  const int gain = which == 0 ? GAIN_NINV : (which == 1 ? GAIN_MESSENGER : GAIN_LIFT);
  hipStream_t s = S(stream);
  MM_TRY(sweep_filter(plan, nullptr, x, SRC_PM, B_FILTER, gain, which == 1 ? lambda : 1.0, 1.0, s));
  MM_TRY_HIP(launch_unshift(plan->dp, plan->d_work, out, s));
  return MM_OK;
}

mm_status mm_noise_grad(mm_plan_t plan, const void* d, const double* m, const double* z, double* grad_dev,
                        mm_stream_t stream) {
  if (!plan || !d || !m || !z || !grad_dev) return fail(MM_E_ARG, "null argument");
  // two rows of both residuals per workgroup: 4 M1 complex values in LDS (at most 64 KB); each
  // residual's rows are transformed by a call of their own
  if (plan->lds_g > 65536) return fail(MM_E_LEN, "chunk rows too long for the two-spectrum gradient pass");
  hipStream_t s = S(stream);
  if (!plan->d_work2) return fail(MM_E_ARG, "the plan was built without with_adjoint (no second TOD buffer)");
  const bool pm = plan->pm_mode != 0;
  if (pm) MM_TRY_HIP(launch_project(plan->dp, m, plan->d_pm, s));
  MM_TRY_HIP(launch_interleave(plan->dp, m, s));  // no-op without an interleaved copy
  MM_TRY_HIP(launch_pass_a(plan->dp, plan->d_itemsAC, (int)plan->itemsAC.size(), d, m,
                           pm ? SRC_D_MINUS_PMBUF : SRC_D_MINUS_PM, plan->d_work, plan->lds_ac, s, plan->d_pm));
  if (pm) MM_TRY_HIP(launch_project(plan->dp, z, plan->d_pm, s));
  MM_TRY_HIP(launch_interleave(plan->dp, z, s));
  MM_TRY_HIP(launch_pass_a(plan->dp, plan->d_itemsAC, (int)plan->itemsAC.size(), nullptr, z,
                           pm ? SRC_PMBUF : SRC_PM, plan->d_work2, plan->lds_ac, s, plan->d_pm));
  MM_TRY_HIP(launch_grad(plan->dp, plan->d_itemsG, (int)plan->itemsG.size(), plan->d_chunk_itemG_begin,
                         plan->d_work, plan->d_work2, plan->d_chi2_part, grad_dev, plan->lds_g, s));
  return MM_OK;
}

mm_status mm_cg_solve(mm_plan_t plan, const void* d, const double* rhs_map, int32_t maxiter, double rtol,
                      const double* m0, double* m_out, double* chi2_hist_dev, double* rz_hist_dev,
                      int32_t* iters_done, mm_stream_t stream) {
  if (!plan || !m_out || maxiter < 0) return fail(MM_E_ARG, "invalid argument");
  if ((d == nullptr) == (rhs_map == nullptr)) return fail(MM_E_ARG, "give exactly one of d and rhs_map");
  if (chi2_hist_dev && !d) return fail(MM_E_ARG, "the chi^2 history needs the data");
  if (!(rtol >= 0)) return fail(MM_E_ARG, "rtol must be >= 0");
  const int64_t n = mapn(plan);
  double* x = m_out;
  double* b = plan->d_map[0];
  double* r = plan->d_map[1];
  double* z = plan->d_map[2];
  double* p = plan->d_map[3];
  double* q = plan->d_map[4];
  double* zero = plan->d_map[5];
  double* sc = plan->d_scal;  // 0: p.q  1: chi2(0)  2: x.b  3: x.r
  double* rzh = rz_hist_dev;
  if (!rzh) {
    if ((int64_t)maxiter + 1 > kCgHistCap)
      return fail(MM_E_ARG, "maxiter above " + std::to_string(kCgHistCap - 1) + " needs a caller history (rz_hist_dev)");
    rzh = plan->d_hist;
  }
  int it = 0;
  // the whole solve on stream s; with rtol > 0 the host reads r^T z every 10 iterations
  auto body = [&](hipStream_t s) -> mm_status {
    // b = P^T N^-1 d (or the given map)
    if (d)
      MM_TRY(apply_op(plan, GAIN_NINV, 1.0, nullptr, d, b, s));
    else
      MM_TRY_HIP(launch_copy(b, rhs_map, n, s));
    // x0, r0 = b - A x0
    if (m0) {
      if (m0 != x) MM_TRY_HIP(launch_copy(x, m0, n, s));
      MM_TRY(apply_op(plan, GAIN_NINV, 1.0, x, nullptr, q, s));
      MM_TRY_HIP(launch_sub(r, b, q, n, s));
    } else {
      MM_TRY_HIP(launch_fill(x, n, 0.0, s));
      MM_TRY_HIP(launch_copy(r, b, n, s));
    }
    MM_TRY_HIP(launch_winv_apply(plan->dp, r, z, s));
    MM_TRY_HIP(launch_copy(p, z, n, s));
    MM_TRY(dot(plan, r, z, rzh + 0, s));
    auto record_chi2 = [&](int i) -> mm_status {
      MM_TRY(dot(plan, x, b, sc + 2, s));
      MM_TRY(dot(plan, x, r, sc + 3, s));
      MM_TRY_HIP(launch_cg_chi2(sc + 1, sc + 2, sc + 3, chi2_hist_dev + i, s));
      return MM_OK;
    };
    if (chi2_hist_dev) {
      MM_TRY_HIP(launch_fill(zero, n, 0.0, s));
      MM_TRY(chi2_device(plan, d, zero, 1.0, sc + 1, nullptr, s));
      MM_TRY(record_chi2(0));
    }
    const int nb = dot_blocks(plan->npix);
    double rz0 = -1.0;
    for (it = 0; it < maxiter; ++it) {
      MM_TRY(apply_op(plan, GAIN_NINV, 1.0, p, nullptr, q, s));
      MM_TRY(dot(plan, p, q, sc + 0, s));
      MM_TRY_HIP(launch_cg_update_xr(plan->dp, x, r, z, p, q, rzh + it, sc + 0, plan->d_part, nb, s));
      MM_TRY_HIP(launch_reduce(plan->d_part, nb, rzh + it + 1, s));
      MM_TRY_HIP(launch_cg_update_p(p, z, rzh + it + 1, rzh + it, n, s));
      if (chi2_hist_dev) MM_TRY(record_chi2(it + 1));
      if (rtol > 0 && ((it + 1) % 10 == 0 || it + 1 == maxiter)) {
        double h[2];
        if (rz0 < 0) {
          MM_TRY_HIP(hipMemcpyAsync(&h[0], rzh, sizeof(double), hipMemcpyDeviceToHost, s));
        }
        MM_TRY_HIP(hipMemcpyAsync(&h[1], rzh + it + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        MM_TRY_HIP(hipStreamSynchronize(s));
        if (rz0 < 0) rz0 = h[0];
        if (h[1] <= rtol * rtol * rz0) {
          ++it;
          break;
        }
      }
    }
    return MM_OK;
  };
  if (rtol > 0) {
    MM_TRY(body(S(stream)));
  } else {
    // a fixed iteration count: the whole solve is captured into the plan's cached graph, like
    // mm_solve's schedule (replayed when called again with the same buffers and count)
    const std::vector<double> key = {2.0, (double)(uintptr_t)d, (double)(uintptr_t)rhs_map, (double)(uintptr_t)m0,
                                     (double)(uintptr_t)m_out, (double)(uintptr_t)chi2_hist_dev,
                                     (double)(uintptr_t)rzh, (double)maxiter};
    MM_TRY(run_graph(plan, key, stream, body));
    it = maxiter;
  }
  if (iters_done) *iters_done = it;
  return MM_OK;
}

}  // extern "C"
