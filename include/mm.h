/*
 * mm.h -- messenger-field CMB mapmaking on one MI355X (gfx950).
 *
 * C ABI of libmm.so.  The library solves the minimum-variance mapmaking
 * equation (P^T N^-1 P) m = P^T N^-1 d of Huffenberger & Naess, "Cosmic
 * Microwave Background Mapmaking with a Messenger Field":
 *   - Section 2: data model d = P m + n, eqn. (mapmaking), eqn. (chi2);
 *   - Section 2.1: the messenger iteration, compact form eqn. (mcompact),
 *     the cooling parameter lambda and chi^2(m, lambda);
 *   - Section 3.1: the cooling schedule and the diagonal-preconditioned
 *     conjugate-gradient comparison;
 *   - Section 4.2: a messenger variance tau per detector chunk.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Samples      The time-ordered data (TOD) of all detector chunks are
 *               concatenated; chunk c holds samples [chunk_off[c], chunk_off[c+1]).
 *               A chunk is one stationary stretch of one detector; its noise
 *               covariance is circulant (diagonal in the chunk's discrete
 *               Fourier basis).  Every chunk length must be even and half of it
 *               must factor into 2, 3 and 5 only (MM_E_LEN otherwise).
 *  Pointing     pix[j] is the map pixel of sample j (int32); a negative value
 *               means the sample is off the map (its row of P is zero but it
 *               still enters the noise filter and chi^2).  With three Stokes
 *               components sample j sees I + Q cos 2psi_j + U sin 2psi_j.
 *  Noise        Chunk c has N(f) = sigma_c^2 (1 + (f / fknee_c)^alpha_c) at the
 *               rfft frequencies f_k = k fsample_c / n_c; the f = 0 bin takes the
 *               value at f_1.  The messenger covariance is T = tau_c I on chunk c
 *               (default tau_c = sigma_c^2, the minimum of the spectrum).
 *  Maps         float64, layout [ncomp][npix], pixel p = y * nx + x.
 *  Memory       Arguments documented "device" are device pointers on the
 *               current HIP device; "host" are host pointers.  All are
 *               borrowed: the library never frees or keeps them past the
 *               call, except pix / psi and the workspace, which a plan reads
 *               at every iteration and which must stay valid (pix / psi also
 *               unchanged) until mm_plan_destroy.  A plan allocates no device
 *               memory: every table and work buffer lies in the caller's
 *               workspace, whose size mm_plan_workspace_bytes reports.
 *  Streams      Every call is ordered on the given stream and returns without
 *               waiting for it, except mm_plan_workspace_bytes(_noalloc) and
 *               mm_plan (they wait for their passes over the pointing),
 *               mm_chi2 (returns a host scalar) and mm_cg_solve when rtol > 0.
 *               Pass 0 for the default stream.  A plan is not thread-safe; use
 *               it from one host thread and one stream at a time.
 *  Errors       Every entry point returns an mm_status.  On error nothing is
 *               written to the output arguments and mm_last_error() gives a
 *               thread-local description.  Errors of earlier asynchronous work
 *               surface as MM_E_HIP at a later call.
 *  Determinism  Pixel binning is a fixed-order segmented reduction over
 *               samples sorted by pixel: results are bitwise reproducible run
 *               to run on the same device.
 */
#ifndef MM_H
#define MM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_plan_s* mm_plan_t;
typedef void* mm_stream_t; /* a hipStream_t */

typedef enum {
  MM_OK = 0,
  MM_E_ARG = 1,       /* invalid argument or descriptor field */
  MM_E_LEN = 2,       /* a chunk length the transforms do not support */
  MM_E_NOMEM = 3,     /* device or host allocation failed */
  MM_E_HIP = 4,       /* a HIP runtime error (possibly from earlier asynchronous work) */
  MM_E_SINGULAR = 5,  /* no pixel has a solvable weight block */
  MM_E_NONFINITE = 6  /* a non-finite chi^2 (NaN or Inf in the data or the map) */
} mm_status;

enum { MM_FP64 = 0, MM_MIXED = 1 };                              /* precision */
enum { MM_PSI_NONE = 0, MM_PSI_F64 = 1, MM_PSI_F32 = 2, MM_PSI_U16 = 3 }; /* psi storage */
enum { MM_MAP_AUTO = 0, MM_MAP_GATHER = 1, MM_MAP_PROJECTED = 2 };        /* map_access */
enum { MM_TUNE_MEASURE = 0, MM_TUNE_STATIC = 1, MM_TUNE_PICK0 = 16 };    /* tune */
enum { MM_BIN_SORTED = 0, MM_BIN_ATOMIC = 1 };                            /* binning */

/*
 * Problem description (Section 2 data model; Section 4.2 per-chunk tau).
 *  ncomp        1 (temperature) or 3 (I, Q, U).
 *  precision    MM_FP64: TOD, transforms and filter in float64 (d is double*).
 *               MM_MIXED: TOD, transforms and filter in float32 (d is float*);
 *               map, weight blocks, binning sums, chi^2 and CG scalars stay float64.
 *  npix, nx     map size; nx > 0 is the row length used to form square pixel
 *               tiles for binning (0 treats the map as one long row).
 *  nchunk       number of chunks; chunk_off (host, nchunk+1 int64, increasing,
 *               chunk_off[0] = 0) gives their extents.
 *  fsample, sigma, fknee, alpha   host, nchunk doubles: the noise law above.
 *  tau          host, nchunk doubles, or NULL for sigma^2; must satisfy
 *               0 < tau_c <= sigma_c^2 so that N - T stays positive semidefinite.
 *  pix          device, N_s int32 (N_s = chunk_off[nchunk]).
 *  psi          device, N_s angles (radians) of type psi_kind: MM_PSI_F64
 *               (double), MM_PSI_F32 (float) or MM_PSI_U16 (uint16 index into
 *               psi_table); NULL / MM_PSI_NONE when ncomp == 1.  Angles must be
 *               finite with |psi| < 1e5 (MM_E_ARG otherwise).
 *  psi_table    host, psi_table_len floats (only for MM_PSI_U16).
 *  map_access   how the time-domain sweeps read P m: MM_MAP_GATHER gathers the
 *               map per sample; MM_MAP_PROJECTED keeps a plan-owned N_s-sample
 *               buffer holding P m, written in pixel-tile order by the binning
 *               pass (or a projection pass) and read in time order; MM_MAP_AUTO
 *               picks PROJECTED when ncomp * npix * 8 bytes exceeds 4 MiB.  The
 *               results agree to rounding (MM_MIXED rounds P m to float32 there).
 *  tune         layout of each chunk length's transforms (split M = M1 M2 of the
 *               n/2-point complex transform, column-block width, radix order):
 *               MM_TUNE_MEASURE times the candidate layouts on the GPU at plan
 *               time for chunks of n/2 >= 16384 and keeps the fastest (the timing
 *               reads the TOD streams the plan's column pass reads: d, and P m
 *               under projected access, both halves of it with composite
 *               pointing; cached per process, length and stream count; with the
 *               environment variable MM_TUNE_CACHE
 *               naming a file, also persisted there, keyed by the device
 *               architecture, the HIP runtime version and the library build, and
 *               read back by later processes instead of timing again; the file
 *               is replaced by a rename, and a file that cannot be read or
 *               written only disables the persistence); MM_TUNE_STATIC takes the first candidate of
 *               a fixed rule.  Layouts differ only in rounding; MM_TUNE_STATIC
 *               gives bitwise identical results across processes.
 *               MM_TUNE_PICK0 + i takes candidate i of the rule's order for every
 *               length (clamped to the last one), to exercise each layout.
 *  binning      how the iterations form P^T y: MM_BIN_SORTED (default) reduces the
 *               samples of each pixel tile in pixel-sorted order, a fixed summation
 *               order (bitwise reproducible); MM_BIN_ATOMIC adds every sample into the
 *               map with FP64 atomics in time order (a measured alternative: the
 *               rounding varies from run to run).  The plan precompute (hits, W)
 *               always uses the sorted reduction.
 *  with_adjoint 1 reserves a second TOD-sized buffer in the workspace for
 *               mm_noise_grad and for mm_solve with a map right-hand side; 0
 *               leaves it out (those calls then return MM_E_ARG).
 *  tile_pixels  pixels per binning tile: 0 picks about npix / 2048, within
 *               16..512; 16..1024 asks for that many.  Larger tiles hold longer
 *               time-contiguous runs of each scan (fewer partly used cache lines
 *               when the binning pass reads the filtered TOD) but take more LDS.
 *  pix_b, psi_b, weight_a, weight_b
 *               composite pointing P = P_A + P_B (Section 2.2, Appendix B): NULL
 *               pix_b is the single pencil beam.  Otherwise every sample j also
 *               sees the map through a second component at pixel pix_b[j] (device,
 *               N_s int32, < 0: no second entry) with angle psi_b[j] (device, same
 *               type as psi; NULL when ncomp == 1):
 *                 (P m)_j = weight_a a(psi_j) m[pix_j] + weight_b a(psi_b_j) m[pix_b_j],
 *               a(psi) = (1, cos 2psi, sin 2psi).  A differential instrument has
 *               weights +1 and -1.  The messenger covariance is split T_A = T_B =
 *               T/2, so the per-pixel blocks the iteration inverts are
 *               W_AB = 2 (weight_a^2 P_A^T T^-1 P_A + weight_b^2 P_B^T T^-1 P_B)
 *               (eqn. mdiffcompact), and the lambda = inf step is a weighted Jacobi
 *               step (no longer the binned map).  Hits count the entries of both
 *               components.  Needs map_access AUTO or PROJECTED (it takes the
 *               projected access, with a 2 N_s-sample buffer) and binning SORTED;
 *               mm_lift_rhs, mm_tod_apply(which = 2) and mm_solve with a map
 *               right-hand side return MM_E_ARG (their lifting needs
 *               W = P^T T^-1 P).  Weights must be finite.
 *  with_gapfill 1 reserves two more TOD-sized buffers (the fields d_0 and t_0 of
 *               mm_solve_gapfill) and takes the projected map access; 0 leaves
 *               them out.  Not with composite pointing or map_access GATHER.
 *  pad_         unused (zero).
 */
typedef struct {
  int32_t ncomp;
  int32_t precision;
  int64_t npix;
  int64_t nx;
  int64_t nchunk;
  const int64_t* chunk_off;
  const double* fsample;
  const double* sigma;
  const double* fknee;
  const double* alpha;
  const double* tau;
  const int32_t* pix;
  const void* psi;
  int32_t psi_kind;
  int32_t map_access;
  const float* psi_table;
  int64_t psi_table_len;
  int32_t tune;
  int32_t binning;
  int32_t with_adjoint;
  int32_t tile_pixels;
  const int32_t* pix_b;
  const void* psi_b;
  double weight_a;
  double weight_b;
  int32_t with_gapfill;
  int32_t pad_;
} mm_plan_desc;

/* Cooling schedule (Section 3.1): optionally one lambda = inf step, then
 * nlevel levels, level l running iters[l] iterations at lambda[l] (host arrays). */
typedef struct {
  int32_t nlevel;
  int32_t first_inf;
  const double* lambda;
  const int32_t* iters;
} mm_schedule;

/*
 * Device bytes of the workspace a plan of this description needs (the
 * problem statement of Section 2: chunk table, pointing, noise law).  The
 * size depends on the pointing through the pixel-tile lists of the
 * deterministic binning, so the call validates the description and walks the
 * device pointing on `stream` (two passes over pix, one over psi; it waits for
 * them): pixel indices must be < npix, angles finite with |psi| < 1e5 (or
 * table indices < psi_table_len), MM_E_ARG otherwise.  It allocates a small
 * device buffer for its counters and the chunk table (freed before it
 * returns).  The result is the same for every call with the same description
 * and pointing, on any stream.
 */
mm_status mm_plan_workspace_bytes(const mm_plan_desc* desc, mm_stream_t stream, size_t* bytes);

/*
 * mm_plan_workspace_bytes for callers that cannot allocate device memory
 * (code under graph capture elsewhere on the device, serving loops, harnesses
 * that forbid hipMalloc).  Same result, but its counters and the chunk table
 * live in a fixed 1 MiB device array of the library (one per GPU, held until
 * the process ends), so nchunk is limited to 131039 (MM_E_ARG beyond).  Calls
 * on one GPU share that array: calls that overlap on one GPU (other host
 * threads, other streams) race and must be serialized by the caller.
 */
mm_status mm_plan_workspace_bytes_noalloc(const mm_plan_desc* desc, mm_stream_t stream, size_t* bytes);

/*
 * Build a plan in the caller's workspace (device, 256-byte aligned,
 * workspace_bytes >= what mm_plan_workspace_bytes reports, MM_E_NOMEM
 * otherwise): validates the descriptor, sorts the pointing by pixel tile for
 * deterministic binning (on the device), selects transform splits (timing
 * candidates in the workspace with MM_TUNE_MEASURE), and runs the precompute
 * kernels on `stream`: hit counts, the weight blocks
 * W_p = sum_{j at p} a_j a_j^T / tau_c (P^T T^-1 P of Section 2.1) and their
 * inverses.  A pixel is solvable when it has hits and, for 3x3 blocks,
 * det(W_p) / (W_p,00 W_p,11 W_p,22) >= 1e-8 (its angles separate Q from U);
 * unsolvable pixels are held at 0.
 * Waits for the stream.  MM_E_SINGULAR if no pixel is solvable.  The workspace
 * belongs to the plan until mm_plan_destroy, which waits for the device.
 */
mm_status mm_plan(const mm_plan_desc* desc, void* workspace, size_t workspace_bytes, mm_stream_t stream,
                  mm_plan_t* out);
mm_status mm_plan_destroy(mm_plan_t plan);
/* Binning structures of the plan (host out[7]): pixel tiles, tile width and
 * height (pixels), sub-batches, time-contiguous segments, pixel-sorted entries
 * (padded), and the workspace bytes in use. */
mm_status mm_plan_binning_stats(mm_plan_t plan, int64_t* out);
/* Copy the bit-exact hit counts (int32 [npix]) into hits_dev (device). */
mm_status mm_plan_hits(mm_plan_t plan, int32_t* hits_dev, mm_stream_t stream);
/* Copy the solvable mask (uint8 [npix]) into mask_dev (device). */
mm_status mm_plan_solvable(mm_plan_t plan, uint8_t* mask_dev, mm_stream_t stream);
/* Number of solvable pixels (host). */
mm_status mm_plan_nsolvable(mm_plan_t plan, int64_t* count);
/* The map access the plan uses (host): MM_MAP_GATHER or MM_MAP_PROJECTED
 * (MM_MAP_AUTO resolved). */
mm_status mm_plan_map_access(mm_plan_t plan, int32_t* access);
/* Transform layout of chunk `chunk` (host outputs): M1, M2 (M = n/2 = M1 M2),
 * cb (columns per column item), `pick` (index of the chosen candidate in the
 * fixed rule's order) and `ncand` (number of candidates). */
mm_status mm_plan_chunk_layout(mm_plan_t plan, int64_t chunk, int64_t* M1, int64_t* M2, int32_t* cb,
                               int32_t* pick, int32_t* ncand);

/*
 * One messenger iteration, eqn. (mcompact) of Section 2.1:
 *   m_out = m_in + W^-1 P^T (lambda^-1 (N - T) + T)^-1 (d - P m_in)
 * on solvable pixels (0 elsewhere).  lambda >= 1 or INFINITY; lambda = inf
 * gives the binned map W^-1 P^T T^-1 d directly (no transforms).
 * d: device TOD (double* for MM_FP64, float* for MM_MIXED).  m_in, m_out:
 * device maps (may be the same buffer).  chi2_dev: device double or NULL;
 * receives chi^2(m_in) of eqn. (chi2) (computed from the same transform).
 */
mm_status mm_messenger_iter(mm_plan_t plan, const void* d, double lambda, const double* m_in,
                            double* m_out, double* chi2_dev, mm_stream_t stream);

/*
 * Full cooled messenger solve (Section 3.1).  Captures the whole schedule in
 * one HIP graph and launches it on `stream`; a call with the same buffers and
 * the same schedule as the previous one replays that graph without capture.
 * The plan keeps only the latest graph: a call that captures a new one first
 * waits on the host until the previous graph's last launch has completed, then
 * destroys it.  Exactly one of d (device TOD) and rhs_map (device map g) is
 * given.  With rhs_map the solve runs on the lifted data N T^-1 P W^-1 g (see
 * mm_lift_rhs), so it converges to (P^T N^-1 P)^-1 g: the adjoint solve of a
 * map gradient, with the cooling behaviour of real data (needs with_adjoint).
 * m0: device start map or NULL for zero.  m_out: device result.  chi2_hist_dev: device array of
 * (first_inf + sum(iters) + 1) doubles or NULL; entry i is chi^2(m_i) of the
 * map entering iteration i, the last entry chi^2 of the final map.
 */
mm_status mm_solve(mm_plan_t plan, const void* d, const double* rhs_map, const mm_schedule* sched,
                   const double* m0, double* m_out, double* chi2_hist_dev, mm_stream_t stream);

/*
 * The cooled messenger solve in its map-sized form (Section 2.1, eqns. md and F;
 * Section 4.1): each level first forms m_d(lambda) = W^-1 P^T (lambda^-1 N-bar + T)^-1 d
 * (one sweep that reads the data), and its iterations then apply
 * m_{i+1} = m_d(lambda) + F(lambda) m_i, F(lambda) m = m - W^-1 P^T (lambda^-1 N-bar + T)^-1 P m,
 * without reading d.  Equal to mm_solve's iterates in exact arithmetic (Woodbury); the
 * lambda = inf step is the binned map as there.  Same schedule, start map and graph
 * capture/replay as mm_solve (the one cached graph is shared); no chi^2 history (the
 * iterations never form d - P m: use mm_chi2 on the result).
 */
mm_status mm_solve_mapsized(mm_plan_t plan, const void* d, const mm_schedule* sched, const double* m0,
                            double* m_out, mm_stream_t stream);

/*
 * The cooled solve with gap filling: composite noise N = N_0 + N_1 (Appendix C), N_1 diagonal
 * in time with infinite variance in the gaps and eps_c = sigma_c^2 - tau_c elsewhere, N_0 =
 * N - eps_c I (so that outside the gaps the noise is the chunk's law N).  Every iteration sets
 * the four fields of the appendix to their conditional means in its order:
 *   t_1 = d outside the gaps, d_0 inside (T_1 = eps I, the largest allowed);
 *   d_0 = t_1 + A (t_0 - t_1),  A = eps / (eps + N-bar_0) per Fourier bin;
 *   t_0 = P m + tau (lambda^-1 N-bar_0 + T_0)^-1 (d_0 - P m);
 *   m   = W^-1 P^T T_0^-1 t_0 (W^-1 P^T T_0^-1 P = I on the solvable pixels),
 * with T_0 = tau I and N-bar_0 = N_0 - T_0 = sigma^2 (f/f_knee)^alpha (the DC bin clamped), lambda
 * on T_0 as in Section 2.1.  The fixed point at lambda = 1 is the generalised least-squares
 * map of the samples outside the gaps; d_0 is the gap-filled data.  Start: d_0 = d outside the
 * gaps and 0 inside, t_0 = d_0, m = m0 (NULL: zero).
 * The plan needs with_gapfill, single-beam pointing and 0 < tau_c < sigma_c^2 (tau_c < sigma_c^2
 * sets eps_c > 0); MM_E_ARG otherwise.  d: device TOD (the plan's precision).  gaps: device
 * N_s bytes, nonzero for a sample whose data are unusable (its pointing still counts in W and
 * P m); the data there are never read.  d0_out: device TOD receiving d_0 (time order), or NULL.
 * Each iteration runs two filter sweeps (the d_0 and the t_0 updates), two time-domain steps
 * and the binning pass.  Runs uncaptured on `stream`; no chi^2 history.
 */
mm_status mm_solve_gapfill(mm_plan_t plan, const void* d, const uint8_t* gaps, const mm_schedule* sched,
                           const double* m0, double* m_out, void* d0_out, mm_stream_t stream);

/*
 * Geometric cooling levels (Section 3.1): lambda_l = lambda_max^((nlevel-1-l)/(nlevel-1)),
 * ending at exactly 1.  lambda_max <= 0 selects the rule lambda_max = max_c N_c(f_0) / tau_c
 * (lambda tau spans the noise power).  out: host array of nlevel doubles.
 */
mm_status mm_cooling_levels(mm_plan_t plan, int32_t nlevel, double lambda_max, double* out);

/*
 * Diagonal-preconditioned conjugate gradients on (P^T N^-1 P) m = P^T N^-1 d
 * (Sections 1, 2 and 3.1), preconditioner W^-1 = (P^T T^-1 P)^-1 per pixel.
 * d: device TOD, or NULL when rhs_map (device map) gives P^T N^-1 d directly.
 * m0: device start map or NULL (zero, as in Section 3.1).  Runs maxiter
 * iterations, or stops when r^T W^-1 r <= rtol^2 r_0^T W^-1 r_0 (checked on
 * the host every 10 iterations, which waits for the stream) if rtol > 0.
 * chi2_hist_dev (device, maxiter+1 doubles, or NULL) gets chi^2 of each iterate
 * from the recursion chi^2(x) = d^T N^-1 d - x^T b - x^T r (needs d).
 * rz_hist_dev (device, maxiter+1 doubles, or NULL) gets r^T W^-1 r; without it
 * the plan keeps the history itself, which limits maxiter to 16383.
 * iters_done (host, or NULL) gets the number of iterations run.  With rtol = 0
 * (a fixed count) the solve is captured into the plan's one cached HIP graph and
 * replayed by a later call with the same buffers and count (as mm_solve's schedule);
 * with rtol > 0 it runs uncaptured.
 */
mm_status mm_cg_solve(mm_plan_t plan, const void* d, const double* rhs_map, int32_t maxiter,
                      double rtol, const double* m0, double* m_out, double* chi2_hist_dev,
                      double* rz_hist_dev, int32_t* iters_done, mm_stream_t stream);

/*
 * chi^2(m, lambda) = (d - P m)^T N'(lambda)^-1 (d - P m), N' = N + (lambda - 1) T
 * (eqn. chi2 for lambda = 1; Section 2.1 otherwise), summed over the Fourier
 * modes of every chunk.  chi2_host: host double (the call waits for the
 * stream).  per_chunk_dev: device array of nchunk doubles or NULL.
 * MM_E_NONFINITE if the sum is not finite.
 */
mm_status mm_chi2(mm_plan_t plan, const void* d, const double* m, double lambda, double* chi2_host,
                  double* per_chunk_dev, mm_stream_t stream);

/*
 * chi^2 per Fourier mode, a diagnostic of the noise model (Section 3.1 reads
 * chi^2 mode by mode; each mode's term |r-hat_k|^2 / (n N'_k) has unit mean when
 * the noise model is right): for the nsel chunks listed in `chunks` (host),
 * with r = d - P m and N' = N + (lambda - 1) T (lambda = 1: eqn. chi2),
 *   modes_dev (device, sum over the listed chunks of n_i/2 + 1 doubles, chunk i
 *   after those before it): term k = omega_k |r-hat_k|^2 / (n N'_k), k = 0..n/2,
 *   omega_k = 1 for k = 0 and n/2, else 2 (they sum to the chunk's chi^2);
 *   bins_dev (device, [nsel][nbins][2]): per log-spaced bin, the sum of the terms
 *   and the number of real modes they stand for (sum of omega_k).
 * Bins: k = 0 in bin 0; k >= 1 in bin 1 + s o + floor(s (k - 2^o) / 2^o),
 * o = floor(log2 k), s = per_octave (1..64); nbins must equal
 * 1 + s (floor(log2 max_i n_i/2) + 1) (MM_E_ARG otherwise).  One forward sweep
 * over the whole TOD plus the listed chunks' row transforms; deterministic.
 */
mm_status mm_chi2_modes(mm_plan_t plan, const void* d, const double* m, double lambda, int32_t nsel,
                        const int64_t* chunks, int32_t per_octave, double* modes_dev, double* bins_dev, int32_t nbins,
                        mm_stream_t stream);

/*
 * Apply the map-space operators once (building blocks for adjoint solves and
 * tests): out = P^T G P x or P^T G d with G = N^-1 (which == 0) or
 * G = (lambda^-1 (N - T) + T)^-1 (which == 1).  x: device map, d: device TOD
 * (exactly one of them non-NULL).  out: device map.
 */
mm_status mm_apply(mm_plan_t plan, int32_t which, double lambda, const double* x, const void* d,
                   double* out, mm_stream_t stream);

/*
 * Lift a map-space vector g to TOD space: out = N T^-1 P W^-1 g, so that
 * P^T N^-1 out = g on solvable pixels.  Running mm_solve on `out` then solves
 * (P^T N^-1 P) z = g with the messenger iteration (the adjoint solve of the
 * map gradient).  out: device TOD of the plan's TOD type.
 */
mm_status mm_lift_rhs(mm_plan_t plan, const double* g, void* out, mm_stream_t stream);

/*
 * Replace the noise parameters of every chunk (host arrays of nchunk doubles;
 * tau NULL for sigma^2) and recompute what depends on them: the noise
 * spectrum, the weight blocks P^T T^-1 P, their inverses and the solvable
 * mask.  The pointing sort is kept.  Waits for the stream.
 */
mm_status mm_plan_set_noise(mm_plan_t plan, const double* sigma, const double* fknee, const double* alpha,
                            const double* tau, mm_stream_t stream);

/*
 * TOD-space image of a map: out = G P x with G = N^-1 (which == 0),
 * (lambda^-1 (N - T) + T)^-1 (which == 1) or N T^-1 (which == 2).  x: device
 * map; out: device TOD of the plan's TOD type.  With x = z = A^-1 g (A the
 * normal matrix P^T N^-1 P of eqn. mapmaking), which == 0 gives the gradient
 * of a loss L(m) of the solved map with respect to the data, N^-1 P z.
 */
mm_status mm_tod_apply(mm_plan_t plan, int32_t which, double lambda, const double* x, void* out,
                       mm_stream_t stream);

/*
 * Gradient of a loss of the solved map m = A^-1 P^T N^-1 d (eqn. mapmaking)
 * with respect to each chunk's noise parameters (sigma, fknee, alpha):
 *   dL/dtheta_c = -(1/n_c) sum_k omega_k Re(conj(Zhat_k) Rhat_k) (dN_k/dtheta_c) / N_k^2
 * with r = d - P m, Zhat = rfft of P z and z = A^-1 (dL/dm) the adjoint map
 * (obtain it with mm_lift_rhs + mm_solve, or mm_cg_solve with rhs_map).
 * omega_k is the multiplicity of rfft bin k.  d: device TOD; m, z: device
 * maps; grad_dev: device [nchunk][3] doubles.  Needs the plan's second
 * TOD-sized buffer (with_adjoint).  MM_E_LEN when two rows of two residuals
 * do not fit one workgroup's LDS.
 */
mm_status mm_noise_grad(mm_plan_t plan, const void* d, const double* m, const double* z, double* grad_dev,
                        mm_stream_t stream);

/*
 * Per-pass timing for measurement.  With timing enabled, every pass launched
 * by mm_messenger_iter, mm_chi2, mm_apply and mm_cg_solve (not mm_solve, which
 * replays a graph) is bracketed by HIP events recorded on the stream it runs
 * on.  mm_get_timing waits for the recorded events, returns the summed
 * milliseconds and launch counts per pass (ms and launches: 5 entries each;
 * index 0..4 = passes A, B, C, D and the map projection: gather + column
 * transforms, row transforms + filter, inverse column transforms, binning +
 * map update, P m in pixel-tile order for large maps) and clears the record.
 * With timing enabled mm_solve runs its iterations on the stream directly
 * instead of capturing a graph, so that they are timed too.
 */
mm_status mm_set_timing(mm_plan_t plan, int32_t enable);
mm_status mm_get_timing(mm_plan_t plan, double* ms, int64_t* launches);

const char* mm_status_str(mm_status s);
const char* mm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
