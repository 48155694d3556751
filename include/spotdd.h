/*
 * spotdd.h -- C ABI of libspotdd: brute-force incoherent dedispersion of an
 * 8-bit multichannel filterbank over many trial dispersion measures (DMs),
 * followed by a boxcar matched-filter single-pulse S/N search, on one
 * AMD Instinct MI355X (gfx950) GPU.
 *
 * Method (paper: "Searching For Fast Radio Transients And Radio Pulsars Using
 * SPOTLIGHT"):
 *   - Chapter 1, Eq. (1): the dispersion delay of channel frequency f at
 *     dispersion measure DM, relative to the top frequency, is proportional
 *     to DM * (f^-2 - f_top^-2).
 *   - Section 3.2: brute-force dedispersion sums all channels of the dynamic
 *     spectrum along that delay curve, per trial DM; the series may be
 *     downsampled by a user factor.
 *   - Section 2.1: many trial DMs are dedispersed, then a single-pulse search
 *     by time-domain boxcar filtering reports pulses above a user threshold.
 *
 * Conventions the paper leaves open (fixed here and used by every call):
 *   delay   d(c,i) = floor(v + 0.5), v = 4.148808e3 * DM_i * (1/(f_c*f_c) -
 *           1/(f_top*f_top)) / (dec * t_samp), FP64, evaluated left to right;
 *           f in MHz, t_samp in s, f_top = max listed frequency.
 *   decim.  a DM range with decimation dec > 1 dedisperses the exact sums of
 *           dec consecutive input samples (groups aligned to input sample 0).
 *   extent  O = max_r (maxdelay_r + w_max - 1) * dec_r native samples
 *           (w_max = 1 with no widths). For nsamp_in input samples the call
 *           owns N = nsamp_in - O native samples; range r owns
 *           N_r = N / dec_r (floor) samples and its plane has
 *           cols_r = N_r + w_max - 1 columns:
 *           plane_r[i][j] = sum_c x_r[c][j + d_r(c,i)], j < cols_r (uint32,
 *           exact).
 *   search  for owned start j < N_r and width w: B_w[j] = sum_{k<w} y[j+k];
 *           S/N = (B_w[j] - w*mu) / (sigma*sqrt(w)) in FP64, mu = S1/n,
 *           sigma = sqrt(n*S2 - S1^2)/n, n = N_r, S1/S2 the exact sums of y and
 *           y^2 over the owned samples. A constant series (n*S2 == S1^2) has
 *           S/N 0 everywhere and no candidate. Best = first maximum in
 *           (j ascending, w ascending) order. A candidate is the best of one
 *           cell of cand_block owned starts, kept if S/N > threshold
 *           (strict); candidates are ordered by (range, DM index, sample).
 *
 * General rules:
 *   - Every call returns sdd_status (0 = ok, < 0 = error); nothing throws
 *     across the ABI. sdd_last_error() returns a thread-local message for the
 *     last failing call on the calling thread.
 *   - "d_" pointers are device pointers on the plan's device; "host_"
 *     pointers are host memory. The caller owns every buffer it passes.
 *   - stream is a hipStream_t (NULL = the null stream). Compute calls only
 *     enqueue work; results are valid once the stream has been synchronised.
 *   - Integer sums are exact by construction: plan creation refuses (ERANGE)
 *     a plan whose plane sums could exceed 2^32 - 1 or whose S2 could exceed
 *     2^64 - 1 (the latter is also checked per call against N_r).
 */
#ifndef SPOTDD_H
#define SPOTDD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDD_ABI_VERSION 1
#define SDD_MAX_RANGES 16
#define SDD_MAX_WIDTHS 32
#define SDD_MAX_WMAX 8192

typedef enum sdd_status {
  SDD_OK = 0,
  SDD_EINVAL = -1,    /* bad argument: null pointer, size, ordering, layout */
  SDD_ERANGE = -2,    /* exact integer sums could overflow */
  SDD_ENOMEM = -3,    /* workspace too small, or device allocation failed */
  SDD_EDEVICE = -4,   /* HIP error; message in sdd_last_error() */
  SDD_EAGAIN = -5,    /* (server) no room now: retry later */
  SDD_ESTATE = -6,    /* (server) call out of order: sequence gap, closed stream */
  SDD_ETIMEDOUT = -7  /* (server) poll timed out with no result */
} sdd_status;

/* Input layouts. Time-major is the spectra order a beamformer writes
 * (Section 2.2): byte (t, c) at d_in[t * in_pitch + c]. Channel-major:
 * byte (c, t) at d_in[c * in_pitch + t]. */
enum { SDD_CHAN_MAJOR = 0, SDD_TIME_MAJOR = 1 };

/* One DM range: DM_i = lo + i*step (FP64) for i < floor((hi-lo)/step + 0.5),
 * dedispersed at time decimation `decimation` (>= 1). */
typedef struct sdd_dm_range {
  double dm_lo, dm_hi, dm_step;
  int32_t decimation;
  int32_t reserved;
} sdd_dm_range;

typedef struct sdd_plan_desc {
  const double* freqs_mhz;     /* [nchan] channel centre frequencies, any order, > 0 */
  const double* dm_list;       /* [ndm] explicit trial DMs (>= 0, decimation 1), or NULL */
  const sdd_dm_range* ranges;  /* [nranges] DM ranges, or NULL; exactly one of the two */
  const int32_t* widths;       /* [nwidths] boxcar widths, strictly ascending, >= 1;
                                  nwidths == 0: plane only, no search */
  double t_samp_s;             /* native sampling time, > 0 */
  int32_t nchan;               /* >= 1 */
  int32_t ndm;                 /* entries of dm_list */
  int32_t nranges;             /* entries of ranges, <= SDD_MAX_RANGES */
  int32_t nwidths;             /* <= SDD_MAX_WIDTHS, w_max <= SDD_MAX_WMAX */
  int32_t cand_block;          /* owned starts per candidate cell, >= 1 (0: 1024) */
  float threshold;             /* candidate when S/N > threshold */
  int32_t layout;              /* SDD_CHAN_MAJOR or SDD_TIME_MAJOR */
  int32_t device;              /* HIP device ordinal */
} sdd_plan_desc;

typedef struct sdd_plan sdd_plan;

typedef struct sdd_plan_info {
  int32_t nchan, nranges, ndm_total, nwidths;
  int32_t w_max, cand_block, layout, device;
  int64_t overlap;                         /* O, native samples */
  int32_t ndm[SDD_MAX_RANGES];             /* trials per range */
  int32_t dm_offset[SDD_MAX_RANGES];       /* global index of the range's first trial */
  int32_t decimation[SDD_MAX_RANGES];
  int32_t max_delay[SDD_MAX_RANGES];       /* largest delay of the range, its own samples */
} sdd_plan_info;

/* Per-call sizes for nsamp_in input samples. */
typedef struct sdd_geometry {
  int64_t nsamp_in, overlap, n_owned;      /* n_owned = N = nsamp_in - O */
  int64_t n_owned_r[SDD_MAX_RANGES];       /* N_r */
  int64_t plane_cols[SDD_MAX_RANGES];      /* N_r + w_max - 1 */
  int64_t ncells[SDD_MAX_RANGES];          /* ceil(N_r / cand_block), 0 without widths */
  int64_t workspace_bytes;                 /* caller passes its own planes */
  int64_t workspace_bytes_planes;          /* planes live inside the workspace */
} sdd_geometry;

typedef struct sdd_candidate {
  int32_t range;      /* DM range */
  int32_t dm_index;   /* trial index within the range */
  int64_t sample;     /* window start j, in the range's own (decimated) samples */
  int32_t width;      /* boxcar width, the range's own samples */
  float snr;          /* S/N (FP64 rounded to float) */
} sdd_candidate;

typedef struct sdd_dm_best {   /* best (S/N, j, w) of one trial over all owned starts */
  float snr;
  int32_t width;
  int64_t sample;
} sdd_dm_best;

typedef struct sdd_dm_stats {  /* moments of the owned samples of one trial */
  int64_t n;
  uint64_t s1, s2;
  double mean, std;
} sdd_dm_stats;

/* Tile shape of the dedispersion kernel (a fixed menu; see sdd_tile_menu).
 * kind 0: direct kernel (one thread per DM and 4 samples, no LDS);
 * kind 1 + flags: LDS-tiled kernel (Section 3.2's brute-force sum, staged
 * per channel window in LDS). kind 1: vector form (byte align + widen with
 * v_perm, two channels per v_add3 into 16-bit fields); kind 3: the same
 * with two 64-bit LDS reads per 8 samples instead of 64 + 32 bits; kind 9:
 * vector form for uint16 ranges (decimation > 1 only) that keeps four copies
 * of each window, shifted by 0, 2, 4 and 6 bytes, so each channel costs one
 * aligned 64-bit read and no v_perm per 4 samples; kind 5:
 * matrix-core form (the shifted channel sum as an int8 product with a 0/1
 * selection matrix, two channels per v_mfma_i32_16x16x64_i8, int32 sums;
 * uint8 ranges only); kind 21: kind 5 that reads a channel pair's data words
 * once for two neighbouring trials when both windows start in the same
 * 16-byte words (the default for ranges with fine DM steps, where most
 * groups do). The other fields apply to the LDS kernels. */
typedef struct sdd_tile {
  int32_t kind;
  int32_t dm_per_wave;     /* DM trials per wavefront */
  int32_t waves_dm;        /* wavefronts along DM per workgroup */
  int32_t waves_time;      /* wavefronts along time per workgroup */
  int32_t pairs_per_lane;  /* 2-sample pairs per lane (samples per lane / 2) */
  int32_t chan_stage;      /* channels staged in LDS per step */
} sdd_tile;

/* ---- library ------------------------------------------------------------ */

/* ABI version (SDD_ABI_VERSION of the built library). */
int32_t sdd_abi_version(void);
/* Message of the last failing call on this thread ("" if none). The pointer
 * stays valid until the next sdd_* call on the same thread. */
const char* sdd_last_error(void);
/* Static name of a status code. */
const char* sdd_status_string(int32_t status);

/* ---- plan (host only: these calls touch no GPU) -------------------------- */

/* Builds the FP64 delay tables (Chapter 1, Eq. (1)), the overlap and the
 * exactness guards. Copies everything it needs from desc. EINVAL on a bad
 * descriptor, ERANGE on an overflow risk. *out is owned by the caller and
 * freed with sdd_plan_destroy. */
sdd_status sdd_plan_create(const sdd_plan_desc* desc, sdd_plan** out);
/* Frees the plan and its device tables. NULL is accepted. The caller must not
 * destroy a plan with work still in flight that uses it. */
sdd_status sdd_plan_destroy(sdd_plan* plan);
sdd_status sdd_plan_query(const sdd_plan* plan, sdd_plan_info* out);
/* Copies range r's delay table, int32 [ndm_r][nchan] row-major, to host_out. */
sdd_status sdd_plan_delays(const sdd_plan* plan, int32_t range, int32_t* host_out);
/* Copies range r's trial DMs, double [ndm_r], to host_out. */
sdd_status sdd_plan_dms(const sdd_plan* plan, int32_t range, double* host_out);
/* Sizes for nsamp_in samples. EINVAL if nsamp_in < O + dec_max (some range
 * would own no sample); ERANGE if S2 could overflow at that length. */
sdd_status sdd_plan_geometry(const sdd_plan* plan, int64_t nsamp_in, sdd_geometry* out);
/* Tile used for range r (set by the heuristic, sdd_plan_set_tile or
 * sdd_autotune). */
sdd_status sdd_plan_get_tile(const sdd_plan* plan, int32_t range, sdd_tile* out);
/* Forces range r's tile (range -1: every range). EINVAL if the shape is not
 * in the built menu or cannot hold the range's delay span. Results never
 * depend on the tile: the sums are exact. */
sdd_status sdd_plan_set_tile(sdd_plan* plan, int32_t range, const sdd_tile* tile);
/* Noise estimate (mu, sigma) of the search's S/N = (B - w*mu)/(sigma*sqrt(w))
 * (Sections 2.1 and 3.3: the median resists outliers better than the mean):
 *   SDD_STATS_MOMENTS    mean and population std of the owned samples
 *                        (default);
 *   SDD_STATS_CLIPPED    from those, `iters` passes keeping the samples with
 *                        |y - mu| <= k * sigma (FP64) and recomputing mu and
 *                        sigma from their exact integer moments (a pass that
 *                        keeps none stops);
 *   SDD_STATS_MEDIAN_MAD mu = lower median, sigma = 1.4826 * lower median of
 *                        |y - mu| (exact selections).
 * sdd_dm_stats then reports this mu and sigma as mean and std (n, s1, s2
 * stay the plain moments). EINVAL on an unknown mode, or k <= 0 or iters
 * outside 1..64 for SDD_STATS_CLIPPED. Like sdd_plan_set_tile and
 * sdd_plan_set_dereddening, it changes the plan for calls made afterwards
 * (cached batch graphs are rebuilt); it must not run while another thread
 * (or a server stream) is making calls with the plan. */
enum { SDD_STATS_MOMENTS = 0, SDD_STATS_CLIPPED = 1, SDD_STATS_MEDIAN_MAD = 2 };
sdd_status sdd_plan_set_stats(sdd_plan* plan, int32_t mode, double k, int32_t iters);
/* Running-median de-reddening of every searched series (Section 3.3: the
 * slowly varying baseline is removed by subtracting a running median whose
 * window exceeds twice the widest pulse). The window moves in strides of a
 * block of `block` samples: block k (samples [k*block, (k+1)*block) of the
 * trial's N_r + w_max - 1 columns) gets base_k = lower median of the samples
 * of blocks k-half .. k+half (clipped to the series), and the search (its
 * moments, noise estimate, boxcar sums and candidates) runs on
 *   y''[j] = clip(y[j] - base_{j / block} + M/2, 0, M),
 * M = nchan * 255 * dec the range's full scale (integer M/2; the clip acts
 * only on samples more than M/2 from their baseline, and the offset moves
 * mu, not sigma or the S/N). The DM-time planes themselves are left as
 * dedispersed. sdd_dm_stats then reports the moments of y''.
 * block = 0 turns it off. EINVAL unless block is a power of two in 64..4096,
 * half >= 1, (2*half+1)*block <= 4096 and > 2 * the widest boxcar, and the
 * plan has boxcar widths; ERANGE if nchan * 255 * dec_max >= 2^30. The
 * workspace grows by ndm_total * ceil(max columns / block) * 4 bytes. */
sdd_status sdd_plan_set_dereddening(sdd_plan* plan, int32_t block, int32_t half);
/* Writes up to max menu entries to host_out; *n_out = menu size. */
sdd_status sdd_tile_menu(sdd_tile* host_out, int32_t max, int32_t* n_out);
/* Picks each DM range's tile by timing every fitting menu shape on the
 * device with synthetic input of nsamp_in samples in the range's element
 * type (uint8 rows, or uint16 rows of nsamp_in / dec samples for a decimated
 * range; enqueued on stream, then synchronised). cache_path (may be NULL) is a text file of earlier choices
 * keyed by (nchan, ndm, decimation, delay spans, plane width): a hit skips the
 * timing, a miss appends the new choice. Allocates temporary device buffers
 * (input and one plane). Results never depend on the tile. */
sdd_status sdd_autotune(sdd_plan* plan, int64_t nsamp_in, const char* cache_path, void* stream);

/* ---- compute (enqueue on stream) ---------------------------------------- */

/* Every device workspace passed to this library (d_workspace / d_ws) must be
 * 256-byte aligned, as hipMalloc and torch allocations are: it holds 64-bit
 * atomics and 128-bit vectors at 256-byte offsets. A misaligned workspace is
 * refused with EINVAL before anything is enqueued. */

/* Dedisperses one chunk (Section 3.2, Section 2.1): corner turn (time-major
 * input), decimation (ranges with dec > 1), then every range's plane.
 *   d_in       uint8 input, layout as planned, nsamp_in samples per channel
 *   in_pitch   bytes between rows (time-major: >= nchan; channel-major:
 *              >= nsamp_in)
 *   d_planes   [nranges] device pointers (host array) to uint32 planes
 *              [ndm_r][plane_pitch[r]]; plane_pitch[r] >= cols_r elements
 *   d_workspace / ws_bytes: device scratch, >= geometry.workspace_bytes
 * The call uploads the plan's delay tables on first use on a device
 * (a synchronous copy). */
sdd_status sdd_dedisperse(const sdd_plan* plan, const uint8_t* d_in, int64_t nsamp_in,
                          int64_t in_pitch, uint32_t* const* d_planes,
                          const int64_t* plane_pitch, void* d_workspace, int64_t ws_bytes,
                          void* stream);

/* Single-pulse boxcar search (Section 2.1) of planes made by sdd_dedisperse
 * for the same nsamp_in.
 *   d_best   [ndm_total] per-trial best (global trial order: range by range)
 *   d_stats  [ndm_total] per-trial moments (may be NULL)
 *   d_cands  [cap] candidates in (range, dm, sample) order; *d_ncand receives
 *            the total number found, which may exceed cap (only the first
 *            cap are written)
 * EINVAL if the plan has no widths. */
sdd_status sdd_search_boxcar(const sdd_plan* plan, const uint32_t* const* d_planes,
                             const int64_t* plane_pitch, int64_t nsamp_in,
                             sdd_dm_best* d_best, sdd_dm_stats* d_stats,
                             sdd_candidate* d_cands, int32_t cap, int32_t* d_ncand,
                             void* d_workspace, int64_t ws_bytes, void* stream);

/* sdd_dedisperse followed by sdd_search_boxcar. d_planes may be NULL: the
 * planes then live in the workspace (>= geometry.workspace_bytes_planes) and
 * are not returned. */
sdd_status sdd_dedisperse_search(const sdd_plan* plan, const uint8_t* d_in, int64_t nsamp_in,
                                 int64_t in_pitch, uint32_t* const* d_planes,
                                 const int64_t* plane_pitch, sdd_dm_best* d_best,
                                 sdd_dm_stats* d_stats, sdd_candidate* d_cands, int32_t cap,
                                 int32_t* d_ncand, void* d_workspace, int64_t ws_bytes,
                                 void* stream);

/* sdd_dedisperse_search for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same path and results, with every scratch buffer (corner-
 * turned rows, decimated rows, search partials; the planes too when d_planes
 * is NULL) in a static device array of the library, 256 MiB, one copy per
 * device, held until the process ends. It calls no hipMalloc, hipFree or
 * other allocating routine. ENOMEM if the chunk needs more than 256 MiB of
 * scratch (geometry.workspace_bytes, or workspace_bytes_planes with NULL
 * planes); ESTATE if the plan's device tables do not exist yet (any other
 * compute call with the plan creates them); other errors as
 * sdd_dedisperse_search. Every call on one device shares that device's
 * array, which keeps the last call's contents: calls that overlap on one
 * device (other host threads, or other streams before the first call's work
 * is done) race and corrupt each other's results. */
sdd_status sdd_dedisperse_search_static(const sdd_plan* plan, const uint8_t* d_in,
                                        int64_t nsamp_in, int64_t in_pitch,
                                        uint32_t* const* d_planes, const int64_t* plane_pitch,
                                        sdd_dm_best* d_best, sdd_dm_stats* d_stats,
                                        sdd_candidate* d_cands, int32_t cap, int32_t* d_ncand,
                                        void* stream);

/* ---- batches of chunks (many beams, uneven lengths) ---------------------- */

/* One chunk of one beam in a batch; fields as in sdd_dedisperse_search.
 * d_planes may be NULL (planes live in the batch workspace, not returned);
 * plans without widths only dedisperse (d_best ... d_ncand unused). */
typedef struct sdd_batch_item {
  const sdd_plan* plan;
  const uint8_t* d_in;
  int64_t nsamp_in;
  int64_t in_pitch;
  uint32_t* const* d_planes;
  const int64_t* plane_pitch;
  sdd_dm_best* d_best;
  sdd_dm_stats* d_stats;
  sdd_candidate* d_cands;
  int32_t cap;
  int32_t reserved;
  int32_t* d_ncand;
} sdd_batch_item;

/* flags of sdd_batch_dedisperse_search */
enum {
  SDD_BATCH_PER_ITEM = 1, /* one launch per (chunk, range) instead of the persistent
                             multi-chunk dedispersion launch */
  SDD_BATCH_GRAPH = 2     /* capture the batch's launch sequence as a HIP graph on the
                             first call and replay it on later calls with identical
                             items, flags, workspace and stream (EINVAL on the null
                             stream, which cannot be captured) */
};

/* Workspace bytes for a batch (all items on one device). */
sdd_status sdd_batch_workspace_size(const sdd_batch_item* items, int32_t n, int64_t* bytes);
/* Dedisperses and searches every item (Section 2.1 over many beams, the
 * beam-level parallelism of Section 2.2). By default the dedispersion of all
 * items whose DM ranges share an LDS tile shape runs as one persistent launch:
 * the tile list is cut into one contiguous part per XCD and that XCD's
 * workgroups walk it in rounds, so beams of uneven length leave no tail per
 * beam. With SDD_BATCH_PER_ITEM every (chunk, range) is its own grid launch;
 * for chunks of 2^16 samples or more this is the faster mode on MI355X (two
 * or more streams then overlap one launch's tail with the next). Results
 * equal per-item sdd_dedisperse_search calls bit for bit. A graph replay (SDD_BATCH_GRAPH) re-runs the captured launches
 * on the same buffers: the caller rewrites inputs in place between calls. */
sdd_status sdd_batch_dedisperse_search(const sdd_batch_item* items, int32_t n, int32_t flags,
                                       void* d_ws, int64_t ws_bytes, void* stream);
/* Destroys every cached batch graph. */
sdd_status sdd_batch_graph_clear(void);

/* ---- streaming server (continuous batching of many beams) ---------------- */
/* Section 2.2: beams arrive as blocks of spectra that a ring buffer of recent
 * data holds long enough to absorb the pipeline's delay, and many beams are
 * searched side by side. Here each beam's ring lives in device memory and
 * keeps the max-delay overlap (plus the widest boxcar) between chunks, so
 * output chunk k is the one-shot sdd_dedisperse_search of stream samples
 * [kN, (k+1)N + O); ready chunks of all beams are batched onto the device
 * as slots free up (continuous batching), and beams are admitted by their
 * HBM footprint. */

typedef struct sdd_server sdd_server;
typedef struct sdd_stream sdd_stream;

/* flags of sdd_server_desc */
enum { SDD_SERVER_FAKE = 1 /* no GPU: batches sleep fake_exec_us and yield empty
                              results (for testing the scheduling logic) */ };

typedef struct sdd_server_desc {
  int64_t hbm_budget;     /* device bytes the server may hold: rings + slot buffers */
  int32_t device;
  int32_t max_beams;      /* open streams at most */
  int32_t nstreams;       /* batch slots (HIP streams) running concurrently, 1..16 */
  int32_t max_batch;      /* output chunks per batch, 1..256 */
  int32_t ring_chunks;    /* ring depth beyond the overlap, in chunks (>= 2) */
  int32_t cap;            /* candidates kept per output chunk */
  int32_t batch_flags;    /* SDD_BATCH_PER_ITEM (recommended) or 0 (persistent launch) */
  int32_t flags;          /* SDD_SERVER_FAKE */
  int32_t fake_exec_us;   /* batch duration in fake mode */
  int32_t fake_fail_every; /* fake mode: every n-th batch fails with SDD_EDEVICE (0: none) */
} sdd_server_desc;

/* One output chunk of one stream. best/cands are host memory owned by the
 * server until sdd_result_release. Times are steady-clock nanoseconds:
 * t_ready = the submit that completed the chunk's input returned, t_start =
 * its batch was launched, t_done = its results reached host memory. */
typedef struct sdd_result {
  uint64_t tag;                /* the stream's tag */
  int64_t chunk;               /* k: owned native samples [k*N, (k+1)*N) of the stream */
  int32_t status;              /* SDD_OK or the device error of its batch */
  int32_t ncand;               /* candidates found (may exceed the server's cap) */
  int32_t ndm;                 /* entries of best */
  int32_t reserved;
  const sdd_dm_best* best;     /* [ndm] */
  const sdd_candidate* cands;  /* [min(ncand, cap)] in (range, dm, sample) order */
  int64_t t_ready_ns, t_start_ns, t_done_ns;
  void* handle;
  /* DM-time planes of the chunk, only for streams with sdd_stream_keep_planes
   * on (nplanes = 0 otherwise): device memory owned by the server until
   * sdd_result_release, range r as [plane_rows[r]][plane_pitch[r]] uint32
   * (plane_rows[r] = the range's trials) with plane_cols[r] defined columns:
   * the sdd_dedisperse plane of the same window of spectra. */
  int32_t nplanes;
  int32_t plane_rows[SDD_MAX_RANGES];
  const uint32_t* d_planes[SDD_MAX_RANGES];
  int64_t plane_pitch[SDD_MAX_RANGES];
  int64_t plane_cols[SDD_MAX_RANGES];
} sdd_result;

typedef struct sdd_server_stats {
  int32_t open_streams;
  int32_t queued_results;
  int64_t hbm_used;
  int64_t batches;
  int64_t chunks;
  double busy_ms;              /* summed batch time (launch to results on host) */
} sdd_server_stats;

/* Starts the scheduler and completion threads. */
sdd_status sdd_server_create(const sdd_server_desc* desc, sdd_server** out);
/* Closes every open stream (waiting for their batches) and frees the server;
 * unreleased results are freed too. */
sdd_status sdd_server_destroy(sdd_server* server);
/* Ring bytes a stream of this plan and chunk length would hold. */
sdd_status sdd_stream_footprint(const sdd_server* server, const sdd_plan* plan,
                                int64_t chunk_nsamp, int64_t* bytes);
/* Opens a beam: time-major plan, chunks of chunk_nsamp samples (a multiple of
 * the plan's largest decimation). SDD_EAGAIN if max_beams are open or the
 * beam's ring (plus slot growth) does not fit the HBM budget. The plan must
 * outlive the stream. */
sdd_status sdd_stream_open(sdd_server* server, const sdd_plan* plan, int64_t chunk_nsamp,
                           uint64_t tag, sdd_stream** out);
/* Copies chunk seq (spectra [nsamp][nchan], host or device memory) into the
 * beam's ring; the caller may reuse its buffer on return. seq must count
 * 0, 1, 2, ... (SDD_ESTATE on a gap or after close). SDD_EAGAIN when the ring
 * slot still holds samples of an unfinished output chunk: poll, then retry. */
sdd_status sdd_stream_submit(sdd_stream* stream, const uint8_t* chunk, int64_t nsamp,
                             uint64_t seq, int32_t on_device);
/* Checkpoint of a beam (resume after a restart or a move to another server):
 * the next sequence number, the next output chunk not yet scheduled, and the
 * spectra that chunk and the later ones still need (samples next_out * N ..
 * submitted * N - 1, at most the ring). Output chunks already scheduled
 * finish and are polled as usual and are not part of the checkpoint.
 * host_out == NULL: *needed receives the size only; otherwise host_out must
 * hold *needed bytes (SDD_ENOMEM if bytes is smaller). The caller must not
 * submit to the stream during the call. The stream stays open. */
sdd_status sdd_stream_snapshot(sdd_stream* stream, void* host_out, int64_t bytes,
                               int64_t* needed);
/* Opens a beam from a checkpoint: like sdd_stream_open with the checkpoint's
 * chunk length, its ring refilled with the saved spectra; the next submit
 * takes the saved next sequence number and the saved unscheduled output
 * chunks are produced (bit for bit what the original stream would have
 * produced). EINVAL if the checkpoint is malformed or does not fit the plan
 * (channel count, overlap) or the ring; the sdd_stream_open errors otherwise. */
sdd_status sdd_stream_restore(sdd_server* server, const sdd_plan* plan, const void* snapshot,
                              int64_t bytes, uint64_t tag, sdd_stream** out);
/* Plane retention for one beam (off by default). When on, each output chunk
 * scheduled afterwards also writes its DM-time planes into a device buffer
 * that the server allocates for that chunk (hipMalloc, outside the HBM
 * budget: sum_r ndm_r * plane_pitch_r * 4 bytes) and frees at
 * sdd_result_release; the result's d_planes describe it. A chunk whose buffer
 * cannot be allocated comes back with SDD_ENOMEM. Meant for checking served
 * planes against one-shot calls, not for the real-time loop: the allocation
 * and the free (which waits for the device) sit on the serving path. */
sdd_status sdd_stream_keep_planes(sdd_stream* stream, int32_t on);
/* Copies a polled result's planes into caller buffers on `stream` (device
 * to device; d_dst[r] rows of dst_pitch[r] >= plane_cols[r] elements).
 * EINVAL if the result holds no planes. */
sdd_status sdd_result_copy_planes(sdd_server* server, const sdd_result* result,
                                  uint32_t* const* d_dst, const int64_t* dst_pitch,
                                  void* stream);
/* Stops the beam: no more submits, unscheduled output chunks are dropped,
 * scheduled ones finish (their results stay queued); frees the ring. */
sdd_status sdd_stream_close(sdd_stream* stream);
/* Takes up to max finished results, waiting up to timeout_us (< 0: until one
 * arrives or the server stops). SDD_ETIMEDOUT with *n_out = 0 if none came. */
sdd_status sdd_stream_poll(sdd_server* server, sdd_result* out, int32_t max, int32_t timeout_us,
                           int32_t* n_out);
/* Returns a polled result's host memory to the server. */
sdd_status sdd_result_release(sdd_server* server, sdd_result* result);
sdd_status sdd_server_query(sdd_server* server, sdd_server_stats* out);

/* ---- RFI pre-conditioning (before dedispersion) --------------------------- */

/* Bandpass correction with time- and frequency-domain flagging of one chunk
 * (Section 2.1 and the paper's figure of its RFI tool), as exact integer
 * maps applied while the chunk is staged for dedispersion:
 *   m_c   mean of channel c over the unflagged samples (all samples in the
 *         first round), FP64 of the exact integer sum;
 *   b_c   lower median of m over the median_window channels centred on c
 *         (clipped to the band): the bandpass;
 *   channel c flagged when |r_c - median(r)| > chan_sigma * 1.4826 * MAD(r),
 *         r = m - b (lower medians; a zero MAD flags nothing);
 *   z_t   sum of x[c][t] over unflagged channels; sample t flagged when
 *         |z_t - median(z)| > time_sigma * 1.4826 * MAD(z);
 *   repeated `rounds` times, each round from the previous round's flags.
 * Output: lut [nchan][256] with lut[c][v] = 0 for a flagged channel, else
 * clip(v - floor(b_c + 0.5) + floor(median(b) + 0.5), 0, 255); time mask
 * [nsamp_in], 1 = keep; optionally the channel flags [nchan]. */
typedef struct sdd_rfi_desc {
  int32_t median_window;  /* odd, 1..63 (21) */
  int32_t rounds;         /* 1..16 (2) */
  double chan_sigma;      /* (4.0) */
  double time_sigma;      /* (3.0) */
} sdd_rfi_desc;

/* Device scratch for sdd_rfi_estimate on chunks of nsamp_in samples. */
sdd_status sdd_rfi_workspace_size(const sdd_plan* plan, int64_t nsamp_in, int64_t* bytes);
/* Estimates the maps from one chunk in the plan's layout (d_in, in_pitch as
 * for sdd_dedisperse). d_chan_flags may be NULL. Enqueued on stream. */
sdd_status sdd_rfi_estimate(const sdd_plan* plan, const uint8_t* d_in, int64_t nsamp_in,
                            int64_t in_pitch, const sdd_rfi_desc* desc, uint8_t* d_lut,
                            uint8_t* d_time_mask, int32_t* d_chan_flags, void* d_workspace,
                            int64_t ws_bytes, void* stream);
/* Workspace bytes of sdd_dedisperse_search_pre (lib_planes != 0: planes kept
 * in the workspace, as d_planes == NULL). */
sdd_status sdd_pre_workspace_size(const sdd_plan* plan, int64_t nsamp_in, int32_t lib_planes,
                                  int64_t* bytes);
/* sdd_dedisperse_search of the pre-conditioned chunk
 * x'[c][t] = (d_time_mask == NULL || d_time_mask[t]) ? lut[c][x[c][t]] : 0,
 * with d_lut == NULL meaning the identity map. The maps are applied in the
 * corner turn (time-major input) or in a row copy (channel-major input). */
sdd_status sdd_dedisperse_search_pre(const sdd_plan* plan, const uint8_t* d_in, int64_t nsamp_in,
                                     int64_t in_pitch, const uint8_t* d_lut,
                                     const uint8_t* d_time_mask, uint32_t* const* d_planes,
                                     const int64_t* plane_pitch, sdd_dm_best* d_best,
                                     sdd_dm_stats* d_stats, sdd_candidate* d_cands, int32_t cap,
                                     int32_t* d_ncand, void* d_workspace, int64_t ws_bytes,
                                     void* stream);

/* ---- candidate sifting (after the search) -------------------------------- */

/* Removal of redundant candidates of one event with square stencils in the
 * DM-time plane, then density-based (DBSCAN) clustering of the survivors in
 * the DM-time plane, each cluster keeping its highest-S/N member (Section 2.1
 * names both steps; Ester et al. 1996 for DBSCAN). Coordinates of a
 * candidate: its FP64 trial DM from the plan and its window start in native
 * samples (sample * decimation of its range). Candidate q is better than p
 * when its float32 S/N is higher, or equal and q comes earlier in the list.
 *   stencil k (0 <= k < nstencils), half-sizes (stencil_dm[k] pc cm^-3,
 *     stencil_t[k] native samples): a candidate survives the pass when no
 *     better candidate of the pass's input has |dDM| <= stencil_dm[k] and
 *     |dt| <= stencil_t[k]; passes run in order on the previous survivors.
 *   clustering (min_pts >= 1): neighbourhood |dDM| <= eps_dm and
 *     |dt| <= eps_t, a point counting itself; core points have >= min_pts
 *     neighbours; clusters are connected components of core points; a
 *     non-core point with core neighbours joins the cluster of the earliest
 *     one, otherwise it is noise and is dropped. min_pts == 0: no clustering,
 *     every stencil survivor is kept with cluster size 1. */
#define SDD_MAX_STENCILS 8
typedef struct sdd_sift_desc {
  int32_t nstencils;
  int32_t min_pts;
  double stencil_dm[SDD_MAX_STENCILS];
  int64_t stencil_t[SDD_MAX_STENCILS];
  double eps_dm;
  int64_t eps_t;
} sdd_sift_desc;

/* Device scratch for sdd_sift_candidates on lists of up to cap candidates. */
sdd_status sdd_sift_workspace_size(int32_t cap, int64_t* bytes);
/* Sifts the candidate list of one sdd_search_boxcar / sdd_dedisperse_search
 * call of the same plan: d_cands [cap] in (range, dm, sample) order and
 * d_ncand, that call's device count (entries past cap are ignored). Writes
 * the kept candidates (entries naming no trial of the plan are dropped) to
 * d_out [cap] in list order, their number to
 * *d_nout (device), and, if d_sizes is not NULL, each kept candidate's
 * cluster size to d_sizes [cap] (device). Enqueued on stream; nothing is
 * read back to the host. EINVAL on null buffers, cap < 1, nstencils outside
 * 0..SDD_MAX_STENCILS, negative half-sizes or min_pts < 0; ENOMEM when
 * ws_bytes is too small. */
sdd_status sdd_sift_candidates(const sdd_plan* plan, const sdd_candidate* d_cands,
                               const int32_t* d_ncand, int32_t cap, const sdd_sift_desc* desc,
                               sdd_candidate* d_out, int32_t* d_nout, int32_t* d_sizes,
                               void* d_workspace, int64_t ws_bytes, void* stream);

/* ---- FFA folding and the boxcar search of folded profiles ---------------- */

/* Section 3.5: a series of N samples is stacked as m = floor(N / period)
 * rows of `period` samples (samples past m * period are not folded) and the
 * Fast Folding Algorithm (Staelin 1969) turns the stack into m folded
 * profiles. Profile s drifts s bins over the m - 1 row steps, i.e. it folds
 * at the trial frequency f_s = (1/p - s/((m-1) p^2)) / tau0 and period
 * p_s = p^2 / (p - s/(m-1)) * tau0 of Section 3.5 (p = period, tau0 the
 * sampling interval). Recursion: a stack of len > 1 rows splits into
 * h = len/2 head and t = len - h tail rows; its profile s is head profile
 * k_h plus tail profile k_t rolled left by s - k_t bins, with
 * k_h = round(s(h-1)/(len-1)), k_t = round(s(t-1)/(len-1)), round(x) =
 * floor(x + 1/2) (for m a power of two: the classic FFA, k_h = k_t = s/2).
 * Each profile is searched with circular boxcars of the given widths:
 * B_w[j] = sum of bins j .. j+w-1 (mod period), S/N = (B - w m mu) /
 * (sigma sqrt(m w)) with mu, sigma the mean and population deviation of the
 * m * period folded samples (exact integer moments, FP64); the best is the
 * largest S/N, then the smaller bin, then the smaller width; sigma = 0 gives
 * (0, 0, widths[0]). Profile bins are exact uint32 sums. */
#define SDD_FFA_MAX_PERIOD 4096

typedef struct sdd_ffa_best {  /* best boxcar of one folded profile */
  float snr;
  int32_t bin;    /* first bin of the boxcar */
  int32_t width;
  int32_t pad;
} sdd_ffa_best;

/* Device scratch for sdd_ffa_search: two uint32 stacks of nseries * m *
 * period plus the moments. */
sdd_status sdd_ffa_workspace_size(int32_t nseries, int64_t nsamp, int32_t period, int64_t* bytes);

/* Folds and searches nseries series (device, uint32; series k at
 * d_series + k * pitch elements, nsamp samples each, e.g. the rows of a
 * DM-time plane) at one base period on device `device`.
 *   max_value   a bound of every sample (a plane's nchan * 255 * dec); the
 *               call is refused (ERANGE) when m * max_value >= 2^32, so
 *               every profile bin is exact in 32 bits;
 *   widths      host, nwidths (1..SDD_MAX_WIDTHS) strictly increasing
 *               widths within 1 .. period-1;
 *   d_profiles  device uint32 [nseries][m][period] or NULL (not stored);
 *   d_best      device [nseries][m] best boxcar per profile;
 *   d_stats     device [nseries] moments of the folded samples, or NULL.
 * Enqueued on stream; nothing returns to the host. EINVAL on null buffers,
 * period outside 2..SDD_FFA_MAX_PERIOD, nsamp < period, pitch < nsamp or
 * bad widths; ENOMEM when ws_bytes is too small. */
sdd_status sdd_ffa_search(int32_t device, const uint32_t* d_series, int64_t pitch,
                          int32_t nseries, int64_t nsamp, int32_t period, uint32_t max_value,
                          const int32_t* widths, int32_t nwidths, uint32_t* d_profiles,
                          sdd_ffa_best* d_best, sdd_dm_stats* d_stats, void* d_ws,
                          int64_t ws_bytes, void* stream);

/* ---- kernel timing (benchmarks) ----------------------------------------- */

/* Stages whose kernels can be timed. */
enum { SDD_STAGE_CORNER_TURN = 0, SDD_STAGE_DECIMATE = 1, SDD_STAGE_DEDISPERSE = 2,
       SDD_STAGE_SEARCH = 3, SDD_STAGE_SIFT = 4, SDD_STAGE_FFA = 5, SDD_NSTAGES = 6 };

/* on != 0: from now on every stage launch is bracketed by two HIP events
 * recorded on the launch stream; the accumulated times are reset. on == 0:
 * stops recording (pending events are still read by sdd_profile_read).
 * Process-wide; not for concurrent use from several threads. */
sdd_status sdd_profile_enable(int32_t on);
/* Waits for the recorded events and returns the summed GPU time (ms) and the
 * number of launches of one stage since the last enable. */
sdd_status sdd_profile_read(int32_t stage, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* SPOTDD_H */
