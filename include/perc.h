/*
 * perc.h -- percolation inspection of carbon-nanotube fibers on AMD MI355X (gfx950).
 *
 * The method is the Markov-chain inspection of Xu, Xu & Yakobson, "Site-percolation
 * threshold of carbon nanotube fibers -- fast inspection of percolation with Markov
 * stochastic theory": a fiber is a modified FCC lattice of tubes (Sec. II.A, Fig. 1;
 * 12 side contacts + 2 end contacts per tube), each tube metallic with probability p;
 * a random walker hops to a uniformly chosen metallic contact (Eq. 1-2); probability
 * mass is injected on the metallic tubes of one end and pushed forward by repeated
 * sparse matrix-vector products, a detector joined to every metallic tube of the far
 * end absorbs it (Sec. II.B), and the configuration percolates iff the detector ever
 * receives non-zero probability (Eq. 3-4: first-passage probabilities).
 *
 * Conventions shared by every call:
 *  - Geometry. W is the hex radius of the hexagonal cross-section in tube spacings
 *    (3W(W+1)+1 columns); L is the number of (111) layers, stacked A,B,C. Column (q,r)
 *    (axial coordinates) carries the layers k = (q - r) mod 3, +3, +6, ... < L.
 *  - Canonical site order: lexicographic (k, q, r); N sites; site s is bit s % 32 of
 *    word s / 32 of a configuration (LSB first), ceil(N/32) words per configuration,
 *    configurations back to back. Padding bits past N are ignored.
 *  - Surfaces: start = the tubes of layers 0..2 (one per column), far = the tubes of
 *    layers L-3..L-1 (one per column). The start mass is 1/|S0| on each metallic start
 *    tube; deg counts metallic contacts plus the detector edge of a far tube; a
 *    metallic tube of degree 0 keeps its mass (self-loop).
 *  - steps: the number of forward steps the inspection took: d+1 for a percolating
 *    configuration whose nearest far tube is d contacts from the start set (the first
 *    step with non-zero detector probability), else the step at which the reached set
 *    stopped growing; 0 when no start tube is metallic.
 *  - Device pointers are HIP device memory of the current device; host pointers are
 *    ordinary memory. `stream` is a hipStream_t (NULL = the default stream). Calls
 *    marked async enqueue work on `stream` and return; the caller keeps every buffer
 *    alive until the stream is synchronised.
 *  - Work memory: pieces under 64 MiB are taken stream-ordered from the device's
 *    memory pool; larger work memory comes from one buffer per device that the library
 *    keeps between calls (it grows in 1 GiB steps to the largest need seen; a batch
 *    runs in waves of at most 128 GiB and half the free memory) and lends to one call
 *    at a time, stream-ordered behind the previous borrower's work; a call that finds
 *    it lent to another thread allocates its own. The persistent part of a mixed batch
 *    runs on a second stream the library keeps per device, with a second such buffer.
 *    perc_trim releases both buffers.
 *  - Errors: a negative PERC_E* code; perc_last_error() gives a message (per thread,
 *    valid until the next call on that thread). No call aborts the process.
 */
#ifndef PERC_H
#define PERC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PERC_OK = 0,
    PERC_EINVAL = -1,    /* invalid argument */
    PERC_ENOMEM = -2,    /* device or host allocation failed */
    PERC_EHIP = -3,      /* a HIP runtime call failed */
    PERC_EBUSY = -4,     /* server: over the memory budget or queue full */
    PERC_ECANCELED = -5, /* server: request cancelled */
    PERC_ECAP = -6       /* the step cap N+1 was reached (impossible for a valid lattice) */
};

/* Execution forms of an inspection batch (all give identical results). */
enum {
    PERC_FORM_AUTO = 0,    /* chosen from the shape and batch size (autotuned if cached);
                              a batch with at least 2048 jobs on short-walk fibers (below)
                              and some on others runs as PERC_FORM_MIXED */
    PERC_FORM_PLAIN = 1,   /* one configuration at a time; the host checks the stop flags
                              after every step (the paper's per-configuration loop) */
    PERC_FORM_SPAN = 2,    /* many configurations at once, each spread over workgroups;
                              one launch per step over a device-built work list, replayed
                              as a HIP graph */
    PERC_FORM_PERSIST = 3, /* one workgroup per configuration pulled from a device queue;
                              the whole inspection (sampling included) in one launch;
                              it reports PERC_ECAP from the synchronous calls only
                              (perc_pi, perc_pi_ex, perc_batch with groups) */
    PERC_FORM_SPAN2 = 4,   /* the span form advancing two steps per launch: the first step
                              of a tile's halo range is kept in LDS and the second is
                              computed from it, one pass over the state per two steps.
                              PERC_EINVAL for fibers whose outer range (the halo of the
                              halo range) exceeds two columns per thread or LDS */
    PERC_FORM_PERSIST2 = 5, /* the persistent form advancing two steps per pass: one
                              workgroup holds the whole cross-section (one thread per
                              column, no halo), keeps the first step in LDS and writes the
                              second; PERC_EINVAL for fibers of more than 1024 columns
                              (W > 17). Reports PERC_ECAP as the persistent form */
    PERC_FORM_MIXED = 6    /* per fiber: jobs on short-walk fibers (one column tile of at
                              most 512 columns, or column tiles x unit cells ceil(L/3) <=
                              600) in the persistent form on a second stream of the
                              library's, the others in the
                              span form on `stream` beside it (depth, block, grid and
                              graph_steps apply to the span part); outputs and group counts
                              as for one batch, complete when `stream` reaches them */
};

typedef struct perc_options {
    int32_t form;        /* PERC_FORM_* */
    int32_t depth;       /* unit cells one workgroup walks per work item, rounded up to a
                            multiple of 8; 0 = choose */
    int32_t block;       /* threads per workgroup, multiple of 64, <= 1024, at least the
                            widest column tile and half its halo range; 0 = choose */
    int32_t grid;        /* workgroups per launch; 0 = choose */
    int32_t graph_steps; /* span form: steps per graph replay; 0 = choose */
} perc_options;

typedef struct perc_lattice perc_lattice;

/* ---- lattice (Sec. II.A, Fig. 1) ------------------------------------------------ */

/* Build the fiber lattice of hex radius 0 <= W <= 1024 and 1 <= L <= 65535 layers
 * (the sampler's stream tag W<<16 | L is then distinct for every shape). Returns NULL
 * on a bad argument or more than 2^31-1 sites. Owned by the caller; immutable; safe to
 * use from several threads and streams at once. */
perc_lattice* perc_lattice_create(int32_t W, int32_t L);

/* As perc_lattice_create with options: PERC_LATTICE_NO_END_CONTACTS drops the two end
 * contacts of every tube, leaving the regular FCC lattice of the same sites (12 side
 * contacts), the lattice the paper compares its threshold with (Sec. III). Sites, site
 * order, surfaces, the detector edge and the sampler streams are those of the modified
 * lattice, so both variants can be inspected on the same configurations. Unknown flag
 * bits: NULL. */
#define PERC_LATTICE_NO_END_CONTACTS 1
perc_lattice* perc_lattice_create_ex(int32_t W, int32_t L, int32_t flags);
void perc_lattice_destroy(perc_lattice* lat); /* NULL-safe */

int64_t perc_lattice_sites(const perc_lattice* lat);   /* N */
int64_t perc_lattice_words(const perc_lattice* lat);   /* ceil(N/32) */
int32_t perc_lattice_columns(const perc_lattice* lat); /* 3W(W+1)+1 */
/* Device bytes one configuration occupies while it is inspected (state and codes). */
int64_t perc_lattice_state_bytes(const perc_lattice* lat);

/* Coordinates of canonical site s (host). PERC_EINVAL if s is out of range. */
int perc_site_coord(const perc_lattice* lat, int64_t s, int32_t* q, int32_t* r, int32_t* k);

/* The contacts of canonical site s, ascending (host): side contacts (FCC nearest
 * neighbours) and end contacts (same column, 3 layers away). nbr must hold 14
 * entries; *count receives the number written. */
int perc_site_neighbors(const perc_lattice* lat, int64_t s, int64_t* nbr, int32_t* count);

const char* perc_last_error(void);

/* ---- sampling (Sec. II.A: each tube metallic with probability p) ----------------- */

/* Occupancy bits of configurations cfg0 .. cfg0+n_cfg-1 (device, async). Tube s of
 * configuration c is metallic iff word s%4 of Philox4x32-10 (Salmon et al., SC'11) with
 * counter (s/4, c mod 2^32, c / 2^32, W<<16 | L) and key (seed mod 2^32, seed / 2^32)
 * is below floor(p * 2^32). p in [0, 1]. The stream does not depend on p, so lower p
 * occupies a subset of the tubes of higher p (common random numbers). */
int perc_sample(const perc_lattice* lat, double p, uint64_t seed, int64_t cfg0, int64_t n_cfg,
                uint32_t* occ_bits, void* stream);

/* Fixed-count ensemble (Sec. II.A: Np of the N tubes are chosen metallic, uniformly):
 * each configuration has exactly K = floor(N p + 1/2) metallic tubes, the K with the
 * smallest 64-bit keys, ties by tube index; tube s's key is words 2(s%2) (high) and
 * 2(s%2)+1 (low) of Philox4x32-10 with counter (s/2, c mod 2^32, c / 2^32,
 * (W<<16 | L) | 2^31) and key (seed mod 2^32, seed / 2^32). Same layout and ownership
 * as perc_sample (device bits, async). */
int perc_sample_fixed(const perc_lattice* lat, double p, uint64_t seed, int64_t cfg0, int64_t n_cfg,
                      uint32_t* occ_bits, void* stream);

/* ---- inspection (Sec. II.B) --------------------------------------------------------- */

/* Decide percolation of n_cfg >= 0 configurations given as canonical occupancy bits
 * (device, n_cfg * words uint32). perc (device, n_cfg bytes) receives 0/1 and steps
 * (device, n_cfg int32, may be NULL) the step counts. Async (work memory as the
 * conventions above state). */
int perc_inspect(const perc_lattice* lat, const uint32_t* occ_bits, int64_t n_cfg, uint8_t* perc,
                 int32_t* steps, void* stream);

/* As perc_inspect, with the execution form chosen by `opt` (NULL = automatic) and the
 * optional output hit (device, n_cfg float, may be NULL): the probability that the
 * walker hits the detector for the first time at step `steps` (0 if not percolating),
 * computed in FP32 -- it underflows to 0 on long paths, the decision never uses it. */
int perc_inspect_ex(const perc_lattice* lat, const uint32_t* occ_bits, int64_t n_cfg, uint8_t* perc,
                    int32_t* steps, float* hit, const perc_options* opt, void* stream);

/* For callers that cannot allocate (code under HIP graph capture elsewhere in the
 * program, tight serving loops, harnesses that forbid allocation): perc_inspect_ex in
 * the span form with every work buffer (state, codes, slot tables, the planner's work
 * list, the shape tables) carved from one fixed 256 MiB array per device that the
 * library holds from its first use on that device until the process ends. The call
 * makes no device, pinned-host or pool allocation and builds no graph; it runs in
 * waves of as many configurations as the array holds and returns when the work is
 * complete (synchronous; not capturable). occ_bits, perc, steps (may be NULL), hit
 * (may be NULL): device, as perc_inspect_ex; results equal perc_inspect_ex's bit for
 * bit. PERC_EINVAL when one configuration of the fiber needs more than the array (at
 * 9 bytes per state word: e.g. W=64 fits up to L of about 7,000 layers). Every call on
 * a device shares its array: calls that overlap on one device (other threads, other
 * streams) race and must be serialised by the caller. */
int perc_inspect_noalloc(const perc_lattice* lat, const uint32_t* occ_bits, int64_t n_cfg, uint8_t* perc,
                         int32_t* steps, float* hit, void* stream);

/* ---- percolation probability Pi(p) (Sec. III) ------------------------------------ */

typedef struct perc_pi_out {
    int64_t n_perc;  /* out: number of percolating configurations */
    double pi;       /* out: n_perc / n_cfg (0 when n_cfg = 0) */
    uint8_t* bits;   /* in: device buffer for the n_cfg decisions, or NULL */
    int32_t* steps;  /* in: device buffer for the n_cfg step counts, or NULL */
    float* hit;      /* in: device buffer for the n_cfg first-hit probabilities, or NULL */
} perc_pi_out;

/* Sample configurations 0 .. n_cfg-1 of the Philox stream `seed` at probability p
 * (as perc_sample) and inspect them. Synchronous: returns after n_perc and pi are
 * known; the device buffers in `out` are complete on return. */
int perc_pi(const perc_lattice* lat, double p, int64_t n_cfg, uint64_t seed, perc_pi_out* out, void* stream);
int perc_pi_ex(const perc_lattice* lat, double p, int64_t n_cfg, uint64_t seed, perc_pi_out* out,
               const perc_options* opt, void* stream);

/* ---- batches of uneven shapes ------------------------------------------------------- */

/* One configuration of a batch. Either occ_bits (device, canonical words of `lat`) or,
 * when occ_bits is NULL, the Philox draw (p, seed, cfg) as in perc_sample. `group`
 * selects the Pi count it adds to (0 .. n_groups-1), or -1 for none. */
typedef struct perc_job {
    const perc_lattice* lat;
    const uint32_t* occ_bits;
    double p;
    uint64_t seed;
    int64_t cfg;
    int32_t group;
} perc_job;

/* Inspect n_jobs configurations of possibly different lattices in one batch (one
 * persistent launch, or one span launch per step over every job). perc (device,
 * n_jobs bytes), steps and hit (device, n_jobs entries, may be NULL) are indexed by job.
 * group_count (host, n_groups int64) receives the number of percolating jobs of each
 * group; the call is synchronous when n_groups > 0, else async. The batch runs in the
 * form `opt` names (NULL = automatic): the span form in waves of consecutive jobs that
 * fit the work-memory budget (one wave when the whole batch fits), the persistent form
 * handing out the largest fibers first and, among equal ones, the highest p first (the
 * longest expected inspections). */
int perc_batch(const perc_job* jobs, int64_t n_jobs, uint8_t* perc, int32_t* steps, float* hit,
               int64_t* group_count, int32_t n_groups, const perc_options* opt, void* stream);

/* ---- test hook ------------------------------------------------------------------ */

/* Exactly K >= 0 forward steps of one configuration (occ_bits: device, words uint32)
 * with no early exit. x_out (device, N+1 floats): the probability of each tube after K
 * steps in canonical order (0 at insulating tubes), then the detector's accumulated
 * probability. reach_out (device, N+1 bytes): 1 where the probability is non-zero in
 * exact arithmetic (the reached set), then the detector. Async. */
int perc_state_after(const perc_lattice* lat, const uint32_t* occ_bits, int32_t K, float* x_out,
                     uint8_t* reach_out, void* stream);

/* ---- first-passage outputs (Sec. II.B, Eq. 3; Sec. III) ------------------------- */

/* First-passage probabilities from every tube at once: the backward form of Eq. 3, in
 * which the vector runs from the detector towards the sources. f_out (device, N floats,
 * canonical order) receives, for each tube i, the probability that a walk started on i
 * enters the detector for the first time at move M >= 1: f^(1)_i = 1/deg_i on metallic
 * far-end tubes (0 elsewhere), f^(m)_i = (1/deg_i) sum over metallic contacts k of
 * f^(m-1)_k (a metallic tube of degree 0 keeps its value; insulating tubes hold 0). The
 * forward first-hit probability of the inspection at step m equals the mean of f^(m)
 * over the metallic start tubes. FP32 with the step kernel's fixed summation order;
 * values the exact recursion makes zero may read as denormals up to about M * 2^-149
 * (the kernel keeps every word that was once non-zero at least 2^-149). occ_bits:
 * device, words uint32, canonical order. Work memory is taken from and returned to the
 * stream-ordered pool of `stream`. Async. Errors: PERC_EINVAL for M < 1 or NULL
 * pointers, PERC_ENOMEM, PERC_EHIP. */
int perc_first_passage(const perc_lattice* lat, const uint32_t* occ_bits, int32_t M, float* f_out, void* stream);

/* perc_first_passage for n_cfg configurations of one lattice at once (occ_bits: device,
 * n_cfg x words; f_out: device, n_cfg x N floats, configuration i at i * N): every move
 * is one launch over all of them. Results equal perc_first_passage's bit for bit. The
 * call returns after its set-up copies; the computation is async on `stream`. Errors:
 * as perc_first_passage, and PERC_EINVAL for n_cfg outside [0, 2^20]. */
int perc_first_passage_batch(const perc_lattice* lat, const uint32_t* occ_bits, int64_t n_cfg, int32_t M,
                             float* f_out, void* stream);

/* Histogram of the stop step m* (Sec. III: the first step with a non-zero detector
 * probability is the length of the shortest spanning path, m* tubes) over the
 * percolating configurations of an inspection: hist[min(m*, nbins - 1)] += 1 for every
 * i < n with perc[i] == 1. perc (device, n bytes), steps (device, n int32) as written by
 * perc_inspect / perc_batch; hist: device, nbins uint64, accumulated into (the caller
 * zeroes it). Async. Errors: PERC_EINVAL for n < 0, nbins < 1 or NULL pointers,
 * PERC_EHIP. */
int perc_steps_hist(const uint8_t* perc, const int32_t* steps, int64_t n, int32_t nbins, uint64_t* hist,
                    void* stream);

/* ---- profiling of the step kernel (span and plain forms) ------------------------- */

typedef struct perc_profile {
    int64_t step_launches;      /* step-kernel launches timed */
    double step_ms;             /* sum of their durations (HIP events on the launching stream) */
    int64_t tube_steps;         /* tube slots those launches advanced by one step */
    int64_t persist_launches;   /* the persistent launches among them */
    double persist_ms;          /* their part of step_ms */
    int64_t persist_tube_steps; /* their part of tube_steps */
} perc_profile;

/* Process-wide switch; resets the counters. While on, the span form and the server's
 * ticks launch their steps directly (HIP reports no elapsed time for events recorded as
 * graph nodes) with an event pair around each step launch, or around each pair of step
 * launches that run back to back between two plans (counted as two launches), on the
 * caller's (server's) stream, and count the tube slots the planner schedules; the
 * persistent form times its one persistent launch (initialisation and finishing
 * included, so its rate is a lower bound; sampling is a launch of its own) and counts
 * the tube slots of its steps, and runs synchronously (the two parts of a mixed batch
 * then run one after the other). */
int perc_profile_enable(int32_t on);
int perc_profile_read(perc_profile* out);

/* ---- measurement: the HBM ceiling ------------------------------------------------- */
/* Copy `bytes` (a multiple of 16; src and dst device, 16-byte aligned, not overlapping)
 * with the step kernels' memory access pattern and none of their arithmetic: `grid`
 * workgroups of 512 threads (0: the span step's 4096), each copying one contiguous chunk
 * with 16-byte loads and non-temporal 16-byte stores. Timing it gives the practical
 * read+write bandwidth the step kernels' HBM traffic is compared with. Async. */
int perc_stream_copy(const void* src, void* dst, int64_t bytes, int32_t grid, void* stream);

/* ---- work memory ----------------------------------------------------------------- */
/* Release the work buffers the library keeps on the current device (waiting for the work
 * of their last borrowers first). PERC_EBUSY if a call is using one; the next call that
 * needs large work memory allocates it again. */
int perc_trim(void);

/* ---- autotuning of the execution settings -------------------------------------- */
/* Time candidate settings (span form with 32/64/80/128 cells per work item and one or two
 * block sizes, persistent form with 64/128/256, the two-step forms where the shapes allow
 * them, the mixed form with 64/80 cells per span item when the sample holds fibers of both
 * kinds) on the sample `jobs` (as perc_batch; group must be -1; a sample spread over the
 * batch's p values and shapes represents it best) and return the fastest in *best (wall
 * time of the whole sample, ms, in *best_ms; either may be NULL). If every job has the
 * same (W, L), the choice is also
 * remembered for PERC_FORM_AUTO calls on that shape with a batch of about n_target
 * configurations (n_target <= 0: the sample size). Synchronous; the outputs of the
 * timing runs are discarded. */
int perc_autotune(const perc_job* jobs, int64_t n_jobs, int64_t n_target, perc_options* best, double* best_ms,
                  void* stream);

/* ---- serving: continuous batching of single inspections -------------------------- */
/* A server keeps the state of every admitted inspection resident on the GPU and advances
 * all of them together, a tick at a time; requests that arrive meanwhile wait in a FIFO
 * queue and are admitted at the next tick as a slot and HBM (the pool below) free up.
 * A request is one configuration: fiber (W, L), metallic probability p, the Philox
 * configuration cfg of stream seed (the same draw as perc_pi_ex's configuration cfg and
 * perc_batch's Philox jobs), so its result is bitwise the result of inspecting that
 * configuration alone (Sec. II.B method, outputs as perc_inspect_ex). */
typedef struct perc_server perc_server;

typedef struct perc_server_config {
    int64_t hbm_bytes;   /* device pool for resident state (0: half the free memory, <= 64 GiB) */
    int32_t max_slots;   /* inspections in flight at once (0: 1024) */
    int32_t tick_steps;  /* iteration steps per tick (0: 16) */
    int32_t max_w;       /* widest fiber accepted (0: 64; at most 128) */
    int32_t host_only;   /* 1: no GPU work, every admitted request completes at the next
                            tick with status PERC_OK and zero outputs (scheduler tests) */
    perc_options opt;    /* item length (depth), block, grid of the step launches */
    int32_t max_queue;   /* requests that may wait at once (0: 2^20); a submit beyond it
                            is refused with PERC_EBUSY (load shedding) */
    int32_t lookahead;   /* admission: 0 = strict FIFO (a request that does not fit waits,
                            and so do the ones behind it); k > 0 = the first k requests
                            behind a waiting head may be admitted past it when they fit */
} perc_server_config;

typedef struct perc_result {
    uint64_t tag;        /* the caller's request id */
    int32_t W, L;
    double p;
    uint64_t seed, cfg;
    int32_t status;      /* PERC_OK; PERC_ECAP if the step cap was reached; PERC_ECANCELED
                            (perc_server_cancel); PERC_EBUSY (refused by perc_server_run's
                            submit: queue full) */
    uint8_t perc;        /* percolates */
    int32_t steps;       /* as perc_inspect */
    float hit;           /* first-hit probability at the stop (0 if not percolating) */
    int64_t t_arrive_ns, t_admit_ns, t_done_ns;  /* host steady clock */
} perc_result;

typedef struct perc_server_stats {
    int64_t queued, in_flight, completed, ticks;
    int64_t pool_bytes, pool_used_bytes;
    int64_t rejected;    /* submits refused with PERC_EBUSY */
    int64_t cancelled;   /* requests retired with PERC_ECANCELED */
} perc_server_stats;

/* Create a server on the current device, working on `stream` (hipStream_t or NULL); the
 * server owns its device memory (allocated here, freed by destroy). NULL on failure
 * (see perc_last_error). */
perc_server* perc_server_create(const perc_server_config* cfg, void* stream);
void perc_server_destroy(perc_server* srv);

/* Queue one request; t_arrive_ns < 0 stamps the current steady-clock time. PERC_EINVAL
 * for W outside [0, max_w], L outside [1, 65535] or p outside [0, 1]; PERC_EBUSY (not
 * queued) when max_queue requests already wait, or when the request's resident state
 * exceeds the whole pool (it could never be admitted). */
int perc_server_submit(perc_server* srv, int32_t W, int32_t L, double p, uint64_t seed, uint64_t cfg, uint64_t tag,
                       int64_t t_arrive_ns);

/* Cancel every request with this tag: a waiting one leaves the queue at once, one in
 * flight stops at the next tick (its slot and pool room are freed then). Each cancelled
 * request is retired with status PERC_ECANCELED and zero outputs (poll returns it).
 * Returns the number of requests cancelled (>= 0; 0 if none had the tag, or all had
 * already finished). */
int perc_server_cancel(perc_server* srv, uint64_t tag);

/* One tick: admit queued requests (in queue order, as lookahead allows, while a slot and
 * pool room are free), sample and initialise them, advance every resident inspection by
 * tick_steps steps, retire the finished and the cancelled ones. Returns the number
 * retired (>= 0) or an error. Synchronous. */
int perc_server_tick(perc_server* srv);

/* Move up to max finished results (retirement order) into out; returns the count. */
int perc_server_poll(perc_server* srv, perc_result* out, int32_t max);
int perc_server_stats_read(const perc_server* srv, perc_server_stats* out);

/* Serve a whole request stream natively: request i arrives t_arrive_ns[i] after the
 * start (non-decreasing); the loop submits arrivals as their time comes, ticks while
 * anything is queued or in flight, sleeps otherwise, and writes the n results (in
 * retirement order, t_arrive_ns on the same clock as t_done_ns) to out. A request the
 * queue refuses (PERC_EBUSY at submit) gets a result with that status at once. */
typedef struct perc_request {
    int64_t t_arrive_ns;
    int32_t W, L;
    double p;
    uint64_t seed, cfg, tag;
} perc_request;
int perc_server_run(perc_server* srv, const perc_request* reqs, int64_t n, perc_result* out);

#ifdef __cplusplus
}
#endif

#endif /* PERC_H */
