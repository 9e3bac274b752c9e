/*
 * tnc.h - exact output amplitudes of open-boundary 1D brickwork circuits by
 * the deterministic temporal-boundary tensor-network contraction, on one
 * AMD Instinct MI355X (gfx950).  C ABI; no C++ or framework types cross it.
 *
 * Method (arXiv 2608.13110):
 *   - circuit family: n qubits on an open chain, d layers of nearest-
 *     neighbour entanglers alternating between the pairs (1,2),(3,4),... and
 *     (2,3),(4,5),... (1-based), a layer of one-qubit gates (any 2x2)
 *     around each of them, d + 1 in all (Sec. 2.1); every entangler must have operator
 *     Schmidt rank <= 2 (Sec. 2.1, the operator-Schmidt-rank equation);
 *   - the amplitude psi(x) = <x|U|0^n> (Sec. 2.2) is contracted by the
 *     unsliced sweep of Alg. 1 (Sec. 3.1), width ceil(d/2) (Prop.
 *     constructive-memory); with k open output legs the batch
 *     Z[b] = <a, b|U|0^n> over the last k qubits is contracted by Alg. 2
 *     (Sec. 4.3) at the same width for 1 <= k <= floor(d/4) (Prop. batched
 *     width).
 *
 * Conventions (0-based): qubit j is row j of the chain.  A bitstring is n
 * bytes, byte j = output value (0/1) of qubit j.  For k open legs the batch
 * output index is b = sum_j x_{n-k+j} * 2^(k-1-j), i.e. the last k qubits
 * read most-significant first, so (a, b) read MSB-first is the full index.
 * one-qubit layer l (0..d) acts after entangling layer l; its gate on qubit q
 * is one_qubit[(l*n + q)*4 + 2*row + col] (row = output, col = input).
 *
 * Errors: every entry point returns TNC_OK (0) or a negative status and never
 * throws; tnc_last_error() gives a message for the calling thread.
 *
 * Threading: a plan is immutable once built (schedules for each k and the
 * device tables are created lazily under a lock).  Calls of
 * tnc_amplitudes on different streams with different workspaces may overlap.
 */
#ifndef TNC_H
#define TNC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tnc_plan_s* tnc_plan_t;

typedef struct {
  double re, im;
} tnc_c128;

#define TNC_OK 0
#define TNC_E_INVALID (-1)   /* malformed input (bad pattern, pointer, size) */
#define TNC_E_DOMAIN (-2)    /* outside the supported range (k, n, d, width) */
#define TNC_E_RANK (-3)      /* an entangler has operator Schmidt rank > 2 */
#define TNC_E_NOMEM (-4)     /* workspace too small or device allocation failed */
#define TNC_E_DEVICE (-5)    /* a HIP call failed */

#define TNC_GATE_CZ 0     /* diag(1, 1, 1, -1); m ignored */
#define TNC_GATE_DENSE4 1 /* m: 4x4 row-major [out][in], basis 2*x_q + x_{q+1} */

/* Storage of the boundary tensor in HBM.  The updates always compute in
 * complex FP32; the 16-bit modes store each entry as two FP16 or BF16 halves
 * (re, im) of the entry divided by its block's FP32 power-of-two scale, with
 * one scale per block of 4096 entries written together by one tile (fewer in
 * tiles below 2^12 entries); the scale puts the block's largest component
 * in [2^14, 2^15).  This halves the bytes each pass moves, at a precision the
 * format sets (about 2^-11 relative per store for FP16, 2^-8 for BF16, for
 * entries near their block's maximum).  The join and the late phase read the
 * decoded values in FP64 as in the complex64 mode. */
#define TNC_STORE_C64 0             /* complex64 (8 bytes per entry) */
#define TNC_STORE_F16_BLOCKSCALE 1  /* 2 x FP16 + FP32 scale per block (about 4 bytes per entry) */
#define TNC_STORE_BF16_BLOCKSCALE 2 /* 2 x BF16 + FP32 scale per block */

/* One two-qubit gate of entangling layer `layer` (1..d) on qubits (q, q+1). */
typedef struct {
  int32_t layer;
  int32_t q;
  int32_t kind;
  int32_t reserved;
  tnc_c128 m[16];
} tnc_gate2;

/* Tiling options of the pass kernels; zero fields take the defaults. */
typedef struct {
  int32_t max_tile_bits; /* entries per pass tile = 2^max_tile_bits (default 13, 6..14) */
  int32_t reg_bits;      /* entries per thread = 2^reg_bits (default 5, 1..5); at most 512
                            threads per tile: max_tile_bits - reg_bits <= 9 */
  int32_t low_bits;      /* contiguous low slots in every non-bottom tile (default 4):
                            HBM runs of 2^low_bits * 8 bytes */
  int32_t math;          /* 0: vector-ALU updates (default); 2: runs of three updates without
                            output-bit variants fused into one complex 8x8 per control value,
                            on v_mfma_f32_16x16x4f32 (tiles of 64 threads or more); two of the
                            three targets sit in lane bits, so such a phase carries up to
                            reg_bits + 2 updates.  Other values: TNC_E_INVALID */
  int32_t late_fold;     /* k >= 1: late removals folded on the host into the join launch
                            (0: automatic, 7 for boundary tensors of 2^35 entries, 5 for
                            2^30 or more, 3 for 2^26 or more, else none; -1: none; 1..8:
                            that many; the host fold costs O(2^(3k + late_fold))) */
  int32_t reg_adapt;     /* 1: a pass takes reg_bits - 1 when that needs no more register
                            phases and its tile fits 256 threads (more resident waves);
                            0: every pass uses reg_bits (default) */
  int32_t bond;          /* bond dimension of the lowering (Sec. 6.2, Effect of bond dimension):
                            0 (default) the smallest that holds every entangler: 2 when all have
                            operator Schmidt rank <= 2, else 4; 2: rank > 2 is TNC_E_RANK; 4: two
                            legs per crossing for every entangler.  Bond 4 needs even d, gives a
                            boundary tensor of d - 1 slots (the width min(n, d-1) for n >= d-1)
                            updated by dense 4x4s, and k = 0 only (TNC_E_DOMAIN otherwise) */
  int32_t reserved;
  uint64_t mem_cap_bytes; /* device memory the plan may use per call, 0: no cap.  A batch whose
                             workspace exceeds it: TNC_E_NOMEM (tnc_workspace_bytes,
                             tnc_amplitudes, tnc_amplitudes_host).  tnc_amplitudes uses at most the
                             cap of the caller's workspace and tnc_amplitudes_host allocates at
                             most the cap; the batches then run in groups that fit */
} tnc_options;

typedef struct {
  int32_t width;              /* W(P): log2 of the largest intermediate (Sec. 2.2) */
  int32_t boundary_bits;      /* h = max crossings of a cut: device tensor has 2^h entries */
  int32_t live_slots_fixed;   /* legs of the boundary tensor after the fixed rows */
  int32_t n_ops;              /* boundary updates in the fixed sweep */
  int32_t n_passes;           /* HBM passes of the fixed sweep */
  int32_t n_phases;           /* register phases over all passes */
  int32_t n_late_launches;    /* device launches of the late phase */
  int32_t fixed_rows;         /* rows contracted by the sweep (Alg. 2: q_1..q_{n-k}) */
  int32_t early_layers;       /* c = 2k entangling layers in the early region */
  int32_t late_layers;        /* d - c layers absorbed after the join */
  double log2_cost;           /* log2 C(P), C = sum |I||J||K| (Sec. 2.2) */
  uint64_t workspace_per_batch; /* device bytes per concurrent batch (0: width above 40, planned only) */
  int32_t bond;               /* bond dimension of the lowering (2 or 4) */
  int32_t reserved;
} tnc_info;

/*
 * Build a plan for an n-qubit, d-layer circuit.
 *   one_qubit: (d+1)*n*4 entries (see Conventions); copied.
 *   gates:     n_gate2 gates; each must belong to its layer's brickwork
 *              pattern (patterns alternate; the first gate fixes the parity;
 *              with no gates layer 1 uses the 1-based pairs (2,3),(4,5),...).
 *              Pattern pairs without a gate are identity.  Copied.
 *   opt:       may be NULL.
 * Host only: no device memory is touched.  Returns TNC_OK and *out, or
 * TNC_E_INVALID / TNC_E_DOMAIN (n < 2, d < 2, a bond-two width above 40, a
 * bond-four width above 69, bond four at odd d with n > d) / TNC_E_RANK (an
 * entangler of rank > 2 with opt->bond = 2).  Bond-four plans of width 41..69
 * are planned only (tnc_plan_info; the amplitude calls return TNC_E_DOMAIN).
 */
int tnc_plan(int32_t n, int32_t d, const tnc_c128* one_qubit, int32_t n_gate2, const tnc_gate2* gates,
             const tnc_options* opt, tnc_plan_t* out);

/* Path metrics and launch counts for k open legs (0 <= k <= min(n-1, 10), 2k <= d). */
int tnc_plan_info(tnc_plan_t plan, int32_t k, tnc_info* info);

/*
 * Build and upload the device tables for k open legs on the current HIP
 * device (synchronous).  tnc_amplitudes does this on first use; call it
 * beforehand when the launches will be captured into a HIP graph.
 */
int tnc_prepare(tnc_plan_t plan, int32_t k);

/* Device workspace needed to run n_batches batches at once with storage mode
 * `storage` (TNC_STORE_*): per batch the tensor (8 or 4 bytes per entry),
 * for the 16-bit modes two arrays of block scales, and the late-phase
 * buffers.  The 16-bit modes need low_bits >= 2 (TNC_E_INVALID otherwise). */
int tnc_workspace_bytes(tnc_plan_t plan, int32_t k, int32_t n_batches, int32_t storage, uint64_t* bytes);

/*
 * Exact amplitude batches on the device, enqueued on `stream` (asynchronous).
 *   d_bits:   device, n_batches*n bytes; the last k bits of each are ignored.
 *   d_out:    device, n_batches * 2^k amplitudes (index b above), FP64.
 *   d_workspace / workspace_bytes: device scratch owned by the caller; when
 *             it holds fewer than n_batches batches (tnc_workspace_bytes),
 *             the batches run in consecutive groups.  At least one batch must
 *             fit (else TNC_E_NOMEM).
 *   stream:   hipStream_t (NULL = default stream).
 * Arithmetic: boundary updates in complex FP32; the row-0 build-up, the join
 * and all later reductions in FP64.
 */
int tnc_amplitudes(tnc_plan_t plan, int32_t n_batches, const uint8_t* d_bits, int32_t k, int32_t storage,
                   tnc_c128* d_out, void* d_workspace, uint64_t workspace_bytes, void* stream);

/*
 * tnc_amplitudes for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same launches, with the workspace taken from a scratch array that the
 * library holds on each GPU (tnc_noalloc_scratch_bytes() bytes, 256 MiB:
 * one batch up to about 2^22 boundary entries with k >= 1) until the process
 * ends.  No hipMalloc, hipFree or other allocating call is made.
 *   d_bits, d_out, stream: as for tnc_amplitudes (caller-owned device memory).
 *   The device tables for k must already be on the current device
 *   (tnc_prepare, or an earlier tnc_amplitudes call): TNC_E_INVALID otherwise.
 *   A batch whose workspace exceeds the scratch: TNC_E_NOMEM.  Batches that
 *   fit together run in groups, as with a small workspace.
 * Every call on one GPU shares that GPU's scratch, so calls that overlap on
 * one GPU (different streams or threads) race; calls in one stream do not.
 * Nothing in the scratch is read before this call writes it.
 */
int tnc_amplitudes_noalloc(tnc_plan_t plan, int32_t n_batches, const uint8_t* d_bits, int32_t k, int32_t storage,
                           tnc_c128* d_out, void* stream);
/* Size of the per-GPU scratch of tnc_amplitudes_noalloc, in bytes. */
uint64_t tnc_noalloc_scratch_bytes(void);

/* Same with host buffers: allocates device memory, runs, synchronizes. */
int tnc_amplitudes_host(tnc_plan_t plan, int32_t n_batches, const uint8_t* bits, int32_t k, int32_t storage,
                        tnc_c128* out);

/*
 * log-XEB of Sec. 5.2 (Eq. normalized-log-xeb) in FP64 on the device:
 *   F = gamma + n ln 2 + (1/N) sum_i ln |amp_i|^2,  SE = sd / sqrt(N).
 *   d_amp:    device, n_batches * 2^k amplitudes.
 *   d_select: device, n_batches indices b (one component per batch), or NULL
 *             to use every component.
 *   d_result: device, 5 doubles {F, SE, F - 1.96 SE, F + 1.96 SE, N}.
 */
int tnc_logxeb(const tnc_c128* d_amp, int32_t n_batches, int32_t k, const int32_t* d_select, int32_t n_qubits,
               double* d_result, void* stream);

/*
 * Batched sampling, Sec. 4.2 (steps 3-4 of the batched sampler): for each
 * batch (one prefix a, its 2^k amplitudes from tnc_amplitudes) the
 * probabilities p(a, b) = |Z[b]|^2 and Q_a = sum_b p(a, b) in FP64, and one
 * suffix b drawn from p(b | a) = p(a, b) / Q_a: the smallest b whose prefix
 * sum p(a, 0) + ... + p(a, b) exceeds u Q_a (2^k - 1 if rounding leaves
 * none).  The prefix a itself is the caller's uniform draw.
 *   d_amp: device, n_batches * 2^k amplitudes (index b as in tnc_amplitudes).
 *   d_u:   device, n_batches uniforms in [0, 1) (the caller's random numbers).
 *   d_b:   device, n_batches sampled suffixes (out).
 *   d_q:   device, n_batches marginals Q_a (out).
 *   0 <= k <= 10; n_batches = 0 does nothing.  Asynchronous on `stream`.
 */
int tnc_sample_batched(const tnc_c128* d_amp, int32_t n_batches, int32_t k, const double* d_u, int32_t* d_b,
                       double* d_q, void* stream);

/*
 * Frugal rejection, Sec. 4.1 (steps 2-3): for each candidate amplitude,
 * z = 2^n |amp|^2 and acceptance when u < min(1, z / M).  Candidates are the
 * caller's uniform draws (their amplitudes from tnc_amplitudes with k = 0, or
 * the entries of batches).
 *   d_amp:    device, count amplitudes.
 *   d_u:      device, count uniforms in [0, 1).
 *   d_accept: device, count bytes, 1 = accepted (out).
 *   d_z:      device, count rescaled probabilities z (out).
 *   1 <= n_qubits <= 1000; M > 0 finite.  Asynchronous on `stream`.
 */
int tnc_frugal_accept(const tnc_c128* d_amp, int64_t count, int32_t n_qubits, double M, const double* d_u,
                      uint8_t* d_accept, double* d_z, void* stream);

/*
 * Ring geometry by structure-aware slicing (Sec. 6.3).  Gates as in tnc_plan,
 * plus CZ gates listed at q = n-1, which act on the wrap pair (n-1, 0); in
 * their layers qubits n-1 and 0 must be idle in the chain pattern.  Each
 * wrap CZ is cut as sum_a P_a (x) Z^a (P_a = |a><a| on qubit n-1, Z^a on
 * qubit 0, both folded into the one-qubit layer that follows); each of the
 * 2^m assignments of the m cut bonds is an open-chain plan of width
 * ceil(d/2), and the ring's amplitudes are the sum over all slices.
 *   m <= 12 (else TNC_E_DOMAIN); wrap gates other than CZ: TNC_E_INVALID.
 * The ring plan owns its 2^m slice plans until tnc_ring_release.
 */
typedef struct tnc_ring_plan_s* tnc_ring_plan_t;
int tnc_plan_ring(int32_t n, int32_t d, const tnc_c128* one_qubit, int32_t n_gate2, const tnc_gate2* gates,
                  const tnc_options* opt, tnc_ring_plan_t* out);
/* Slice count, width of each slice, and device workspace for n_batches
 * batches (a group of slices run together: their workspaces, results and
 * launch segment tables; host only). */
int tnc_ring_info(tnc_ring_plan_t ring, int32_t k, int32_t n_batches, int32_t* n_slices, int32_t* width,
                  uint64_t* workspace_bytes);
/* Ring amplitudes, with the arguments of tnc_amplitudes (complex64 storage):
 * the slices run in groups of up to 1024 on `stream` (the i-th launches of a
 * group's slices as one grouped launch), their results added to d_out in
 * slice order in FP64.  The workspace must hold what tnc_ring_info reports.
 * The ring plan's pinned staging is reused call to call: one thread at a
 * time per ring plan. */
int tnc_ring_amplitudes(tnc_ring_plan_t ring, int32_t n_batches, const uint8_t* d_bits, int32_t k, tnc_c128* d_out,
                        void* d_workspace, uint64_t workspace_bytes, void* stream);
/* Host emulation of every slice (tnc_debug_emulate_device) summed on the
 * host: a CPU check of the slicing. */
int tnc_debug_ring_emulate(tnc_ring_plan_t ring, int32_t n_batches, const uint8_t* bits, int32_t k, tnc_c128* out);
/* NULL-safe. */
void tnc_ring_release(tnc_ring_plan_t ring);

/*
 * Kernel timing with HIP events recorded on the launch stream around every
 * launch of tnc_amplitudes while profiling is on (process-wide).
 * tnc_profile_end waits for the recorded events and returns the summed
 * durations per kernel class (row-0 build-up, sweep passes, late phase).
 */
typedef struct {
  double init_ms;
  double pass_ms;
  double late_ms;
  int64_t init_launches;
  int64_t pass_launches;
  int64_t late_launches;
  double pass_bytes;  /* algorithmic bytes of the passes: 2 * 2^h * 8 per batch and pass */
} tnc_profile;

int tnc_profile_begin(void);
int tnc_profile_end(tnc_profile* out);
/* The launches timed by the last tnc_profile_end, in issue order: class
 * (0 build-up / variant resolution, 1 pass, 2 late phase) and duration in
 * ms; *n = their number, at most cap are written. */
int tnc_profile_launches(int32_t* cls, double* ms, int64_t cap, int64_t* n);

/* The HBM passes of the fixed sweep for k open legs, in launch order: seven
 * int32 per pass, {low slots, window start, window length, register bits,
 * updates, register phases, fused phases}; *n_passes = their number, at most
 * cap are written.  Host only. */
int tnc_plan_passes(tnc_plan_t plan, int32_t k, int32_t* out, int32_t cap, int32_t* n_passes);

/*
 * Tile autotuner.  Times each candidate tile option set on the current
 * device for an n-qubit, d-layer brickwork CZ circuit with seeded random
 * one-qubit unitaries (width and pass structure depend only on n, d and k,
 * never on the gate values: the invariance of width and cost stated in Sec. 1 and Sec. 7) and
 * reports the fastest.
 *   candidates: n_candidates option sets (NULL entries not allowed);
 *   reps:       timed batches per candidate (after one untimed warm-up);
 *   times_ms:   n_candidates doubles, median time per batch of each
 *               candidate (infinity for a candidate the library rejects);
 *   best:       index of the fastest candidate.
 * Allocates its own device memory (one batch of workspace); synchronous.
 */
int tnc_autotune(int32_t n, int32_t d, int32_t k, int32_t storage, const tnc_options* candidates,
                 int32_t n_candidates, int32_t reps, int32_t* best, double* times_ms);

/*
 * Serving: a continuous-batching request loop on the current device
 * (batches of one circuit share its plan: Sec. 5.2).  Requests of any shape
 * are submitted at any time from any thread; planner threads build (or find
 * in the plan cache, keyed by the circuit's contents) the plan and upload
 * its tables; the dispatcher admits a prepared request as soon as one of
 * n_streams HIP streams is free and the device arena has room for its
 * footprint (workspace + bits + output), oldest first, letting younger
 * requests that fit pass an older one that does not at most 16 times.
 * Small requests (boundary tensor of <= small_bits bits) run together: the
 * ready complex64 requests of the admitted one's width (up to max_group)
 * form a group whose launches are merged, launch by launch, into grouped
 * launches of one kernel each (one segment per member).  A small request
 * whose (plan, k, batches, storage) has been served before runs as a cached
 * HIP graph, built node by node from its launches (never by stream capture),
 * which owns its device region (within a quarter of the arena) and is
 * replayed, from any stream, while idle.  No stream is ever put in capture
 * mode, so other threads may use the device freely meanwhile.
 * Results are bit-identical to tnc_amplitudes with the same plan options.
 */
typedef struct tnc_server_s* tnc_server_t;

typedef struct {
  uint64_t arena_bytes;  /* device memory reserved at creation for all requests (> 0) */
  int32_t n_streams;     /* concurrent requests or groups on the device (default 4, at most 16) */
  int32_t n_planners;    /* planner threads (default 4, at most 16) */
  int32_t small_bits;    /* grouped / graph-replayed requests: boundary bits <= small_bits (0: none, at most 24) */
  int32_t max_graphs;    /* cached graph executables (default 256) */
  int32_t max_group;     /* requests per group (default 16, at most 256; 1: never group) */
  int32_t group_window_us; /* a ready small complex64 request waits up to this long for max_group
                            requests of its width to be ready (default 0: no wait) */
  int32_t reserved[2];
} tnc_server_options;

typedef struct {
  double plan_ms;        /* submit -> plan ready (planning, table upload) */
  double queue_ms;       /* submit -> admitted to a stream */
  double run_ms;         /* admitted -> results copied back */
  double total_ms;       /* submit -> done */
  int32_t boundary_bits;
  int32_t mode;          /* 0: its own launches; 1: a cached graph; 2: in a group */
} tnc_request_stats;

typedef struct {
  int64_t completed;
  int64_t graph_launches, graph_builds, graph_failures, plain_launches;
  int64_t groups, grouped_requests, grouped_launches;  /* groups of >= 2 requests; their merged launches */
  int64_t plan_cache_hits, plan_cache_misses;
  int32_t max_inflight;  /* most requests seen running at once */
  int32_t reserved;
  double latency_ms_p50, latency_ms_p99, latency_ms_max;  /* submit -> done */
  double elapsed_s;      /* first submit -> last completion */
} tnc_server_stats;

/* Create / destroy (destroy finishes every submitted request first). */
int tnc_server_create(const tnc_server_options* opt, tnc_server_t* out);
void tnc_server_destroy(tnc_server_t server);

/* Tile options for plans whose width (boundary bits) is boundary_bits
 * (unset widths use the defaults); applies to plans built afterwards. */
int tnc_server_set_tuning(tnc_server_t server, int32_t boundary_bits, const tnc_options* opt);

/*
 * Submit one request (asynchronous).  The circuit arguments are as for
 * tnc_plan, bits as for tnc_amplitudes_host (host, n_batches*n bytes); both
 * are copied.  `out` (host, n_batches * 2^k amplitudes) is written when the
 * request completes and must stay valid until tnc_server_wait returns.
 * *id identifies the request for tnc_server_wait.
 */
int tnc_server_submit(tnc_server_t server, int32_t n, int32_t d, const tnc_c128* one_qubit, int32_t n_gate2,
                      const tnc_gate2* gates, int32_t n_batches, const uint8_t* bits, int32_t k, int32_t storage,
                      tnc_c128* out, uint64_t* id);

/* Block until request `id` is done; returns its status and timings (stats
 * may be NULL).  Each id can be waited for once. */
int tnc_server_wait(tnc_server_t server, uint64_t id, tnc_request_stats* stats);

/* Counters and latency quantiles over every completed request. */
int tnc_server_summary(tnc_server_t server, tnc_server_stats* stats);

/* Free a plan and its device tables.  NULL is ignored. */
void tnc_release(tnc_plan_t plan);

const char* tnc_strerror(int code);
const char* tnc_last_error(void);

/*
 * Planner self-checks, host only, FP64 (tests; the device path never calls
 * them).  execute_host runs the plan's own update tables on the host;
 * emulate_device runs the device tables through a host emulation of the
 * pass kernel's thread / LDS mapping, with the given storage mode.
 * Width <= 24.
 */
int tnc_debug_execute_host(tnc_plan_t plan, int32_t n_batches, const uint8_t* bits, int32_t k, tnc_c128* out);
int tnc_debug_emulate_device(tnc_plan_t plan, int32_t n_batches, const uint8_t* bits, int32_t k, int32_t storage,
                             tnc_c128* out);

/*
 * Complex128 reference path (tests and the accuracy report; not tuned): the
 * same plan, with the boundary tensor in complex128 and every update of the
 * sweep applied in FP64 by its own launch (no fusion, no tiles), then the
 * same FP64 join and late phase.  The paper measures its complex64 runs
 * against complex128 ones by the TV of the conditional distributions
 * (Sec. 5.1).  Arguments as for tnc_amplitudes (complex64 storage modes do
 * not apply); the workspace holds the complex128 tensor and the late
 * buffers per batch (tnc_debug_workspace_c128), and the update tables are
 * uploaded on first use (synchronous).  Bond-dimension-2 plans only (a
 * bond-4 plan: TNC_E_DOMAIN).
 */
int tnc_debug_workspace_c128(tnc_plan_t plan, int32_t k, int32_t n_batches, uint64_t* bytes);
int tnc_debug_amplitudes_c128(tnc_plan_t plan, int32_t n_batches, const uint8_t* d_bits, int32_t k, tnc_c128* d_out,
                              void* d_workspace, uint64_t workspace_bytes, void* stream);

/* Planner self-check of the LDS placement: over every register phase of the
 * pass tables for k, stats[0] = phases, stats[1] = phases in which two of the
 * 16 lanes of a bank cycle (lanes 16 c .. 16 c + 15) meet the same slot
 * modulo 16, stats[2] = the same for 32-lane cycles modulo 32 (8-byte slots).
 * Host only. */
int tnc_debug_lds_conflicts(tnc_plan_t plan, int32_t k, int64_t* stats);

/* Host self-check of the serving loop's device-arena allocator: n_ops
 * seeded random allocations and releases, checked for overlap, bounds and
 * full coalescing at the end.  TNC_OK or TNC_E_INVALID (message says why). */
int tnc_debug_arena_check(uint64_t seed, int32_t n_ops);

#ifdef __cplusplus
}
#endif

#endif /* TNC_H */
