/*
 * greedy_code.h -- C ABI of the MI355X (gfx950) greedy code construction
 * library, libgreedy_code.so.
 *
 * The operation (Paliwal, Tiwary, Chaudhury, Gupta, "Generating Binary
 * Optimal Codes Using Heterogeneous Parallel Computing", arXiv:1507.05398,
 * section "Greedy Algorithms and Different Orderings"): order all 2^n vectors
 * of F_2^n, start from the zero vector and append each vector in turn to the
 * code C when its Hamming distance to every word already in C is at least d
 * (section "Hamming Distance": distance = popcount(a XOR b)).  The result is
 * the ordered list of accepted words; it is unique, and every entry point
 * returns it bit for bit, in acceptance order.
 *
 * Words are uint32 bit masks: coordinate x_1 (the leftmost character of the
 * paper's strings, e.g. "011") is bit n-1, x_n is bit 0.
 *
 * Orderings (section "Ordering Implementation"; the paper names them, the
 * definitions are fixed here; GC_BORDER is described with gc_problem):
 *   GC_LEX      position p holds the word with value p (Example 1's listing).
 *   GC_GRAY     binary-reflected Gray code, p XOR (p >> 1).
 *   GC_GRLEX    weight ascending; equal weights by increasing value.
 *   GC_GREVLEX  weight ascending; equal weights by the graded reverse
 *               lexicographic monomial order (Cox, Little, O'Shea): the word
 *               with a 1 at the lowest differing bit comes first.
 *
 * Error codes: every entry point returns GC_OK (0) or a negative code; the
 * thread-local message of the last failure is available from gc_last_error().
 * No C++ exception crosses this boundary.
 *
 * Threading: calls may run concurrently from different threads on different
 * streams; each call owns its device workspace.  A call does not return until
 * its work on the given stream has finished (the result codes depend on it).
 */
#ifndef GREEDY_CODE_H
#define GREEDY_CODE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { GC_LEX = 0, GC_GRAY = 1, GC_GRLEX = 2, GC_GREVLEX = 3, GC_BORDER = 4 };

enum {
    GC_OK = 0,
    GC_EINVAL = -1,    /* n outside [1,32], d < 1, unknown ordering, NULL pointer */
    GC_ECAPACITY = -2, /* more words than the capacity given; the count is set to
                          greedy_code_capacity(n, d) (host API) or the number of
                          words that fit (device API) */
    GC_EDEVICE = -3,   /* a HIP call failed; see gc_last_error() */
    GC_ENOMEM = -4,    /* device or host allocation failed */
    GC_ETIMEOUT = -5,  /* a bounded device-side wait expired (no forward progress) */
    GC_EBUSY = -6      /* server: the job has not finished yet */
};

/* Server job states (gc_server_poll). */
enum { GC_JOB_WAITING = 0,   /* submitted, waiting for device memory */
       GC_JOB_ADMITTED = 1,  /* published to the device queue */
       GC_JOB_DONE = 2,      /* finished; words resident in the arena */
       GC_JOB_FAILED = 3 };

/* Work counters of one call (optional output).  checks_* count executed
 * distance checks (candidate x codeword pairs) by the kernel phase that ran
 * them; they measure the device's total work, which includes speculation. */
typedef struct gc_stats {
    uint64_t count;           /* |C| */
    uint64_t windows;         /* candidate windows processed */
    uint64_t resolve_rounds;  /* deep-scan rounds over all windows */
    uint64_t survivors;       /* window candidates that passed the near screen */
    uint64_t checks_near;     /* near-screen checks executed */
    uint64_t checks_deep;     /* deep-scan checks executed */
    uint64_t checks_pairs;    /* in-window pair checks executed */
    float kernel_ms;          /* device time of the construction kernel */
    /* device time by phase (including the barrier that ends the phase):
     * near screen, survivor list + conflict pairs, resolve, deep scans */
    double near_ms, survivors_ms, resolve_ms, deep_ms;
} gc_stats;

/* Tuning knobs (optional input; zero fields take the built-in defaults). */
typedef struct gc_tuning {
    uint64_t near_depth;    /* newest code words screened before the in-window
                               resolve; 0 = default, UINT64_MAX = whole code */
    uint32_t target_survivors; /* window survivors aimed for (<= 1024) */
    uint32_t grid_blocks;   /* persistent workgroups; 0 = one per compute unit */
    uint32_t resolve_mode;  /* 0 = by ordering, 1 = tentative (deep-scan only the
                               tentatively accepted survivors, repeat until
                               stable), 2 = deep-scan every survivor once */
    uint32_t deep_tile;     /* candidates per tile of the deep scan: 256, 512 or
                               1024 (0 = 1024).  The workgroups of a tile sweep
                               the old code together, newest first; smaller
                               tiles mean fewer workgroups per sweep, so a
                               candidate killed deep is dropped sooner. */
    uint32_t valu_screen;   /* 0 = distance screens on the matrix cores (bits as
                               signed bytes, one int8 matrix product per 32
                               words x 32 candidates); 1 = popcounts of XORs
                               on the vector ALU.  Self-orthogonal screens
                               always use the vector ALU. */
} gc_tuning;

/* Capacity (in words) that always suffices for (n, d): the sphere-packing
 * bound 2^n / V(n, floor((d-1)/2)), using A(n, d) = A(n-1, d-1) for even d
 * (every code of minimum distance d has at most this many words; the greedy
 * code is one).  2^n for d <= 1, 1 for d > n.  Returns 0 for invalid n, d. */
uint64_t greedy_code_capacity(int n, int d);

/* Host-memory entry point.  out_words: caller-owned host array; *out_count on
 * input is its capacity in words, on return the code size |C|.  The words
 * are written in acceptance order.  Allocates and frees its own device memory
 * and runs on the null stream.  GC_ECAPACITY: *out_count set to
 * greedy_code_capacity(n, d), out_words contents unspecified. */
int greedy_code(int n, int d, int ordering, uint32_t *out_words, uint64_t *out_count);

/* Device-memory entry point: the words go to d_words (device array of
 * `capacity` uint32, caller-owned, e.g. a torch tensor's data_ptr), the count
 * to *d_count (one device uint64), both written on `hip_stream` (a
 * hipStream_t, NULL = null stream).  The call uses a device workspace of
 * about 154 KiB from a pool the library keeps per device (allocated with
 * hipMalloc the first time a call needs one, reused by later calls, held
 * until the process ends; concurrent calls get distinct workspaces).
 * GC_ECAPACITY: the first `capacity` words and *d_count = capacity. */
int greedy_code_device(int n, int d, int ordering, uint32_t *d_words, uint64_t capacity,
                       uint64_t *d_count, void *hip_stream);

/* As greedy_code_device, with optional tuning (may be NULL) and work counters
 * (may be NULL). */
int greedy_code_device_ex(int n, int d, int ordering, uint32_t *d_words, uint64_t capacity,
                          uint64_t *d_count, void *hip_stream, const gc_tuning *tuning,
                          gc_stats *stats);

/* The paper's other problems, with the same greedy rule and the same
 * guarantees (the result is the unique greedy list, bit for bit):
 *
 *   ordering GC_BORDER (section "B-ordering Implementation"): an ordered
 *     basis b_1 .. b_n of F_2^n lists the vectors as 0, b_1, b_2, b_2+b_1,
 *     b_3, ...: position p holds the XOR of b_{j+1} over the set bits j of p
 *     (LEX is the basis b_{j+1} = 2^j, GRAY the basis 1, 3, 6, 12, ...).
 *   weight w >= 0 (section "Brief overview of the Greedy Algorithm and
 *     Codes": constant-weight codes): only the vectors of weight w are
 *     candidates, in increasing value (GC_LEX or GC_GRLEX) or in the graded
 *     reverse lexicographic order (GC_GREVLEX).
 *   self_orthogonal = 1 (section "Self Orthogonal Greedy Codes
 *     Implementation"): a candidate is accepted only if it has even weight
 *     and an even number of ones in common (popcount of the AND) with every
 *     accepted word, besides distance >= d; the candidates are the
 *     even-weight vectors of the ordering, in its order.
 *   start, stop, prefix (checkpoint and resume): only positions [start,
 *     stop) of the walk are screened (stop 0 = its end), and the code buffer
 *     already holds the `prefix` words the greedy accepted before `start`
 *     (what a call that stopped at `start` returned).  Screening [0, P) and
 *     then [P, end) with the first call's words as prefix gives exactly the
 *     code of one call over [0, end).
 *
 * Rules: n in [1, 32]; the basis (GC_BORDER only; entries past n ignored)
 * must be linearly independent with every b_j < 2^n; a weight needs GC_LEX,
 * GC_GRLEX or GC_GREVLEX; self_orthogonal cannot be combined with
 * GC_BORDER; start <= stop <= the walk's length (gc_problem_positions);
 * otherwise GC_EINVAL.  A self-orthogonal problem with an odd weight has no
 * candidates (its code is the prefix). */
typedef struct gc_problem {
    int n, d, ordering;      /* ordering: GC_LEX .. GC_GREVLEX, or GC_BORDER */
    int weight;              /* -1: every weight; w in [0, n]: constant weight w */
    int self_orthogonal;     /* 0 or 1 */
    uint32_t basis[32];      /* GC_BORDER: b_1 .. b_n in basis[0 .. n) */
    uint64_t start, stop;    /* screened positions [start, stop); stop 0 = the end */
    uint64_t prefix;         /* words already in the output buffer */
} gc_problem;

/* Fill *p with the plain problem (n, d, ordering): every weight, not
 * self-orthogonal, the whole walk, no prefix, zero basis.  GC_EINVAL for a
 * NULL p. */
int gc_problem_init(gc_problem *p, int n, int d, int ordering);

/* Number of positions of the walk (candidates): 2^n, 2^(n-1) if
 * self-orthogonal, C(n, w) with a weight (0 if self-orthogonal and w odd).
 * 0 for an invalid problem. */
uint64_t gc_problem_positions(const gc_problem *p);

/* Capacity (words, prefix included) that always suffices: the sphere-packing
 * bound of greedy_code_capacity; with a weight the Johnson bound
 * A(n, 2e, w) <= floor(n/w * A(n-1, 2e, w-1)) (2e = d rounded up to even:
 * two words of one weight are at even distance), 1 once w < e; if
 * self-orthogonal also 2^floor(n/2) (the span of the code is a
 * self-orthogonal code, of dimension at most n/2); never more than
 * prefix + the number of positions screened.  0 for an invalid problem. */
uint64_t gc_problem_capacity(const gc_problem *p);

/* Host-memory entry point of a problem: out_words (caller-owned host array;
 * *out_count on input = its capacity in words) holds the prefix words on
 * input and the whole code (prefix first) on return, *out_count = its size.
 * Runs on the null stream.  GC_ECAPACITY: *out_count = gc_problem_capacity. */
int greedy_code_problem(const gc_problem *p, uint32_t *out_words, uint64_t *out_count);

/* Device-memory entry point of a problem: d_words (device array of
 * `capacity` uint32, 16-byte aligned, holding the prefix words) receives the
 * code after the prefix, *d_count (device uint64) its total size; tuning and
 * stats as in greedy_code_device_ex (may be NULL).  Errors as in
 * greedy_code_device. */
int greedy_code_problem_device(const gc_problem *p, uint32_t *d_words, uint64_t capacity,
                               uint64_t *d_count, void *hip_stream, const gc_tuning *tuning,
                               gc_stats *stats);

/* Constant-weight greedy code over words of up to 64 coordinates (section
 * "Brief overview of the Greedy Algorithm and Codes": the candidates are the
 * weight-w vectors; section "Some Examples" reports such codes up to length
 * 35, past 32-bit words).  Candidates are the weight-w vectors of length n in
 * increasing value (as integers); a candidate is appended when its Hamming
 * distance to every word already in the code is at least d.  n in 1..64,
 * w in 0..n, d >= 1, at most 2^32 candidates (C(n, w)).  The words go to
 * d_words (device array of `capacity` uint64, 8-byte aligned, caller-owned),
 * the count to *d_count (device uint64, may be NULL).  Runs on hip_stream and
 * returns when the code is complete; uses a small device workspace from the
 * library's per-device pool.  GC_EINVAL: an argument out of range;
 * GC_ECAPACITY: the first `capacity` words and *d_count = capacity;
 * GC_EDEVICE: launch or device failure. */
int greedy_code_cw64(int n, int w, int d, uint64_t *d_words, uint64_t capacity, uint64_t *d_count,
                     void *hip_stream);

/* No-allocation variant of greedy_code_device, for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as greedy_code_device, but
 * the call allocates nothing: its device workspace (barrier block, queue, one
 * job and one team workspace, about 154 KiB) is a fixed array that the
 * library holds on every device it runs on until the process ends, and the
 * job descriptor reaches the device as a kernel argument.  A launch needs a
 * fixed workspace size, checked against the array's (GC_EINVAL if it were
 * larger).  All calls on one device share that array: calls that overlap on
 * one device (different threads or streams) race and must be serialised by
 * the caller.  The tuning remembered by greedy_code_tune applies. */
int greedy_code_device_noalloc(int n, int d, int ordering, uint32_t *d_words, uint64_t capacity,
                               uint64_t *d_count, void *hip_stream);

/* One code of a batch.  Inputs: n, d, ordering, d_words (device array of
 * `capacity` uint32, 16-byte aligned, caller-owned), d_count (device uint64 or
 * NULL).  Outputs, filled in by greedy_code_batch: status (GC_OK or an error
 * code), count (|C|), device_ms (device time from the moment a team picked the
 * job up to its completion). */
typedef struct gc_job {
    int n, d, ordering;
    uint32_t *d_words;
    uint64_t capacity;
    uint64_t *d_count;
    int status;
    uint64_t count;
    double device_ms;
} gc_job;

/* Build many codes (batched workload; no paper counterpart: the paper
 * builds one code per run) in one persistent launch on `hip_stream`: the
 * workgroups form `teams` teams by XCD (1, 2, 4 or 8; 0 = 4 teams from 4
 * jobs up, fewer below) and each team pulls the next job from a device
 * queue that holds the jobs longest first, so codes of uneven size share the
 * GPU.  Every code is bit-identical to what
 * greedy_code_device returns for it.  Returns GC_OK when every job succeeded,
 * otherwise the first failing job's code (each job's status is set).
 * kernel_ms (may be NULL) receives the device time of the launch. */
int greedy_code_batch(gc_job *jobs, int njobs, int teams, void *hip_stream, float *kernel_ms);

/* Captured batch (no paper counterpart): the batch launch of `jobs` (same
 * rules as greedy_code_batch, tunings as remembered at creation) recorded once
 * into a HIP graph -- job-table upload from pinned host memory, reset kernel,
 * cooperative persistent launch, download of the outputs into pinned host
 * memory -- so that each rebuild of the same codes is one hipGraphLaunch.
 * The graph keeps the jobs' d_words / d_count pointers: those buffers must
 * stay allocated while it exists.  Allocates its device workspace and pinned
 * buffers at creation and nothing afterwards. */
typedef struct gc_batch_graph gc_batch_graph;
int gc_batch_graph_create(const gc_job *jobs, int njobs, int teams, gc_batch_graph **out);
/* Enqueue one replay on `hip_stream` (asynchronous). */
int gc_batch_graph_launch(gc_batch_graph *graph, void *hip_stream);
/* After the replay's stream has synchronized: per-job status, count and
 * device_ms into jobs[0..njobs) (the array given at creation, same order).
 * Returns GC_OK or the first failing job's code. */
int gc_batch_graph_results(gc_batch_graph *graph, gc_job *jobs);
/* Free the graph (no replay may be in flight). */
int gc_batch_graph_destroy(gc_batch_graph *graph);

/* Autotuner (no paper counterpart).  Builds (n, d, ordering) once per
 * candidate tuning on `hip_stream` (near-screen depth of the whole code or the
 * newest 65536, 16384 or 4096 words, with either deep-scan policy; then the
 * fastest so far with a larger window target, then with deep-scan tiles of 512
 * and of 256 candidates), checks that every candidate built the same code word
 * for word, and returns the fastest in *best (its device time in *best_ms, may
 * be NULL).  The choice is remembered per device and
 * (n, d, ordering): later builds of that instance that pass no tuning
 * (greedy_code, greedy_code_device, greedy_code_device_ex with tuning NULL,
 * batch jobs, server jobs) use it.  Allocates a scratch code buffer
 * (hipMalloc) for the duration of the call.  d <= 1 or d > n: nothing to tune,
 * *best is zeroed.  GC_EDEVICE if two candidates disagree. */
int greedy_code_tune(int n, int d, int ordering, void *hip_stream, gc_tuning *best, float *best_ms);

/* Forget every remembered tuning (builds return to the built-in defaults). */
void greedy_code_tune_reset(void);

/* Team-count tuner for a batch: runs greedy_code_batch with 1, 2, 4 and 8
 * teams and returns the fastest count in *best_teams (device time in
 * *best_ms, may be NULL).  The jobs' outputs are those of the last run (every
 * run builds the same codes). */
int greedy_code_batch_tune(gc_job *jobs, int njobs, void *hip_stream, int *best_teams, float *best_ms);

/* Job server (served workload; no paper counterpart): continuous
 * batching over one persistent launch.  Callers: anything that wants codes
 * built as requests arrive.  A job is admitted once the device arena has room
 * for its worst-case code (greedy_code_capacity(n, d) words); admitted jobs
 * go to a queue in pinned host memory that the running kernel's teams pull
 * from, so a job arriving while others build starts as soon as a team frees
 * up.  With teams 2 or 4, a job whose exhaustive work bound
 * 2^n * greedy_code_capacity(n, d) is at least 2^38 ("wide") goes to a wide
 * queue, served by one team spanning 8 - teams of the eight XCDs; the other
 * jobs go to a narrow queue, served by `teams` teams of one XCD each and by
 * the wide team whenever no wide job waits.  Each queue runs in arrival
 * order; narrow jobs never wait behind a wide one, and may be admitted past a
 * wide job that waits for arena space until it has waited 1 s.  Finished
 * codes stay resident in the arena until released.  The kernel
 * exits after about 0.1 s without work and is relaunched on demand.  If a
 * bounded device-side wait expires, every unfinished job fails with
 * GC_ETIMEOUT (gc_server_poll reports GC_JOB_FAILED) and the server accepts
 * no further jobs.  Not thread-safe across servers' destroy; every call on
 * one server is serialised by an internal lock. */
typedef struct gc_server gc_server;

/* arena_bytes: device memory for resident codes (the server also allocates
 * as much pinned host memory: each finished code is written there by the
 * kernel itself, so fetching a result needs no device copy while the kernel
 * holds the GPU); teams: 1 (one team spanning the GPU) or 8 (one team per
 * XCD): every job in one queue, in arrival order; 2 or 4: the wide team of
 * 8 - teams XCDs plus `teams` narrow teams of one XCD. */
int gc_server_create(size_t arena_bytes, int teams, gc_server **out);
/* Queue a job; *ticket identifies it.  GC_ENOMEM if its worst-case code can
 * never fit the arena. */
int gc_server_submit(gc_server *srv, int n, int d, int ordering, uint64_t *ticket);
/* *state = GC_JOB_*; *count (may be NULL) = |C| once done. */
int gc_server_poll(gc_server *srv, uint64_t ticket, int *state, uint64_t *count);
/* Device address of a finished job's words (valid until released). */
int gc_server_words(gc_server *srv, uint64_t ticket, const uint32_t **d_words, uint64_t *count);
/* Copy a finished job's words into host memory (cap words available); a host
 * memcpy from the pinned mirror. */
int gc_server_fetch(gc_server *srv, uint64_t ticket, uint32_t *host_words, uint64_t cap,
                    uint64_t *count);
/* Work counters and device time of a finished job (either may be NULL). */
int gc_server_stats(gc_server *srv, uint64_t ticket, gc_stats *stats, double *device_ms);
/* Free a finished job's arena space (and admit waiting jobs). */
int gc_server_release(gc_server *srv, uint64_t ticket);
/* Wait until no job is waiting or building; timeout_ms < 0 waits forever. */
int gc_server_drain(gc_server *srv, int timeout_ms);
/* Stop the kernel and free everything (jobs not yet claimed by the device are
 * abandoned; the kernel finishes the ones it is building first). */
int gc_server_destroy(gc_server *srv);

/* Measurement probes (no paper counterpart; they measure the machine the
 * construction runs on).  gc_probe_block_loop runs the screen's block loop
 * alone (four rows of 64 candidates against broadcast code words: v_xor_b32,
 * v_bcnt_u32_b32 and v_min3_u32, 2.5 VALU ops per distance check) in
 * wgs_per_cu (1 or 2) workgroups of 1024 threads per compute unit for
 * `iters` calls per wave, and returns the distance checks per second.
 * gc_probe_matrix_loop runs the matrix-core screen's segment loop alone (one
 * workgroup of 1024 threads per compute unit, each call 1024 candidates
 * against 1024 staged words with int8 v_mfma_i32_32x32x32_i8 products and the
 * max-fold, nothing killed) for `iters` calls and returns the distance checks
 * per second.  gc_probe_barrier times `iters` team-wide barriers of the
 * persistent kernel (one team spanning the GPU) and returns microseconds per
 * barrier.  All run on the null stream and synchronize. */
int gc_probe_block_loop(int wgs_per_cu, int iters, double *checks_per_s);
int gc_probe_matrix_loop(int iters, double *checks_per_s);
int gc_probe_barrier(int iters, double *us_per_barrier);

/* Message of the last failed call on this thread ("" if none). */
const char *gc_last_error(void);

/* Library version string. */
const char *gc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GREEDY_CODE_H */
