/*
 * ofl.h -- C ABI of the GA-driven GPU offload library for AMD MI355X (gfx950).
 *
 * The method (Yamato et al., "Study of Automatic GPU Offloading Technology for
 * Open IoT", Sec. 3.3 and Sec. 4): the for-loop nests of an application are
 * checked one by one for parallelisability; the ``a`` nests that pass each get
 * one bit of a gene (1 = run on the GPU, 0 = run on the CPU); a Simple GA
 * searches the genes, the fitness of each coming from the measured run time
 * of the application under that pattern (Sec. 5.1.2: fitness = time^-1/2,
 * roulette selection with one elite, one-point crossover Pc = 0.9, bit-flip
 * mutation Pm = 0.05), and a pattern measured before is not measured again.
 *
 * Here every offloaded nest runs as a hand-written HIP kernel for gfx950 and
 * every CPU nest as serial host code; host<->device copies follow from the
 * pattern (Sec. 3.3: transfer overhead is why the combination of individually
 * parallelisable loops is searched rather than all offloaded).
 *
 * Conventions for every function below
 *  - Return value: OFL_OK (0) or a negative OFL_E_* code; ofl_status_str()
 *    names a code and ofl_last_error() gives the detail of the calling
 *    thread's last failure.  No function aborts the process.
 *  - Ownership: an ofl_app owns the parsed application, the verdicts, the
 *    pinned host copies of every buffer and a small device scratch area (both
 *    allocated on first use and released by ofl_app_free).  The caller owns the
 *    device buffers (one per application buffer, at least ofl_buf_info's
 *    byte size, 16-byte aligned) and the stream; the library never frees them.
 *  - Layouts: matrices row-major; grids p[i][j][k] with k contiguous; f32 and
 *    f64 IEEE, bf16 as raw 16-bit patterns.
 *  - Genes: uint8 arrays of length a (ofl_app_info's gene_len), each byte 0 or
 *    1; bit i belongs to the i-th accepted nest in program order.
 *  - Streams: a hipStream_t passed as void* (NULL = the null stream).  Run
 *    and evaluation calls synchronise the stream before returning.
 *  - Threads: one ofl_app must not be used by two threads at once.
 */
#ifndef OFL_H
#define OFL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
enum {
    OFL_OK = 0,
    OFL_E_ARG = -1,          /* null pointer, bad size or enum value */
    OFL_E_IO = -2,           /* application file cannot be read */
    OFL_E_PARSE = -3,        /* malformed JSON or expression */
    OFL_E_IR = -4,           /* invalid application: unknown op, shape or dtype
                                mismatch, out-of-bounds access, accepted nest
                                without a device kernel */
    OFL_E_GENE_LEN = -5,     /* gene length differs from a */
    OFL_E_GENE_BIT = -6,     /* gene byte not 0 or 1 */
    OFL_E_NOT_PARALLEL = -7, /* a rejected nest asked to run on the GPU */
    OFL_E_BUF = -8,          /* device buffer missing, misaligned or n_bufs wrong */
    OFL_E_HIP = -9,          /* HIP runtime error (detail in ofl_last_error) */
    OFL_E_TIMEOUT = -10,     /* run exceeded its deadline and was abandoned */
    OFL_E_MISMATCH = -11,    /* output check failed */
    OFL_E_STATE = -12,       /* call out of order (e.g. read before any run) */
    OFL_E_NOMEM = -13,       /* host or device allocation failed */
    OFL_E_RANGE = -14,       /* index out of range */
    OFL_E_UNSUPPORTED = -15  /* batch: a nest without a grouped kernel, or
                                instances that differ in structure */
};

/* Parallelisability verdict of a nest and the reason of a rejection
 * (the compile-error kinds listed in Sec. 4 of the paper). */
enum { OFL_PARALLEL = 0, OFL_PARALLEL_REDUCTION = 1, OFL_REJECT = 2 };
enum { OFL_R_NONE = 0, OFL_R_DATA_DEP = 1, OFL_R_EXTERNAL_CALL = 2, OFL_R_BREAK = 3,
       OFL_R_NO_KERNEL = 4   /* a host_code nest: no GPU form (Sec. 4's compile
                                that fails for other reasons) */ };

/* Transfer policies (see ofl_plan_transfers) and run flags. */
enum { OFL_POLICY_RESIDENT = 0, OFL_POLICY_PER_REGION = 1, OFL_POLICY_SECTIONS = 2 };
enum {
    OFL_RUN_PRESTAGED = 1,   /* set-up content already on the device when the
                                timed region starts (restored device-side,
                                outside the timed region) */
    OFL_RUN_KEEP_OUTPUTS = 2, /* leave outputs on the device (no final D2H);
                                ofl_read_buffer fetches them afterwards */
    OFL_RUN_GRAPH = 4,       /* replay the run as HIP graphs captured once per
                                (gene, policy, flags): a reset graph (untimed)
                                and a run graph holding the copies, kernels and
                                host nodes for the CPU nests (led by one more
                                host node that stamps the run's start);
                                deadlines are not applied to single graph runs.
                                Plans and results are those of the eager run. */
    OFL_RUN_BATCHED = 8,     /* population evaluation (ofl_eval_population,
                                ofl_ga_run, ofl_ga_run_table) only: all
                                uncached genes of a population / generation are
                                measured together, ONE submission per round of
                                runs (each warm-up round, then each timed
                                round) -- the reset and run graphs of every
                                gene queued back to back with an event pair
                                around each run graph, one synchronisation per
                                round; a gene's time is the median of its
                                timed event intervals (GPU timeline, host nodes
                                included).  Implies OFL_RUN_GRAPH.  A deadline
                                applies to every run's interval and to the host
                                nests: each run's graph stamps its start, and a
                                host nest still running at start + limit stops
                                (checked between its rows or planes, as in an
                                eager run); a run over the limit or cut there
                                makes the gene OFL_ST_TIMEOUT at the limit and
                                leaves it out of the later rounds, as an eager
                                measurement ends at its first run over the
                                limit; GPU work is not cut.  In the GA every
                                gene of a generation gets the limit taken at
                                the start of that generation.  ofl_ga_run
                                submits a generation only once the best run
                                so far is shorter than 20 ms
                                (OFL_BATCH_EAGER_S in the environment sets
                                the threshold in seconds); before that (the
                                first generation included) it measures the
                                genes one after the other with eager runs,
                                exactly as without this flag: for longer runs
                                capturing each gene's graphs costs more than
                                the launch overhead a submission saves. */
    OFL_RUN_PROGRESS = 16,   /* ofl_ga_run only: one line per generation on
                                stderr (generation, best time so far, genes
                                measured, wall time), for long searches */
    OFL_RUN_CONCURRENT = 32  /* eager runs: the application's components --
                                groups of nests that share no buffer (nor the
                                product workspace) -- run at the same time,
                                each on a stream of its own (default priority,
                                created by the library; the caller's stream
                                carries the first) and from a host thread of
                                its own, each in program order, so that a
                                memory-bound part overlaps a compute-bound one
                                and a host nest holds up only its own part.
                                Results are those of the sequential run (no
                                data is shared between components); plans,
                                copies and byte counts are the same.  Graph
                                runs (OFL_RUN_GRAPH / OFL_RUN_BATCHED) stay
                                sequential. */
};

/* Buffer element types. */
enum { OFL_F32 = 0, OFL_F64 = 1, OFL_BF16 = 2 };

/* Run status inside evaluation / GA traces. */
enum { OFL_ST_OK = 0, OFL_ST_TIMEOUT = 1, OFL_ST_FAILED = 2,
       OFL_ST_MISMATCH = 3   /* outputs differ from the all-CPU run's (see
                                verify_rtol); fitness 0 */ };

typedef struct ofl_app ofl_app;

typedef struct {
    int32_t policy;          /* OFL_POLICY_* */
    int32_t flags;           /* OFL_RUN_* bits */
    double deadline_s;       /* wall-time limit of the run, 0 = none */
    double verify_rtol;      /* > 0: check the run's outputs against those of
                                the all-zero gene (the program as written, all
                                on the CPU; that run is made once, untimed and
                                without a deadline, and kept until the inputs
                                change): at up to 4096 probe elements of every
                                output buffer (every element of a smaller
                                one; the same positions each time),
                                |x - ref| <= verify_rtol * max |ref over the
                                buffer's probes|, NaN only where the reference
                                has NaN.  A failed check returns
                                OFL_E_MISMATCH with status OFL_ST_MISMATCH.
                                0 = no check */
} ofl_run_opts;

typedef struct {
    double t_total_s;        /* host wall time of the timed region: first nest
                                to outputs in place, transfers included */
    uint64_t bytes_h2d, bytes_d2h;
    int32_t n_copies;        /* number of host<->device copies */
    int32_t n_launches;      /* kernel launches */
    int32_t n_host_nests;    /* nest executions on the CPU */
    int32_t status;          /* OFL_ST_* */
} ofl_run_stats;

typedef struct {
    int32_t reps;            /* timed runs per gene; time = median (>= 1) */
    int32_t warmup;          /* untimed runs before them (>= 0) */
    int32_t policy, flags;   /* as ofl_run_opts */
    double deadline_s;       /* per run, 0 = none */
    double verify_rtol;      /* > 0: each distinct gene's outputs are checked
                                once, as ofl_run_opts.verify_rtol describes,
                                on its first run (with OFL_RUN_BATCHED, on one
                                run of its graphs before the submission); a
                                gene that fails gets OFL_ST_MISMATCH and no
                                timed runs */
} ofl_eval_opts;

typedef struct {
    int32_t M, T;            /* individuals, evaluated generations (incl. the first) */
    double Pc, Pm;           /* crossover rate per pair, mutation rate per bit */
    double p;                /* fitness = time^-p (the paper uses 1/2) */
    uint64_t seed;           /* SplitMix64 seed of the GA's random stream */
    int32_t reps, warmup;    /* measurement of one gene, as ofl_eval_opts */
    int32_t policy, flags;   /* transfer policy and run flags */
    double deadline_factor;  /* > 0: measure the all-zero gene first and give
                                every later run the limit
                                min(t_all0, deadline_factor * t_best); 0 = none */
    double timeout_s;        /* > 0: no run (the all-zero one included) goes on
                                past this wall time; one that would is a
                                TIMEOUT with fitness 0, like a trial cut off
                                by a timeout (Sec. 5.2); 0 = none.  With
                                deadline_factor the limit is the smaller one */
    double verify_rtol;      /* > 0: output check of every measured gene, as in
                                ofl_eval_opts; a gene that fails has fitness 0 */
    const char *cache_path;  /* NULL or "": the measurements live only in this
                                call.  Otherwise a log file of the search (the
                                same-pattern skip of Sec. 4 kept across calls,
                                for resuming): created if missing, else read
                                first -- its measurements are taken in order
                                instead of measuring again, which retraces the
                                logged search exactly -- and every fresh
                                measurement (gene, time, status) and every
                                generation's end (the random stream's state)
                                is appended and flushed as one JSON line.  The
                                log's first line names the search (every
                                parameter above except T, and the application
                                or table); a log of another search, or one that
                                disagrees on the way, gives OFL_E_STATE. */
} ofl_ga_params;

typedef struct {
    uint8_t *best_gene;      /* [a] caller-owned, filled */
    uint8_t *pop_trace;      /* [T*M*a] caller-owned or NULL */
    double *time_trace;      /* [T*M] or NULL */
    int32_t *status_trace;   /* [T*M] or NULL */
    double best_time, best_fitness;
    double t_all0;           /* all-zero gene time when measured, else -1 */
    int32_t n_measured;      /* fresh measurements (cache misses) */
    int32_t n_generations;
    double search_wall_s;    /* wall time of the whole search */
    double time_to_best_s;   /* wall time until the final best was measured */
} ofl_ga_result;

/* ------------------------------------------------------------ application */

/* Parse an application description (JSON: params, buffers, program of loop
 * nests with affine accesses and repeat blocks), validate it and run the
 * parallelisability check of every nest (Sec. 4: loops found and counted,
 * each checked on its own; the accepted ones define the gene).  A nest may
 * also be a function block, a library call given one gene bit (Sec. 3.2,
 * steps 1-2 and 1-3, name FFT library calls beside loops): op "fft_rows",
 * the forward DFT of every row of an f32 buffer [R][2n] (n complex values per
 * row, interleaved; n a power of two up to 4096), or with args "inverse":
 * true / 1 the inverse DFT scaled by 1/n, or with "real": true / 1 the DFT
 * of rows of n real values [R][n] (2 <= n <= 4096), written in place packed
 * as [X0, X(n/2), Re X1, Im X1, ..., Re X(n/2-1), Im X(n/2-1)]; both flags:
 * such packed spectra replaced by their real rows (scaled by 1/n).  `seed` drives the
 * application's random-initialisation nests.  Allocates nothing on the GPU
 * (the device scratch, and for an FFT call its twiddle tables, come with the
 * first run).  A nest of op "host_code" (args {"symbol": name}) is a loop
 * nest whose body no library operation matches, compiled from its own source
 * text into the shared object the description names as "host_object" (its
 * entry point void name(void *const *host_bufs, const int64_t *repeat_env)
 * gets the host copy of every buffer, in declaration order, and the values
 * of the repeat variables, by repeat id); such a nest always runs on the CPU
 * (verdict OFL_REJECT, its own reason or OFL_R_NO_KERNEL) and its transfers
 * follow from its declared accesses.  Every nest's loops must span exactly
 * the index space of its operation (the whole arrays; the interior of the
 * grid for the sweep and the interior copy).  A grid of the interior copy
 * must hold under 2 GiB, one of the sweep under 2 GiB with six planes added
 * (both address their grids with 32-bit byte offsets).  Errors: OFL_E_IO (file or host
 * object cannot be read), OFL_E_PARSE, OFL_E_IR, OFL_E_ARG, OFL_E_NOMEM. */
int ofl_app_load(const char *path, uint64_t seed, ofl_app **out);
int ofl_app_load_json(const char *json_text, uint64_t seed, ofl_app **out);
void ofl_app_free(ofl_app *app);

/* Counts: nests in program order, gene length a, buffers. */
int ofl_app_info(const ofl_app *app, int32_t *n_nests, int32_t *gene_len, int32_t *n_bufs);

/* Verdict of nest `nest` (OFL_PARALLEL / _REDUCTION / OFL_REJECT), reason
 * (OFL_R_*), and its gene position (-1 when rejected).  OFL_E_RANGE. */
int ofl_nest_info(const ofl_app *app, int32_t nest, int32_t *verdict, int32_t *reason,
                  int32_t *gene_pos);
int ofl_nest_name(const ofl_app *app, int32_t nest, char *out, int32_t cap);

/* Size in bytes, element type (OFL_F32/F64/BF16) and output flag of buffer
 * `buf`.  OFL_E_RANGE. */
int ofl_buf_info(const ofl_app *app, int32_t buf, uint64_t *bytes, int32_t *dtype,
                 int32_t *is_output);
int ofl_buf_name(const ofl_app *app, int32_t buf, char *out, int32_t cap);

/* Extents of buffer `buf`, outermost first: *ndim set to the rank, the first
 * min(rank, cap) extents written to dims.  OFL_E_RANGE. */
int ofl_buf_dims(const ofl_app *app, int32_t buf, int64_t *dims, int32_t cap, int32_t *ndim);

/* Replace the set-up content of buffer `buf` (what its host copy holds when a
 * run starts) by `bytes` bytes copied from host memory `src`; `bytes` must be
 * the buffer's size.  The benchmark input of the application, supplied by the
 * caller.  Errors: OFL_E_RANGE, OFL_E_ARG, OFL_E_NOMEM. */
int ofl_set_input(ofl_app *app, int32_t buf, const void *src, uint64_t bytes);

/* Convert a per-nest placement mask (n_nests bytes, 1 = GPU) to a gene.
 * OFL_E_NOT_PARALLEL when a rejected nest is set, OFL_E_GENE_BIT on a byte
 * other than 0/1. */
int ofl_mask_to_gene(const ofl_app *app, const uint8_t *mask, int32_t n_nests, uint8_t *gene_out);

/* ---------------------------------------------------------------- planning */

/* Host<->device copies implied by a gene (pure host computation).  Per nest a
 * buffer is read when any access reads it or when it is written only in part,
 * written when any access writes it.  Buffer state (host_valid, dev_valid)
 * starts (1,0) ((1,1) with OFL_RUN_PRESTAGED).
 *   RESIDENT: before a GPU nest copy in every read buffer not valid on the
 *     device; before a CPU nest copy out every read buffer not valid on the
 *     host; after a nest its written buffers are valid only where it ran; at
 *     the end copy out outputs not valid on the host (unless KEEP_OUTPUTS).
 *   PER_REGION: the directive compiler's implicit copies (Sec. 2 of the
 *     paper): every GPU nest copies in all it reads and copies out all it
 *     writes.
 *   SECTIONS: RESIDENT, but a CPU nest that only reads a buffer stale on the
 *     host copies out just the bounding box of the elements its plain reads
 *     touch (the array section a data clause would name), unless a box of
 *     that buffer copied out earlier and still current contains it; a box
 *     equal to the whole buffer is a whole copy; any write drops the boxes.
 *     Each box copy counts as one copy of its bytes.
 * Errors: OFL_E_GENE_LEN, OFL_E_GENE_BIT, OFL_E_ARG. */
int ofl_plan_transfers(const ofl_app *app, const uint8_t *gene, int32_t gene_len, int32_t policy,
                       int32_t flags, uint64_t *bytes_h2d, uint64_t *bytes_d2h, int32_t *n_copies);

/* ---------------------------------------------------------------- running */

/* Run the application once under `gene` (Sec. 4: the pattern is built, run and
 * its time measured): host copies reset to the set-up content (untimed), then
 * the timed region executes every nest in program order -- GPU nests as HIP
 * kernels on `stream` into the caller's device buffers `dev_bufs[n_bufs]`
 * (device pointers, one per application buffer), CPU nests serially on the
 * host copies -- with the planned copies in between, and ends when the outputs
 * are in place.  Synchronous.  With a deadline, a run that exceeds it stops at
 * the next nest boundary (or inside a CPU nest) and returns OFL_E_TIMEOUT with
 * stats->status = OFL_ST_TIMEOUT.  Errors: gene errors, OFL_E_BUF, OFL_E_HIP,
 * OFL_E_TIMEOUT, OFL_E_NOMEM. */
int ofl_run_pattern(ofl_app *app, const uint8_t *gene, int32_t gene_len, void *const *dev_bufs,
                    int32_t n_bufs, void *stream, const ofl_run_opts *opts, ofl_run_stats *stats);

/* Measure `pop` genes (row-major pop x gene_len): per gene `warmup` untimed
 * runs and `reps` timed runs, time = median.  Genes that occur more than once
 * are measured once.  time_out[pop], status_out[pop] (OFL_ST_*); a failed or
 * timed-out gene gets its status and the time it reached.  Returns OFL_OK
 * unless the arguments are invalid or a HIP error leaves the device unusable. */
int ofl_eval_population(ofl_app *app, const uint8_t *genes, int32_t pop, int32_t gene_len,
                        void *const *dev_bufs, int32_t n_bufs, void *stream,
                        const ofl_eval_opts *opts, double *time_out, int32_t *status_out);

/* The Simple GA (Sec. 3.3, Sec. 4, Sec. 5.1.2) with measured fitness.
 * Random stream: SplitMix64(seed); initial bits next()>>63; per generation
 * M-1 roulette draws (first m whose running fitness sum exceeds u*total,
 * uniform next()%M when all fitness is 0), pairs in draw order with one u()
 * against Pc and a point 1 + next()%(a-1), then per non-elite child and bit
 * one u() against Pm; u() = (next()>>11) * 2^-53.  The elite (highest fitness,
 * lowest index on ties) is copied unchanged to position 0.  Cached genes are
 * not re-measured.  Result: best gene over all measurements (earliest on
 * ties).  Errors: OFL_E_ARG plus those of ofl_run_pattern. */
int ofl_ga_run(ofl_app *app, const ofl_ga_params *params, void *const *dev_bufs, int32_t n_bufs,
               void *stream, ofl_ga_result *result);

/* The same GA over an injected time table (host only, no GPU): the time of
 * gene g is t_table[idx(g)] with idx = sum g_i 2^i, its status
 * status_table[idx] (NULL = all OK); with deadline_factor > 0 a time above the
 * limit becomes OFL_ST_TIMEOUT at the limit.  gene_len <= 24. */
int ofl_ga_run_table(int32_t gene_len, const ofl_ga_params *params, const double *t_table,
                     const int32_t *status_table, ofl_ga_result *result);

/* Copy the current content of buffer `buf` after a run into host memory
 * (from the host copy or the device, whichever holds the newest values).
 * Errors: OFL_E_STATE before any run, OFL_E_RANGE, OFL_E_ARG (bytes too
 * small), OFL_E_HIP. */
int ofl_read_buffer(ofl_app *app, int32_t buf, void *host_dst, uint64_t bytes);

/* ---------------------------------------------------------------- profiling */

/* Enable (1) / disable (0) per-kernel timing with HIP events recorded on the
 * run's stream around every launch; enabling clears the totals.  Graph runs
 * (OFL_RUN_GRAPH) use graphs captured while timing is on, which hold an event
 * record node before and after every GPU nest; their intervals are added
 * after each replay. */
int ofl_set_kernel_timing(ofl_app *app, int32_t enable);

/* Restrict kernel timing to nests of the kinds listed in `op`, names
 * separated by commas (e.g. "stencil19" or "stencil19,copy_interior"); NULL
 * or "" times every kind.  Errors: OFL_E_ARG for an unknown kind (the
 * previous selection stays). */
int ofl_set_kernel_timing_op(ofl_app *app, const char *op);

/* Time only every stride-th execution of each timed kind in a run: the
 * executions i = phase, phase + stride, ... (counted per kind from 0 in each
 * run).  Default 1, 0 (all).  Errors: OFL_E_ARG unless stride >= 1 and
 * 0 <= phase < stride. */
int ofl_set_kernel_timing_sample(ofl_app *app, int32_t stride, int32_t phase);

/* Timed executions of nests of kind `op` (e.g. "stencil19", "gemm") and
 * their total kernel time (ms) since timing was enabled.  Unknown op: zeros.
 * The time of an execution covers all of the nest's launches.  A "stencil19"
 * nest launches the sweep; the sum of its per-wave residual partials runs
 * as one extra block of the "copy_interior" launch when that nest follows on
 * the GPU, else as a one-block kernel before the next step (counted in the
 * run's launches, timed with neither nest). */
int ofl_kernel_stats(const ofl_app *app, const char *op, int64_t *executions, double *total_ms);

/* ---------------------------------------------------------------- nest calls */

/* One sweep of the 19-point nest on caller-owned device grids, the offloaded
 * form of the iterated stencil nest as a call of its own (Sec. 3.2: a call
 * the offloader can substitute, like a library call's GPU implementation).
 * p, q: distinct I x J x K f32 grids, p[i][j][k] with k contiguous, 16-byte
 * aligned; res_slot: one double in device memory, 8-byte aligned.  Writes
 * q on the interior (1 <= i < I-1, 1 <= j < J-1, 1 <= k < K-1):
 *   q = (p/4 + F/16) + E/32, F = (a_{i-1} + a_{i+1}) + x_i,
 *   E = (x_{i-1} + x_{i+1}) + y_i, with the plane partial sums
 *   a = p, x = (p[j-1] + p[j+1]) + (p[k-1] + p[k+1]),
 *   y = (p[j-1][k-1] + p[j-1][k+1]) + (p[j+1][k-1] + p[j+1][k+1])
 * (weights 1/4, 1/16, 1/32 on the centre, the 6 face and the 12 edge
 * neighbours; FP32, no contraction); the boundary of q is not touched; and
 * adds sum over the interior of ((double)q - (double)p)^2 to res_slot[0] in
 * a fixed order (reproducible bits).  Launches on `stream` (a hipStream_t;
 * NULL = the null stream) and does not synchronise.  Scratch: the sweep's
 * per-wave residual partials, in device memory the library allocates on the
 * first call on each device (grown when needed, kept until the process
 * ends); calls that overlap on one device race on it.  Errors: OFL_E_ARG
 * (null or misaligned pointer, p == q), OFL_E_RANGE (an extent < 1, or the
 * grid plus six planes 2 GiB or more: 32-bit byte offsets), OFL_E_NOMEM,
 * OFL_E_HIP. */
int ofl_sweep19(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res_slot, void *stream);

/* ofl_sweep19 for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, result bits, launches and errors, but it allocates nothing.
 * The residual partials live in a fixed array of the library, 16384 doubles
 * (128 KiB) on every device it runs on, held until the process ends; a grid
 * whose sweep needs more partials than that (more than about 2000 CUs) is
 * rejected with OFL_E_RANGE.  Every call on one device shares that device's
 * array and leaves its partials there; calls that overlap on one device (on
 * different streams or threads, or overlapping ofl_sweep19_noalloc launches
 * of several callers) race on it and must be serialised by the caller. */
int ofl_sweep19_noalloc(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res_slot,
                        void *stream);

/* ---------------------------------------------------------------- instance batches */

/* Many instances of one application description that differ only in their
 * parameter values (sizes) and seeds, run with every nest on the GPU: the
 * batching configuration (uneven instance sizes in one persistent launch per
 * nest, the iterated sweeps captured in a HIP graph, tile shapes chosen by the
 * library's own tuner).  Each nest of the program runs as ONE grouped launch
 * that covers that nest in all instances; results equal those of running
 * every instance alone under the all-GPU gene (bit-identical wherever the
 * arithmetic is fixed; the product within the FP32 GEMM tolerance, as its
 * tile shape is tuned).  Supported nests: init_uniform, FP32 gemm, stencil19,
 * copy_interior.  Buffers: bufs[inst * n_bufs + buf], caller-owned device
 * pointers, 16-byte aligned, sized by ofl_batch_buf_bytes. */
typedef struct ofl_batch ofl_batch;

enum {
    OFL_BATCH_LOOP = 0,           /* per-instance launches, instance after instance */
    OFL_BATCH_GROUPED = 1,        /* one grouped launch per nest execution */
    OFL_BATCH_GROUPED_GRAPH = 2   /* the grouped launches as one captured HIP graph */
};

typedef struct {
    int32_t gemm_cfg;               /* tile shape index: 0..7 = (64,16) (64,32) (64,64)
                                       (128,16) (128,32) (128,64) (256,16) (256,32) as
                                       (BM = BN, BK); (256,64) is not offered: its double-
                                       buffered slabs need 272 KB of LDS (160 KB per CU) */
    int32_t gemm_blocks_per_cu;     /* persistent blocks per CU (1..8, <= occupancy) */
    int32_t stencil_rows;           /* rows per sweep item: 2, 4 or 8 */
    int32_t stencil_planes;         /* planes per sweep item (>= 1) */
    int32_t stencil_blocks_per_cu;  /* persistent blocks per CU */
} ofl_batch_config;

typedef struct {
    double t_total_s;        /* wall time from the first launch to completion */
    int32_t n_launches;      /* kernel launches (inside the graph for mode 2) */
    int32_t n_submissions;   /* host submissions: launches, or 1 graph launch */
    int32_t status;          /* OFL_ST_* */
} ofl_batch_stats;

typedef struct {
    int32_t phase;           /* 0 = product, 1 = sweep */
    ofl_batch_config cfg;    /* the candidate */
    double ms;               /* median launch time */
} ofl_tune_entry;

/* Parse `app_json` once per instance with its parameter values
 * param_values[inst * n_params + p] for the names param_names[p] (each must
 * be a parameter the description declares) and its seed seeds[inst].
 * Errors: OFL_E_ARG, OFL_E_PARSE, OFL_E_IR, OFL_E_NOT_PARALLEL (a rejected
 * nest), OFL_E_UNSUPPORTED, OFL_E_NOMEM. */
int ofl_batch_create(const char *app_json, int32_t n_inst, const char *const *param_names, int32_t n_params,
                     const int64_t *param_values, const uint64_t *seeds, ofl_batch **out);
void ofl_batch_free(ofl_batch *batch);
int ofl_batch_info(const ofl_batch *batch, int32_t *n_inst, int32_t *n_bufs, int32_t *n_nests);
/* Size in bytes, dtype (OFL_F32 / OFL_F64 / OFL_BF16) and rank of buffer `buf`
 * of instance `inst`; its extents (min(rank, cap) written); its name (the
 * same in every instance, NUL-terminated, truncated to cap).  OFL_E_RANGE. */
int ofl_batch_buf_info(const ofl_batch *batch, int32_t inst, int32_t buf, uint64_t *bytes, int32_t *dtype,
                       int32_t *rank);
int ofl_batch_buf_dims(const ofl_batch *batch, int32_t inst, int32_t buf, int64_t *dims, int32_t cap);
int ofl_batch_buf_name(const ofl_batch *batch, int32_t buf, char *name, int32_t cap);

/* Write every buffer's set-up content (sine fields, zeros) into the device
 * buffers; synchronous, untimed.  Errors: OFL_E_BUF, OFL_E_HIP, OFL_E_NOMEM. */
int ofl_batch_setup(ofl_batch *batch, void *const *bufs, int32_t n_ptrs, void *stream);

/* Run the program of every instance once in `mode` on `stream`; synchronous.
 * Errors: OFL_E_ARG, OFL_E_BUF, OFL_E_HIP, OFL_E_NOMEM. */
int ofl_batch_run(ofl_batch *batch, void *const *bufs, int32_t n_ptrs, void *stream, int32_t mode,
                  ofl_batch_stats *stats);

int ofl_batch_get_config(const ofl_batch *batch, ofl_batch_config *cfg);
/* Errors: OFL_E_ARG for a value outside the ranges above. */
int ofl_batch_set_config(ofl_batch *batch, const ofl_batch_config *cfg);

/* Autotune the grouped product and sweep: every tile shape x blocks per CU
 * in {1,2,4,8} within occupancy (product), every rows in {2,4,8} x planes in
 * {8,16,32} x blocks per CU (sweep), each timed as the median of `reps`
 * launches after one warm-up on the batch's own buffers (contents change:
 * call ofl_batch_setup afterwards).  The fastest of each phase becomes the
 * configuration; min(cap, count) entries are written, *n_entries = count.
 * Errors: as ofl_batch_run. */
int ofl_batch_tune(ofl_batch *batch, void *const *bufs, int32_t n_ptrs, void *stream, int32_t reps,
                   ofl_tune_entry *entries, int32_t cap, int32_t *n_entries);

/* ---------------------------------------------------------------- status */
const char *ofl_status_str(int32_t code);
const char *ofl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* OFL_H */
