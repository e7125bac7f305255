/*
 * hj.h -- C ABI of libhj, the MI355X (gfx950) Jacobi pressure sweep.
 *
 * What is computed (the Himeno workload's Poisson solve by Jacobi iteration,
 * paper section 5.1.1). The paper prints no stencil; this library fixes it as
 * a 19-point variable-coefficient operator on an nx*ny*nz grid (k contiguous)
 * whose one-cell shell is a Dirichlet boundary that is never written. One
 * iteration, on every interior cell and from the field before the iteration:
 *   s0 = a0 p(i+1,j,k) + a1 p(i,j+1,k) + a2 p(i,j,k+1)
 *      + b0 [p(i+1,j+1,k) - p(i+1,j-1,k) - p(i-1,j+1,k) + p(i-1,j-1,k)]
 *      + b1 [p(i,j+1,k+1) - p(i,j-1,k+1) - p(i,j+1,k-1) + p(i,j-1,k-1)]
 *      + b2 [p(i+1,j,k+1) - p(i-1,j,k+1) - p(i+1,j,k-1) + p(i-1,j,k-1)]
 *      + c0 p(i-1,j,k) + c1 p(i,j-1,k) + c2 p(i,j,k-1) + wrk1
 *   ss   = (s0 a3 - p) bnd          wrk2 = p + omega ss
 *   gosa = sum over the interior of ss^2, accumulated in FP64
 * after which wrk2 becomes the field. Sums are evaluated left to right as
 * written, without fused multiply-add, in FP64 (HJ_F64) or FP32 (HJ_F32;
 * ss is widened to FP64 before it is squared).
 *
 * Data stays on the device. Following the paper's transfer rule (sections 3.2
 * and 3.3: transfer once at the outermost level, mark resident data present,
 * block implicit transfers), inputs are uploaded once, any number of sweeps
 * run with no host transfer except the FP64 gosa values, and the field is
 * downloaded once.
 *
 * Conventions for every function:
 *  - Return 0 (HJ_OK) or a negative HJ_ERR_* code. Nothing aborts or throws.
 *    hj_last_error() gives a thread-local message for the last failure.
 *  - Shapes include the shell and must be >= 3 on every axis; nx*ny*nz must
 *    fit the device. Host arrays are dense C order [nx][ny][nz], k fastest.
 *  - Host pointers are borrowed for the duration of the call only.
 *  - Work is ordered on the handle's HIP stream (the caller's, or one the
 *    library creates). Calls that return host results synchronize with it.
 *  - Different handles may be used from different threads; one handle must
 *    not be used by two threads at once.
 */
#ifndef HJ_H
#define HJ_H

#ifdef __cplusplus
extern "C" {
#endif

enum hj_status {
    HJ_OK = 0,
    HJ_ERR_ARG = -1,     /* bad argument (null pointer, field, count, config) */
    HJ_ERR_SHAPE = -2,   /* a dimension below 3, or sizes that overflow */
    HJ_ERR_DTYPE = -3,   /* dtype other than HJ_F64 / HJ_F32 */
    HJ_ERR_OOM = -4,     /* device or host allocation failed */
    HJ_ERR_HIP = -5,     /* a HIP runtime call failed (see hj_last_error) */
    HJ_ERR_STATE = -6,   /* e.g. sweep before every input field is uploaded */
    HJ_ERR_HANDLE = -7,  /* null, destroyed or unknown handle */
    HJ_ERR_TUNE = -8     /* autotuning found no candidate that passed */
};

enum hj_dtype { HJ_F64 = 0, HJ_F32 = 1 };

/* Field ids: 13 inputs, then the ping-pong partner of p. */
enum hj_field {
    HJ_P = 0, HJ_A0, HJ_A1, HJ_A2, HJ_A3, HJ_B0, HJ_B1, HJ_B2,
    HJ_C0, HJ_C1, HJ_C2, HJ_BND, HJ_WRK1, HJ_WRK2, HJ_NFIELDS
};

/* Kernel choice. kernel: HJ_KERNEL_DIRECT (one thread per cell, neighbours
 * read through the caches), HJ_KERNEL_MARCH (a (j,k) tile per workgroup
 * marching along i, p planes staged in an LDS ring) or HJ_KERNEL_FLAT (a
 * run of 64*bj consecutive interior cells of the flattened (j,k) plane per
 * workgroup, marching along i, so no lane idles at the end of a k row; only
 * for grids where the rows a run touches fit 10 KiB of LDS, e.g. nz up to
 * about 600 in FP32 at bj 4; bj 2, 4 or 8, vec 1). bj: rows of 64*vec
 * cells per workgroup (1, 2, 4, 8). vec: consecutive k cells per lane (1, 2,
 * or 4 for HJ_F32; 1 or 2 for HJ_F64). ichunk: i planes per workgroup for the
 * march kernel (>= 1; splits the march so the grid fills the chip).
 * nontemporal: stream the 12 single-use arrays with non-temporal loads and
 * stores. use_graph: replay the sweep loop as a captured HIP graph.
 * xcd_remap: renumber workgroups so neighbouring tiles share an XCD's L2
 * (two-iteration single solves: within windows of the workgroups resident
 * at once, queried when the configuration is installed; one-iteration
 * kernels and batches: over the whole grid or tile list).
 * persistent (batches only): launch as many workgroups as stay resident and
 * let each loop over tiles, instead of one workgroup per tile.
 * tsteps: Jacobi iterations per pass over memory. 1, or 2: the march
 * kernel computes the first iteration of a tile and its one-cell halo into
 * LDS and the second from it, so each coefficient is read once per two
 * iterations. Needs kernel HJ_KERNEL_MARCH, not persistent, and a row
 * layout in vec: 1, tiles of 62-cell rows, each a 64-lane row with its halo
 * (bj 2, 4, 6, 8 or 14; bj+2 waves); 2, tiles of 64-cell rows, one more
 * wave computing the halo columns (bj 2, 4, 6, 8 or 12; bj+3 waves); 4,
 * tiles of 30-cell rows, two 32-lane rows per wave (bj 6, 14, 22 or 30;
 * (bj+2)/2 waves). An odd remainder runs one single-iteration launch. 0
 * means 1. The results are bitwise those of tsteps 1. In FP32 these kernels
 * address a plane with 32-bit byte offsets, so they refuse (HJ_ERR_ARG) a
 * grid whose plane (ny rows of the padded k pitch) holds 4 GiB or more.
 * reread (tsteps 2 only): 0 holds each cell's coefficients in registers
 * between its two iterations, 1 reads them again for the second (an L2 hit
 * when nontemporal is 0), which frees registers for more resident waves. */
typedef struct hj_config {
    int kernel;
    int bj;
    int vec;
    int ichunk;
    int nontemporal;
    int use_graph;
    int xcd_remap;
    int persistent;
    int tsteps;
    int reread;
} hj_config;

enum { HJ_KERNEL_DIRECT = 0, HJ_KERNEL_MARCH = 1, HJ_KERNEL_FLAT = 2 };

typedef struct hj_solver_s* hj_solver;
typedef struct hj_batch_s* hj_batch;

/* ---- single solve ------------------------------------------------------ */

/* Bytes of device memory a solve of this shape needs (for hj_attach).
 * Paper section 3.3 / section 4: the arrays get a GPU-side area of their own
 * that the transfers fill, so no transfer happens implicitly in the loop.
 * The area holds the 14 fields (rows padded to 128-byte lines) and, after
 * them, a compact copy of the coefficients on the k tile edges (12 arrays x
 * nx x ceil((nz-2)/64) x ny x 2 elements) that hj_upload fills. */
int hj_slab_bytes(int dtype, int nx, int ny, int nz, unsigned long long* bytes);

/* Create a solve that owns its device memory (the GPU-side area of paper
 * sections 3.3 and 4). stream: a hipStream_t, or NULL for a library-created
 * non-blocking stream. */
int hj_create(hj_solver* out, int dtype, int nx, int ny, int nz, void* stream);

/* Create a solve on caller-owned device memory of at least hj_slab_bytes
 * bytes, 256-byte aligned (e.g. a torch uint8 tensor): the same GPU-side
 * area (paper section 3.3), supplied by the caller. The caller keeps it
 * alive and unused until hj_destroy. */
int hj_attach(hj_solver* out, int dtype, int nx, int ny, int nz, void* device_slab,
              unsigned long long slab_bytes, void* stream);

/* Paper sections 3.3 and 4: what the CPU defines and the GPU reads is sent
 * once, before the GPU work, at the outermost level (a data copy batched
 * over the loop, not a transfer per iteration).
 * Upload one input field from a dense host array in the handle's dtype
 * (hj_upload) or in FP64 (hj_upload_f64, rounded to nearest even for HJ_F32
 * handles). Uploading HJ_P also resets the ping-pong partner to p and makes
 * p current. HJ_WRK2 cannot be uploaded (HJ_ERR_ARG). Synchronous. A pinned
 * host array (hipHostMalloc, a torch pin_memory tensor) is copied directly;
 * a pageable one is staged through the library's pinned buffers (one host
 * copy more), as is any FP64 source of an HJ_F32 handle. A device pointer
 * is refused (HJ_ERR_ARG), here and wherever the ABI takes a host array. */
int hj_upload(hj_solver h, int field, const void* host_src);
int hj_upload_f64(hj_solver h, int field, const double* host_src);

/* Paper sections 3.3 and 4: results come back once, after all the GPU work.
 * Download a field into a dense host array of the handle's dtype. HJ_P and
 * HJ_WRK2 both return the current field (the last sweep's wrk2 once any
 * sweep has run). Synchronous. Pinned host memory is written directly, as
 * for hj_upload. */
int hj_download(hj_solver h, int field, void* host_dst);

/* Send the current field to the host while later work proceeds: enqueues,
 * on the handle's stream, a dense copy of p into a device buffer the handle
 * owns (allocated at the first call, nx*ny*nz elements), then the copy of that buffer
 * to host_dst (a dense host array of the handle's dtype) on a second stream
 * of the handle. Returns without waiting: sweeps enqueued afterwards run
 * while the transfer proceeds. host_dst must stay valid, and unread, until
 * hj_snapshot_wait; the transfer overlaps only if host_dst is pinned. A
 * further snapshot is ordered after the previous one's transfer. This is the
 * overlapped form of observing the field every k iterations: a transfer the
 * paper's section 3.3 would hoist out of the loop, when the host needs the
 * field inside it. */
int hj_snapshot(hj_solver h, void* host_dst);

/* Wait until the last hj_snapshot's host array is written. HJ_OK with none
 * pending. hj_destroy also waits. */
int hj_snapshot_wait(hj_solver h);

/* The offloaded loop: the Himeno workload's Jacobi iteration (paper section
 * 5.1.1), run on arrays already resident (section 3.3: present data, no
 * transfer inside the loop; only the FP64 gosa values come back).
 * Run n_iter Jacobi iterations with relaxation omega on the resident arrays.
 * gosa_last (nullable) receives the last iteration's gosa, gosa_hist
 * (nullable, n_iter doubles) every iteration's, each computed from the field
 * before that iteration's update. Synchronous. n_iter == 0 is a no-op. */
int hj_sweep(hj_solver h, int n_iter, double omega, double* gosa_last, double* gosa_hist);

/* Paper section 5.1.1 and 3.3 as for hj_sweep.
 * As hj_sweep, but only enqueued on the handle's stream: the per-iteration
 * gosa goes to dev_gosa_hist (nullable device pointer, n_iter doubles). */
int hj_sweep_async(hj_solver h, int n_iter, double omega, double* dev_gosa_hist);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * iterations as hj_sweep_async, with the same results bit for bit, but the
 * call allocates nothing. The per-tile gosa partials go to a file-scope
 * device array of HJ_NOALLOC_SCRATCH_DOUBLES doubles (4 MiB) instead of the
 * handle's buffer, and the kernels are enqueued one by one on the handle's
 * stream (no graph is instantiated). The array's address is looked up when
 * a handle is created on a device. Only enqueued: dev_gosa_hist (device
 * pointer, required, n_iter doubles) receives every iteration's gosa.
 * Errors: HJ_ERR_ARG for a NULL dev_gosa_hist, a current device other than
 * the one the handle was created on, or a configuration whose per-iteration
 * partials (one per tile, of the configured kernel or of the one-iteration
 * kernel that runs remainders) do not fit the array (one iteration's worth,
 * two for two-iteration passes); HJ_ERR_STATE before every input is
 * uploaded. Every call on a GPU shares that GPU's array: calls whose work
 * overlaps on one GPU (other streams, other threads) race and must be
 * ordered by the caller. Nothing needs clearing between calls (each tile
 * writes its own slot before it is read). Captured into a caller's graph,
 * the call records launches between the two field buffers as they stand at
 * capture time; each launch swaps them, so a replay continues the solve
 * only if the call makes an even number of launches (n_iter a multiple of 4
 * with two iterations per pass, even with one); the handle's own record of
 * which buffer holds the field advances once, at the call. */
#define HJ_NOALLOC_SCRATCH_DOUBLES 524288
int hj_sweep_noalloc(hj_solver h, int n_iter, double omega, double* dev_gosa_hist);

/* gosa of the current field, without updating it: the residual sum of the
 * Jacobi iteration of paper section 5.1.1 (the paper names the workload; the
 * sum is this library's reading, stated at the top of this file).
 * Synchronous. */
int hj_residual(hj_solver h, double* gosa);

/* The knobs of paper section 3.2's tuning list (coalesced access, use of the
 * memory levels, occupancy, parallel granularity) as this kernel's
 * configuration. The configuration the next sweep runs with: the library default, the
 * tuning cache's entry for this problem, the last autotune winner or the
 * last hj_set_config. The default of a new solve is the two-iteration
 * kernel on 64-cell rows (kernel HJ_KERNEL_MARCH, bj 8, vec 2, tsteps 2,
 * reread 0, nontemporal 0, xcd_remap 1, use_graph 1) with the i-chunk that
 * keeps its grid to one wave of resident workgroups on the device; when the
 * occupancy query fails, the one-iteration kernel (bj 4 (FP64) or 8 (FP32),
 * vec 2 or 4, nontemporal 1, tsteps 1). hj_set_config returns HJ_ERR_ARG for a configuration
 * the library does not build (see hj_config) or a flat kernel that does not
 * fit the grid, and leaves the previous one in place. */
int hj_get_config(hj_solver h, hj_config* out);
int hj_set_config(hj_solver h, const hj_config* cfg);

/* Paper section 4: candidates are measured on the real program and the
 * fastest measured one is the solution; the result is checked against a
 * reference (there the CPU, with PCAST) before it is used.
 * Measure the candidate configurations on this handle's arrays and keep the
 * fastest one whose field is bitwise equal to the reference configuration's
 * after the same sweeps. The solve's state (p) is restored afterwards.
 * With the environment variable HJ_TUNE_CACHE=<file>, the winner is recorded
 * there (one text line per GPU architecture, dtype and shape), and handles
 * created later for the same problem start from it. A candidate that fails
 * to launch or to match the reference is never chosen.
 * n_sweeps per timing (>= 1; an even count times two-iteration passes
 * without a one-iteration remainder), repeats (>= 1): the median of the
 * repeats is scored.
 * best (nullable) receives the chosen configuration, best_ms its time.
 * HJ_ERR_TUNE when no candidate passed; the configuration then stays as it
 * was. On any error the field is restored and the previous configuration
 * kept. The device memory the search uses (a saved copy of the field and the
 * parity reference) is freed before the call returns.
 * Environment: HJ_TUNE_LOG=<file> appends one CSV line per measurement
 * (configuration, median ms, and "ok", "launch-failed" or "parity-failed").
 * HJ_TUNE_INJECT exercises the failure paths from the host: rules separated
 * by ';', each "launch:" or "parity:" followed by field=value pairs joined by
 * ',' (field names of hj_config), e.g. "launch:tsteps=2;parity:kernel=2". A
 * candidate whose fields match a launch rule scores as a failed launch
 * without running; one matching a parity rule runs and then scores as a
 * parity failure. No kernel is altered. */
int hj_autotune(hj_solver h, int n_sweeps, int repeats, hj_config* best, double* best_ms);

/* The paper's genetic search (sections 4 and 5.1.2) as the search strategy
 * of the autotuner, instead of trying every candidate. A gene is 11 bits and
 * every value names a configuration (hj_gene_config gives the bits).
 * population x generations individuals are measured as by hj_autotune (same
 * parity gate) with fitness (time)^(-1/2); a failed measurement or a gene
 * that names no configuration counts as 1000 s.
 * Roulette selection with elitism, one-point crossover with probability pc,
 * per-bit mutation with probability pm (the paper uses 0.9 and 0.05, and a
 * population and generation count no larger than the gene length). Random
 * numbers come from a counter-based SplitMix64 stream of `seed`. Identical
 * genes are measured once; evaluations (nullable) receives how many were.
 * The winner is installed, recorded in the tuning cache and returned. */
int hj_autotune_ga(hj_solver h, int population, int generations, unsigned long long seed, double pc,
                   double pm, int n_sweeps, int repeats, hj_config* best, double* best_ms,
                   int* evaluations);

/* Paper section 4: a gene of one bit per decision.
 * The configuration a gene names for this problem; every gene names one, and
 * every one of them is among the configurations hj_autotune (or, for batch
 * != 0, hj_batch_autotune) measures, so both searches cover the same space.
 * bit 10: two iterations per pass (1) or one (0).
 * Two iterations (march kernel, nontemporal 0, xcd_remap 1, the settings the
 * exhaustive search keeps for them): bit 0 the row layout (set: vec 2, 64-cell
 * rows, for single solves; vec 4, 30-cell rows, for batches; clear: vec 1,
 * 62-cell rows); bits 1-2 bj (vec 1: 4, 6, 8, 14; vec 2: 4, 6, 8, 12; vec 4:
 * 6, 14, 22, 30); bit 3 reread; bits 5-7 the i-chunk (single solves: the
 * longest that keeps the grid within 256, 512, 768, 1024, 1536, 2048, 4096 or
 * 16384 workgroups; batches: 8, 12, 16, 24, 32, 48, 64 or 128 planes); bits
 * 4, 8 and 9 unused.
 * One iteration: bit 0 the march kernel when set; when clear, for single
 * solves the flat kernel if bit 3 is set, else the direct kernel, and for
 * batches the flat kernel; bits 1-2 bj 1, 2, 4, 8 (flat and direct read 1 as
 * 2); bits 3-4 the march kernel's vec 1, 2, 1, 2 (FP64) or 1, 2, 4, 4 (FP32);
 * bits 5-6 the i-chunk (single solves: the grid of about 1024, 2048, 4096 or
 * 8192 workgroups; batches: 2, 4, 8 or 16 planes); bit 7 unused; bit 8
 * nontemporal; bit 9 the march kernel's xcd_remap (single solves) or the
 * persistent grid (batches). A flat kernel that does not fit the grid reads
 * as the march kernel. Returns HJ_ERR_ARG for an unknown dtype. Host only. */
int hj_gene_config(int dtype, int nx, int ny, int nz, int batch, unsigned gene, hj_config* out);

/* Paper sections 4 and 5.1.2 (the search itself, without a GPU).
 * The same genetic search with the time of every gene given by a table
 * (time_of_gene[g] in seconds for g < 2^gene_bits, gene_bits <= 20). Host
 * only: no GPU is used. history (nullable) receives the genes of every
 * generation, [generations][population]. */
int hj_ga_run(int gene_bits, int population, int generations, unsigned long long seed, double pc,
              double pm, const double* time_of_gene, unsigned* best_gene, double* best_time,
              unsigned* history, int* evaluations);

/* Runtime plumbing (no passage of the paper): wait for all work queued on
 * the handle's stream. */
int hj_sync(hj_solver h);

/* Runtime plumbing: the HIP stream used by the handle (a hipStream_t). */
int hj_get_stream(hj_solver h, void** stream);

/* Wait for the handle's queued work, then release it: its device memory
 * when it owns it (hj_create), its library-created stream, and the handle
 * itself, which is invalid afterwards (HJ_ERR_HANDLE). */
int hj_destroy(hj_solver h);

/* ---- batch of independent solves ---------------------------------------- */

/* Not in the paper: many independent solves of paper section 5.1.1's
 * workload, each resident as section 3.3 prescribes, advanced together so
 * that small grids still fill the GPU.
 * n >= 1 independent solves (the same operator, each with its own shape
 * nx[t] x ny[t] x nz[t], every side >= 3, else HJ_ERR_SHAPE naming the
 * instance) held in one device slab the batch owns, and advanced together:
 * each pass is one launch over a flattened list of every instance's tiles
 * (one iteration, or two with tsteps 2, where an odd remainder runs one
 * one-iteration pass), and the loop is replayed as a captured HIP graph.
 * The shape arrays are read during the call only. stream as for hj_create. */
int hj_batch_create(hj_batch* out, int dtype, int n, const int* nx, const int* ny,
                    const int* nz, void* stream);

/* Paper sections 3.3 and 4, per instance (as hj_upload / hj_download).
 * Upload / download one field of instance inst (0 <= inst < n) as hj_upload
 * / hj_upload_f64 / hj_download do for a single solve (dense host array of
 * that instance's shape; HJ_P also resets the partner; HJ_WRK2 cannot be
 * uploaded). Synchronous. */
int hj_batch_upload(hj_batch b, int inst, int field, const void* host_src);
int hj_batch_upload_f64(hj_batch b, int inst, int field, const double* host_src);
int hj_batch_download(hj_batch b, int inst, int field, void* host_dst);

/* Paper section 5.1.1's iteration on every instance (as hj_sweep).
 * n_iter iterations of every instance (HJ_ERR_STATE until every input field
 * of every instance is uploaded). gosa_last (nullable, n doubles),
 * gosa_hist (nullable, n_iter*n doubles, [iteration][instance]), each
 * instance's sum in a fixed order. Synchronous. */
int hj_batch_sweep(hj_batch b, int n_iter, double omega, double* gosa_last, double* gosa_hist);

/* gosa of every instance's current field (n doubles), no update (as
 * hj_residual). */
int hj_batch_residual(hj_batch b, double* gosa);
int hj_batch_get_config(hj_batch b, hj_config* out);
/* Any supported configuration but the direct kernel; a flat kernel must fit
 * every instance (else HJ_ERR_ARG). xcd_remap and reread are kept for
 * two-iteration passes (tsteps 2, not persistent) and cleared otherwise. */
int hj_batch_set_config(hj_batch b, const hj_config* cfg);
/* Paper section 4 (as hj_autotune).
 * As hj_autotune, over the batch's candidates (one configuration for all
 * instances); the parity gate compares every instance's current field, and
 * the cache line is keyed by a hash of the instance shapes. */
int hj_batch_autotune(hj_batch b, int n_sweeps, int repeats, hj_config* best, double* best_ms);
/* Genetic search over the batch's configuration (as hj_autotune_ga, with
 * the batch reading of the gene that hj_gene_config documents). */
int hj_batch_autotune_ga(hj_batch b, int population, int generations, unsigned long long seed, double pc,
                         double pm, int n_sweeps, int repeats, hj_config* best, double* best_ms,
                         int* evaluations);
/* As hj_destroy: waits, then frees the slab and the handle. */
int hj_batch_destroy(hj_batch b);

/* ---- diagnostics ---------------------------------------------------------- */

const char* hj_status_string(int status);
const char* hj_last_error(void);

/* Measurement (paper section 3.2: how well a loop does on the GPU is known
 * only by measuring it). Device time, in milliseconds, of the last hj_sweep / hj_batch_sweep on this
 * thread, measured with HIP events around the launched work. */
double hj_last_sweep_ms(void);

/* Bandwidth probe with the sweep's access pattern: n_rep launches that read
 * the same 13 arrays and write the same one per interior cell, in the same
 * layout, with no stencil; ms receives the average time per launch. The
 * solve's state is unchanged. */
int hj_stream_probe(hj_solver h, int vec, int ichunk, int n_rep, double* ms);

/* Stream a plain device-to-device copy of `bytes` bytes between two device
 * buffers with the library's copy kernel (the bandwidth ceiling probe). */
int hj_copy_probe(void* dst, const void* src, unsigned long long bytes, void* stream, double* ms);

#ifdef __cplusplus
}
#endif
#endif /* HJ_H */
