/*
 * katz.h -- C ABI of the MI355X (gfx950) certified top-k Katz ranking library.
 *
 * Method: van der Grinten, Bergamini, Green, Bader, Meyerhenke, "Scalable Katz
 * Ranking Computation in Large Static and Dynamic Graphs", ESA 2018.
 *
 *   Katz centrality     c(v) = sum_{i>=1} alpha^i omega_i(v), omega_i(v) the number
 *                       of walks of length i that start at v (Section 1, Eq. (katz)).
 *   Walk recurrence     omega_i(v) = sum_{v->x} omega_{i-1}(x), omega_0 = 1
 *                       (Section 3.2, Eq. (basic_recurrence)): one sparse
 *                       matrix-vector product per iteration.
 *   Bounds after r      l_r = c_r (+ alpha^{r+1} omega_r on undirected graphs),
 *   iterations          u_r = c_r + alpha^{r+1} omega_r gamma,
 *                       gamma = deg_max / (1 - alpha deg_max), alpha < 1/deg_max
 *                       (Section 3.1, Theorem 1; monotone in r by Lemma 2).
 *   Top-k criterion     stop once the k nodes with the largest lower bounds are
 *                       eps-separated, l(w) > u(v) - eps, from each other and from
 *                       every other node (Section 3.1, Eq. (epsilon_sep);
 *                       Algorithm 1 with its converged() test).
 *   Dynamic update      edge insertions I and deletions D, I n E = {}, D c E;
 *                       recompute the walk counts of the affected nodes level by
 *                       level, reactivate, resume (Section 4, Algorithm 2).
 *
 * Conventions shared by every entry point
 *   - Pointers marked "host or device" may point to host memory or to device
 *     memory of the current HIP device; the library detects which with
 *     hipPointerGetAttributes.  Host inputs are copied to the device; host
 *     outputs are written by a device-to-host copy that has completed when the
 *     call returns.
 *   - `stream` is a hipStream_t (NULL = the default stream) of the current
 *     device.  Every call orders its device work on `stream` after earlier
 *     work on that stream.  katz_bounds with both outputs in device memory is
 *     asynchronous: it returns once its work is enqueued, and the outputs are
 *     valid when the stream (or an event recorded on it after the call) has
 *     completed.  Every other call is blocking: when it returns, all its
 *     device work has finished and every output is written (convergence is
 *     data dependent, so the host reads a device flag while iterating).  A
 *     call on another stream that reuses the library's workspace waits for
 *     the previous call's work first.
 *   - The caller owns every input and output buffer; the library never frees
 *     them and keeps no pointer to them after returning (katz_state copies the
 *     graph).  The library allocates its own workspace on the current device.
 *   - Return value: 0 = KATZ_OK; > 0 = a warning, the outputs are written;
 *     < 0 = an error, no output is written and a state passed in is unchanged.
 *     Argument errors are detected before any device work is enqueued.
 *   - Node ids are int32 (0 <= id < n <= 2^31 - 1); arc counts are int64.
 *   - Distinct states may be used from different host threads at once; a single
 *     state is not re-entrant.
 */
#ifndef KATZ_H_
#define KATZ_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define KATZ_OK                  0
#define KATZ_W_ITER_LIMIT        1  /* max_iter reached before certification          */
#define KATZ_W_PRECISION_LIMIT   2  /* FP32 form: bound widths stopped shrinking below */
                                    /* the rounding margin; not certified             */
#define KATZ_W_EXACT_TIES        3  /* walks died out (bounds exact) and a pair is a   */
                                    /* true tie that eps = 0 cannot separate          */
#define KATZ_E_INVALID_ARG      -1  /* null pointer, k < 1, k > n, eps < 0 or NaN, r < 1 */
#define KATZ_E_ALPHA            -2  /* alpha <= 0, NaN, or alpha * deg_max >= 1        */
#define KATZ_E_CSR              -3  /* malformed CSR (see katz_params.validate)        */
#define KATZ_E_UPDATE           -4  /* update batch violates I n E = {}, D c E, ...    */
#define KATZ_E_DEGREE_CAP       -5  /* insertion would exceed the state's degree cap   */
#define KATZ_E_OOM              -6  /* device allocation failed                        */
#define KATZ_E_HIP              -7  /* a HIP runtime call failed                       */
#define KATZ_E_UNSUPPORTED      -8  /* valid request outside what the library supports */
#define KATZ_E_SCRATCH          -9  /* katz_rank_static_noalloc: the problem needs more */
                                    /* workspace than the fixed scratch array holds     */
#define KATZ_E_CANCELLED       -10  /* server: the request was cancelled (or still      */
                                    /* queued when the server was destroyed); it never  */
                                    /* ran                                              */
#define KATZ_E_TIMEOUT         -11  /* server: the request did not finish within the    */
                                    /* wait's time limit; its ticket stays valid        */
#define KATZ_E_BUSY            -12  /* server: the request is on the device or finished */
                                    /* and can no longer be cancelled                   */

/* ---- precision forms ------------------------------------------------------ */
#define KATZ_FP64         0  /* walk vector, sums and bounds in FP64 (the plain method)  */
#define KATZ_FP32_MARGIN  1  /* walk vector and row sums in FP32; c, bounds and the     */
                             /* rounding-error margin that widens both bounds in FP64    */

/* ---- stopping criteria (Section 3.1) -------------------------------------- */
#define KATZ_TOPK         0  /* the k nodes with the largest lower bounds are eps-     */
                             /* separated from each other and from every other node  */
#define KATZ_RANKING      1  /* every node eps-separated from every other: the top-k  */
                             /* criterion with k = n (katz_params.k is ignored)       */
#define KATZ_SCORE        2  /* every score known to within eps: u - l < eps for all  */
                             /* nodes; the output lists all n nodes (k is ignored)    */
#define KATZ_PAIR         3  /* the two nodes pair_u, pair_v are eps-separated; the   */
                             /* output lists those two nodes (k is ignored)           */

/* ---- CSR validation levels -------------------------------------------------- */
#define KATZ_VALIDATE_NONE    0  /* trust the caller                                   */
#define KATZ_VALIDATE_BASIC   1  /* row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz,  */
                                 /* 0 <= col < n (default)                             */
#define KATZ_VALIDATE_STRICT  2  /* BASIC + rows strictly increasing (no duplicates),   */
                                 /* no self-loops, and symmetry when undirected = 1     */

/* ---- option flags (katz_params.flags) --------------------------------------- */
#define KATZ_FLAG_NO_REORDER  1  /* keep the caller's node order on the device.  By     */
                                 /* default static calls and dynamic states renumber    */
                                 /* nodes internally by degree class (rows of similar   */
                                 /* length contiguous, high-degree nodes first) so the  */
                                 /* walk vector's most gathered entries share cache     */
                                 /* lines; results, ids and tie order are the same      */
                                 /* either way (a state keeps each row in the caller-id */
                                 /* order of its entries).  A batch (count > 1) is      */
                                 /* renumbered graph by graph only when some graph's    */
                                 /* walk vector is larger than 4 MiB (one XCD's L2;     */
                                 /* smaller ones stay cached whatever the order) or a   */
                                 /* graph sets KATZ_FLAG_REORDER; NO_REORDER on any     */
                                 /* graph of a batch turns it off.                      */
#define KATZ_FLAG_REORDER     2  /* renumber a batch even where its graphs are small.   */
#define KATZ_FLAG_INBOUND     4  /* inbound Katz centrality (Section 2.1): count the     */
                                 /* walks that end at each node.  It equals the         */
                                 /* outbound centrality of the reverse graph, which the */
                                 /* library builds on the device (a stable transpose:  */
                                 /* each reversed row lists its sources in ascending    */
                                 /* order, so runs stay deterministic) and ranks in     */
                                 /* place of the graph.  Directed graphs only; on an    */
                                 /* undirected graph (its own reverse) the flag changes */
                                 /* nothing.  Offsets and column ids are always checked */
                                 /* before the transpose.  Taken by every ranking call, */
                                 /* batches included, katz_bounds, katz_solve and       */
                                 /* states (update pairs (u, v) still denote the        */
                                 /* caller's arc u -> v); katz_rank_static_noalloc      */
                                 /* returns E_UNSUPPORTED for it (the reverse graph     */
                                 /* needs a workspace of its own).                      */

/* A graph in compressed sparse row form.  Row v lists the out-neighbours of v:
 * arcs v -> col[j] for row_ptr[v] <= j < row_ptr[v+1].  An undirected graph
 * stores both arcs of each edge (Section 2.1) and sets undirected = 1, which
 * enables the improved lower bound of Section 3.1.  row_ptr and col: host or
 * device, read only. */
typedef struct katz_csr {
  int64_t n;              /* number of nodes, 1 <= n <= 2^31 - 1                    */
  int64_t nnz;            /* number of arcs = row_ptr[n]                            */
  const void* row_ptr;    /* n + 1 offsets: int32 if row_ptr_64 = 0, else int64     */
  const int32_t* col;     /* nnz target ids                                         */
  int32_t row_ptr_64;     /* 0: row_ptr is int32 (needs nnz < 2^31); 1: int64       */
  int32_t undirected;     /* 1: symmetric adjacency                                 */
} katz_csr;

/* Problem parameters (Section 3: alpha, k, eps and the stopping criterion). */
typedef struct katz_params {
  double alpha;           /* attenuation, 0 < alpha < 1/deg_max (Theorem 1);        */
                          /* 0.0 selects 1/(1 + deg_max) (Section 3.1)              */
  double epsilon;         /* separation tolerance eps >= 0 (absolute); 0 = strict   */
  int32_t k;              /* top-k: 1 <= k <= n (batches and states: k <= 4096)     */
  int32_t max_iter;       /* iteration cap; 0 selects 1000                          */
  int32_t precision;      /* KATZ_FP64 or KATZ_FP32_MARGIN                          */
  int32_t criterion;      /* KATZ_TOPK, KATZ_RANKING, KATZ_SCORE or KATZ_PAIR       */
  int32_t validate;       /* KATZ_VALIDATE_*; applies to the input CSR              */
  int32_t flags;          /* KATZ_FLAG_* bits; 0 = defaults                         */
  int64_t degree_cap;     /* states only: the largest deg_max that edge insertions  */
                          /* may create; 0 = the initial deg_max.  alpha must obey  */
                          /* alpha * degree_cap < 1.                                */
  int32_t pair_u;         /* KATZ_PAIR: the two distinct node ids to separate;      */
  int32_t pair_v;         /* ignored by the other criteria                          */
} katz_params;

/* Output of a ranking call.  topk_ids, lower, upper: caller-owned arrays of
 * k elements (KATZ_TOPK), n elements (KATZ_RANKING, KATZ_SCORE) or 2 elements
 * (KATZ_PAIR), host or device, written in ranking order (lower bound
 * descending, ties by ascending id).  The scalar fields are written by the
 * library. */
typedef struct katz_result {
  int32_t* topk_ids;       /* [k] node ids                                          */
  double* lower;           /* [k] l_r of each ranked node (FP32 form: widened)      */
  double* upper;           /* [k] u_r of each ranked node (FP32 form: widened)      */
  double rest_upper_max;   /* max u_r over the nodes outside the top-k; -inf if k=n */
  double alpha_used;       /* the alpha the run used                                */
  double eta;              /* FP32 form: relative error bound of the walk vector at */
                           /* the last iteration; 0 for FP64                        */
  int64_t active_final;    /* |M| when the run stopped (k once certified)           */
  int32_t iterations;      /* r                                                     */
  int32_t status;          /* same value as the return code                         */
  double separated_fraction; /* KATZ_RANKING, KATZ_SCORE: fraction of the n(n-1)/2  */
                           /* unordered node pairs {w, v} that the final bounds     */
                           /* separate, l(w) > u(v) or l(v) > u(w) (the separation  */
                           /* measure of Table 1); NaN for the other criteria       */
} katz_result;

/* Library-owned, device-resident state for dynamic updates: a copy of the graph
 * (CSR with per-row slack), the walk-vector history x_0..x_r, c_r and the active
 * set M (Section 4: Algorithm 2 resumes from Algorithm 1's state). */
typedef struct katz_state katz_state;

/*
 * katz_rank_static -- Algorithm 1 (Section 3.2) with a stopping criterion of
 * Section 3.1 (katz_params.criterion).
 *
 * Ranks `count` independent graphs: g[i] with parameters p[i] into out[i].
 * count = 1 is the plain call; count > 1 runs all graphs together (one walk
 * sparse matrix-vector product per iteration over every graph that is still
 * iterating, per-graph selection and separation test), each with its own alpha,
 * k and eps.
 *
 * Criteria: KATZ_TOPK takes any 1 <= k <= n (past 4096 the top-k is sorted by
 * a device-wide sort instead of one workgroup's LDS sort); KATZ_RANKING is the
 * top-k test with k = n; KATZ_SCORE stops once u - l < eps for every node and
 * then lists all n nodes; KATZ_PAIR stops once pair_u and pair_v are
 * eps-separated.  Batches (count > 1) and states take KATZ_TOPK with
 * k <= 4096 only.
 *
 * states: NULL, or an array of `count` pointers that receives one new
 *         katz_state per graph for later katz_rank_update calls (FP64 or
 *         FP32 form, undirected or directed; free each with katz_state_free).
 *         An FP32 state sizes its scales and error tables (Section 3.3) for
 *         the degree cap, so they hold for every graph its updates may reach.
 * Errors: E_INVALID_ARG (also: pair ids out of range or equal), E_ALPHA,
 *         E_CSR, E_UNSUPPORTED (a batch or a state with a criterion other than
 *         top-k or k > 4096), E_OOM, E_HIP.  With
 *         count > 1 the first failing graph's error is returned and nothing is
 *         written for any graph.
 */
int katz_rank_static(int32_t count, const katz_csr* g, const katz_params* p,
                     katz_result* out, katz_state** states, void* stream);

/*
 * katz_rank_update -- Algorithm 2 (Section 4): apply one batch of insertions
 * (ins_u[i], ins_v[i]) and deletions (del_u[i], del_v[i]) to the state's
 * graph, recompute the walk counts of every affected node for levels 1..r,
 * patch c_r, recompute the bounds, reactivate nodes whose upper bound reaches
 * min_{x in M} l(x) - eps, and iterate further until converged() holds.
 * An FP32 state re-walks each level with the scale it was first computed
 * with, so its recomputed entries carry the history's arithmetic; should a
 * re-walked entry exceed 2^64 (the scales no longer fit the graph), the
 * update instead re-runs Algorithm 1 from level 1 on the new graph.
 * On an undirected graph each pair is an edge (both arcs); on a directed graph
 * it is the arc u -> v (the reverse arc is a different arc), and the affected
 * nodes are found by a search over reverse arcs, which the state keeps as a
 * second CSR.  An inbound state (KATZ_FLAG_INBOUND) takes the caller's arcs
 * and stores each as its reverse.  The batch is atomic: it is validated whole
 * (ids in range, no self-loops, no pair twice, inserted edges or arcs absent,
 * deleted ones present, none both inserted and deleted, degree cap) and
 * rejected with E_UPDATE / E_DEGREE_CAP before the state changes.
 * The id arrays: host or device; n_ins or n_del may be 0 (arrays then unused).
 * The result has the state's k.  Errors: E_INVALID_ARG, E_UPDATE,
 * E_DEGREE_CAP, E_OOM, E_HIP.
 */
int katz_rank_update(katz_state* st, const int32_t* ins_u, const int32_t* ins_v,
                     int64_t n_ins, const int32_t* del_u, const int32_t* del_v,
                     int64_t n_del, katz_result* out, void* stream);

/*
 * katz_bounds -- exactly r iterations of Algorithm 1 without a convergence test,
 * then l_r and u_r of every node (Section 3.1, Theorem 1).  This is the score
 * surface used for parity checks.  lower, upper: caller-owned arrays of n
 * doubles, host or device, indexed by node id.  p->k, p->epsilon and
 * p->max_iter are ignored.  With both arrays in device memory the call is
 * stream-ordered and asynchronous (every error, E_CSR included, is returned
 * before it enqueues the iterations); otherwise it blocks until the host
 * arrays are written.  Errors: E_INVALID_ARG (r < 1), E_ALPHA, E_CSR, E_OOM,
 * E_HIP.
 */
int katz_bounds(const katz_csr* g, const katz_params* p, int32_t r,
                double* lower, double* upper, void* stream);

/*
 * katz_rank_static_noalloc -- katz_rank_static for one graph (count = 1, no
 * states), for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  It calls no
 * hipMalloc, hipHostMalloc, hipFree or hipHostFree: its workspace is a static
 * device array of 64 MiB that every device using the library holds until the
 * process ends, and its flag read-backs go to static host memory (so the host
 * waits for each iteration instead of reading the stop flag one iteration
 * behind).  The first call on a device looks up that device's copy of the
 * array (hipGetSymbolAddress).  The phase timers (katz_timing_*) are not
 * recorded.
 *
 * Arguments, outputs and results are those of katz_rank_static with
 * count = 1 and states = NULL; the results are bitwise the same.  A graph
 * whose workspace (about 140 bytes per node plus 4 bytes per arc, more for
 * host inputs or outputs) exceeds the array returns E_SCRATCH before any
 * device work.  Every call on a device shares that device's array, and it
 * keeps the last call's contents: calls that overlap on one device (from
 * several host threads or on several streams) race and must be serialised
 * by the caller.
 * Errors: those of katz_rank_static, and E_SCRATCH.
 */
int katz_rank_static_noalloc(const katz_csr* g, const katz_params* p,
                             katz_result* out, void* stream);

/* ---- the paper's comparison methods (Sections 2.2 and 5) ----------------------
 * Score vectors by the methods the paper compares against, on the same device
 * kernels (the walk step's sparse matrix-vector product y = alpha A v, FP64,
 * in the caller's node order), for comparison with the bound-based ranking.
 *   KATZ_SOLVE_FOSTER  Foster's heuristic (Section 2.2): f_0 = 1,
 *                      f_{i+1} = alpha A f_i + 1, stopped once the largest
 *                      change of an entry, max_v |f_{i+1}(v) - f_i(v)|, is below
 *                      tol; scores = f - 1.  No correctness guarantee.
 *   KATZ_SOLVE_CG      conjugate gradients without preconditioning on Eq.
 *                      (la), (I - alpha A) z = 1, from z = 0, stopped once the
 *                      relative residual ||1 - (I - alpha A) z||_2 / sqrt(n) is
 *                      below tol; scores = alpha A z (Section 1).  Undirected
 *                      graphs only (the matrix must be symmetric).
 */
#define KATZ_SOLVE_FOSTER 0
#define KATZ_SOLVE_CG     1

typedef struct katz_solve_info {
  int32_t iterations;      /* sparse matrix-vector products of the iteration        */
  int32_t converged;       /* 1: the stopping test held; 0: max_iter was reached   */
  double residual;         /* the last tested quantity (max change / rel. residual) */
  double alpha_used;
} katz_solve_info;

/*
 * katz_solve -- Katz scores of every node by Foster's heuristic or by CG.
 * p->alpha (0.0 selects 1/(1 + deg_max)), p->max_iter (0 selects 1000) and
 * p->validate are used; the other fields are ignored.  scores: caller-owned
 * array of n doubles, host or device, indexed by node id.  info may be NULL.
 * Blocking.  Returns KATZ_OK when the stopping test held, W_ITER_LIMIT when
 * max_iter was reached first (scores hold the last iterate).  Errors:
 * E_INVALID_ARG (method, tol <= 0), E_ALPHA, E_CSR, E_UNSUPPORTED (CG on a
 * directed graph), E_OOM, E_HIP.
 */
int katz_solve(const katz_csr* g, const katz_params* p, int32_t method, double tol,
               double* scores, katz_solve_info* info, void* stream);

/* Frees a state from katz_rank_static (NULL is ignored). */
void katz_state_free(katz_state* st);

/*
 * katz_state_save / katz_state_load -- checkpoint and resume of a dynamic state
 * (Section 4: Algorithm 2 continues from Algorithm 1's walk counts, bounds and
 * active set).  save writes the state's graph (slack CSR, and the reverse CSR
 * of a directed state), its renumbering, the walk history x_1..x_r, c_r, the
 * active set M and the run flags to the file at `path` (host file system); it
 * waits for the state's device work first.  load recreates the state on the
 * current device: updates applied to it then give bitwise the results they
 * give on the saved state.  A file written by a library with another state
 * layout is refused.  Errors: E_INVALID_ARG (null arguments, a file that
 * cannot be opened, read or written, or is not a state file of this layout),
 * E_OOM, E_HIP.
 */
int katz_state_save(katz_state* st, const char* path);
int katz_state_load(const char* path, katz_state** out, void* stream);
/* The node count n and the k of a state (for a caller that restored one). */
int katz_state_size(const katz_state* st, int64_t* n, int32_t* k);

/* A static, human-readable description of a status code. */
const char* katz_strerror(int code);

/* ---- serving: continuous admission of update batches -------------------------
 * A server owns dynamic states (katz_rank_update, Algorithm 2 of Section 4)
 * and a pool of `slots` worker threads, each with its own HIP stream on the
 * device current at creation.  An update runs in two halves: the host half
 * (the batch validated on its own and its arcs grouped by row; it reads no
 * graph state) and the device half (existence checks against the graph, the
 * merge, the re-walk, the re-certification).  The device halves of one
 * graph's requests run in submission order, one at a time, so the result of
 * a request reflects exactly that graph's batches up to it; their host halves
 * run ahead, on idle slots, while earlier requests of the same graph are on
 * the device.  Requests of different graphs run concurrently and overlap on
 * the device.  A prepared request is admitted when a slot is free and its
 * device-memory estimate (batch buffers, row merges, one more walk-history
 * level and the slack-pool growth of its insertions) fits `memory_budget`
 * bytes (0 = unlimited).  All buffers passed to these calls are host memory. */
typedef struct katz_server katz_server;

/* 1 <= slots <= 64.  Errors: E_INVALID_ARG, E_HIP. */
int katz_server_create(int32_t slots, int64_t memory_budget, katz_server** out);
/* Ranks g statically (katz_rank_static with a state, FP64 or FP32 form;
 * undirected, directed or inbound) and registers it; writes its initial result to out and its id to graph_id. */
int katz_server_add_graph(katz_server* sv, const katz_csr* g, const katz_params* p, katz_result* out,
                          int32_t* graph_id);
/* Queues one batch (arrays are copied before returning) and returns a ticket. */
int katz_server_submit(katz_server* sv, int32_t graph_id, const int32_t* ins_u, const int32_t* ins_v,
                       int64_t n_ins, const int32_t* del_u, const int32_t* del_v, int64_t n_del,
                       int64_t* ticket);
/* Blocks until the ticket's request has run; writes its result (out's arrays:
 * host, k entries), its latency from submission and its service time in ms
 * (either pointer may be NULL).  Returns the request's status code. */
int katz_server_wait(katz_server* sv, int64_t ticket, katz_result* out, double* latency_ms,
                     double* service_ms);
/* katz_server_wait with a time limit (timeout_ms >= 0): E_TIMEOUT when the
 * request has not finished by then; the ticket stays valid and may be waited
 * for again or cancelled.  Other errors as katz_server_wait. */
int katz_server_wait_for(katz_server* sv, int64_t ticket, int64_t timeout_ms, katz_result* out,
                         double* latency_ms, double* service_ms);
/* Cancels a request that has not reached the device: it leaves its graph's
 * queue, never runs (later requests of the graph do not include its batch),
 * and its waiter gets E_CANCELLED.  Returns OK, E_BUSY (already on the device
 * or finished) or E_INVALID_ARG (unknown or already collected ticket). */
int katz_server_cancel(katz_server* sv, int64_t ticket);
/* Stops the server: requests that have not started their device half end
 * with E_CANCELLED (a thread blocked in katz_server_wait on one returns that
 * code), requests on the device finish, then the workers stop, the call waits
 * for every katz_server_wait in progress to return, and the states are freed.
 * No call on sv may start once destroy has begun.  add_graph, submit and wait
 * may otherwise be called from any thread while requests run. */
void katz_server_destroy(katz_server* sv);

/* ---- device timing (instrumentation for benchmarks and profiles) ----------
 * While enabled, every ranking and bounds call records hipEvent pairs on its own stream
 * around each of its phases and adds the elapsed device times to process-wide
 * counters when the call has finished.  walk_step covers the walk
 * sparse matrix-vector product of iterations r >= 2 (one kernel launch per
 * iteration); walk_first covers iteration 1 (x_0 = 1 needs no gather, plus the
 * column-range check); select covers the selection and converged() kernels of
 * every iteration.  Recording adds a little host work per launch. */
typedef struct katz_timing {
  double walk_step_ms;       int64_t walk_step_launches;
  double walk_first_ms;      int64_t walk_first_launches;
  double select_ms;          int64_t select_iterations;
  double prep_ms;            /* staging, binning, d_max read-back              */
  double result_ms;          /* output kernels                                 */
  double call_ms;            /* first to last event of each call, summed       */
  int64_t calls;
  /* Walk step 2 of renumbered static calls, which also renames the column ids
   * (counted here, not in walk_step_*).                                        */
  double renumber_step_ms;   int64_t renumber_step_launches;
} katz_timing;

/* on = 1: reset the counters and start recording; on = 0: stop. */
void katz_timing_enable(int on);
/* Copies the counters; E_INVALID_ARG if out is NULL. */
int katz_timing_read(katz_timing* out);

/* ---- launch tuning of the walk kernels ------------------------------------
 * Process-wide launch shape of the walk step (the degree-binned SpMV of Eq.
 * (basic_recurrence), Section 3.2).  No setting but split_hot_bytes and
 * bin_bounds changes any result bit: every row is still summed by the same
 * lane schedule, and the LDS copy holds exact walk entries.
 *   hub_bytes            single-graph static calls with the internal
 *                        renumbering: bytes of LDS per workgroup that hold a
 *                        copy of the first walk entries (after the renumbering,
 *                        the nodes with the longest rows, which most arcs point
 *                        to); 0 = no copy.  0 .. 65536, a multiple of 16
 *                        (0 .. 162816 with walk_groups = 4).
 *   blocks_per_cu        single-graph calls: persistent walk grid of this many
 *                        workgroups per compute unit, each taking work items
 *                        with a grid stride; 0 = one workgroup per work item.
 *                        0 .. 32.  A non-zero hub_bytes needs a non-zero
 *                        blocks_per_cu (the copy is filled once per workgroup).
 *   batch_blocks_per_cu  the same for the batched form (count > 1); 0 .. 32.
 *   batch_tile           batched form: row groups per work item of the short-row
 *                        bins (each wave sums its rows group after group, each row
 *                        still by the same lanes); 0 or 1 = one group, up to 16.
 *   walk_groups          single-graph calls: 4 = workgroups of four 256-thread
 *                        groups that share one LDS copy of hub_bytes, each group
 *                        working as one workgroup does (blocks_per_cu then counts
 *                        these 1024-thread workgroups); 0 or 1 = 256-thread
 *                        workgroups.
 *   batch_xcd            batched form: 1 = give every graph to one of the eight
 *                        XCDs (balanced by arcs) and let the workgroups that the
 *                        hardware places on an XCD take only its graphs' work
 *                        items, so each XCD's L2 holds the walk vectors of an
 *                        eighth of the batch; 0 = any workgroup takes any item.
 *   split_hot_bytes      single-graph static calls with the internal
 *                        renumbering, walk steps 3, 4, ...: the walk step runs
 *                        in two passes, the first summing each row's entries
 *                        of the hottest nodes (the first split_hot_bytes of
 *                        the walk vector: a set that stays in an XCD's L2),
 *                        the second the others and adding the first pass's
 *                        partial sum (one more rounding level, counted in the
 *                        FP32 margin).  0 = one pass (default); > 0 = two
 *                        passes with this hot set (a multiple of 16, at most
 *                        64 MiB).  The split changes the order of
 *                        additions, so results differ from one-pass runs in
 *                        their rounding (both certified); the autotuner leaves
 *                        it unchanged.
 *   bin_bounds           the row-length classes of the degree binning: rows of
 *                        length 1..b0 are summed by one lane, b0+1..b1 by one,
 *                        b1+1..b2 by 2, b2+1..b3 by 4, b3+1..b4 by 16 lanes,
 *                        b4+1..b5 by a wave, b5+1..4096 by a workgroup, longer
 *                        rows by 4096-arc segments.  All 0 = the defaults
 *                        {4, 8, 16, 32, 128, 1024}.  The classes fix the order
 *                        of each row's additions, so results differ from
 *                        other classes in their rounding (both certified);
 *                        the autotuner searches a few tables.  A state keeps
 *                        the classes of its creation.
 * Defaults: all 0.  Calls already running keep the setting they started with. */
typedef struct katz_tuning {
  int32_t hub_bytes;
  int32_t blocks_per_cu;
  int32_t batch_blocks_per_cu;
  int32_t batch_tile;
  int32_t batch_xcd;         /* 0 or 1 */
  int32_t walk_groups;       /* 0, 1 or 4 */
  int32_t split_hot_bytes;   /* 0, or 16 .. 64 MiB */
  int32_t bin_bounds[6];     /* all 0, or 1 <= b0 < b1 < ... < b5 < 4096 */
  int32_t reserved;          /* must be 0 */
} katz_tuning;

/* Copies the current setting; E_INVALID_ARG if t is NULL. */
int katz_tuning_get(katz_tuning* t);
/* Replaces the setting; E_INVALID_ARG (and no change) for values out of range. */
int katz_tuning_set(const katz_tuning* t);
/* Autotuner: times katz_rank_static(count, g, p) on `stream` under each
 * candidate launch shape (two calls each, the second timed), installs the
 * fastest and copies it to *best (may be NULL).  count = 1 tunes hub_bytes and
 * blocks_per_cu, count > 1 tunes batch_blocks_per_cu and batch_tile; the other
 * fields keep their values.  Inputs as for katz_rank_static; returns the first error of a
 * ranking call (the setting is then left unchanged), or KATZ_OK. */
int katz_autotune(int32_t count, const katz_csr* g, const katz_params* p, katz_tuning* best, void* stream);
/* Autotuner cache: with a path set, katz_autotune first looks its workload up
 * in that text file and, on a hit, installs the stored setting without timing
 * anything; after tuning it appends the result.  A workload is keyed by the
 * device (architecture, compute units), the graph count, the total nodes and
 * arcs, and the precision, criterion, flags and direction of the first graph.
 * One line per entry: the key, a tab, the 13 katz_tuning fields before
 * `reserved` as decimal integers; the last valid line of a key wins, and lines
 * that do not parse or hold an invalid setting are ignored.  The file is read
 * and appended by plain stdio calls (no locking between processes).  path =
 * NULL or "" turns the cache off (the default).  Returns KATZ_OK. */
int katz_autotune_cache(const char* path);

#ifdef __cplusplus
}
#endif

#endif /* KATZ_H_ */
