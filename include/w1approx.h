/*
 * w1approx: approximate 1-Wasserstein distance between persistence diagrams
 * on one AMD Instinct MI355X (gfx950), after Dey & Zhang, "Approximating
 * 1-Wasserstein Distance between Persistence Diagrams by Graph
 * Sparsification" (Alg. 3, the approximate W1 algorithm).
 *
 * The library runs the data-parallel part of the method as HIP kernels:
 *   a0  0-condensation of A u B into net weighted locations (Sec. 4.3),
 *   a1  RWMD lower bound L (Alg. 1, Sec. 5.1),
 *   a2  delta-condensation onto a power-of-two grid (Alg. 2,
 *       Prop. delta-condensation),
 *   a3  binary radix tree over Morton-ordered cells (the hierarchy for the
 *       WSPD, Sec. 5.3 split-tree paragraph),
 *   a4  s-WSPD pairs (Alg. 4-6),
 *   a5  the sparse transshipment network: biarcs, diagonal arcs (Alg. 7) and
 *       supplies, as compressed sparse rows with the arcs sorted by tail,
 *       then head (Appendix, representation of the transshipment network),
 * and then solves the uncapacitated min-cost flow of that network on the host
 * with an integer network simplex (Sec. 5.4), timed separately.  The solve
 * leaves out the cell arcs that cost at least both ends' diagonal arcs
 * together (on the Euclidean network, plus a margin for its rounded costs):
 * some optimal flow never uses them, so F* is that of the whole network,
 * which is still what the result holds; pivots count the reduced solve.
 *
 * Ground metric: L-infinity by default.  Distance to the diagonal of (b, d):
 * (d - b)/2.  Costs of the network are integers in units of g/2,
 * g = 2^grid_exp.  w1 = (g/2)(F* + n), w1_paper = (g/2) F*.
 * Guarantee: exact_W1 <= w1 <= (1 + eps) * exact_W1 and
 *            lower_bound <= exact_W1.
 *
 * Euclidean metric (W1_METRIC_L2, the paper's own, Sec. 4.2): distance to
 * the diagonal (d - b)/sqrt(2), computed as (d - b) R with R the double
 * nearest to 1/sqrt(2).  The RWMD cost of a location is min(sqrt(q), (d - b)
 * R) with q the smallest (b - b')^2 + (d - d')^2 over the other diagram, in
 * IEEE doubles.  The grid satisfies g <= sqrt(2) eps_c L / n (a point moves by
 * at most half a cell diagonal).  Two nodes are separated when their
 * Euclidean box gap is at least s times the larger box diagonal (exact on
 * integer squares); the longer diagonal is split.  Network costs are 64-bit
 * integers in units of g 2^-K (K = cost_shift = min(30, 59 - bitlen(n) -
 * bitlen(X)), X the largest shifted cell coordinate): between cells
 * ceil(sqrt(di^2 + dj^2) 2^K), to the diagonal ceil((j - i) R 2^K), each from
 * IEEE doubles.  w1 = g (F* 2^-K + n R), w1_paper = g F* 2^-K.  The same
 * guarantee holds up to the rounding of one square root per cost and of R
 * (relative 2^-52).  The pair records' cost word is 0 with this metric.
 *
 * Conventions for every entry point
 *   - returns W1_OK (0) or a negative W1_E* code; never aborts, never throws;
 *   - input point arrays are borrowed for the duration of the call; rows are
 *     (birth, death) pairs, row-major, FP32 or FP64 as given by `dtype`;
 *     death == birth rows lie on the diagonal and are ignored; death < birth
 *     or a non-finite value gives W1_EINVAL;
 *   - `stream` is a hipStream_t (NULL = the null stream).  Device inputs
 *     must be ready on that stream.  The call synchronises the stream before
 *     it returns;
 *   - a w1_ctx is not thread-safe: use one per host thread.  It keeps its
 *     device buffers between calls (they only grow);
 *   - arrays inside a w1_result are allocated by the library and released by
 *     w1_result_free only.
 */
#ifndef W1APPROX_H
#define W1APPROX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define W1_OK 0
#define W1_EINVAL (-1)    /* bad argument or invalid diagram point          */
#define W1_ERANGE (-2)    /* grid extent >= 2^30 cells, coordinates too      */
                          /* large for exact integer snapping, or a network  */
                          /* too large for its row form: more than 2^22      */
                          /* cells in one launch group, or bucket and head   */
                          /* bits above 32 (above 2^21 cells in one pair)    */
#define W1_ENOMEM (-3)    /* device or host allocation failed                */
#define W1_EHIP (-4)      /* HIP runtime error (see w1_ctx_hip_error)        */
#define W1_EOVERFLOW (-5) /* internal work list capacity exceeded            */
#define W1_ENODEV (-6)    /* no usable gfx950 device                         */

/* ---- w1_result.status --------------------------------------------------- */
#define W1_OPTIMAL 0      /* flow solved to optimality (or not requested)    */
#define W1_STALLED 1      /* pivot_cap reached: the flow is not optimal.  If */
                          /* it meets every supply, flow_cost is its cost    */
                          /* and w1 >= exact W1 still holds (without the     */
                          /* (1 + eps) bound); otherwise flow_solved = 0,    */
                          /* flow_cost = -1 and w1 = w1_paper = NaN          */

/* ---- dtypes -------------------------------------------------------------- */
#define W1_F32 0
#define W1_F64 1

/* ---- w1_params.flags ------------------------------------------------------ */
#define W1_INPUT_DEVICE 1u /* w1_pd.xy are device pointers                  */
#define W1_COUNT_ONLY 2u   /* stop after counting WSPD pairs (no arcs, flow) */
#define W1_NO_FLOW 4u      /* build the network on the device, skip the flow */
#define W1_KEEP_NETWORK 8u /* copy the network into the result (host)       */
#define W1_KEEP_STAGES 16u /* copy stage intermediates into the result      */
#define W1_PRUNE 32u       /* leave out diagonal-dominated WSPD pairs: a    */
                           /* node pair U, V whose box gap (in grid cells)  */
                           /* is at least half of (U.maxj - U.mini) +       */
                           /* (V.maxj - V.mini), with everything below it   */
                           /* in the WSPD recursion.  Each such arc costs   */
                           /* at least its two ends' diagonal arcs, so the  */
                           /* optimal flow cost F*, w1 and w1_paper are     */
                           /* unchanged and the network is smaller (not in  */
                           /* the paper; follows from the matching costs of */
                           /* Sec. 4.3: the distance to the diagonal is     */
                           /* 1-Lipschitz, and the zero-cost diagonal arc   */
                           /* carries at least the cell-to-cell flow).      */
                           /* n_pairs then counts the pairs kept.  Not with */
                           /* W1_METRIC_L2 (W1_EINVAL).                     */
#define W1_METRIC_L2 64u   /* Euclidean ground metric, the paper's own      */
                           /* (Sec. 4.2), instead of L-infinity: see the    */
                           /* Euclidean notes at the top of this file       */
#define W1_PAPER_GRID 128u /* with s_override > 0: the paper's own grid for */
                           /* that s (Alg. 2, Alg. 3): eps_c = 8/(s - 4) for */
                           /* s >= 12 and 1 below, in place of kappa * eps  */
                           /* (eps and kappa are then unused); the grid    */
                           /* bound g <= 2 eps_c L / n is unchanged.        */
                           /* Without s_override W1_EINVAL                  */

typedef struct w1_ctx w1_ctx;

/* One persistence diagram: n rows of (birth, death). */
typedef struct {
  const void *xy;
  int64_t n;
  int32_t dtype;    /* W1_F32 or W1_F64 */
  int32_t reserved; /* must be 0 */
} w1_pd;

typedef struct {
  double eps;         /* target relative error, 0 < eps <= 1                  */
  double cond_frac;   /* share kappa of eps spent on grid condensation,        */
                      /* 0 < kappa < 0.5; 0 selects 0.1                         */
  int32_t s_override; /* > 0: use this WSPD separation s instead of the one   */
                      /* derived from eps (the (1+eps) bound then does not     */
                      /* hold; this is the paper's sparsity-parameter mode of */
                      /* Sec. 5.5; s <= 2 has no stretch bound at all, as for */
                      /* its s = 1 runs in Sec. 7, but w1 is still an upper   */
                      /* bound on W1); < 0 is W1_EINVAL                        */
  uint32_t flags;     /* W1_* flags above                                      */
  int64_t pivot_cap;  /* network simplex pivot limit, 0 = unlimited            */
} w1_params;

/* Per-stage timings in milliseconds (t_ms index). */
#define W1_T_CONDENSE0 0 /* a0 */
#define W1_T_RWMD 1      /* a1 */
#define W1_T_GRID 2      /* a2 */
#define W1_T_TREE 3      /* a3 */
#define W1_T_WSPD 4      /* a4 */
#define W1_T_ARCS 5      /* a5 */
#define W1_T_D2H 6       /* network copy to the host */
#define W1_T_FLOW 7      /* host min-cost flow */

typedef struct {
  double w1;          /* (g/2)(F* + n): certified, exact <= w1 <= (1+eps) exact */
  double w1_paper;    /* (g/2) F*: the paper's value on the condensed network  */
  double lower_bound; /* RWMD lower bound L (exact fixed-point sum, rounded down) */
  double grid;        /* g = 2^grid_exp                                          */
  int32_t grid_exp;
  int32_t s;          /* WSPD separation used                                    */
  int32_t status;     /* W1_OPTIMAL / W1_STALLED, or a negative W1_E* for this pair */
  int32_t flow_solved;/* 1 if w1 / w1_paper / flow_cost come from a flow solve   */
  int64_t n_points;   /* n = nA + nB after co-located A/B points cancel          */
  int64_t n_a, n_b;
  int64_t n_locations;/* distinct (birth, death) locations with net mass != 0    */
  int64_t n_cells;    /* grid cells = network nodes other than the two diagonal nodes */
  int64_t n_pairs;    /* WSPD pairs = biarcs                                    */
  int64_t n_arcs;     /* directed arcs: 2 n_pairs + n_diag (0 with COUNT_ONLY) */
  int64_t flow_cost;  /* F* in units of g/2 (-1 if not solved)                 */
  int64_t pivots;     /* network simplex pivots                                 */
  /* Streamed emission (W1_COUNT_ONLY with w1_tuning.stream_arena_pairs > 0):
   * the pairs written through the arena, and an order-independent checksum
   * of them (test bookkeeping): with h(u, v, c) = (((u + 1) K1 + (v + 1)) K2
   * + c) K3 mod 2^64 over the pair records (u = representative of the
   * pair's first node, v of its second, c the cost, local cell ids; under
   * W1_METRIC_L2 the records carry no cost and c = 0),
   * K1 = 0x9E3779B97F4A7C15, K2 = 0xC2B2AE3D27D4EB4F,
   * K3 = 0x165667B19E3779F9: pair_checksum = (sum h, sum h^2) mod 2^64.
   * The checksum covers all of the pair's n_pairs when n_pairs_streamed
   * equals n_pairs. */
  int64_t n_pairs_streamed;
  uint64_t pair_checksum[2];

  /* Network (W1_KEEP_NETWORK), built on the device in compressed sparse row
   * form.  Node ids: cells 0..n_cells-1 in Morton order of (cell_i, cell_j),
   * the diagonal node of A is n_cells, the diagonal node of B is n_cells+1.
   * The arcs of node v are row_ptr[v] .. row_ptr[v+1]-1 (row_ptr has
   * n_cells + 3 entries, row_ptr[0] = 0, row_ptr[n_cells + 2] = n_arcs),
   * with heads col[] in strictly increasing order and costs cost[] in units
   * of g/2:
   *   cell -> cell: both orientations of every WSPD pair, cost
   *                 2 max(|di|, |dj|) of the two cells;
   *   cell -> A-diagonal: for cells with A mass, cost cell_j - cell_i;
   *   B-diagonal -> cell: for cells with B mass, cost cell_j - cell_i;
   *   B-diagonal -> A-diagonal: cost 0 (the A-diagonal row is empty).
   * supply[v] = out-flow minus in-flow at v: cell_ca - cell_cb for a cell,
   * -n_a for the A-diagonal node, n_b for the B-diagonal node. */
  int32_t *cell_i, *cell_j;   /* n_cells, shifted grid coordinates */
  int32_t *cell_ca, *cell_cb; /* n_cells, multiplicities from A and from B */
  int64_t *supply;            /* n_cells + 2 */
  int64_t *row_ptr;           /* n_cells + 3 */
  uint32_t *col;              /* n_arcs: head of each arc */
  int32_t *cost;              /* n_arcs (L-infinity; NULL with W1_METRIC_L2) */
  int64_t *cost64;            /* n_arcs (W1_METRIC_L2; NULL otherwise), see below */
  int64_t n_diag;             /* arcs at a diagonal node: #A cells + #B cells + 1 */
  int32_t metric_l2;          /* 1 if computed with W1_METRIC_L2 */
  int32_t cost_shift;         /* W1_METRIC_L2: costs are in units of g 2^-cost_shift */

  /* Stage intermediates (W1_KEEP_STAGES). */
  double *loc_b, *loc_d; /* n_locations, sorted by (birth, death) */
  int32_t *loc_w;        /* net multiplicity: count in A minus count in B */
  double *loc_t;         /* RWMD: cost of the cheapest arc out of the location */
  int64_t rwmd_sum_a, rwmd_sum_b;     /* fixed-point sums (int64)        */
  int32_t rwmd_shift_a, rwmd_shift_b; /* L_x = sum_x * 2^-shift_x       */
  int32_t *node_lo, *node_hi; /* n_cells-1 internal nodes: cell range    */
  int32_t *node_left, *node_right; /* child: >= 0 internal node, < 0 leaf ~cell */
  int32_t *node_box;          /* 4 per node: min_i, min_j, max_i, max_j  */

  double t_ms[8];
} w1_result;

/* Device-resident network of the last w1_approx on a context (batch entry
 * k of the last call), in the layout of the w1_result network above: the
 * rows of pair k with row_ptr local to it (row_ptr[0] = 0), col / cost
 * pointing at its first arc.  Pointers stay valid until the next call on
 * ctx. */
typedef struct {
  int64_t n_cells, n_pairs, n_arcs;
  const int32_t *cell_ij; /* 2 per cell: i, j */
  const int32_t *cell_ca, *cell_cb;
  const int64_t *supply;  /* n_cells + 2 */
  const int64_t *row_ptr; /* n_cells + 3 */
  const uint32_t *col;    /* n_arcs */
  const int32_t *cost;    /* n_arcs (L-infinity; NULL with W1_METRIC_L2) */
  const int64_t *cost64;  /* n_arcs (W1_METRIC_L2; NULL otherwise) */
} w1_device_network;

/* Create a context on HIP device `device` (must be gfx950). */
int w1_ctx_create(int device, w1_ctx **out);
int w1_ctx_destroy(w1_ctx *ctx);
/* Last HIP error code seen by the context (hipError_t as int). */
int w1_ctx_hip_error(const w1_ctx *ctx);

/* Approximate W1 of one pair (Alg. 3).  `out` is filled even on per-pair
 * errors (status < 0); release it with w1_result_free. */
int w1_approx(w1_ctx *ctx, const w1_pd *a, const w1_pd *b, const w1_params *params, void *stream,
              w1_result *out);

/* k pairs (a[i], b[i]) processed together: every stage runs once over all
 * pairs.  out[i] receives pair i.  All diagrams must share one dtype and
 * one memory kind (host or device, W1_INPUT_DEVICE). */
int w1_approx_batch(w1_ctx *ctx, const w1_pd *a, const w1_pd *b, int64_t k, const w1_params *params,
                    void *stream, w1_result *out);

/* RWMD lower bound L (Alg. 1) of each of k pairs, without the rest
 * (flags: W1_INPUT_DEVICE, W1_METRIC_L2). */
int w1_rwmd(w1_ctx *ctx, const w1_pd *a, const w1_pd *b, int64_t k, uint32_t flags, void *stream,
            double *L_out);

/* w1_rwmd for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and results as w1_rwmd (flags: W1_INPUT_DEVICE, W1_METRIC_L2), but the
 * call makes no device allocation (no hipMalloc, hipFree or allocating
 * library routine) and no host allocation: every device buffer it needs is a
 * slice of one fixed scratch array of 128 MiB per GPU, which the library
 * holds from the first context created on that GPU until the process ends.
 * Limits: at most 2^19 points in all k pairs together and k <= 1024;
 * larger inputs return W1_ERANGE before any work.  Calls on one GPU share
 * that array (it keeps the last call's contents; the call clears what it
 * needs), so calls that overlap in time on one GPU, from any contexts or
 * streams, race and must not be issued.  The context's own buffers are not
 * touched. */
int w1_rwmd_noalloc(w1_ctx *ctx, const w1_pd *a, const w1_pd *b, int64_t k, uint32_t flags, void *stream,
                    double *L_out);

/* Device pointers to the network of pair k of the last call on ctx
 * (requires that call to have been made without W1_COUNT_ONLY, and pair k
 * to be in the call's last launch group, see w1_tuning). */
int w1_device_network_get(w1_ctx *ctx, int64_t k, w1_device_network *out);

/* Tunables of the WSPD traversal and of batching (Alg. 4-6 run as a
 * persistent traversal over a work list of node pairs):
 *   stack_depth    per-lane DFS stack entries in LDS (8..32); work-list items
 *                  are expanded until the tree heights of their two nodes sum
 *                  to less than this;
 *   work_cap       items are expanded until |U| |V| <= work_cap (cells).
 *                  A pair of n cells with n^2 / 2 < 2^14 work_cap uses a
 *                  smaller cap: the largest power of two c >= 16 with
 *                  2^14 c <= n^2 / 2, else 16 (smaller items spread a small
 *                  pair's traversal over more waves);
 *   chunk_items    work-list items per chunk of the persistent passes;
 *   blocks_per_cu  resident blocks per compute unit of those passes (1..16);
 *   max_points_per_launch  w1_approx_batch runs its pairs in launch groups of
 *                  consecutive pairs holding at most this many points (a
 *                  single larger pair forms its own group).  This bounds the
 *                  device memory of one launch;
 *   compact_records 1 (default): when every grid coordinate of a launch group
 *                  is below 2^28, the count pass reads a split's two child
 *                  boxes from one 32-byte record of 28-bit fields; 0: from
 *                  the children's full 32-byte records, as the emit pass
 *                  always does.
 * The set of WSPD pairs, every count, the network and W1 do not depend on
 * these; the order of the pairs within a diagram pair's output does (it is
 * deterministic for a given tuning, and compact_records does not change it).
 * stream_arena_pairs and stream_max_rounds (see w1_tuning) only apply to
 * W1_COUNT_ONLY calls: the WSPD pairs are then written, in runs that reuse
 * one arena, without building the network -- emission measured at sizes
 * whose pair list does not fit in memory.
 * set_tuning returns W1_EINVAL for out-of-range values. */
typedef struct {
  int32_t stack_depth, work_cap, chunk_items, blocks_per_cu;
  int64_t max_points_per_launch;
  int32_t compact_records;
  int32_t stream_max_rounds;  /* streamed emission: at most this many arena */
                              /* fills (0 = until every pair is written)    */
  int64_t stream_arena_pairs; /* streamed emission: with W1_COUNT_ONLY and  */
                              /* a value > 0, the emit pass also runs, over */
                              /* consecutive runs of work-list chunks whose */
                              /* pairs fit this many 12-byte records, each  */
                              /* run overwriting the one device arena; the  */
                              /* result then carries n_pairs_streamed and   */
                              /* pair_checksum, and kernel time [4] the     */
                              /* emit time.  A chunk larger than the arena  */
                              /* gives W1_EOVERFLOW.  0 = off               */
  int32_t blocked_emit;       /* network of a single pair with at least   */
                              /* 4096 work-list chunks: 1 emits the pair   */
                              /* records into blocks that the waves take  */
                              /* as they fill them, sized by a count over  */
                              /* every 16th chunk, instead of counting     */
                              /* every chunk first; 0 (default) = always   */
                              /* count first.  The network is the same.    */
                              /* Experimental: not yet validated on the    */
                              /* GPU                                       */
  int32_t sort_window_words;  /* row sort: bitmap window in 32-bit words   */
                              /* (0 = as large as the largest pair needs,  */
                              /* up to 24576); rows of pairs with more     */
                              /* cells are sorted window by window.  The   */
                              /* network does not depend on it             */
  int64_t emit_block_limit;   /* blocked emission: at most this many blocks */
                              /* of 2048 records (0 = as sized); when they */
                              /* run out the pass is redone with every     */
                              /* chunk counted first (same result)         */
  int32_t fused_expand_cells; /* launch groups of at most this many cells  */
                              /* (0..65536) expand their WSPD work list in */
                              /* one workgroup, with no host wait between  */
                              /* rounds; 0 = always round by round.  The   */
                              /* work list is the same either way.         */
                              /* Default 4096                              */
  int32_t fused_expand_items; /* room of that expansion, in work-list items */
                              /* kept and per frontier (0 = 64 n_cells +   */
                              /* 4096 kept, 16 n_cells + 4096 frontier);   */
                              /* out of room, the rounds run one by one    */
  int32_t stream_graph;       /* streamed emission: 1 (default) captures   */
                              /* one arena fill (its ranges taken from a   */
                              /* device table, then the emit pass) in a    */
                              /* HIP graph and replays it for every fill,  */
                              /* with no host wait between fills; 0        */
                              /* launches each fill directly.  Same        */
                              /* records and checksums either way          */
} w1_tuning;

int w1_ctx_get_tuning(const w1_ctx *ctx, w1_tuning *out);
int w1_ctx_set_tuning(w1_ctx *ctx, const w1_tuning *t);

/* Device times (ms, HIP events on the call's stream) of the last call's
 * WSPD and network kernels: [0] work-list build (expansion rounds, item
 * sort, chunking), [1] count pass (with blocked emission: the count over
 * every 16th chunk), [2] emit pass (which also takes the network's bucket
 * histogram), [3] the number of pairs emitted; [4] the streamed emission's
 * emit passes, all arena fills together (0 unless streaming); then the
 * passes that sort the network into rows: [5] bucket scatter, [6] row
 * histogram, [7] row scatter (with the degree scan before it), [8] row sort
 * (with the diagonal rows and row pointers); [9] the blocks the blocked
 * emission filled (0: counted layout); [10] how the work list was expanded:
 * 1 in one workgroup, -1 tried so but out of room (then round by round),
 * 0 round by round; [11] the words per pair record the emit pass wrote
 * for the network: 2 (u, v), 3 (u, v, cost), 0 when nothing was emitted.
 * n is the capacity of ms (>= 4); entries beyond 11 are 0. */
int w1_ctx_last_kernel_times(const w1_ctx *ctx, double *ms, int n);

/* Host network simplex on any uncapacitated network with non-negative integer
 * costs (the solver used inside w1_approx).  Arcs src[k] -> dst[k] with cost
 * cost[k]; supply[v] = out-flow minus in-flow.  flow_out (m) and pot_out
 * (n_nodes, reduced cost cost + pot[src] - pot[dst] >= 0 at optimum) may be
 * NULL.  Returns W1_OK, W1_EINVAL (infeasible / bad input) or W1_ENOMEM;
 * *status_out is W1_OPTIMAL or W1_STALLED.  After a stall *cost_out is the
 * cost of the flow reached if that flow meets every supply, else -1.  Arc
 * numbers are 64-bit inside the solver: m is limited by memory only; node
 * numbers must be below 2^31 - 1. */
int w1_flow_solve(int64_t n_nodes, int64_t m, const uint32_t *src, const uint32_t *dst, const int32_t *cost,
                  const int64_t *supply, int64_t pivot_cap, int64_t *cost_out, int64_t *flow_out,
                  int64_t *pot_out, int64_t *pivots_out, int32_t *status_out);

/* WSPD separation s for eps and kappa (0 selects 0.1): the smallest s with
 * t + (t + 1) kappa eps <= 1 + eps, t = (s + 2)/(s - 2). */
int w1_separation_for_eps(double eps, double kappa);

void w1_result_free(w1_result *r);
const char *w1_strerror(int code);

/* ======================================================================
 * Learned form: a DeepSets surrogate of W1 and 1-NN search.
 *
 * The nearest-neighbour problem (Sec. 6, Problem NN): given database
 * diagrams A_1..A_m and a query B, find argmin_i W1(B, A_i).  Here W1 is the
 * certified value `w1` that w1_approx computes at the given eps, and ties go
 * to the lowest index.  The surrogate only orders the candidates.  Every
 * answer comes from the method itself.  A candidate is skipped only when
 * its RWMD lower bound (Alg. 1) exceeds the best W1 found so far, so it
 * cannot be the answer.  Answers are identical in every search mode.
 *
 * Network: phi(x) = ReLU(W2 ReLU(W1 x + b1) + b2), with x = (birth,
 * death - birth) and shapes 2 -> 128 -> 128.  It is summed over the points
 * of a diagram (a point of multiplicity k counts k times; diagonal points
 * are ignored).  Then e = W3 pool + b3 (128 -> 64), and the prediction is
 * ||e_A - e_B||_2.  W1, b1, W2 and the first hidden layer are BF16 on the
 * matrix cores with FP32 accumulation; x enters as a two-term BF16
 * expansion.  b2, pooling and rho are FP32; master parameters are FP32.
 *
 * Parameter vector (W1_SURR_NPARAM floats, FP32), in this order:
 *   W1 [128][2], b1 [128], W2 [128 out][128 in], b2 [128], W3 [64][128], b3 [64]
 * ====================================================================== */
#define W1_SURR_NPARAM 25152
#define W1_SURR_EMB 64

typedef struct w1_surrogate w1_surrogate;

typedef struct {
  int32_t epochs;      /* passes over the labelled pairs                        */
  int32_t batch_pairs; /* pairs per Adam step                                   */
  float lr, beta1, beta2, adam_eps; /* Adam; 0 selects 1e-3, 0.9, 0.999, 1e-8    */
  uint64_t seed;       /* pair shuffling                                        */
} w1_train_params;

/* New surrogate on the context's device.  The parameters are drawn from a
 * counter-based generator seeded by `seed` (uniform fan-in scaling), and the
 * Adam state starts at zero.  The surrogate is bound to ctx's device; use it
 * only with contexts on that device.  Like a context, a surrogate (and an
 * nn index) is not thread-safe: calls that share one must not overlap.
 * Every call synchronises the stream it is given before it returns. */
int w1_surrogate_create(w1_ctx *ctx, uint64_t seed, w1_surrogate **out);
int w1_surrogate_destroy(w1_surrogate *s);
/* Copy the FP32 master parameters to / from host memory (n = W1_SURR_NPARAM).
 * set_params resets the Adam state. */
int w1_surrogate_get_params(const w1_surrogate *s, float *out, int64_t n);
int w1_surrogate_set_params(w1_surrogate *s, const float *in, int64_t n);

/* Embeddings of k diagrams: emb_out (host) receives k x 64 FP32, row-major.
 * Diagrams are host arrays, or device arrays with W1_INPUT_DEVICE in flags.
 * Invalid points (non-finite, death < birth) give W1_EINVAL. */
int w1_surrogate_embed(w1_ctx *ctx, w1_surrogate *s, const w1_pd *d, int64_t k, uint32_t flags, void *stream,
                       float *emb_out);

/* Loss and gradient over labelled pairs, without an update.  Pair j joins
 * diagrams pa[j] and pb[j] (indices into d[0..k)) and has label w[j] > 0.
 * loss = (1/P) sum_j ((||e_pa - e_pb|| - w_j) / w_j)^2.  grad_out (host,
 * W1_SURR_NPARAM) gets d loss / d parameters: the BF16 roundings pass
 * gradients unchanged, and a ReLU at exactly 0 passes none. */
int w1_surrogate_grad(w1_ctx *ctx, w1_surrogate *s, const w1_pd *d, int64_t k, const int64_t *pa,
                      const int64_t *pb, const double *w, int64_t npairs, uint32_t flags, void *stream,
                      double *loss_out, float *grad_out);

/* Train with Adam on labelled pairs, entirely on the device (the forward
 * and backward kernels of this library).  epoch_loss_out (host, `epochs`
 * entries, may be NULL) gets the mean pair loss of each epoch as it was
 * computed during that epoch. */
int w1_surrogate_train(w1_ctx *ctx, w1_surrogate *s, const w1_pd *d, int64_t k, const int64_t *pa,
                       const int64_t *pb, const double *w, int64_t npairs, const w1_train_params *tp,
                       uint32_t flags, void *stream, double *epoch_loss_out);

/* Timings of the surrogate's last embed call: [0] forward kernel ms (HIP
 * events), [1] points embedded, [2] diagrams embedded.  n >= 3. */
int w1_surrogate_last_times(const w1_surrogate *s, double *out, int n);

/* ---- 1-NN search ---------------------------------------------------------- */
typedef struct w1_nn_index w1_nn_index;

/* Search modes.  All return the same answers.
 *   W1_NN_RWMD        the method without the surrogate: the RWMD bound of
 *                     every (query, database) pair, then candidates in
 *                     increasing RWMD order until RWMD > best.
 *   W1_NN_SURROGATE   verify the seed_k nearest candidates by surrogate
 *                     distance first; drop every candidate whose dual bound
 *                     exceeds the best W1 so far; compute RWMD only for the
 *                     rest, then continue as W1_NN_RWMD on them.  The dual
 *                     bound is max_c |sum_A f_c - sum_B f_c| over the test
 *                     functions f_c(x) = max(0, d_diag(x) - c), c = 0 and
 *                     2^-20 .. 2^11.  Each f_c is 1-Lipschitz in L-infinity
 *                     and vanishes on the diagonal, so the bound is <= W1
 *                     (Kantorovich duality).  Its per-diagram sums are FP64,
 *                     and a margin of 1e-8 (sum_A f_c + sum_B f_c) covers
 *                     their rounding.
 *   W1_NN_EXHAUSTIVE  verify every database diagram.
 *   W1_NN_SPARSE      the cheap sparse stage of the paper's 1-NN pipelines
 *                     (Sec. 7), kept exact: the RWMD bound of every pair; the
 *                     method at s = 1 on the paper's own grid for s = 1
 *                     (w1_approx with s_override = 1 and W1_PAPER_GRID) for
 *                     the `keep` candidates of smallest RWMD; the seed_k of
 *                     those with the smallest s = 1 value (an upper bound on
 *                     W1, ties to the earlier in RWMD order) are verified
 *                     first; then as W1_NN_RWMD.  Same answers as above.
 *   W1_NN_PIPELINE    the paper's keep-seed_k-1 pipeline (Sec. 7, with RWMD
 *                     in place of its first stage), NOT exact: the candidates
 *                     left after both cuts of W1_NN_SPARSE are verified and
 *                     the best of them is returned.  It is the nearest
 *                     neighbour only when that survives both cuts (what the
 *                     paper measures as accuracy).
 * Verifications run w1_approx with W1_PRUNE (the same w1, a smaller flow). */
#define W1_NN_RWMD 0
#define W1_NN_SURROGATE 1
#define W1_NN_EXHAUSTIVE 2
#define W1_NN_SPARSE 3
#define W1_NN_PIPELINE 4
#define W1_NN_NSTATS 33 /* test functions of the dual bound */

typedef struct {
  double eps;       /* eps of the method that verifies candidates               */
  int32_t mode;     /* W1_NN_*                                                  */
  int32_t seed_k;   /* W1_NN_SURROGATE / W1_NN_SPARSE: candidates verified     */
                    /* first (0 selects 1); W1_NN_PIPELINE: candidates kept    */
                    /* after the s = 1 stage (0 selects 3)                     */
  int32_t keep;     /* W1_NN_SPARSE / W1_NN_PIPELINE: candidates kept after    */
                    /* RWMD for the s = 1 stage (0 selects 15)                 */
  int32_t reserved; /* must be 0                                               */
} w1_nn_params;

typedef struct {
  int64_t verifications; /* full-method W1 evaluations, all queries          */
  int64_t rwmd_evals;    /* RWMD bounds computed, all queries                 */
  int64_t rounds;        /* verification rounds (one candidate per live query) */
  double t_rwmd_ms;      /* RWMD bounds                                        */
  double t_embed_ms;     /* query embedding, surrogate distances, dual bounds  */
  double t_verify_ms;    /* full-method verifications (GPU + host flow)         */
  double t_total_ms;
  int64_t sparse_evals;  /* s = 1 evaluations (W1_NN_SPARSE, W1_NN_PIPELINE)    */
  double t_sparse_ms;    /* s = 1 evaluations (GPU + host flow)                 */
} w1_nn_stats;

/* Index over m database diagrams: a device copy of their points and, when s
 * is not NULL, their embeddings under s.  The index does not keep s. */
int w1_nn_build(w1_ctx *ctx, w1_surrogate *s, const w1_pd *db, int64_t m, uint32_t flags, void *stream,
                w1_nn_index **out);
int w1_nn_destroy(w1_nn_index *idx);
/* Nearest database diagram of each of nq queries.  nn_out[q] = index,
 * w1_out[q] = its certified W1 (may be NULL), verif_out[q] = verifications
 * spent on query q (may be NULL).  W1_NN_SURROGATE needs the surrogate the
 * index was built with (s); the other modes ignore s. */
int w1_nn_query(w1_ctx *ctx, w1_nn_index *idx, w1_surrogate *s, const w1_pd *q, int64_t nq,
                const w1_nn_params *p, uint32_t flags, void *stream, int64_t *nn_out, double *w1_out,
                int64_t *verif_out, w1_nn_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* W1APPROX_H */
