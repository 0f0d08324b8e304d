/*
 * bp.h -- C ABI of the MI355X (gfx950) exact O(mM) belief-propagation library.
 *
 * Method: Coughlan & Shen, "An Embarrassingly Simple Speed-Up of Belief
 * Propagation with Robust Potentials".  For a pairwise MRF on a 4-connected
 * H x W grid (Sec. 1, Eq. 1) with M labels and the truncated-linear robust
 * potential f(x_i, x_j) = exp(-alpha |x_i - x_j|) for |x_i - x_j| <= T and a
 * constant fbar otherwise (Sec. 1, Sec. 6), each message update
 *   sum-product (Sec. 4, Eq. 7):
 *     m(x_j) = fbar * sum_x h(x) + sum_{|x - x_j| <= T} (f(x, x_j) - fbar) h(x)
 *   max-product (Sec. 5, Eq. 11, product domain):
 *     m(x_j) = max(fbar * max_x h(x), max_{|x - x_j| <= T} f(x, x_j) h(x))
 * costs O(mM) with m = 2T + 1 instead of the O(M^2) of Eq. 2 / Eq. 9, with
 * h(x) = g(x) * product of the incoming messages except the target's (Eq. 5).
 * Every message is normalised to sum 1 after it is computed (Sec. 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Status: every int-returning call returns BP_OK (0) or a negative
 *   bp_status.  bp_status_string() names a code; bp_last_error() returns a
 *   thread-local description of the most recent failure on this thread.
 * - Memory: the caller owns all device memory (unary, outputs, workspace);
 *   pointers marked "device" must be device (HBM) pointers of the GPU that
 *   was current at bp_init_grid.  The library keeps only host-side state.
 *   Borrowed pointers must stay valid until they are replaced or the handle
 *   is destroyed.
 * - Asynchrony: device work is enqueued on the handle's HIP stream and the
 *   call returns before it runs; the caller synchronises that stream.
 *   Argument and call-order errors are detected synchronously, before any
 *   work is enqueued.  Launch failures are reported as BP_EHIP.
 * - Threads: a handle must not be used by two threads at once.
 * - Tracing: with the environment variable BP_ROCTX=1 (read once), the
 *   calls that enqueue updates or readouts (bp_iterate, bp_iterate_dense,
 *   bp_readout and the other readouts, bp_autotune, bp_iterate_multiscale,
 *   bp_forward_ckpt, bp_backward, bp_batch_iterate, bp_fg_iterate) each
 *   open a roctx range named after the call (rocprofv3 --marker-trace);
 *   roctx is looked up at run time, and without it nothing is traced.
 * - Layouts (row-major, float32, labels contiguous):
 *     unary g        [H][W][M]      g >= 0, finite, every pixel's row nonzero
 *     beliefs        [H][W][M]      each row sums to 1
 *     labels         [H][W]         int32 in [0, M)
 *     messages       [4][H][W][M]   inbox planes: plane k at pixel p holds the
 *                                   message into p from its neighbour in
 *                                   direction k = 0 left, 1 right, 2 up,
 *                                   3 down.  Slots whose neighbour is off the
 *                                   grid are never read nor written by an
 *                                   update; bp_reset_messages sets them to 1/M.
 */
#ifndef BP_H
#define BP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bp_grid bp_grid;   /* opaque single-grid handle */
typedef struct bp_batch bp_batch; /* opaque handle for many independent grids */
typedef struct bp_fgraph bp_fgraph; /* opaque factor-graph handle */

enum bp_status {
    BP_OK = 0,
    BP_EINVAL = -1,       /* bad argument (null pointer, size, range, alignment) */
    BP_ESTATE = -2,       /* call out of order (e.g. iterate before set_unary) */
    BP_ENOMEM = -3,       /* workspace too small or host allocation failed */
    BP_EHIP = -4,         /* a HIP runtime call or kernel launch failed */
    BP_EUNSUPPORTED = -5  /* valid request this library does not implement */
};

enum bp_mode { BP_SUM_PRODUCT = 0, BP_MAX_PRODUCT = 1 };

enum bp_schedule {
    BP_SCHED_SYNC = 0,        /* Jacobi: every message from the previous state */
    BP_SCHED_CHECKERBOARD = 1, /* bipartite: pass t updates messages sent by
                                  pixels with (row + col) % 2 == t % 2, in place */
    BP_SCHED_SWEEP = 2         /* directional sweeps (Sec. 6): one sweep is four
                                  in-place passes, messages travelling left,
                                  right, up, then down; each pass walks every
                                  row (left/right) or column (up/down) from
                                  its far end, each message using the one its
                                  sender has just received in the same pass */
};

#define BP_MAX_LABELS 256     /* largest M this library accepts */
#define BP_FBAR_TIED (-1.0f)  /* bp_set_potential: fbar := f(T) = exp(-alpha T) */

/* Create a handle for an H x W grid (H, W >= 1, H*W < 2^31 / 4): the pairwise
 * MRF of Eq. 1 on the 4-connected pixel lattice of the stereo model (Sec. 6),
 * one node per pixel and one pairwise factor per pair of horizontal or
 * vertical neighbours.
 * hip_stream: a hipStream_t, or NULL for the default stream.  The GPU that is
 * current on the calling thread becomes the handle's device.
 * Errors: BP_EINVAL (sizes, null out), BP_EHIP (no usable device). */
int bp_init_grid(bp_grid** out, int32_t H, int32_t W, void* hip_stream);

/* Change the stream later work is enqueued on. */
int bp_set_stream(bp_grid* grid, void* hip_stream);

/* Set the truncated-linear potential (Sec. 1, Sec. 6; sparse compatibility
 * Sec. 4): f(d) = exp(-alpha |d|) for |d| <= T, fbar for |d| > T, where
 * Nbd(x_j) = {x : |x - x_j| <= T, 0 <= x < M} (clipped at the label range).
 * fbar = exp(-alpha T) gives exp(-alpha min(|d|, T)); fbar = 0 gives Eq. 8.
 * fbar = BP_FBAR_TIED ties fbar to f(T): fbar := exp(-alpha T) rounded to
 * float32, the same value as the table's f(T), so the potential is exactly
 * exp(-alpha min(|d|, T)) in float32 and d fbar / d alpha = -T fbar.
 * The table is built in double on the host and rounded to float32.
 * Requires 1 <= M <= BP_MAX_LABELS, 0 <= T < M, alpha finite, fbar finite
 * and >= 0 or BP_FBAR_TIED (else BP_EINVAL).  Changing M invalidates the workspace and the
 * unary (attach and set them again); changing only T, alpha or fbar keeps
 * the messages. */
int bp_set_potential(bp_grid* grid, int32_t M, int32_t T, float alpha, float fbar);

/* Bytes of device workspace needed after bp_set_potential: the message
 * state of BP on the Eq. 1 grid (one M-label message per directed edge,
 * Sec. 3, stored as four inbox planes) in two buffers for the synchronous
 * ping-pong, plus the tables of the Eq. 10
 * max-product update sized for any T < M), or a negative status. */
int64_t bp_workspace_bytes(const bp_grid* grid);

/* Attach caller-owned device workspace (>= bp_workspace_bytes, 256-byte
 * aligned); resets the messages to 1/M.  Errors: BP_ESTATE before
 * set_potential, BP_ENOMEM if too small, BP_EINVAL on misalignment. */
int bp_attach_workspace(bp_grid* grid, void* dev_ptr, int64_t bytes);

/* Borrow the unary table g (the per-node factor of Eq. 1; in the stereo
 * model of Sec. 6 the data term of each disparity) (device, [H][W][M],
 * 16-byte aligned) until the
 * next bp_set_unary, a change of M, or bp_destroy.  Every entry must be
 * finite and >= 0, with a positive entry in every row (otherwise the
 * pixel's messages are 0/0 under Eq. 5 and the normalisation).  With the
 * environment variable BP_VALIDATE=1 this is checked on the device: the call
 * then waits for the stream, returns BP_EINVAL on a violating table (keeping
 * the previous one), and BP_ESTATE if no workspace is attached yet. */
int bp_set_unary(bp_grid* grid, const float* g_dev);

/* All messages := 1/M: the uniform start of the iteration of Eq. 2 / Eq. 9
 * (Sec. 3 leaves the start open; uniform is the usual choice).  Returns
 * BP_ESTATE before a workspace is attached. */
int bp_reset_messages(bp_grid* grid);

/* Run n_iters >= 0 iterations of the O(mM) update (Eq. 7 for sum-product,
 * Eq. 11 for max-product) with the given schedule.  For the checkerboard
 * schedule n_iters counts passes (two passes update every message once) and
 * the pass parity continues across calls until the next reset; for the sweep
 * schedule it counts whole sweeps (each updates every message once).
 * Eq. 11 equals Eq. 9 only when f >= fbar on every compatible pair (Sec. 5),
 * i.e. fbar <= f(T) as rounded to float32.  Otherwise max-product runs the
 * exact Eq. 10 (the largest h outside each window times fbar) through the
 * general kernel, for every schedule.  Sum-product accepts any fbar >= 0.
 * After bp_set_sparse_potentials the general kernel runs instead, for every
 * schedule (bp_iterate_dense returns BP_EUNSUPPORTED). */
int bp_iterate(bp_grid* grid, int32_t mode, int32_t n_iters, int32_t schedule);

/* Arithmetic of the update.  BP_ARITH_F64 (the default): h, the window sums,
 * the normaliser and the normalisation in double, every stored message its
 * exact value rounded once to float32.  BP_ARITH_F32: the same Eq. 7
 * sum-product update entirely in float32 (a few roundings per message,
 * contracted by sum-product; results agree with BP_ARITH_F64 to rounding,
 * not bit for bit), where it is compiled: sum-product of the window
 * potential with fbar > 0 (with fbar = 0 messages reach zero and the
 * denormal range, where float32 products lose their precision), the
 * synchronous, checkerboard or sweep schedule, T within the
 * register windows (T <= 16, 12 for M <= 16), M = 4 * ceil-pow2(M / 4) (16,
 * 32, 64, 128, 256) and 4*H*W*M bytes below 2^32.  Everything else (max-
 * product, dense, general potentials, multi-scale, the gradient)
 * computes in double whatever this says; batches have their own setting
 * (bp_batch_set_arithmetic).  BP_EINVAL for another value. */
enum bp_arith { BP_ARITH_F64 = 0, BP_ARITH_F32 = 1 };
int bp_set_arithmetic(bp_grid* grid, int32_t arith);

/* Launch mapping of the two-iteration launches (synchronous iterations and
 * checkerboard pass pairs of the window potential, Eq. 7 / Eq. 11; see
 * bp_set_sync_fusion).  layout: BP_PAIR_STRIPS runs one
 * workgroup per block of consecutive pixels of a grid row, the blocks of a
 * row padded to a multiple of the 8 XCDs so that each XCD holds the same
 * column strips in every row; BP_PAIR_BANDS the same blocks remapped so that
 * each XCD holds a contiguous band of rows; BP_PAIR_WIDE the same blocks
 * remapped so that each XCD holds one contiguous strip of 1/8 of the
 * columns, every row (the default); BP_PAIR_SLOTS one pixel group
 * per slot in row-major order (the only form when M is not 4 * ceil-pow2(M /
 * 4) or a message plane reaches 2^32 bytes, where the first two fall back to
 * it; float32 arithmetic has the row blocks only, where BP_PAIR_SLOTS runs
 * BP_PAIR_STRIPS); BP_PAIR_WALK, for synchronous launches with M = 32 or 64,
 * one workgroup per strip of columns walking down a chunk of rows, each
 * grid row's unary and inbox staged once in LDS (checkerboard pairs and
 * other M run BP_PAIR_WIDE); BP_PAIR_TILE, for synchronous launches with
 * M = 16, 32, 64 or 128 and checkerboard pass pairs with M = 32, 64 or 128,
 * one workgroup per pixel tile whose rows and halo are staged once in LDS
 * (other M run BP_PAIR_WIDE).
 * cap: the
 * most workgroups per compute unit the
 * launch's LDS request allows (0 none, 1..64, -1 the default: 4 with float32
 * arithmetic, none with double; BP_PAIR_WALK's LDS ring and BP_PAIR_TILE's
 * tile set their own, whatever the cap).  Until this call or bp_autotune
 * chooses one, the mapping follows the arithmetic (bp_set_arithmetic):
 * BP_PAIR_TILE with float32 arithmetic, BP_PAIR_WIDE with double, cap -1.
 * Every setting computes the same messages
 * bit for bit; only the speed differs.  BP_EINVAL for a null handle, a
 * layout outside the enum or a cap outside -1..64.  Kept per grid; used by
 * every launch of the grid, including bp_forward_ckpt and multi-scale. */
/* Convergence and failure check of the message state (Sec. 3: the messages
 * of one iteration computed from those of the previous).  *max_change
 * (device float, may be null): the largest |m - m'| over the inbox entries
 * finite in both, m the current messages and m' the grid's other message
 * buffer, which after a synchronous launch holds the state that launch
 * read (one iteration back after a one-iteration launch, two after a
 * two-iteration launch; after bp_reset_messages, bp_set_messages or
 * in-place checkerboard passes it holds an older state).  *non_finite
 * (device int32, may be null): the number of entries of m that are NaN or
 * infinite.  Both are written on the grid's stream (no host sync; no
 * memset, so a graph may capture the call).  BP_EINVAL for a null handle or
 * no output, BP_ESTATE without a potential or a workspace. */
int bp_message_stats(bp_grid* grid, float* max_change, int32_t* non_finite);

enum bp_pair_layout {
    BP_PAIR_STRIPS = 0,
    BP_PAIR_BANDS = 1,
    BP_PAIR_SLOTS = 2,
    BP_PAIR_WIDE = 3,
    BP_PAIR_WALK = 4,
    BP_PAIR_TILE = 5
};
int bp_set_launch_tuning(bp_grid* grid, int32_t layout, int32_t cap);
int bp_get_launch_tuning(const bp_grid* grid, int32_t* layout, int32_t* cap);

/* Time the current setting, every row-block and slot layout above with caps
 * 0, 4 and 3, BP_PAIR_WALK and BP_PAIR_TILE, on this grid's own state, and keep the fastest (another setting
 * replaces the best only when at least 1% faster) for `mode` and `schedule`
 * (BP_SCHED_SYNC or
 * BP_SCHED_CHECKERBOARD): trial_iters iterations (even, >= 2) per candidate
 * after two warm-up iterations, timed with events on the grid's stream, in
 * two rounds over the candidates, each keeping its faster trial
 * (synchronises with the stream).  Needs the potential, the unary and the workspace;
 * the messages are reset to uniform afterwards (the trials iterate them).
 * *best_us (if not null): microseconds per iteration of the winner.
 * BP_EINVAL for a bad mode, schedule or trial_iters; BP_ESTATE when the grid
 * is not ready; BP_EHIP on a device error (the previous setting is kept). */
int bp_autotune(bp_grid* grid, int32_t mode, int32_t schedule, int32_t trial_iters, float* best_us);

/* Synchronous iterations and checkerboard passes of the window potential
 * run two per launch by default (where a register window is compiled: T <=
 * 16, 12 for M <= 16; not for Eq. 10): each pixel computes the four
 * messages its neighbours send it, then its own four, so the intermediate
 * messages stay on chip.  A checkerboard pair writes the grid's other
 * message buffer in full (single passes stay in place).  The results are
 * the same bits as single launches; enable = 0 selects single launches (for
 * comparison and timing).  Errors: BP_EINVAL on a null handle. */
int bp_set_sync_fusion(bp_grid* grid, int32_t enable);

/* Same contract as bp_iterate, but each message is the plain O(M^2) sum or
 * max over all sender labels (Eq. 2 / Eq. 9) with the same potential table.
 * The comparison point for the sparse update (Sec. 6 compares the two under
 * the sweep schedule); requires M <= 128 and the table to fit the device's
 * LDS (else BP_EUNSUPPORTED). */
int bp_iterate_dense(bp_grid* grid, int32_t mode, int32_t n_iters, int32_t schedule);

/* ------------------------------------------------------------------------
 * General sparse-compatible potentials (Sec. 4: f_ij with its own constant
 * fbar_ij outside a set of compatible pairs that may differ from node to
 * node; Sec. 7: potentials that are not functions of x_i - x_j).  A type is
 * given in CSR form over the label y of the second node of a pair (the
 * right or bottom pixel): col_ptr[y] .. col_ptr[y+1]-1 index the compatible
 * labels x of the first node (left or top pixel), strictly increasing, with
 * the potential values f(x, y) >= 0; every other pair has the value fbar.
 * Each message costs O(entries in its list + M) (Eq. 7; Eq. 11 when every
 * listed f >= fbar, else Eq. 10, exactly).
 * ---------------------------------------------------------------------- */
typedef struct bp_sparse_potential {
    const int32_t* col_ptr;  /* host, [M + 1], col_ptr[0] = 0, non-decreasing */
    const int32_t* row_idx;  /* host, [col_ptr[M]], labels in [0, M) */
    const float* val;        /* host, [col_ptr[M]], finite and >= 0 */
    float fbar;              /* finite and >= 0 */
} bp_sparse_potential;

/* Device bytes of the tables bp_set_sparse_potentials builds for these
 * n_types (1..16) types at the grid's M (after bp_set_potential), or a
 * negative status (BP_EINVAL for a malformed type). */
int64_t bp_sparse_table_bytes(const bp_grid* grid, int32_t n_types, const bp_sparse_potential* types);

/* Use n_types potential types instead of the truncated-linear potential.
 * table_dev: caller-owned device buffer (>= bp_sparse_table_bytes, 256-byte
 * aligned) that receives the tables (copied on the grid's stream; the host
 * arrays may be freed when the call returns).  type_h_dev (device, [H][W-1])
 * and type_v_dev (device, [H-1][W]) give the type of every horizontal and
 * vertical pair (uint8, < n_types), or NULL for type 0 everywhere; they are
 * borrowed and checked once here.  Keeps the messages.  bp_set_potential
 * switches back to the truncated-linear potential.  Blocks until earlier
 * work on the grid's stream has drained. */
int bp_set_sparse_potentials(bp_grid* grid, int32_t n_types, const bp_sparse_potential* types, void* table_dev,
                             int64_t table_bytes, const uint8_t* type_h_dev, const uint8_t* type_v_dev);

/* ------------------------------------------------------------------------
 * Multi-scale (coarse-to-fine) BP in tandem with the O(mM) update (Sec. 2,
 * Sec. 6).  Level l+1 groups the 2 x 2 blocks of level l (ceil(H/2) x
 * ceil(W/2)); a block's unary is the product of its children's unaries
 * divided by its maximum over labels (computed in double, rounded once);
 * the potential is the same at every level.  The coarsest level starts
 * from uniform messages, every finer level from its parent's inbox (each
 * pixel copies the inbox of its block), and level l runs iters[l]
 * synchronous iterations.  A fresh solve: the grid's messages are
 * overwritten and hold the level-0 result afterwards (slots of off-grid
 * neighbours, which no update reads, hold prolonged values rather than 1/M).
 * ---------------------------------------------------------------------- */

/* Device bytes of the levels 1..levels (0..12): their unaries and message
 * buffers (level 0 uses the grid's own), or a negative status. */
int64_t bp_multiscale_workspace_bytes(const bp_grid* grid, int32_t levels);

/* Run the multi-scale solve (mode as for bp_iterate).  The potential is the
 * grid's: the truncated-linear one (max-product with fbar above some f(d)
 * runs Eq. 10 at every level), or general sparse potentials set without
 * type maps (one potential on every edge; with type maps BP_EUNSUPPORTED,
 * since they describe the finest grid only).
 * iters: host, [levels + 1], iters[0] for the finest level.  ms_ws: caller-
 * owned device workspace (>= bp_multiscale_workspace_bytes, 256-byte
 * aligned; unused when levels = 0), busy until the grid's stream drains. */
int bp_iterate_multiscale(bp_grid* grid, int32_t mode, int32_t levels, const int32_t* iters, void* ms_ws,
                          int64_t ms_bytes);

/* ------------------------------------------------------------------------
 * Factor graphs with sparse-compatible higher-order factors (Sec. 7): a
 * factor over K = 2 or 3 variables equals a constant fbar except on a set C
 * of compatible tuples, so its message to slot i costs O(C + M):
 *   sum: fbar * prod_{j != i} S_j + sum over the tuples with x_i = x of
 *        (f - fbar) * prod_{j != i} n_j(x_j),   S_j = sum of n_j;
 *   max: max(fbar * prod_{j != i} max n_j, max over those tuples of
 *        f * prod_{j != i} n_j(x_j))   (when f >= fbar on C; otherwise the
 *        split form of bp_fg_iterate).
 * Variable-to-factor messages n are g times the variable's other incoming
 * factor messages (factor order).  One iteration computes every n from the
 * current factor messages, then every factor message (synchronous); every
 * message is normalised in double and stored in float32.
 * ---------------------------------------------------------------------- */
typedef struct bp_factor_type {
    int32_t arity;          /* 2 or 3 */
    int32_t n_tuples;       /* |C| >= 0 */
    const int32_t* tuples;  /* host, [n_tuples][arity], labels in [0, M), no duplicates */
    const float* val;       /* host, [n_tuples], f(tuple), finite and >= 0 */
    float fbar;             /* value of every other tuple, finite and >= 0 */
} bp_factor_type;

/* n_vars variables with M labels (1..BP_MAX_LABELS); factor a is of type
 * factor_type[a] over the variables factor_vars[3a .. 3a+arity-1] (host;
 * distinct, the third entry is ignored for arity 2).  dense_tables != 0 also
 * builds the complete tuple lists (M^arity per type, at most 2^24) for the
 * plain O(M^K) update of bp_fg_iterate(..., dense = 1).  Host copies are
 * taken; the arrays may be freed afterwards. */
int bp_fg_init(bp_fgraph** out, int32_t n_vars, int32_t M, int32_t n_factors, const int32_t* factor_vars,
               const int32_t* factor_type, int32_t n_types, const bp_factor_type* types, int32_t dense_tables,
               void* hip_stream);
int bp_fg_set_stream(bp_fgraph* fg, void* hip_stream);
/* Device bytes for the graph, the tables and both message sets. */
int64_t bp_fg_workspace_bytes(const bp_fgraph* fg);
/* Attach caller-owned workspace (256-byte aligned), upload the graph and the
 * tables, reset the messages to 1/M. */
int bp_fg_attach_workspace(bp_fgraph* fg, void* dev_ptr, int64_t bytes);
/* Borrow the unary table (device, [n_vars][M], 16-byte aligned). */
int bp_fg_set_unary(bp_fgraph* fg, const float* g_dev);
int bp_fg_reset_messages(bp_fgraph* fg);
/* n_iters synchronous iterations; dense = 1 visits every tuple (the O(M^K)
 * comparison).  Max-product with some f < fbar in C runs the split form
 * (Eq. 10's analogue: the listed tuples with their own f, and fbar times
 * the largest product over the completions outside C), exact and equal to
 * the dense form bit for bit; it needs at most 31 listed labels of a slot's
 * other slots per label (else BP_EUNSUPPORTED). */
int bp_fg_iterate(bp_fgraph* fg, int32_t mode, int32_t n_iters, int32_t dense);
/* Beliefs (device [n_vars][M], rows sum to 1) and/or MAP labels (device
 * [n_vars] int32, lowest label on ties); either may be NULL. */
int bp_fg_beliefs(bp_fgraph* fg, float* beliefs_dev, int32_t* labels_dev);
/* Copy the factor->variable (m, [n_factors][3][M]) and variable->factor (n)
 * messages out (device; either may be NULL; unused slots of arity-2
 * factors are unspecified). */
int bp_fg_get_messages(const bp_fgraph* fg, float* m_dev, float* n_dev);
int bp_fg_destroy(bp_fgraph* fg);

/* Beliefs (Eq. 3) from the current messages into out_dev (device,
 * [H][W][M]); rows sum to 1.  For max-product they are sum-normalised
 * max-marginals. */
int bp_beliefs(bp_grid* grid, float* out_dev);

/* MAP labels, the disparity map of Sec. 6: argmax over labels of the
 * float32 beliefs bp_beliefs would return (Eq. 3), lowest label on ties,
 * into out_dev (device, [H][W] int32). */
int bp_map_labels(bp_grid* grid, int32_t* out_dev);

/* Beliefs and MAP labels in one pass over the messages (Eq. 3 and its
 * argmax): the same values bp_beliefs and bp_map_labels write, into either
 * output or both (device, [H][W][M] float32 16-byte aligned and [H][W]
 * int32; BP_EINVAL when both are null or beliefs_dev is misaligned). */
int bp_readout(bp_grid* grid, float* beliefs_dev, int32_t* labels_dev);

/* Copy the current message state out of / into the handle (device,
 * [4][H][W][M] layout above); for checkpoints and warm starts.  set_messages
 * keeps the checkerboard pass parity. */
int bp_get_messages(const bp_grid* grid, float* dst_dev);
int bp_set_messages(bp_grid* grid, const float* src_dev);

/* ------------------------------------------------------------------------
 * Differentiation of unrolled sum-product BP.  The paper motivates
 * sum-product BP by applications that need marginals, such as
 * maximum-likelihood and CRF parameter estimation (Sec. 1, Sec. 2, Sec. 7);
 * these calls return gradients of a loss on the beliefs with respect to the
 * log-unary theta = log g and the smoothness weight alpha.
 *
 * Usage: bp_forward_ckpt, then bp_beliefs (the loss is computed by the
 * caller from those beliefs), then bp_backward with dL/dbeliefs.  Any call
 * that changes the state in between (iterate, reset, set_*, attach) makes
 * bp_backward return BP_ESTATE.
 * Supported: T <= 16 (T <= 12 when M <= 16), the compiled register-window
 * variants, and fbar > 0; otherwise BP_EUNSUPPORTED.  The reverse pass works
 * with adjoints of log messages and divides by each unnormalised message
 * u(y); fbar > 0 keeps u(y) >= fbar * sum(h) > 0, while fbar = 0 (Eq. 8)
 * lets u(y) vanish where h is zero across the window.
 * ---------------------------------------------------------------------- */

/* Device bytes bp_forward_ckpt / bp_backward need for n_iters >= 0
 * synchronous iterations with a message checkpoint every ckpt_every >= 1
 * iterations: ceil(n/k)-1 checkpoints, k recompute buffers, two adjoint
 * buffers (4*H*W*M floats each) and one float per workgroup. */
int64_t bp_grad_workspace_bytes(const bp_grid* grid, int32_t n_iters, int32_t ckpt_every);

/* Reset the messages to 1/M and run n_iters synchronous sum-product
 * iterations (Eq. 7), storing the state every ckpt_every iterations in the
 * caller-owned device workspace gws (>= bp_grad_workspace_bytes, 256-byte
 * aligned).  Afterwards the handle holds the final state m^n, exactly as
 * bp_iterate would leave it. */
int bp_forward_ckpt(bp_grid* grid, int32_t n_iters, int32_t ckpt_every, void* gws, int64_t bytes);

/* Reverse pass.  dL_db (device, [H][W][M]): gradient of the caller's loss
 * with respect to the normalised beliefs of the final state.  Writes
 * dtheta (device, [H][W][M]) = dL/dlog g, and dalpha (device, one float) =
 * dL/dalpha, where fbar moves with alpha (d fbar/d alpha = -T fbar) if it was
 * set with BP_FBAR_TIED and is constant otherwise.  States between
 * checkpoints are recomputed; the alpha reduction has a fixed order, so the
 * result is deterministic.  Accumulation is float32. */
int bp_backward(bp_grid* grid, const float* dL_db, float* dtheta, float* dalpha);

/* Free the handle (host memory only; the caller frees its device memory
 * after its stream has drained). */
int bp_destroy(bp_grid* grid);

/* ------------------------------------------------------------------------
 * Batches: many independent grid MRFs, each with its own H, W, M, T, alpha,
 * fbar and unary (the Sec. 6 stereo model on images of different sizes and
 * disparity ranges), advanced together by the same synchronous O(mM) update
 * (Eq. 7 / Eq. 11).  Instances are grouped by code path (lanes per pixel and
 * window width) and packed, largest first, into launches of up to 8
 * instances whose descriptors travel in the kernel arguments; the launches of
 * different groups touch disjoint instances and their chains of iterations
 * run concurrently on up to 4 private streams (default priority) forked from
 * and joined back into the batch's stream.  The n iterations of
 * bp_batch_iterate are captured once into a HIP graph (per mode, n and
 * buffer parity) and replayed on the batch's stream.  Results do not depend
 * on the plan (streams, passes, grid size): bit for bit those of running
 * each instance alone.
 * Per instance: H, W >= 1; 1 <= M <= BP_MAX_LABELS; 0 <= T <= 8; T < M
 * (else BP_EUNSUPPORTED for T > 8, BP_EINVAL for bad values).
 * Outputs are concatenated in instance order: instance j's beliefs start at
 * float offset sum_{i<j} H_i*W_i*M_i, its labels at sum_{i<j} H_i*W_i.
 * ---------------------------------------------------------------------- */
typedef struct bp_grid_desc {
    int32_t H, W, M, T;
    float alpha;
    float fbar;            /* >= 0, or BP_FBAR_TIED */
    const float* unary;    /* device [H][W][M], 16-byte aligned, borrowed */
} bp_grid_desc;

/* Copy n >= 1 descriptors into a new batch handle on the current device. */
int bp_batch_init(bp_batch** out, int32_t n, const bp_grid_desc* descs, void* hip_stream);
int bp_batch_set_stream(bp_batch* batch, void* hip_stream);

/* Device bytes for every instance's two message buffers. */
int64_t bp_batch_workspace_bytes(const bp_batch* batch);

/* Attach caller-owned workspace (256-byte aligned), build the launch plan
 * and reset all messages to 1/M (enqueued on the batch's stream). */
int bp_batch_attach_workspace(bp_batch* batch, void* dev_ptr, int64_t bytes);

int bp_batch_reset_messages(bp_batch* batch);

/* n_iters synchronous iterations of every instance (mode: BP_SUM_PRODUCT or
 * BP_MAX_PRODUCT; max-product requires f >= fbar for each instance, as for
 * bp_iterate). */
int bp_batch_iterate(bp_batch* batch, int32_t mode, int32_t n_iters);

/* enable = 0: launch the kernels directly on every call instead of
 * replaying captured graphs (results are identical). */
int bp_batch_set_graphs(bp_batch* batch, int32_t enable);

/* Arithmetic of the batch's sum-product updates (Eq. 7), as
 * bp_set_arithmetic for one grid: with BP_ARITH_F32, the instances that
 * qualify for it there (fbar > 0, M = 4 * ceil-pow2(M / 4), 4*H*W*M bytes
 * below 2^32; every batch window is a register window) compute in float32,
 * each equal bit for bit to its single-grid solve with BP_ARITH_F32; the
 * others, and max-product, compute in double.  An instance runs in float32
 * only when every instance launched with it (same lanes per pixel and
 * window width) qualifies.  Drops captured graphs; keeps the messages.
 * BP_EINVAL for a null handle or another value. */
int bp_batch_set_arithmetic(bp_batch* batch, int32_t arith);

/* Work plan: passes[c] = passes per workgroup for instances of lane class c
 * (M <= 16, 32, 64, 128, 256; a pass covers 256 threads' worth of pixels at
 * 4, 8, 16, 32 or 64 lanes per pixel), grid_blocks = workgroups per launch
 * (>= 1; a launch with more pixel ranges than that strides over them; more
 * workgroups than ranges means one range per workgroup).  Keeps the
 * messages, drops captured graphs. */
int bp_batch_set_plan(bp_batch* batch, const int32_t passes[5], int32_t grid_blocks);
int bp_batch_get_plan(const bp_batch* batch, int32_t passes[5], int32_t* grid_blocks);

/* Plan: run the launch chains on at most n_streams (1..4) streams; 1 runs
 * every launch in order on the batch's stream.  Keeps the messages, drops
 * captured graphs.  bp_batch_get_streams returns the current value (or a
 * negative status). */
int bp_batch_set_streams(bp_batch* batch, int32_t n_streams);
int bp_batch_get_streams(const bp_batch* batch);

/* Time a fixed family of candidate plans (streams x passes x grid sizes) for
 * trial_iters >= 1 iterations each on this batch and keep the fastest.
 * Blocks; resets the messages afterwards.  best_us (optional, host) receives
 * the best time per iteration in microseconds. */
int bp_batch_autotune(bp_batch* batch, int32_t mode, int32_t trial_iters, float* best_us);

/* Beliefs (Eq. 3) / MAP labels of every instance (device, concatenated). */
int bp_batch_beliefs(bp_batch* batch, float* out_dev);
int bp_batch_map_labels(bp_batch* batch, int32_t* out_dev);

/* Free the handle and its captured graphs and private streams. */
int bp_batch_destroy(bp_batch* batch);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): one whole solve,
 * messages held in a fixed device array inside the library instead of a
 * caller-attached workspace, and no handle.
 * ---------------------------------------------------------------------- */

/* Bytes of the library's fixed device workspace for bp_solve_noalloc: two
 * message buffers (4*H*W*M floats each, 256-byte aligned) plus the window
 * tables and flag slot of bp_workspace_bytes must fit, i.e. about
 * H*W*M <= 2^21 (for example 256 x 256 x 32 or 288 x 384 x 16). */
#define BP_NOALLOC_WORKSPACE_BYTES (72u * 1024u * 1024u)

/* Uniform start, n_iters iterations (or checkerboard passes, or sweeps) of
 * the O(mM) update of the window potential (arguments as bp_set_potential
 * and bp_iterate), then Eq. 3 beliefs and MAP labels into beliefs_dev
 * ([H][W][M] float32, 16-byte aligned) and/or labels_dev ([H][W] int32),
 * both device, either may be NULL but not both.  g_dev: device unary
 * [H][W][M] as for bp_set_unary.  Enqueued on hip_stream (NULL: default);
 * results equal those of the handle calls bp_init_grid .. bp_readout bit for
 * bit.  Calls no hipMalloc/hipFree: the messages live in a device array of
 * BP_NOALLOC_WORKSPACE_BYTES that each GPU the library runs on keeps until
 * the process ends (looked up on the first call on that device).  All calls
 * on one GPU share that array: calls that overlap in time on one GPU (other
 * streams, other threads) race and give undefined results; calls on one
 * stream in order are safe (each starts from a full reset).
 * Errors: BP_EINVAL (arguments as bp_set_potential / bp_iterate; a problem
 * whose workspace exceeds BP_NOALLOC_WORKSPACE_BYTES), BP_EUNSUPPORTED
 * (max-product with fbar above f(T) and T beyond the register windows, which
 * needs tables staged through host memory), BP_EHIP. */
int bp_solve_noalloc(const float* g_dev, int32_t H, int32_t W, int32_t M, int32_t T, float alpha, float fbar,
                     int32_t mode, int32_t n_iters, int32_t schedule, float* beliefs_dev, int32_t* labels_dev,
                     void* hip_stream);

const char* bp_status_string(int status);
const char* bp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BP_H */
