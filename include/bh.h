/*
 * bh.h -- C ABI of the gfx950 Barnes-Hut tree library.
 *
 * Method: N. Nakasato, "Implementation of a Parallel Tree Method on a GPU"
 * (arXiv:1112.4539).  The library builds the oct-tree of Sec. 4.1 on the GPU
 * (particles in the localized Morton order of Sec. 5), and evaluates the
 * softened gravity of Eq. (1) with the iterative next/more tree walk of
 * Sec. 4.4 and the opening criterion of Eq. (2)/(3).
 *
 * Conventions for every entry point:
 *   - Particle arrays are DEVICE pointers in the caller's order: positions
 *     [n][3] row-major (x, y, z), masses [n], both float (BH_FP32) or double
 *     (BH_FP64), aligned to their element size.  Outputs are device arrays in
 *     the same caller order: acc [n][3], pot [n], same precision as the input.
 *   - The caller owns every buffer, including the workspace (>= 256-byte
 *     aligned); the library allocates no device memory.  A tree handle is a
 *     small host object holding views into the workspace: it must not outlive
 *     the workspace or the input arrays' contents it was built from, and is
 *     freed with bh_tree_release().
 *   - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *     enqueued on it; calls return before the GPU finishes.  Errors found on
 *     the host are returned at once; errors of the GPU work surface on a later
 *     call that synchronises (bh_tree_check, bh_tree_stats, bh_walk_time_ms).
 *   - Return value: BH_OK (0) or a negative status; bh_last_error() gives the
 *     text of the last failure of the calling thread.
 *   - Units: G = 1.  The acceleration on i points toward the sources
 *     (attractive) and the potential is the physical, negative -sum m_j/r.
 *   - Bit-identical results for identical inputs and parameters, whatever the
 *     launch shape (bh_set_walk_config) or target order.
 */
#ifndef BH_H
#define BH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define BH_API __attribute__((visibility("default")))
#else
#define BH_API
#endif

typedef struct bh_tree bh_tree;
typedef struct bh_graph bh_graph;

/* Launch shape of the walk (see bh_set_walk_config); ms = measured walk time. */
typedef struct bh_walk_config {
  int waves_per_block;
  int xcd_chunk;
  int lds_share;
  int persistent;
  int targets_per_lane;
  float ms;
} bh_walk_config;

#define BH_FP32 0
#define BH_FP64 1

#define BH_OK 0
#define BH_EINVAL (-1) /* bad argument: n, pointer, alignment, theta, eps, non-finite input */
#define BH_ENOSPC (-2) /* workspace smaller than bh_workspace_bytes() */
#define BH_EHIP (-3)   /* HIP runtime error; see bh_last_error() */

/* Text of the last error of the calling thread ("" if none). */
BH_API const char *bh_last_error(void);

/* ABI version of this library (bumped on any incompatible change; 3: a
 * per-group theta, the features and the group errors belong to walk groups,
 * runs of 64 of the walk's target order, instead of Morton groups). */
BH_API int bh_version(void);

/* Bytes of workspace a tree of n particles in precision prec needs (an upper
 * bound: the compressed oct-tree has at most 2n-1 nodes).  Returns -1 for an
 * invalid n (n < 0 or n > 2^30 - 1: node and record indices are 32-bit) or prec. */
BH_API int64_t bh_workspace_bytes(int64_t n, int prec);

/* Build the tree of n particles (Sec. 4.1 construction; Sec. 5 Morton order;
 * Sec. 4.4 cell mass, centre of mass and next pointers; Eq. (2) distance s
 * from the cell centre to the centre of mass).
 *   pos [n][3], mass [n]: device, precision prec; must stay unchanged while
 *                        the tree is used (the walk reads sorted copies, but
 *                        bh_tree_check validates the inputs by their bbox pass).
 *   workspace, ws_bytes: device buffer of at least bh_workspace_bytes(n, prec).
 *   out: receives the new handle (host object).
 * The root cube is the coordinate-wise minimum corner with side = the largest
 * extent; cells are cut on its 2^21 grid; a finest-grid cell holding several
 * particles is one leaf.  Non-finite coordinates or masses are flagged on the
 * device and reported by bh_tree_check().  n = 0 is allowed (empty tree). */
BH_API int bh_build_tree(const void *pos, const void *mass, int64_t n, int prec, void *workspace,
                  int64_t ws_bytes, void *stream, bh_tree **out);

/* Synchronise `stream` and report whether the inputs of the build were finite
 * (BH_EINVAL if not), whether the last per-group-theta walk met an invalid
 * theta (BH_EINVAL; see bh_forces_theta) and whether the GPU work failed
 * (BH_EHIP). */
BH_API int bh_tree_check(const bh_tree *t, void *stream);

/* Synchronise `stream` and read the node counts of the tree (any pointer may be NULL). */
BH_API int bh_tree_stats(const bh_tree *t, void *stream, int64_t *n_nodes, int64_t *n_leaves, int64_t *n_internal);

/* Forces on every particle by the tree walk (Sec. 4.4, Fig. 5; opening test
 * Eq. (2): a cell not holding i is used whole iff d^2 > (l/theta + s)^2, d the
 * distance from x_i to the cell's centre of mass, l its side).  Particle and
 * cell terms both use the softened kernel of Eq. (1) with softening eps.
 *   theta: in (0, 2/sqrt(3)) -- beyond it a cell could be accepted by a
 *          particle inside it.  eps >= 0 and finite.
 *   acc [n][3], pot [n]: device outputs, caller order, tree precision.
 * BH_FP32 trees evaluate terms in FP32 (r^2 + eps^2 rounded once, hardware
 * inverse square root) with FP64 opening tests, FP64 offsets and FP64 sums;
 * BH_FP64 trees evaluate every term in FP64. */
BH_API int bh_forces(const bh_tree *t, double theta, double eps, void *acc, void *pot, void *stream);

/* Same walk with one opening parameter per walk group of 64 targets:
 * theta_group [ceil(n/64)] device floats, each in (0, 2/sqrt(3)); group g holds
 * the targets at positions [64g, 64g+64) of the walk's target order (see
 * bh_set_walk_config: the Hilbert order by default; under target_order 0 the
 * Morton positions [64g, 64g+64)).  A value that is not finite or lies outside
 * that range is replaced by 0.5 on the device, and the next bh_tree_check()
 * reports it (BH_EINVAL) until the next per-group walk. */
BH_API int bh_forces_theta(const bh_tree *t, const float *theta_group, double eps, void *acc, void *pot,
                    void *stream);

/* For callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): build + forces in one call
 * for up to BH_NOALLOC_MAX_N particles, with no workspace argument.  Every
 * intermediate array lives in one static device array of the library,
 * BH_NOALLOC_SCRATCH_BYTES per GPU (allocated when the library's code is
 * loaded on a GPU, held until the process ends).  The call allocates no
 * device or host memory.
 *   pos [n][3], mass [n], acc [n][3], pot [n]: device, caller order, precision
 *   prec, as for bh_build_tree + bh_forces, whose results it reproduces bit for
 *   bit (default walk shape).  theta, eps: as for bh_forces.
 *   The work runs on `stream` of the current device.
 * Errors: BH_EINVAL for n outside [0, BH_NOALLOC_MAX_N] or any argument
 * bh_build_tree / bh_forces reject.  Every call on a GPU shares that GPU's
 * array, which keeps the last call's contents (each call rewrites what it
 * reads): calls whose GPU work overlaps on one GPU (other streams, other host
 * threads) race and must be serialised by the caller. */
#define BH_NOALLOC_MAX_N 65536
#define BH_NOALLOC_SCRATCH_BYTES (48 << 20)
BH_API int bh_forces_noalloc(const void *pos, const void *mass, int64_t n, int prec, double theta, double eps,
                             void *acc, void *pot, void *stream);

/* Order of the particle-cell terms of the tree's later walks (bh_forces,
 * bh_forces_theta, bh_walk_stats, bh_graph_create): 1 (default) uses a cell's
 * mass at its centre of mass, the monopole of Eq. (1); 2 adds the quadrupole
 * correction, the second-order Taylor expansion of the cell's softened
 * potential about its centre of mass (Sec. 4.1 allows any higher moment in the
 * particle-cell term; Sec. 7 names higher multipoles as the next step):
 *   acc += M d/rho^3 - 3 (B d)/rho^5 + (15/2 d.B.d/rho^7 - 3/2 T/rho^5) d
 *   pot += -M/rho + (T/rho^3 - 3 d.B.d/rho^5) / 2
 * with d = com - x_i, rho^2 = |d|^2 + eps^2, B the cell's second moments about
 * its centre of mass (sum m y y^T) and T = tr B.  The opening test is the same,
 * so the interaction lists are too.  The first walk of order 2 after a build
 * computes every node's B (FP64) into the workspace.  Order-2 walks take one
 * target per lane (bh_set_walk_config's targets_per_lane is ignored) and read
 * nodes on the scalar route only.  Returns BH_EINVAL for other orders. */
BH_API int bh_set_expansion_order(bh_tree *t, int order);

/* One step of the time loop of Sec. 1 (forces, orbit integration, repeat):
 * a kick-drift-kick leapfrog step of size dt with the tree forces of bh_forces
 * (order 1 or 2, theta, eps as there):
 *   v += dt/2 a;  x += dt v;  rebuild the tree;  a, pot = forces(x);  v += dt/2 a
 * (each update in FP64, rounded once to the state's precision).
 *   pos, vel, acc [n][3], mass, pot [n]: device, precision prec, updated in
 *     place; acc must hold the forces of the current positions on entry (one
 *     bh_forces call before the first step) and holds the new ones on exit.
 *   ids [n] (int64, optional): carried along by the reorder.
 *   reorder: 1 permutes pos, vel, mass, acc, pot and ids into the new tree's
 *     Morton order after the step (Sec. 5: a code that rebuilds its tree every
 *     step gets the localized order for free); the next build then reads
 *     nearly sorted keys, and walking targets in input order walks them nearly
 *     in Morton order.  0 leaves the caller's order.
 *   workspace, ws_bytes: as for bh_build_tree (the step's tree lives there).
 * Errors as for bh_build_tree and bh_forces; BH_EINVAL for a non-finite dt. */
BH_API int bh_leapfrog_step(void *pos, void *vel, void *mass, void *acc, void *pot, int64_t *ids, int64_t n,
                            int prec, double dt, double theta, double eps, int order, int reorder, void *workspace,
                            int64_t ws_bytes, void *stream);

/* Neighbour search by the general tree walk of Sec. 4.3 (Fig. 4): for every
 * particle i, the particles j != i with |x_j - x_i|^2 < radius^2 (FP64 distance
 * of the tree's coordinates), found by walking the tree and skipping every cell
 * that cannot hold such a point.  Outputs in caller order:
 *   count [n] (int32): number of neighbours;
 *   hash [n]: ordered hash of the neighbours' caller indices j, in the walk's
 *     depth-first (Morton) order, h = (h xor (j << 1)) * 1099511628211 from
 *     14695981039346656037 (in a forest j is relative to the cluster's offset
 *     and only the target's own cluster is searched);
 *   lists [n][maxlen] (int64, optional): the first maxlen neighbours, in that
 *     order (entries past the list are left as they were);
 *   rho [n] (optional, tree precision): the SPH density, the per-neighbour work
 *     of proc_particle here: rho_i = m_i W(0, h) + sum_j m_j W(r_ij, h) with
 *     h = radius / 2 and W the M4 cubic spline of support 2h (Monaghan &
 *     Lattanzio 1985), accumulated in FP64.
 * Uses the tree's target order and XCD runs (bh_set_walk_config); overwrites
 * the force walk's node copy (the next force walk rebuilds it). */
BH_API int bh_neighbours(const bh_tree *t, double radius, int32_t *count, uint64_t *hash, int64_t *lists,
                         int64_t maxlen, void *rho, void *stream);

/* The order in which the walk takes its targets, as caller indices: order [n]
 * (device int32), order[64g .. 64g+63] being the targets of wavefront g.  With
 * target_order 2 (the default; bh_set_walk_config) it is the order of the
 * Hilbert index of each particle's cell ten levels below the root cube (fewer
 * in a forest, whose clusters come one after the other), ties in Morton order;
 * 0 gives the Morton order, 1 the caller's order.  Synchronises `stream`. */
BH_API int bh_walk_order(const bh_tree *t, int32_t *order, void *stream);

/* Copy out every node's second moments about its centre of mass (computing
 * them first if no walk of order 2 has since the build): B [n_nodes][6] device
 * doubles, (xx, xy, xz, yy, yz, zz) per node in depth-first preorder.  A leaf
 * sums over its particles (one particle: 0); a cell adds its children's moments
 * shifted to its own centre of mass (parallel-axis theorem), children in octant
 * order.  Synchronises `stream`. */
BH_API int bh_tree_moments2(const bh_tree *t, double *B, void *stream);

/* The walk of bh_forces / bh_forces_theta (theta_group may be NULL) that also
 * records, per particle in caller order, counts [n][2] = (particle terms, cell
 * terms) and hash [n] = ordered-list hash: h = (h xor w) * 1099511628211 from
 * h = 14695981039346656037 over the list words w, w = j<<1 for a particle term
 * with source j (caller index), w = c<<1|1 for a cell term with node c
 * (depth-first preorder id).  In a forest both are relative to the target's
 * cluster (j - offsets[k], c - root of cluster k), so a cluster's words equal
 * those of the same cluster built alone.  If lists != NULL it also writes the first maxlen
 * words of each list to lists [n][maxlen] (entries past the list are left as
 * they were).  If group_steps != NULL it receives, per group of 64 targets of
 * the walk (ceil(n/64) int32; group g is the g-th run of 64 targets of the
 * walk's target order, so the Morton groups only under target_order 0), the
 * number of nodes the group's wavefront visited: sum(counts) / (64 *
 * sum(group_steps)) is the share of useful lanes. */
BH_API int bh_walk_stats(const bh_tree *t, double theta, const float *theta_group, double eps, void *acc,
                  void *pot, int32_t *counts, uint64_t *hash, int64_t *lists, int64_t maxlen,
                  int32_t *group_steps, void *stream);

/* Copy the tree out for inspection: nodes (device, n_nodes records of 64
 * bytes: double com[3], M, l, s; int32 next, first, count, meta with bit 0 =
 * leaf, bit 1 = leaf of several coincident-key particles, bits 8-15 = level)
 * and perm [n] (device int32: Morton position ->
 * caller index).  Either pointer may be NULL.  Synchronises the stream. */
BH_API int bh_tree_export(const bh_tree *t, void *nodes, int32_t *perm, void *stream);

/* Launch shape of the walk: waves_per_block in {1, 2, 4}; xcd_chunk >= -1
 * (runs of workgroups kept on one XCD; 0 = plain order; -1, the default, =
 * 1024 for FP32 trees, about as many one-wave workgroups as an XCD holds at
 * once, so that an XCD's resident waves walk neighbouring groups and share its
 * L2, and 0 for FP64 trees, whose walk measured slower with runs; a run is
 * capped at a 64th of the grid so that every XCD takes at least 8 runs).  target_order 0 =
 * Morton order (groups of Morton-consecutive targets), 1 = caller order (the
 * paper's unsorted experiment, Sec. 5), 2 = Hilbert order (the default):
 * targets sorted by cluster and the Hilbert index of their cell ten levels
 * below the cluster's root cube (fewer in a forest), ties in Morton order, so
 * that a group is a face-connected run of cells; the first walk after each
 * build forms this order with a 4-pass radix sort in the workspace (5 passes
 * beyond 131,072 clusters).  lds_share in [0, 64]: how many waves
 * out of 64 read node records through LDS copies instead of the scalar cache.
 * persistent 0 = one wavefront per group of 64 targets, 1 = a grid that fits
 * the chip at once whose wavefronts take groups from a device counter (kept in
 * the workspace: two walks of one tree must not run concurrently).
 * targets_per_lane 1 or 2: a wavefront walks 64 or 128 Morton-consecutive
 * targets (each node record it reads serves twice as many targets; group_steps
 * of bh_walk_stats then gives each 64-target group its wavefront's count).
 * Results do not depend on any of them. */
BH_API int bh_set_walk_config(bh_tree *t, int waves_per_block, int xcd_chunk, int target_order,
                              int lds_share, int persistent, int targets_per_lane);

/* Enable (1) or disable (0) HIP-event timing of the walk kernel (the force
 * walk of bh_tree_forces and its variants, or the neighbour walk of
 * bh_neighbours); after a timed walk, bh_walk_time_ms synchronises and
 * returns the duration of the last one. */
BH_API int bh_set_timing(bh_tree *t, int enable);
BH_API int bh_walk_time_ms(const bh_tree *t, float *ms);

/* Release a tree handle (host object only; the workspace stays the caller's). */
BH_API void bh_tree_release(bh_tree *t);

/* ---- Batched forest: many independent clusters in one build and one walk.
 * (Sec. 4.4 applied cluster by cluster; the batching itself is beyond the paper.) */

/* Workspace of a forest of n particles in n_clusters clusters (1 <= n_clusters
 * <= 2^24); -1 for invalid arguments.  bh_workspace_bytes(n, p) equals
 * bh_forest_workspace_bytes(n, 1, p). */
BH_API int64_t bh_forest_workspace_bytes(int64_t n, int64_t n_clusters, int prec);

/* Build one tree per cluster: cluster k is the caller's particles [offsets[k],
 * offsets[k+1]) (offsets: device int64 [n_clusters+1], 0 = offsets[0] <= ... <=
 * offsets[n_clusters] = n; may be NULL for one cluster).  Each cluster gets
 * its own root cube, Morton order and tree, exactly as bh_build_tree would
 * build it alone; the clusters' particles stay in their ranges and their
 * subtrees are consecutive preorder ranges (bh_forest_roots).  bh_forces,
 * bh_forces_theta, bh_walk_stats and bh_tree_export then work on the forest: a
 * particle feels only its own cluster, and its result is bit-identical to the
 * single-cluster build.  Bad offsets are reported by bh_tree_check (BH_EINVAL);
 * the build never reads or writes outside its arrays because of them.  The
 * offsets array must stay valid while the tree is used. */
BH_API int bh_build_forest(const void *pos, const void *mass, const int64_t *offsets, int64_t n_clusters,
                           int64_t n, int prec, void *workspace, int64_t ws_bytes, void *stream, bh_tree **out);

/* Copy the preorder id of every cluster's root to roots [n_clusters+1] (device
 * int32; roots[n_clusters] = node count).  Synchronises the stream. */
BH_API int bh_forest_roots(const bh_tree *t, int32_t *roots, void *stream);

/* Capture the whole force pipeline of tree t -- the build from the arrays t was
 * built from (same pointers, re-read at every launch) and bh_forces with theta
 * and eps into acc/pot -- as one HIP graph, with the walk shape set on t at
 * capture time.  The capture runs on a stream of the library's own (after
 * synchronising `stream`) and executes nothing.  bh_graph_launch enqueues one
 * replay on `stream`; t then describes the replayed build.  Replays and other
 * calls on t must not overlap.  The graph holds no memory of its own. */
BH_API int bh_graph_create(bh_tree *t, double theta, double eps, void *acc, void *pot, void *stream,
                           bh_graph **out);
BH_API int bh_graph_launch(bh_graph *g, void *stream);
BH_API void bh_graph_release(bh_graph *g);

/* Pick the walk shape of t by measurement: runs bh_forces (theta, eps, acc, pot)
 * reps times per candidate, one knob at a time (targets_per_lane, persistent,
 * waves_per_block, lds_share, xcd_chunk), keeps the fastest (HIP-event walk time, best of reps),
 * sets it on t and returns it in *best.  If tried != NULL the first max_tried
 * candidates measured are written there and *n_tried gets their number.
 * Synchronises the stream; results of the walk do not depend on the choice. */
BH_API int bh_autotune(bh_tree *t, double theta, double eps, void *acc, void *pot, int reps, void *stream,
                       bh_walk_config *best, bh_walk_config *tried, int max_tried, int *n_tried);

/* ---- Learned opening parameter (beyond the paper, whose theta is one constant
 * in Eq. (2)): per walk group of 64 targets (the groups of bh_forces_theta),
 * features -> MLP -> theta, used by bh_forces_theta.  MLP 8 -> 64 -> 64 -> 1 with tanh-form GELU and
 * theta = 0.2 + 0.8 sigmoid(z); matrix products in bf16 on the matrix cores
 * with FP32 accumulation.  Parameters: flat FP32 device array of n_param = 4801
 * values, W1 [64][8], b1 [64], W2 [64][64], b2 [64], w3 [64], b3 (row-major);
 * bf16 weight copies wbf16 (n_wbf16 uint16, 16-byte aligned) are made by
 * bh_mlp_prepare and refreshed by bh_mlp_adam.  norm: FP32 [16] = mu[8],
 * 1/sd[8]; the network sees bf16((x - mu) / sd). */

/* Features of every walk group g of t (the targets at [64g, 64g+64) of its
 * target order; in a forest the cluster of the group's first Morton position
 * sets N, L and the total mass M): X [ceil(n/64)][8]
 * device FP32, scale-free, with h the half-width of the group's bounding box,
 * c the smallest cell holding the group and l_c its side:
 *   log2(h / (L (64/N)^(1/3) / 2)),
 *   |group centre of mass - centre of mass of c| / l_c,
 *   the same against the ancestor of c three levels up (or the root),
 *   mass-weighted RMS radius about the group's centre of mass / h,
 *   |centre of mass - box centre| / h,
 *   log10 of the density M_c / l_c^3 of c over the mean M / L^3,
 *   the same for the parent of c,
 *   log2(l_c / h).
 * Errors: BH_EINVAL for a null tree or X. */
BH_API int bh_features(const bh_tree *t, float *X, void *stream);

/* Per-group force error against a reference: for every walk group g of t (as
 * in bh_features), rms[g] = RMS over its particles of |acc - acc_ref| /
 * |acc_ref| (acc in the tree's precision, acc_ref FP64, both [n][3] caller
 * order; particles with a zero reference force are left out, and a group of
 * only such particles has rms 0).  If label != NULL: label[g] = max(label[g], theta)
 * where rms[g] <= target -- called for ascending theta it leaves the largest
 * theta of the grid that meets the target.  rms may be NULL. */
BH_API int bh_group_error(const bh_tree *t, const void *acc, const double *acc_ref, double theta, double target,
                          double *rms, float *label, void *stream);

/* Sizes (element counts) of the MLP arrays: parameters, gradient vector (the
 * parameters' gradient followed by the batch loss), bf16 weight copies, and
 * the partial-gradient scratch of bh_mlp_grad for a batch of `batch` rows. */
BH_API int bh_mlp_sizes(int64_t batch, int64_t *n_param, int64_t *n_grad, int64_t *n_wbf16, int64_t *n_partial);

/* Round the weights of params to the bf16 copies wbf16. */
BH_API int bh_mlp_prepare(const float *params, uint16_t *wbf16, void *stream);

/* theta [rows] = min(alpha (0.2 + 0.8 sigmoid(z(X_row))), 1.15) for X [rows][8];
 * a non-finite value is replaced by theta_fallback (the fixed-theta walk). */
BH_API int bh_mlp_infer(const float *params, const uint16_t *wbf16, const float *norm, const float *X,
                        int64_t rows, float alpha, float theta_fallback, float *theta, void *stream);

/* Gradient of the loss mean_b (sigmoid(z_b) - target_b)^2 over the batch rows
 * rows_idx [batch] of X / target (target = (theta* - 0.2) / 0.8):
 * grad [n_grad] (device FP32, last entry = loss).  partial: scratch of
 * n_partial floats.  Deterministic (fixed summation order). */
BH_API int bh_mlp_grad(const float *params, const uint16_t *wbf16, const float *norm, const float *X,
                       const float *target, const int32_t *rows_idx, int64_t batch, float *partial, float *grad,
                       void *stream);

/* One Adam step (Kingma & Ba) on params with gradient grad and moments m, v
 * (FP32 [n_param], zero before the first step, step counts from 1); refreshes
 * the bf16 copies. */
BH_API int bh_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step, float lr, float beta1,
                       float beta2, float eps, uint16_t *wbf16, void *stream);

/* Brute-force sum of Eq. (1) over all j != i for nt targets (Sec. 3):
 * pos [n][3], mass [n] device in precision prec; targets [nt] device int64
 * caller indices in [0, n); acc [nt][3], pot [nt] device outputs in target
 * order.  eps >= 0.  BH_FP64 follows the reference expression in ascending j. */
BH_API int bh_direct(const void *pos, const void *mass, int64_t n, int prec, const int64_t *targets,
              int64_t nt, double eps, void *acc, void *pot, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BH_H */
