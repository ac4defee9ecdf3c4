/*
 * libtpe — discrete tangent-point energy and its vertex gradient on MI355X (gfx950).
 *
 * The energy follows the paper's definition of the tangent-point energy of a closed surface
 * (Sec. 2.2.2 "Self-avoidance", eq. (TP)): with the tangent-point radius
 * R(x,y) = |x-y|^2 / (2 |n(x).(x-y)|),  Phi = rho 2^-alpha / alpha  int_S int_S R^-alpha
 *       = rho / alpha  int_S int_S |n(x).(x-y)|^alpha / |x-y|^(2 alpha).
 * It is discretised on flat triangles with one quadrature point per face (the centroid) or a
 * multi-point rule (TPE_OPT_QUADRATURE), or on curved cubic elements (the *_p3 calls), and
 * pairs of faces that share a vertex index are left out (the continuous integrand has no
 * exclusion; on a mesh those pairs sit on the diagonal of the double integral).  For faces
 * S, T with area a, unit normal n and centroid c:
 *
 *     E(X) = scale * sum_S sum_{T: S,T share no vertex} a_S a_T |n_S.(c_S-c_T)|^q / |c_S-c_T|^p
 *
 * over ORDERED pairs (both orders, as the double integral counts them).  The paper's Phi is
 * q = alpha, p = 2 alpha, scale = rho / alpha (it uses alpha = 6, rho = 1e-4).  The gradient is
 * dE/dX, i.e. the deformation derivative of eq. (dTP) for the discrete surface, evaluated in the
 * reordered form eq. (dTP_reordered) (Sec. 3.2): each face collects its own inner integrals
 * and no pair writes into another face.  The self-avoidance force is -dE/dX.
 *
 * Conventions for every call below:
 *   - Array arguments are DEVICE pointers owned by the caller (e.g. PyTorch tensors) unless the
 *     argument says "host".  X is row-major float64 [V][3]; F is row-major int32 [nF][3], 0-based
 *     vertex indices; face orientation does not matter for the exact path (|.| in the kernel).
 *   - Work is enqueued on the context's stream and is asynchronous.  Outputs are valid once the
 *     stream reaches them.  Calls of one context are ordered among themselves even when the
 *     stream changes between them (tpe_set_stream).  The library owns only opaque objects
 *     (context, scratch arena).
 *   - Return value: TPE_OK or a negative tpe_status; tpe_last_error() gives a message.  Inputs
 *     that can only be checked on the device (vertex indices in range, finite coordinates,
 *     non-degenerate faces, finite result) are checked by the kernels, which never read out of
 *     bounds; with the sync-checks option on (default) the call waits for the stream and
 *     returns the corresponding status, with it off the status is collected by tpe_check().
 *   - A context is not thread-safe; use one per host thread or serialise calls.
 *   - Supported exponents: (q, p) = (6, 12) (the paper's alpha = 6) everywhere.  tpe_energy and
 *     tpe_gradient (with any quadrature rule) and tpe_energy_p3 / tpe_gradient_p3 also take
 *     even q in {2, 4, 6, 8} with even p,
 *     q < p <= 2q (the tangent-point family of Sec. 2.2.2 whose kernel stays in FP32 range on
 *     meshes of unit size); the far field, the learned correction and the confinement energy do
 *     not.  Others return TPE_ERR_UNSUPPORTED.
 *   - Sizes: nF <= 2^24, V <= 2^26.
 */
#ifndef TPE_H
#define TPE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tpe_ctx tpe_ctx;
typedef struct tpe_tree tpe_tree;  /* cluster tree: a k-d ordering of the faces (tpe_build_tree) or of the
                                      quadrature points of curved elements (tpe_build_tree_p3) */
typedef struct tpe_mlp tpe_mlp;    /* learned far-field correction (see tpe_mlp_create) */

typedef enum {
    TPE_OK = 0,
    TPE_ERR_INVALID_ARG = -1, /* null pointer, bad size, vertex index out of range, bad exponents */
    TPE_ERR_DEGENERATE = -2,  /* a face with area <= 1e-300 (curved elements: |J| <= 1e-300 at a
                                 quadrature point) */
    TPE_ERR_NONFINITE = -3,   /* non-finite coordinate, or coincident centroids of a non-adjacent
                                 pair (the energy is infinite for such a non-embedded surface) */
    TPE_ERR_OOM = -4,         /* device allocation of the scratch arena failed */
    TPE_ERR_HIP = -5,         /* a HIP runtime call failed */
    TPE_ERR_UNSUPPORTED = -6  /* exponents outside the supported set */
} tpe_status;

typedef enum {
    TPE_OPT_SYNC_CHECKS = 1,  /* 1 (default): every call synchronises and reports device-side
                                 errors; 0: calls stay asynchronous, tpe_check() reports */
    TPE_OPT_TARGET_WAVES = 2, /* work-groups of the persistent exact pair kernel;
                                 0 (default) = as many as the device keeps resident at once.  The
                                 work is split evenly over them; results agree to rounding */
    TPE_OPT_KERNEL_TIMING = 3, /* 1: record HIP events around every launch of the dominant
                                 kernel (the pair kernel; the far-field evaluation kernel of
                                 tpe_farfield / tpe_farfield_p3, after its classify and launch-order
                                 passes; the whole dual-tree pipeline of tpe_farfield_dual) on the
                                 context's stream; 2: around the finalize + vertex-gather launches;
                                 read back with tpe_kernel_time(); 0 (default): off */
    TPE_OPT_QUADRATURE = 4,   /* quadrature points per face of tpe_energy / tpe_gradient and per
                                 element of tpe_energy_p3 / tpe_gradient_p3 / tpe_build_tree_p3:
                                 1 (default, the centroid), 3 (degree 2) or 6 (degree 4); the
                                 paper integrates both integrals with higher-order rules (Sec.
                                 3.2).  Each point pair of two faces sharing no vertex contributes
                                 W_p W_r a_S a_T |n_S.(x_Sp - x_Tr)|^q / |x_Sp - x_Tr|^p.  The flat
                                 far field and the confinement energy take 1 only (else
                                 TPE_ERR_UNSUPPORTED); at most 2^26 points in all. */
    TPE_OPT_SYMMETRIC = 5     /* 1 (default): tpe_energy / tpe_gradient evaluate every unordered pair
                                 of faces once and credit both faces (the symmetric pair kernel) --
                                 with (q, p) = (6, 12) always, with the other even exponents when
                                 the kernel runs without barriers with 4 or 8 waves per work-group
                                 (the default) -- while its column partial sums fit in 64 GiB of
                                 the context's scratch (about 2,100,000 faces with 8 waves per
                                 work-group, 1,480,000 with 4) and that scratch can be allocated;
                                 0, or otherwise: every ordered pair from its row face (the
                                 row-only kernel).  Results agree to rounding.  The scratch stays
                                 allocated with the context (tpe_destroy frees it) */,
    TPE_OPT_SYM_WAVES = 6     /* waves per work-group of the symmetric pair kernel: 1, 2, 4 or 8 (super
                                 blocks of 128 to 1,024 faces; fewer waves write proportionally
                                 more column partial sums; 8 only without barriers).  0 (default):
                                 4 without barriers (8 where the partials of 4 would exceed 64 GiB,
                                 above about 1,480,000 faces; see TPE_OPT_SYM_BARRIERS); with
                                 barriers, the fewest whose column partial sums fit in 8 GiB (1
                                 up to about 262,000 faces, then 2 up to about 370,000, then 4),
                                 since fewer waves wait less at the barriers.  tpe_exact_plan
                                 tells.  Results agree to rounding */,
    TPE_OPT_SYM_BARRIERS = 7  /* 0 (default): the symmetric pair kernel with 2, 4 or 8 waves per
                                 work-group runs without work-group barriers (each wave stages its
                                 own columns; the waves' column sums meet in a ring of LDS slots,
                                 reduced in wave order by the last wave to arrive); 1: with a
                                 barrier per unit.  The same bits either way */
} tpe_option;

/* Library version as major*10000 + minor*100 + patch. */
int tpe_version(void);

/* Create a context on HIP device `device`, enqueueing on `hip_stream` (a hipStream_t; NULL = the
 * null stream).  The context also owns a second stream of default priority: the far field on
 * curved elements (tpe_farfield_p3) forks its node lists onto it (only the final gather reads
 * them) and joins it back into `hip_stream` before that gather, so every call stays ordered on
 * `hip_stream` as a whole (the flat far field's vertex lists are built once with the tree).
 * *out receives the context; ownership passes to the caller (tpe_destroy). */
int tpe_create(tpe_ctx** out, int device, void* hip_stream);

/* Destroy a context and free its scratch arena.  Waits for the context's stream first. */
int tpe_destroy(tpe_ctx* ctx);

/* Rebind the stream work is enqueued on (e.g. PyTorch's current stream).  The context's calls stay
 * ordered across streams: every call records an event on its stream when it returns, and a call on
 * another stream than the previous call's first makes its stream wait for that event (on the
 * device; no host synchronisation).  Work the caller enqueues itself is ordered by the caller's
 * streams as usual: results of a call on stream A are complete for later work on A. */
int tpe_set_stream(tpe_ctx* ctx, void* hip_stream);

/* Set an option (tpe_option).  Returns TPE_ERR_INVALID_ARG for unknown options or values. */
int tpe_set_option(tpe_ctx* ctx, int option, int64_t value);

/* Message describing the last error on this context ("" if none).  Owned by the context. */
const char* tpe_last_error(const tpe_ctx* ctx);

/* Wait for the context's stream and report device-side errors raised since the last report
 * (only needed with TPE_OPT_SYNC_CHECKS = 0). */
int tpe_check(tpe_ctx* ctx);

/* E_dev (device, one double) <- E(X).  Paper eq. (TP) as discretised above.
 * X: device f64 [V][3]; F: device i32 [nF][3]; V, nF >= 1; q, p exponents; scale multiplies E. */
int tpe_energy(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF,
               double q, double p, double scale, double* E_dev);

/* G_dev (device f64 [V][3]) <- dE/dX and, if E_dev != NULL, E_dev <- E(X).
 * Paper eqs. (dTP) / (dTP_reordered) for the discrete energy above.  Vertices that belong to no
 * face get a zero gradient.  G_dev must not alias X. */
int tpe_gradient(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF,
                 double q, double p, double scale, double* E_dev, double* G_dev);

/* tpe_gradient for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same energy and gradient, computed with the
 * row-only pair kernel (as tpe_gradient with TPE_OPT_SYMMETRIC = 0, to the same bits) in a scratch
 * array of 64 MiB that the library holds on every device it runs on until the process ends, instead
 * of the context's arena.  Makes no device or host allocation (no hipMalloc, no event creation;
 * TPE_OPT_KERNEL_TIMING is ignored).  Meshes whose scratch exceeds 64 MiB (about 147,000 faces
 * with one quadrature point: 456 bytes per face at 327,680) return TPE_ERR_INVALID_ARG with the
 * size in the message.  All calls on one device share that array, which keeps the last call's
 * contents: calls that overlap on one device (other contexts, or other host threads) race and must
 * be serialised by the caller; calls of one context are ordered as usual.  Arguments and errors as
 * for tpe_gradient; flat faces only. */
int tpe_gradient_noalloc(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF,
                         double q, double p, double scale, double* E_dev, double* G_dev);

/* The same energy and gradient on curved cubic (P3) elements, the paper's surface S_h^3 (Sec. 3.1)
 * with its quadrature at the points of the curved elements (Sec. 3.2).
 * X: device f64 [V][3], all nodes; F10: device i32 [nF][10], the nodes of each element at the
 * barycentric lattice points m / 3 in the order
 *     (3,0,0) (0,3,0) (0,0,3) | (2,1,0) (1,2,0) | (0,2,1) (0,1,2) | (1,0,2) (2,0,1) | (1,1,1)
 * (corners, the two nodes of edges 0-1, 1-2 and 2-0 from the edge's first corner, centre);
 * neighbouring elements share corner and edge nodes.  The element maps reference point (s, t) to
 * x(s, t) = sum_k phi_k(1 - s - t, s, t) X_k with the cubic Lagrange basis phi_k.  Quadrature
 * point b (barycentric) of the rule chosen by TPE_OPT_QUADRATURE (1, 3 or 6 points, on both
 * integrals) becomes a record at x(b) with normal J / |J| and weight w_b |J| / 2,
 * J = x_s x x_t, and
 *     E = scale * sum_S sum_{T : S, T share no corner node} sum_{b, c} weight_Sb weight_Tc
 *                 |n_Sb . (x_Sb - x_Tc)|^q / |x_Sb - x_Tc|^p.
 * The gradient is its exact derivative with respect to every node (nodes in no element: zero).
 * Exponents, options (symmetric kernel, work-group count) and errors as for tpe_energy /
 * tpe_gradient; a node index outside [0, V) is TPE_ERR_INVALID_ARG, an element whose |J| vanishes
 * at a quadrature point TPE_ERR_DEGENERATE.  With every node at its lattice point of the flat
 * triangle of the corners the results are those of tpe_energy / tpe_gradient with the same rule
 * (the flat gradient being the pull-back through the node positions). */
int tpe_energy_p3(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F10, int64_t nF,
                  double q, double p, double scale, double* E_dev);
int tpe_gradient_p3(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F10, int64_t nF,
                    double q, double p, double scale, double* E_dev, double* G_dev);

/* Stable LSD radix sort of n (key, value) pairs in place by the low `bits` bits of the keys (the
 * sort that orders faces along the Morton curve and the tree's k-d order, exposed for testing and
 * reuse).  keys, vals: device u32 [n], caller-owned, sorted in place (pairs with equal low bits
 * keep their input order; the keys' other bits travel with them).  1 <= bits <= 32,
 * 0 <= n <= 2^30; uses the context's scratch arena. */
int tpe_sort_pairs(tpe_ctx* ctx, uint32_t* keys, uint32_t* vals, int64_t n, int bits);

/* Confinement energy (paper Sec. 2.2.3, eq. (TPConf)) of the moving surface (X, F) against a fixed
 * confining surface (Y, FY), with the same one-point centroid quadrature:
 *     E_conf = scale * sum_{S in F} sum_{T in FY} a_S a_T |n_S . (c_S - c_T)|^q / |c_S - c_T|^p.
 * Only the moving surface's normal enters (the confinement may be non-smooth), every pair counts
 * once and none is excluded.  The paper's prefactor is scale = rho_conf / alpha, rho_conf = 1e-4.
 * X, Y: device f64 [V][3] / [VY][3]; F, FY: device i32 [nF][3] / [nFY][3]; the confining surface
 * is only read.  E_dev (device, one double) <- E_conf.  Errors as for tpe_energy, for either
 * surface; coincident centroids across the surfaces give TPE_ERR_NONFINITE. */
int tpe_conf_energy(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF, const double* Y,
                    int64_t VY, const int32_t* FY, int64_t nFY, double q, double p, double scale, double* E_dev);

/* G_dev (device f64 [V][3]) <- dE_conf/dX (the confining surface is fixed) and, if E_dev != NULL,
 * E_dev <- E_conf.  G_dev must alias neither X nor Y. */
int tpe_conf_gradient(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF, const double* Y,
                      int64_t VY, const int32_t* FY, int64_t nFY, double q, double p, double scale, double* E_dev,
                      double* G_dev);

/* Build the cluster tree used by tpe_farfield (paper Sec. 3.2: the inner integrals are clustered
 * with precomputed averages over patches of elements, Barnes-Hut style).  The tree is an implicit
 * complete binary tree over leaves of `leaf_size` consecutive faces (1..4096; 32 in the
 * paper-scale workloads); the faces are ordered top-down so that each node's faces are split
 * along the longest axis of their centroid bounding box (k-d order), which keeps every cluster a
 * compact patch.  Only
 * the ordering is stored: the cluster moments are recomputed from the positions passed to each
 * tpe_farfield call, so one tree serves a whole gradient flow as long as the faces stay put in
 * the ordering sense (accuracy, not correctness, depends on it).  Each tpe_farfield call first
 * lists, per target block of 64 faces, its far clusters and near nodes (one walk of the tree), then
 * evaluates the lists; a monopole call (mlp NULL) launches the blocks with the most work first.
 * That changes only when blocks run, never what they compute.  The tree keeps the work of each
 * block of its last call (a device array, written by every call; calls that share one tree on
 * several streams at once are still correct), the vertex -> (face, corner) lists of the gradient's
 * vertex gather in tree order (they depend only on F and the order; 12 B per face), per target
 * block the tiles of 64 faces that hold a face sharing a vertex with it, with a 64-bit exclusion
 * mask per (row, listed tile) that the evaluation tests instead of comparing vertex ids (at most 16
 * tiles: 68 B + 8 KB per block, about 130 B per face), and a checksum of F: every far-field call
 * recomputes the checksum of the F it is given and fails with TPE_ERR_INVALID_ARG if it differs.
 * *out is owned by the caller (tpe_tree_destroy).
 * Synchronises the stream. */
int tpe_build_tree(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF,
                   int32_t leaf_size, tpe_tree** out);

/* Free a tree. */
int tpe_tree_destroy(tpe_tree* tree);

/* perm_dev (device u32 [n], caller-owned) <- the tree's order: perm_dev[i] is the item (face, or
 * point record Q f + point for a tpe_build_tree_p3 tree) at tree position i; node k of the implicit
 * tree (root 1, children 2k and 2k + 1, leaves 2^H .. 2^H + ceil(n / leaf) - 1) holds the positions
 * [(k - 2^l) leaf 2^(H - l), (k - 2^l + 1) leaf 2^(H - l)) clipped to n, l = floor(log2 k).  The
 * order is the k-d order of tpe_build_tree: level by level, the items of every node are sorted
 * stably by key = (node << b) | quantised coordinate, the coordinate being the FP32 centroid's
 * along the longest axis of the node's FP32 centroid box, quantised to b = min(16, 32 - level)
 * bits as (uint32) min(max((x - lo) / extent * (2^b - 1), 0), 2^b - 1) in FP32 (0 for a box of
 * zero extent); the FP32 centroid is the FP64 mean of the three corners, rounded (paper Sec. 3.2
 * leaves the tree open).  n must be the tree's item count (nF, or nF Q). */
int tpe_tree_order(tpe_ctx* ctx, const tpe_tree* tree, uint32_t* perm_dev, int64_t n);

/* Barnes-Hut approximation of E and dE/dX on the tree (paper Sec. 3.2, clustering of the inner
 * integrals of eq. (dTP_reordered)).  Every block of 64 consecutive faces in tree order is
 * enclosed by a ball (C_T, r_T); a cluster B with area A_B, area-weighted centroid C_B, unit
 * mean normal N_B and vertex-bounding radius r_B is far when 2 r_B < theta (|C_T - C_B| - r_T)
 * and then acts on each face of the block as one pseudo-face (C_B, A_B, N_B); every other pair is
 * evaluated exactly, with the shared-vertex exclusion.  r_B is the largest distance from C_B to a
 * vertex of a leaf's faces, and max over the children of |C_child - C_B| + r_child above; r_T the
 * largest distance from C_T (the mean of the block's centroids) to a vertex of the block.  The test
 * is taken in FP32 on the mesh scaled by the power of two 2^k that brings the largest extent of the
 * FP32 centroid box into [0.5, 1): centres relative to that box's centre, rounded to FP32, radii
 * r + 1e-6 (1 + |C|_1) rounded up,
 * |C_T - C_B| = sqrt(fma(dz, dz, fma(dy, dy, dx dx))).  theta in [0, 1] (theta <= 2 keeps faces that
 * share a vertex with the block out of far clusters; else TPE_ERR_INVALID_ARG); theta = 0
 * reproduces tpe_gradient to rounding.  G is the clustered form of eq. (dTP_reordered) (each
 * face's inner integrals with far patches replaced by their averages), not the derivative of E:
 * the paper propagates nothing back to the patches.  mlp: NULL for the plain monopole.  The call
 * lists every block's far clusters and near nodes in its scratch arena (at most ceil(nF / leaf)
 * entries per block, within 8 GiB in all; TPE_ERR_OOM beyond that, which only meshes of several
 * million faces at small theta reach).  E_dev and/or G_dev (device) may be NULL but not
 * both.  X, V, F, nF must describe the mesh the tree was built for (same size, same faces: a face
 * list whose checksum differs from the tree's fails the call with TPE_ERR_INVALID_ARG). */
int tpe_farfield(tpe_ctx* ctx, const tpe_tree* tree, const double* X, int64_t V,
                 const int32_t* F, int64_t nF, double q, double p, double scale, double theta,
                 const tpe_mlp* mlp, double* E_dev, double* G_dev);

/* The same far field on curved cubic elements (F10 and V as for tpe_energy_p3).  The tree
 * (tpe_build_tree_p3) is built over the quadrature points of the elements, with the rule chosen by
 * TPE_OPT_QUADRATURE at build time (1, 3 or 6 points); its items are those point records, so
 * clusters gather points, a cluster acts on each point of a target block as one pseudo-record,
 * and near pairs of points are summed exactly with the exclusion of element pairs sharing a
 * corner node.  theta in [0, 1]; theta = 0 reproduces tpe_gradient_p3 with the same rule to rounding.  The ordering
 * and the per-block work record (as for tpe_build_tree, blocks of 64 points) are kept; positions,
 * weights, normals and moments are recomputed from X on every call. */
int tpe_build_tree_p3(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F10, int64_t nF,
                      int32_t leaf_size, tpe_tree** out);
int tpe_farfield_p3(tpe_ctx* ctx, const tpe_tree* tree, const double* X, int64_t V, const int32_t* F10,
                    int64_t nF, double q, double p, double scale, double theta, const tpe_mlp* mlp,
                    double* E_dev, double* G_dev);

/* Dual-tree (cluster-cluster) approximation of E and dE/dX on the tree: both integrals clustered,
 * the scheme the paper compares against in Sec. 3.2 (its own clusters only the inner integrals),
 * with the derivatives carried back from the clusters to the faces.  A pair of same-level clusters
 * (A, B) (area, area-weighted centroid, unit mean normal, vertex-bounding radius each) is far when
 * 2 max(r_A, r_B) < theta |C_A - C_B| and then counts as one pair of pseudo-faces for all its face
 * pairs; the interaction lists are built level by level (the children of a node's parent's near
 * clusters are its candidates), and the near pairs of the dual leaves (the nodes of 64 faces)
 * are evaluated exactly, with the shared-vertex exclusion.  E is this approximate energy and G
 * its exact gradient (every cluster's derivative passed down to its faces).  theta in [0, 1];
 * theta = 0 reproduces tpe_gradient to rounding (at quadratic cost).  The tree's leaf size must
 * divide 64.  TPE_ERR_OOM if the lists outgrow their scratch (384 entries per node on average;
 * only for theta far below 0.5).  E_dev and/or G_dev may be NULL but not both.  (Not in the
 * paper's own method.) */
int tpe_farfield_dual(tpe_ctx* ctx, const tpe_tree* tree, const double* X, int64_t V, const int32_t* F,
                      int64_t nF, double q, double p, double scale, double theta, double* E_dev, double* G_dev);

/* ---- learned far-field correction (not part of the paper) ------------------------------------
 * A multilayer perceptron 32 -> 64 -> 64 -> 64 -> 16 (ReLU), evaluated and trained with BF16
 * matrix-core (MFMA) products accumulated in FP32, with FP32 master weights and Adam.  Its inputs
 * are 32 features of a (target face, far cluster) pair and its 16 outputs (7 used) correct the
 * monopole's contribution to the face's row sums; see tpe_farfield_samples.  Parameters are one
 * FP32 vector: W1[32][64], b1[64], W2[64][64], b2, W3[64][64], b3, W4[64][16], b4[16]. */

/* Create a network with He-uniform weights drawn from a 64-bit Mersenne twister seeded with
 * `seed` and zero biases.  Only (d_in, width, depth, d_out) = (32, 64, 3, 16) is implemented
 * (TPE_ERR_UNSUPPORTED otherwise).  *out is owned by the caller (tpe_mlp_destroy). */
int tpe_mlp_create(tpe_ctx* ctx, int32_t d_in, int32_t width, int32_t depth, int32_t d_out,
                   uint64_t seed, tpe_mlp** out);
int tpe_mlp_destroy(tpe_mlp* mlp);
/* Number of FP32 parameters (11,472), or -1 for NULL. */
int64_t tpe_mlp_num_params(const tpe_mlp* mlp);
/* Copy the FP32 parameters to / from a host array of exactly tpe_mlp_num_params floats.
 * Synchronise the stream. */
int tpe_mlp_get_params(tpe_ctx* ctx, const tpe_mlp* mlp, float* host, int64_t n);
int tpe_mlp_set_params(tpe_ctx* ctx, tpe_mlp* mlp, const float* host, int64_t n);
/* tpe_farfield applies the correction only to far clusters with r_B / rho >= min_s (default 0:
 * all); rho = |c_S - C_B|.  A wave skips the network for a cluster when none of its 64 faces is
 * inside the gate.  Stored with the network and in checkpoints. */
int tpe_mlp_set_gate(tpe_ctx* ctx, tpe_mlp* mlp, float min_s);
/* *min_s (host) <- the gate of mlp. */
int tpe_mlp_get_gate(tpe_ctx* ctx, const tpe_mlp* mlp, float* min_s);
/* Weight lam >= 0 (default 0) of the training loss's difference term: for consecutive rows i, i+1
 * of one 32-row tile of a training batch, lam w_i w_(i+1) sum_(j<7) ((y_(i+1),j - y_ij) -
 * (t_(i+1),j - t_ij))^2 is added to the loss (same normalisation).  Rows of a tile of the
 * samples tpe_farfield_samples writes are neighbouring faces seeing the same cluster, so the term
 * asks the correction to vary from face to face as the exact one does.  Not stored in
 * checkpoints.  (Not in the paper.) */
int tpe_mlp_set_smoothness(tpe_ctx* ctx, tpe_mlp* mlp, float lam);
/* out (device f32 [n][16]) <- network(feats (device f32 [n][32])), evaluated with the BF16 weights
 * and activations exactly as tpe_farfield evaluates it (bit-identical for the same features). */
int tpe_mlp_forward(tpe_ctx* ctx, const tpe_mlp* mlp, const float* feats, int64_t n, float* out);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, learning rate lr > 0) on the batch feats (device
 * f32 [n][32]) / targets (device f32 [n][16]: columns 0..6 are targets, column 15 the sample
 * weight, 0 = unused row) for the loss sum_i w_i sum_{j<7} (y_ij - t_ij)^2 / (7 sum_i w_i);
 * loss_dev (device f32, nullable) receives the batch loss before the update. */
int tpe_mlp_train_step(tpe_ctx* ctx, tpe_mlp* mlp, const float* feats, const float* targets,
                       int64_t n, float lr, float* loss_dev);
/* grad_dev (device f32 [num_params]) <- d loss / d parameters on the batch, without updating
 * (a hook for checking the hand-written backward pass). */
int tpe_mlp_gradient(tpe_ctx* ctx, tpe_mlp* mlp, const float* feats, const float* targets,
                     int64_t n, float* grad_dev);
/* Checkpoint: magic "TPEMLP02", int32 dims[4], int64 Adam step, float32 gate min_s and 4 bytes of
 * padding, then parameters, first and second Adam moments (FP32 each).  Training resumes exactly
 * from a loaded checkpoint.  Files with magic "TPEMLP01" (no gate field) load with min_s = 0. */
int tpe_mlp_save(tpe_ctx* ctx, const tpe_mlp* mlp, const char* path);
int tpe_mlp_load(tpe_ctx* ctx, const char* path, tpe_mlp** out);

/* Training samples for the learned correction, drawn with the same tree walk as tpe_farfield at
 * opening parameter theta.  A far cluster with at most max_cluster_faces faces is selected with
 * probability ~select_prob (a hash of seed, target block and node; deterministic), up to `quota`
 * clusters per target block of 64 faces (in walk order); cluster B of block b is selected when
 * u = fmix32(fmix32(fmix32(s) ^ b) ^ B) <= floor(select_prob 2^32) (every cluster for select_prob =
 * 1), s = low 32 bits of seed ^ (seed >> 32), fmix32 the 32-bit finaliser of MurmurHash3.  theta in
 * (0, 1].  Each selected (block, cluster) yields one sample per face of the block:
 *   feats   (device f32, rows x 32): features of the (face, cluster) pair in a local frame
 *           e1 = unit(c_S - C_B), e2 = unit part of n_S orthogonal to e1, e3 = e1 x e2:
 *           [4 r_B/rho, n_S.e1, n_S.e2, mean normal of B (3), |N_B|/A_B, M2c/(A_B r_B^2) (6),
 *            M2n/A_B (6), 0 x 13] (the symmetric forms e_a . M e_b in the order 11 12 13 22 23 33),
 *           rho = |c_S - C_B|, r_B the FP32 radius of the admissibility test, M2c / M2n the
 *           area-weighted second moments of centroid offsets (about C_B) and of normals;
 *   targets (device f32, rows x 16): the exact sum over B's faces minus the monopole of the
 *           quantities the face's gradient is made of: K (dE/da), Sd[3] (dE/dn) and the net
 *           C[3] = q (n_S S0 + Sn) - p Sdd (dE/dc), vectors in the frame, divided by
 *           A_B rho^-6 (K, Sd) or A_B rho^-7 (C); columns 7..13 zero; column 14 = the
 *           cluster's node index (as a float); column 15 = weight (1, or 0 for an unused row,
 *           whose other columns are 0).
 * rows = ceil(nF / 64) * quota * 64; the caller allocates the outputs.  If mlp is not NULL, pred
 * (device f32, rows x 16) receives the network's output for each sample computed by the same
 * in-walk (fused) inference tpe_farfield uses; otherwise pred must be NULL. */
int tpe_farfield_samples(tpe_ctx* ctx, const tpe_tree* tree, const double* X, int64_t V,
                         const int32_t* F, int64_t nF, double theta, uint64_t seed, double select_prob,
                         int32_t quota, int64_t max_cluster_faces, const tpe_mlp* mlp, float* feats,
                         float* targets, float* pred);

/* Interaction counts of the last tpe_farfield call on this context, summed over target blocks of
 * 64 faces (each count applies to every face of a block): out_host[0] = far clusters evaluated,
 * [1] = near columns evaluated exactly, [2] = tree nodes visited, [3] = target blocks; and the
 * largest per block: [4] = near columns, [5] = far clusters.  After tpe_farfield_dual: [0] =
 * far cluster pairs, [1] = exactly evaluated face pairs, the rest 0.  Host array of 6 int64.
 * Synchronises the stream. */
int tpe_farfield_stats(tpe_ctx* ctx, int64_t* out_host);

/* How tpe_gradient (grad = 1) or tpe_energy (grad = 0) with (q, p) = (6, 12) would run a mesh of nF
 * faces and V vertices with the context's current options (host only, nothing is launched; other
 * exponents take the row-only kernel): out_host[0] = 1 if the symmetric pair kernel is taken,
 * 2 if it runs without work-group barriers, [1] = its waves per work-group (0 for the row-only kernel),
 * [2] = the bytes of its column partial sums (read back by the merge), [3] = the scratch arena the
 * call needs.  Host array of 4 int64. */
int tpe_exact_plan(tpe_ctx* ctx, int64_t nF, int64_t V, int32_t grad, int64_t* out_host);

/* With TPE_OPT_KERNEL_TIMING on: synchronise the stream, then *total_ms (host) <- summed
 * duration of the dominant-kernel launches (see TPE_OPT_KERNEL_TIMING)
 * recorded since the last call and *count (host) <- their
 * number; the record is cleared. */
int tpe_kernel_time(tpe_ctx* ctx, double* total_ms, int64_t* count);

/* *out_host (host int64) <- number of ordered face pairs (S, T) that share no vertex, i.e. the
 * number of pair interactions one evaluation performs.  Synchronises the stream. */
int tpe_pair_count(tpe_ctx* ctx, const int32_t* F, int64_t nF, int64_t V, int64_t* out_host);

#ifdef __cplusplus
}
#endif

#endif /* TPE_H */
