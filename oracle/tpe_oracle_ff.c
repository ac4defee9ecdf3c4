/*
 * FP64 CPU oracle for the cluster approximations of the tangent-point energy's derivative.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may link, load or call this
 * file: tests compare the HIP far-field kernels against it.  It shares no code, header, table or
 * helper with the HIP library (nor with tpe_oracle.c: its pair kernel and chain rule are written
 * again here, in the per-face form of eq. (dTP_reordered), so that theta = 0 checked against
 * tpeo_gradient compares two independent organisations of the same derivative).
 *
 * What it computes (paper Sec. 3.2, "Assembly of the nonlocal operator"):
 *
 *   eq. (dTP_reordered) writes the derivative as an outer integral over x of three inner
 *   integrals f_K(x), f_nu(x), f(x) over y.  For flat triangles with one quadrature point per face
 *   (centroid c, area a, unit normal n) and k(d; n) = |n.d|^q / |d|^p the inner integrals of the
 *   outer face S are
 *       K_S  = sum_T a_T (k(c_S - c_T; n_S) + k(c_T - c_S; n_T))                 (f_K)
 *       Vn_S = sum_T a_T dk/dn (c_S - c_T; n_S)                                  (f_nu)
 *       Vc_S = sum_T a_T (dk/dd (c_S - c_T; n_S) - dk/dd (c_T - c_S; n_T))        (f)
 *   over the faces T sharing no vertex with S, and
 *       E = scale/2 sum_S a_S K_S,   dE/da_S = scale K_S,   dE/dn_S = scale a_S Vn_S,
 *       dE/dc_S = scale a_S Vc_S,
 *   which the chain rule through a, n and c (a = |w|/2, n = w/|w|, w = (x_j-x_i) x (x_k-x_i),
 *   c = (x_i+x_j+x_k)/3) takes to the vertices.  The paper clusters only these inner integrals:
 *   a patch B of faces that is far from the outer point contributes through precomputed averages,
 *   and nothing is propagated back to the patch.
 *
 *   Readings of what the paper leaves open (the paper defers the admissibility rule to other work):
 *   - Tree: an implicit complete binary tree (node k has children 2k, 2k+1, leaves 2^H..) over
 *     leaves of `leaf` consecutive faces in k-d order: level by level, the faces of every node are
 *     stably sorted by their FP32 centroid coordinate along the longest axis of the node's FP32
 *     centroid box, quantised to min(16, 32 - level) bits; the first child takes the first half of
 *     the node's capacity.  (tpeo_kd_order.)
 *   - Patch averages (monopole): area A_B = sum a, centroid C_B = sum a c / A_B, normal sum
 *     N_B = sum a n; the patch acts as one face (C_B, A_B, N_B/|N_B|) -- the outer face's own n_S
 *     in the forward terms, N_B/|N_B| in the reverse ones.
 *   - Radius r_B: at a leaf the largest distance from C_B to a vertex of its faces, above a leaf
 *     max over the two children of |C_child - C_B| + r_child.
 *   - Admissibility, per target block of 64 consecutive faces in tree order with ball (C_T, r_T)
 *     (C_T the mean of the block's centroids, r_T the largest distance from C_T to a vertex of its
 *     faces): B is far when 2 r_B < theta (|C_T - C_B| - r_T).  Far: monopole for every face of the
 *     block.  Not far: a leaf is summed exactly, face by face; other nodes are opened.
 *   - The test is an integer decision taken in the kernels' precision: in FP32, on the mesh scaled
 *     by the power of two 2^k that brings the largest extent of the FP32 centroid box into
 *     [0.5, 1), with centres taken relative to the centre of that box (in the scaled frame) and
 *     rounded to FP32, and radii r + 1e-6 (1 + |C|_1) (C relative) rounded up to FP32
 *     (the slack covers the FP32 rounding of the centres, so the radii stay bounds), and
 *     dist = sqrt(fma(dz, dz, fma(dy, dy, dx dx))).  The pair sums themselves are FP64.
 *
 *   Learned-correction samples (tpeo_farfield_samples): for a (face S, far cluster B) pair the
 *   features in the frame e1 = (c_S - C_B)/rho, e2 = unit part of n_S orthogonal to e1,
 *   e3 = e1 x e2, and the targets (exact sum over B's faces minus the monopole) of K, Vn/q and Vc in
 *   the units A_B rho^-6 (K, Vn/q) and A_B rho^-7 (Vc).  Selection: cluster B (at most
 *   max_faces faces) of target block b is taken when
 *       fmix32(fmix32(fmix32(s32) ^ b) ^ B) <= floor(select_prob 2^32),  s32 = seed ^ (seed >> 32),
 *   fmix32 being MurmurHash3's 32-bit finaliser (published by Austin Appleby).
 *
 *   Curved cubic elements (tpeo_kd_order_p3, tpeo_farfield_p3, tpeo_farfield_coverage_p3): the same
 *   scheme over the quadrature records of the elements (see the section of that name below).
 *
 *   Dual tree (tpeo_farfield_dual; both integrals clustered, the scheme the paper compares with):
 *   level by level, the candidates of node A are the children of its parent's near list (the
 *   root is its own only near node); B is far from A when 2 max(r_A, r_B) < theta |C_A - C_B|
 *   (FP32 as above, times (1 - 1e-5f)), else near.  Dual leaves are the nodes of 64 faces.
 *       E = scale ( sum_{far (A,B)} A_A A_B k(C_A - C_B; nu_A)
 *                 + sum_{dual leaf A, B near A} sum_{S in A, T in B, no shared vertex} a_S a_T k(c_S - c_T; n_S) )
 *   and the gradient is the derivative of this E, obtained here by the complex-step method
 *   (E evaluated at X + i h e_vd; dE/dx_vd = Im E / h, exact to rounding for this analytic E,
 *   with the lists held fixed).
 *
 * Return codes: 0 ok, -1 invalid argument, -2 degenerate face, -3 non-finite.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FF_OK 0
#define FF_EINVAL -1
#define FF_EDEGEN -2
#define FF_ENONFIN -3
#define BLOCK 64
#define DUAL_SPAN 64

/* ---- geometry --------------------------------------------------------------------------------- */

typedef struct { double a, wn, n[3], c[3]; } fface;

static int ff_face(const double* X, const int32_t* F, int64_t f, fface* g) {
    const double* x0 = X + 3 * (int64_t)F[3 * f];
    const double* x1 = X + 3 * (int64_t)F[3 * f + 1];
    const double* x2 = X + 3 * (int64_t)F[3 * f + 2];
    const double e1[3] = {x1[0] - x0[0], x1[1] - x0[1], x1[2] - x0[2]};
    const double e2[3] = {x2[0] - x0[0], x2[1] - x0[1], x2[2] - x0[2]};
    const double w[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    g->wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    g->a = 0.5 * g->wn;
    if (!(g->a > 1e-300)) return FF_EDEGEN;
    for (int d = 0; d < 3; ++d) {
        g->n[d] = w[d] / g->wn;
        g->c[d] = (x0[d] + x1[d] + x2[d]) / 3.0;
    }
    return FF_OK;
}

static int shares_vertex(const int32_t* F, int64_t s, int64_t t) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (F[3 * s + i] == F[3 * t + j]) return 1;
    return 0;
}

static int check_mesh(const double* X, int64_t V, const int32_t* F, int64_t nF) {
    if (!X || !F || V <= 0 || nF <= 0) return FF_EINVAL;
    for (int64_t i = 0; i < 3 * nF; ++i)
        if (F[i] < 0 || F[i] >= V) return FF_EINVAL;
    for (int64_t i = 0; i < 3 * V; ++i)
        if (!isfinite(X[i])) return FF_ENONFIN;
    return FF_OK;
}

static double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

/* The kernel k(d; n) = |n.d|^q |d|^-p and its partial derivatives (q, p > 0):
 *   dk/dd = q |u|^(q-2) u |d|^-p n - p |u|^q |d|^-(p+2) d,   dk/dn = q |u|^(q-2) u |d|^-p d. */
typedef struct { double k, dd[3], dn[3]; } kval;

static int kernel_eval(const double* d, const double* n, double q, double p, kval* o) {
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(r2 > 0.0)) return FF_ENONFIN;
    const double u = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
    const double au = fabs(u);
    const double rmp = pow(r2, -0.5 * p);
    const double auq = (q == floor(q) && q <= 16.0) ? ipow(au, (int)q) : pow(au, q);
    const double uq1 = (q == floor(q) && q <= 18.0) ? ipow(au, (int)q - 2) * u : pow(au, q - 2.0) * u;
    o->k = auq * rmp;
    for (int i = 0; i < 3; ++i) {
        o->dd[i] = q * uq1 * rmp * n[i] - p * auq * rmp / r2 * d[i];
        o->dn[i] = q * uq1 * rmp * d[i];
    }
    return FF_OK;
}

/* Inner integrals of one outer face S (see the top of the file). */
typedef struct { double K, Vn[3], Vc[3]; } inner_t;

/* Adds the contribution of a face (or pseudo-face) T = (cT, aT, nT) to S's inner integrals. */
static int add_inner(const fface* S, const double* cT, double aT, const double* nT, double q, double p,
                     inner_t* in) {
    double d[3] = {S->c[0] - cT[0], S->c[1] - cT[1], S->c[2] - cT[2]};
    double md[3] = {-d[0], -d[1], -d[2]};
    kval f, r;
    if (kernel_eval(d, S->n, q, p, &f) || kernel_eval(md, nT, q, p, &r)) return FF_ENONFIN;
    in->K += aT * (f.k + r.k);
    for (int i = 0; i < 3; ++i) {
        in->Vn[i] += aT * f.dn[i];
        in->Vc[i] += aT * (f.dd[i] - r.dd[i]);
    }
    return FF_OK;
}

/* Chain rule of one face's (dE/da, dE/dn, dE/dc) to its three vertices; G [V][3]. */
static void face_to_vertices(const double* X, const int32_t* F, int64_t f, const fface* g, double dEda,
                             const double* dEdn, const double* dEdc, double* G) {
    /* g_w = dE/da n / 2 + (I - n n^T) dE/dn / |w|;  dE/dx_i += dE/dc / 3 + (x_j - x_k) x g_w (cyclic) */
    const double nd = g->n[0] * dEdn[0] + g->n[1] * dEdn[1] + g->n[2] * dEdn[2];
    double gw[3];
    for (int d = 0; d < 3; ++d) gw[d] = 0.5 * dEda * g->n[d] + (dEdn[d] - nd * g->n[d]) / g->wn;
    for (int c = 0; c < 3; ++c) {
        const double* xj = X + 3 * (int64_t)F[3 * f + (c + 1) % 3];
        const double* xk = X + 3 * (int64_t)F[3 * f + (c + 2) % 3];
        const double e[3] = {xj[0] - xk[0], xj[1] - xk[1], xj[2] - xk[2]};
        const double cr[3] = {e[1] * gw[2] - e[2] * gw[1], e[2] * gw[0] - e[0] * gw[2], e[0] * gw[1] - e[1] * gw[0]};
        double* o = G + 3 * (int64_t)F[3 * f + c];
        for (int d = 0; d < 3; ++d) o[d] += dEdc[d] / 3.0 + cr[d];
    }
}

/* ---- the FP32 frame of the admissibility decisions ---------------------------------------------- */

/* FP32 centroid of face f as the kernels form it: the FP64 mean of its corners, rounded.  F holds
 * `stride` node ids per face, the three corners first (3 for flat faces, 10 for curved elements). */
static int centroid_f32(const double* X, int64_t V, const int32_t* F, int stride, int64_t f, float* c) {
    const int32_t a = F[stride * f], b = F[stride * f + 1], e = F[stride * f + 2];
    c[0] = c[1] = c[2] = 0.f;
    if (a < 0 || a >= V || b < 0 || b >= V || e < 0 || e >= V) return 0;
    double x[3];
    for (int d = 0; d < 3; ++d) x[d] = (X[3 * (int64_t)a + d] + X[3 * (int64_t)b + d] + X[3 * (int64_t)e + d]) / 3.0;
    if (!isfinite(x[0] + x[1] + x[2])) return 0;
    for (int d = 0; d < 3; ++d) c[d] = (float)x[d];
    return 1;
}

/* s = 2^k with (largest extent of the FP32 centroid box) * s in [0.5, 1) (1 for an empty box), and
 * the box's centre in the scaled frame (the origin of the decisions' FP32 centres). */
static double frame_scale(const double* X, int64_t V, const int32_t* F, int stride, int64_t nF, double* origin) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t f = 0; f < nF; ++f) {
        float c[3];
        if (!centroid_f32(X, V, F, stride, f, c)) continue;
        for (int d = 0; d < 3; ++d) {
            if (c[d] < lo[d]) lo[d] = c[d];
            if (c[d] > hi[d]) hi[d] = c[d];
        }
    }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double e = (double)hi[d] - (double)lo[d];
        if (e > ext && isfinite(e)) ext = e;
    }
    double s = 1.0;
    if (ext > 0.0 && isfinite(ext)) {
        int ex;
        (void)frexp(ext, &ex);
        s = ldexp(1.0, -ex);
    }
    for (int d = 0; d < 3; ++d)
        origin[d] = lo[d] <= hi[d] ? s * (0.5 * ((double)lo[d] + (double)hi[d])) : 0.0;
    return s;
}

static float round_up_f32(double v) {
    float f = (float)v;
    return (double)f >= v ? f : nextafterf(f, INFINITY);
}

/* FP32 ball (centre relative to the origin o, bounding radius) in the scaled frame, of a centre C and
 * radius r given in the original frame. */
static void ball_f32(const double* C, double r, double s, const double* o, float* out) {
    const double sc[3] = {s * C[0] - o[0], s * C[1] - o[1], s * C[2] - o[2]};
    const double slack = 1e-6 * (1.0 + fabs(sc[0]) + fabs(sc[1]) + fabs(sc[2]));
    for (int d = 0; d < 3; ++d) out[d] = (float)sc[d];
    out[3] = round_up_f32(s * r + slack);
}

static float dist_f32(const float* a, const float* b) {
    const float dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
}

/* ---- k-d order ---------------------------------------------------------------------------------- */

static int height_of(int64_t n, int leaf) {
    const int64_t nleaf = (n + leaf - 1) / leaf;
    int H = 0;
    while (((int64_t)1 << H) < nleaf) ++H;
    return H;
}

typedef struct { uint32_t key; int64_t pos; uint32_t val; } kd_item;

static int kd_cmp(const void* x, const void* y) {
    const kd_item* a = (const kd_item*)x;
    const kd_item* b = (const kd_item*)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->pos < b->pos ? -1 : (a->pos > b->pos);  /* stable */
}

/* The k-d order of nF items at the FP32 positions cen (see the top of the file). */
static int kd_core(float (*cen)[3], int64_t nF, int leaf, uint32_t* perm) {
    const int H = height_of(nF, leaf);
    kd_item* it = malloc(sizeof(kd_item) * (size_t)nF);
    if (!it) return FF_EINVAL;
    for (int64_t f = 0; f < nF; ++f) perm[f] = (uint32_t)f;
    for (int level = 0; level < H; ++level) {
        const int64_t node_faces = ((int64_t)1 << (H - level)) * leaf;
        const int qbits = 32 - level < 16 ? 32 - level : 16;
        const float maxq = (float)((1u << qbits) - 1u);
        for (int64_t j0 = 0; j0 < nF; j0 += node_faces) {
            const int64_t j1 = j0 + node_faces < nF ? j0 + node_faces : nF;
            float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int64_t i = j0; i < j1; ++i)
                for (int d = 0; d < 3; ++d) {
                    const float v = cen[perm[i]][d];
                    if (v < lo[d]) lo[d] = v;
                    if (v > hi[d]) hi[d] = v;
                }
            float ext[3];
            for (int d = 0; d < 3; ++d) ext[d] = hi[d] - lo[d];
            int ax = 0;
            if (ext[1] > ext[ax]) ax = 1;
            if (ext[2] > ext[ax]) ax = 2;
            for (int64_t i = j0; i < j1; ++i) {
                const float v = cen[perm[i]][ax];
                float s = ext[ax] > 0.f ? (v - lo[ax]) / ext[ax] * maxq : 0.f;
                s = fminf(fmaxf(s, 0.f), maxq);
                const uint32_t qv = isfinite(s) ? (uint32_t)s : 0u;
                it[i].key = ((uint32_t)(j0 / node_faces) << qbits) | qv;
                it[i].pos = i;
                it[i].val = perm[i];
            }
        }
        qsort(it, (size_t)nF, sizeof(kd_item), kd_cmp);
        for (int64_t i = 0; i < nF; ++i) perm[i] = it[i].val;
    }
    free(it);
    return FF_OK;
}

int tpeo_kd_order(const double* X, int64_t V, const int32_t* F, int64_t nF, int leaf, uint32_t* perm) {
    if (!X || !F || !perm || V <= 0 || nF <= 0 || leaf < 1) return FF_EINVAL;
    float (*cen)[3] = malloc(sizeof(float[3]) * (size_t)nF);
    if (!cen) return FF_EINVAL;
    for (int64_t f = 0; f < nF; ++f) (void)centroid_f32(X, V, F, 3, f, cen[f]);
    const int rc = kd_core(cen, nF, leaf, perm);
    free(cen);
    return rc;
}

/* ---- tree nodes (FP64 patch averages) ------------------------------------------------------------ */

typedef struct {
    double A, C[3], N[3], r;
    double m2c[6], m2n[6]; /* sum a (c - C)(c - C)^T and sum a n n^T: xx xy xz yy yz zz */
    float rec[4];          /* FP32 decision ball (centre, radius) in the scaled frame */
    float af;              /* FP32 area in the scaled frame (a node is used when it is > 0) */
} fnode;

/* A curved element's quadrature record: its tangents x_s, x_t, |J|, rule weight W and point l. */
typedef struct { double xs[3], xt[3], Jn, W, l[3]; } p3aux;

typedef struct {
    int64_t nF, V;  /* nF: the items of the tree -- faces, or the quadrature records of curved elements */
    int leaf, H;
    double s, o[3]; /* scale and origin of the FP32 decision frame */
    const double* X;
    const int32_t* F;     /* node ids, cstride per face or element, its three corners first */
    int cstride, Q;       /* item r belongs to face or element r / Q (Q = 1 for flat faces) */
    const uint32_t* perm; /* tree position -> item */
    fface* g;             /* item geometry by tree position (c, n, a: point, normal, weight) */
    fnode* nodes;         /* 2^(H+1) entries, 1-based heap numbering */
} ftree;

/* The three corner nodes of the face or element holding the item at tree position i. */
static const int32_t* corners_at(const ftree* t, int64_t i) {
    return t->F + (int64_t)t->cstride * (int64_t)(t->perm[i] / (uint32_t)t->Q);
}

/* Excluded pairs: items whose faces (elements) share a corner node -- the same face included. */
static int items_share_corner(const ftree* t, int64_t i, int64_t j) {
    const int32_t* a = corners_at(t, i);
    const int32_t* b = corners_at(t, j);
    for (int u = 0; u < 3; ++u)
        for (int v = 0; v < 3; ++v)
            if (a[u] == b[v]) return 1;
    return 0;
}

static void outer_add(double* m, double w, const double* v) {
    m[0] += w * v[0] * v[0]; m[1] += w * v[0] * v[1]; m[2] += w * v[0] * v[2];
    m[3] += w * v[1] * v[1]; m[4] += w * v[1] * v[2]; m[5] += w * v[2] * v[2];
}

static void node_decision(fnode* n, double s, const double* o) {
    if (n->A > 0.0) {
        ball_f32(n->C, n->r, s, o, n->rec);
        n->af = (float)(s * s * n->A);
    } else {
        n->rec[0] = n->rec[1] = n->rec[2] = n->rec[3] = 0.f;
        n->af = 0.f;
    }
}

/* Positions [p0, p1) of the faces under node k. */
static void node_range(const ftree* t, int64_t k, int64_t* p0, int64_t* p1) {
    int lev = 0;
    while (((int64_t)2 << lev) <= k) ++lev;
    const int64_t span = ((int64_t)1 << (t->H - lev)) * t->leaf;
    *p0 = (k - ((int64_t)1 << lev)) * span;
    *p1 = *p0 + span < t->nF ? *p0 + span : t->nF;
    if (*p0 > t->nF) *p0 = t->nF;
}

/* The tree over n = nE Q items whose geometry (in item order) is `items`: FP32 frame from the
 * corner centroids of the nE faces or elements, leaves of `leaf` consecutive tree positions, and the
 * patch averages bottom-up.  Radii bound the corner nodes of the items' faces or elements. */
static int tree_build_items(ftree* t, const double* X, int64_t V, const int32_t* F, int cstride, int Q, int64_t nE,
                            const fface* items, const uint32_t* perm, int leaf) {
    const int64_t nF = nE * Q;
    t->nF = nF; t->V = V; t->leaf = leaf; t->X = X; t->F = F; t->cstride = cstride; t->Q = Q; t->perm = perm;
    t->H = height_of(nF, leaf);
    t->s = frame_scale(X, V, F, cstride, nE, t->o);
    t->g = malloc(sizeof(fface) * (size_t)nF);
    t->nodes = calloc((size_t)2 << t->H, sizeof(fnode));
    if (!t->g || !t->nodes) return FF_EINVAL;
    char* seen = calloc((size_t)nF, 1);
    if (!seen) return FF_EINVAL;
    for (int64_t i = 0; i < nF; ++i) {
        if (perm[i] >= (uint32_t)nF || seen[perm[i]]) { free(seen); return FF_EINVAL; }
        seen[perm[i]] = 1;
        t->g[i] = items[perm[i]];
    }
    free(seen);
    const int64_t nslot = (int64_t)1 << t->H;
    for (int64_t j = 0; j < nslot; ++j) {
        fnode* n = &t->nodes[nslot + j];
        const int64_t f0 = j * leaf, f1 = f0 + leaf < nF ? f0 + leaf : nF;
        double sc[3] = {0, 0, 0};
        for (int64_t i = f0; i < f1; ++i) {
            const fface* g = &t->g[i];
            n->A += g->a;
            for (int d = 0; d < 3; ++d) { sc[d] += g->a * g->c[d]; n->N[d] += g->a * g->n[d]; }
        }
        if (n->A > 0.0) {
            for (int d = 0; d < 3; ++d) n->C[d] = sc[d] / n->A;
            for (int64_t i = f0; i < f1; ++i) {
                const fface* g = &t->g[i];
                const double dc[3] = {g->c[0] - n->C[0], g->c[1] - n->C[1], g->c[2] - n->C[2]};
                outer_add(n->m2c, g->a, dc);
                outer_add(n->m2n, g->a, g->n);
                const int32_t* cn = corners_at(t, i);
                for (int k = 0; k < 3; ++k) {
                    const double* x = X + 3 * (int64_t)cn[k];
                    const double dv[3] = {x[0] - n->C[0], x[1] - n->C[1], x[2] - n->C[2]};
                    const double r = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
                    if (r > n->r) n->r = r;
                }
            }
        }
        node_decision(n, t->s, t->o);
    }
    for (int64_t k = nslot - 1; k >= 1; --k) {
        fnode* n = &t->nodes[k];
        const fnode* ch[2] = {&t->nodes[2 * k], &t->nodes[2 * k + 1]};
        n->A = ch[0]->A + ch[1]->A;
        if (n->A > 0.0) {
            for (int d = 0; d < 3; ++d) {
                n->C[d] = (ch[0]->A * ch[0]->C[d] + ch[1]->A * ch[1]->C[d]) / n->A;
                n->N[d] = ch[0]->N[d] + ch[1]->N[d];
            }
            for (int c = 0; c < 2; ++c) {
                if (!(ch[c]->A > 0.0)) continue;
                const double dc[3] = {ch[c]->C[0] - n->C[0], ch[c]->C[1] - n->C[1], ch[c]->C[2] - n->C[2]};
                const double r = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]) + ch[c]->r;
                if (r > n->r) n->r = r;
                for (int m = 0; m < 6; ++m) { n->m2c[m] += ch[c]->m2c[m]; n->m2n[m] += ch[c]->m2n[m]; }
                outer_add(n->m2c, ch[c]->A, dc); /* parallel-axis shift */
            }
        }
        node_decision(n, t->s, t->o);
    }
    return FF_OK;
}

/* The tree over the flat faces of (X, F). */
static int tree_build(ftree* t, const double* X, int64_t V, const int32_t* F, int64_t nF, const uint32_t* perm,
                      int leaf) {
    memset(t, 0, sizeof(*t));
    int rc = check_mesh(X, V, F, nF);
    if (rc) return rc;
    if (!perm || leaf < 1) return FF_EINVAL;
    fface* items = malloc(sizeof(fface) * (size_t)nF);
    if (!items) return FF_EINVAL;
    for (int64_t f = 0; f < nF; ++f)
        if ((rc = ff_face(X, F, f, &items[f]))) { free(items); return rc; }
    rc = tree_build_items(t, X, V, F, 3, 1, nF, items, perm, leaf);
    free(items);
    return rc;
}

static void tree_free(ftree* t) {
    free(t->g);
    free(t->nodes);
}

/* Ball of target block b (positions [64 b, min(64 b + 64, nF))), FP32 as the decisions use it. */
static void block_ball(const ftree* t, int64_t b, float* out) {
    const int64_t i0 = b * BLOCK, i1 = i0 + BLOCK < t->nF ? i0 + BLOCK : t->nF;
    double C[3] = {0, 0, 0}, r = 0.0;
    for (int64_t i = i0; i < i1; ++i)
        for (int d = 0; d < 3; ++d) C[d] += t->g[i].c[d];
    for (int d = 0; d < 3; ++d) C[d] /= (double)(i1 - i0);
    for (int64_t i = i0; i < i1; ++i)
        for (int k = 0; k < 3; ++k) {
            const double* x = t->X + 3 * (int64_t)corners_at(t, i)[k];
            const double dv[3] = {x[0] - C[0], x[1] - C[1], x[2] - C[2]};
            const double rr = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
            if (rr > r) r = rr;
        }
    ball_f32(C, r, t->s, t->o, out);
}

static int is_far(const float* tb, const fnode* n, float theta) {
    return 2.0f * n->rec[3] < theta * (dist_f32(tb, n->rec) - tb[3]);
}

/* ---- per-face clustering of the inner integrals ----------------------------------------------------- */

typedef struct { int64_t far, near_cols, visited; } walk_stats;

/* The walk of one target block: every node is tested against the block's ball; far nodes act as one
 * pseudo-face on every face of the block, near leaves are summed exactly, other nodes are opened.
 * visit(node) is called for far nodes (far = 1) and near leaves (far = 0). */
typedef int (*visit_fn)(const ftree* t, int64_t b, int64_t node, int far, void* user);

static int walk(const ftree* t, int64_t b, const float* tb, float theta, int64_t k, walk_stats* st, visit_fn fn,
                void* user) {
    st->visited += 1;
    const fnode* n = &t->nodes[k];
    if (!(n->af > 0.f)) return FF_OK;
    if (is_far(tb, n, theta)) {
        st->far += 1;
        return fn(t, b, k, 1, user);
    }
    if (k >= ((int64_t)1 << t->H)) {
        int64_t p0, p1;
        node_range(t, k, &p0, &p1);
        if (p0 < p1) st->near_cols += p1 - p0;
        return fn(t, b, k, 0, user);
    }
    int rc = walk(t, b, tb, theta, 2 * k, st, fn, user);
    if (!rc) rc = walk(t, b, tb, theta, 2 * k + 1, st, fn, user);
    return rc;
}

typedef struct { double q, p; inner_t* in; } ff_user;

static int ff_visit(const ftree* t, int64_t b, int64_t node, int far, void* user) {
    ff_user* u = (ff_user*)user;
    const int64_t i0 = b * BLOCK, i1 = i0 + BLOCK < t->nF ? i0 + BLOCK : t->nF;
    const fnode* n = &t->nodes[node];
    if (far) {
        const double nn = sqrt(n->N[0] * n->N[0] + n->N[1] * n->N[1] + n->N[2] * n->N[2]);
        const double nu[3] = {nn > 0.0 ? n->N[0] / nn : 0.0, nn > 0.0 ? n->N[1] / nn : 0.0,
                              nn > 0.0 ? n->N[2] / nn : 0.0};
        for (int64_t i = i0; i < i1; ++i)
            if (add_inner(&t->g[i], n->C, n->A, nu, u->q, u->p, &u->in[i])) return FF_ENONFIN;
        return FF_OK;
    }
    int64_t p0, p1;
    node_range(t, node, &p0, &p1);
    for (int64_t i = i0; i < i1; ++i)
        for (int64_t j = p0; j < p1; ++j) {
            if (items_share_corner(t, i, j)) continue;
            if (add_inner(&t->g[i], t->g[j].c, t->g[j].a, t->g[j].n, u->q, u->p, &u->in[i])) return FF_ENONFIN;
        }
    return FF_OK;
}

/* Barnes-Hut approximation of E and dE/dX on the tree given by perm (tree position -> face) and
 * leaf: the inner integrals clustered per target block of 64 faces (see the top of the file).
 * E_out: the energy scale/2 sum_S a_S K_S; G_out (nullable): [V][3].  stats (nullable, 6 int64):
 * far clusters and near columns summed over blocks, visited nodes, blocks, the largest per-block
 * near columns and far clusters -- each block's counts once (they apply to all of its faces). */
int tpeo_farfield(const double* X, int64_t V, const int32_t* F, int64_t nF, const uint32_t* perm, int leaf,
                  double theta, double q, double p, double scale, int nthreads, double* E_out, double* G_out,
                  int64_t* stats) {
    if (!(theta >= 0.0) || !(q >= 2.0) || !(p > q)) return FF_EINVAL;
    ftree t;
    int rc = tree_build(&t, X, V, F, nF, perm, leaf);
    if (rc) { tree_free(&t); return rc; }
    inner_t* in = calloc((size_t)nF, sizeof(inner_t));
    const int64_t nb = (nF + BLOCK - 1) / BLOCK;
    walk_stats* bs = calloc((size_t)nb, sizeof(walk_stats));
    if (!in || !bs) { free(in); free(bs); tree_free(&t); return FF_EINVAL; }
    const float th = (float)theta;
    int err = FF_OK;
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int64_t b = 0; b < nb; ++b) {
        float tb[4];
        block_ball(&t, b, tb);
        ff_user u = {q, p, in};
        if (walk(&t, b, tb, th, 1, &bs[b], ff_visit, &u)) {
#ifdef _OPENMP
#pragma omp critical
#endif
            err = FF_ENONFIN;
        }
    }
    (void)nthreads;
    if (stats) {
        for (int k = 0; k < 6; ++k) stats[k] = 0;
        for (int64_t b = 0; b < nb; ++b) {
            stats[0] += bs[b].far;
            stats[1] += bs[b].near_cols;
            stats[2] += bs[b].visited;
            stats[3] += 1;
            if (bs[b].near_cols > stats[4]) stats[4] = bs[b].near_cols;
            if (bs[b].far > stats[5]) stats[5] = bs[b].far;
        }
    }
    double E = 0.0;
    if (G_out) memset(G_out, 0, sizeof(double) * 3 * (size_t)V);
    for (int64_t i = 0; i < nF && !err; ++i) {
        const fface* g = &t.g[i];
        E += 0.5 * g->a * in[i].K;
        if (G_out) {
            double dn[3], dc[3];
            for (int d = 0; d < 3; ++d) { dn[d] = scale * g->a * in[i].Vn[d]; dc[d] = scale * g->a * in[i].Vc[d]; }
            face_to_vertices(X, F, perm[i], g, scale * in[i].K, dn, dc, G_out);
        }
    }
    if (E_out) *E_out = err ? INFINITY : scale * E;
    free(in); free(bs); tree_free(&t);
    return err;
}

/* Invariants of the walk, checked face by face: cov_visit counts how often every face is reached
 * from the block (far clusters and near leaves alike) and whether a far cluster holds a face that
 * shares a vertex with a face of the block. */
typedef struct { int32_t* seen; int64_t bad_far; } cov_user;

static int cov_visit(const ftree* t, int64_t b, int64_t node, int far, void* user) {
    cov_user* u = (cov_user*)user;
    int64_t p0, p1;
    node_range(t, node, &p0, &p1);
    const int64_t i0 = b * BLOCK, i1 = i0 + BLOCK < t->nF ? i0 + BLOCK : t->nF;
    for (int64_t j = p0; j < p1; ++j) {
        u->seen[j] += 1;
        if (far)
            for (int64_t i = i0; i < i1; ++i)
                if (items_share_corner(t, i, j)) { u->bad_far += 1; break; }
    }
    return FF_OK;
}

/* out[0] <- target blocks from which some face is not reached exactly once; out[1] <- (far
 * cluster face, block) incidences where the face shares a vertex with a face of the block. */
/* The walk's invariants on a built tree (see tpeo_farfield_coverage). */
static int coverage_of(const ftree* t, double theta, int64_t* out) {
    const int64_t nF = t->nF;
    cov_user u = {calloc((size_t)nF, sizeof(int32_t)), 0};
    if (!u.seen) return FF_EINVAL;
    out[0] = out[1] = 0;
    const int64_t nb = (nF + BLOCK - 1) / BLOCK;
    for (int64_t b = 0; b < nb; ++b) {
        float tb[4];
        block_ball(t, b, tb);
        memset(u.seen, 0, sizeof(int32_t) * (size_t)nF);
        walk_stats st = {0, 0, 0};
        walk(t, b, tb, (float)theta, 1, &st, cov_visit, &u);
        for (int64_t j = 0; j < nF; ++j)
            if (u.seen[j] != 1) { out[0] += 1; break; }
    }
    out[1] = u.bad_far;
    free(u.seen);
    return FF_OK;
}

/* out[0] <- target blocks from which some face is not reached exactly once; out[1] <- (far
 * cluster face, block) incidences where the face shares a vertex with a face of the block. */
int tpeo_farfield_coverage(const double* X, int64_t V, const int32_t* F, int64_t nF, const uint32_t* perm, int leaf,
                           double theta, int64_t* out) {
    if (!out || !(theta >= 0.0)) return FF_EINVAL;
    ftree t;
    int rc = tree_build(&t, X, V, F, nF, perm, leaf);
    if (rc) { tree_free(&t); return rc; }
    rc = coverage_of(&t, theta, out);
    tree_free(&t);
    return rc;
}

/* ---- curved cubic elements: the same scheme over quadrature records ----------------------------------
 *
 * For curved (P3) elements (ten nodes per element, the three corners first; paper Sec. 3.1 and 3.2)
 * the items of the tree are the quadrature records of every element: record r = Q e + k at the
 * point l_k of the rule (barycentric, weight W_k) on element e, with position x = x(l_k), normal
 * n = J / |J| (J = x_s x x_t) and weight alpha = W_k |J| / 2.  The tree is the k-d order of the
 * records' FP32 positions; radii, target balls and the exclusion use the elements' corner nodes
 * (records of elements sharing a corner are not paired, the element with itself included), the
 * FP32 frame comes from the elements' corner centroids, and everything else is the scheme above
 * with records in place of faces.  The inner integrals of a record reach the nodes by the chain
 * rule through the record: with g = dE/dalpha = scale K, gn = dE/dn = scale alpha Vn and
 * gx = dE/dx = scale alpha Vc, gJ = g (W/2) n + (I - n n^T) gn / |J|, and node k of the element
 * receives phi_k gx + (dphi_k/ds) (x_t x gJ) + (dphi_k/dt) (gJ x x_s).  The basis is
 * tpeo_p3_basis of tpe_oracle.c (pinned there by cubic reproduction and straight elements). */

int tpeo_p3_basis(const double* l, double* phi, double* ds, double* dt);

static int check_p3(const double* X, int64_t V, const int32_t* F10, int64_t nE, int nq) {
    if (!X || !F10 || V <= 0 || nE <= 0 || nq < 1 || nq > 6) return FF_EINVAL;
    for (int64_t i = 0; i < 10 * nE; ++i)
        if (F10[i] < 0 || F10[i] >= V) return FF_EINVAL;
    for (int64_t i = 0; i < 3 * V; ++i)
        if (!isfinite(X[i])) return FF_ENONFIN;
    return FF_OK;
}

/* x, x_s, x_t of element e at barycentric l */
static void p3_point(const double* X, const int32_t* F10, int64_t e, const double* l, double* x, double* xs,
                     double* xt) {
    double phi[10], ds[10], dt[10];
    tpeo_p3_basis(l, phi, ds, dt);
    for (int d = 0; d < 3; ++d) x[d] = xs[d] = xt[d] = 0.0;
    for (int k = 0; k < 10; ++k) {
        const double* xk = X + 3 * (int64_t)F10[10 * e + k];
        for (int d = 0; d < 3; ++d) {
            x[d] += phi[k] * xk[d];
            xs[d] += ds[k] * xk[d];
            xt[d] += dt[k] * xk[d];
        }
    }
}

/* The records (item order) of every element under the rule (bary[nq][3], w[nq]). */
static int p3_records_of(const double* X, const int32_t* F10, int64_t nE, const double* bary, const double* w,
                         int nq, fface* items, p3aux* aux) {
    for (int64_t e = 0; e < nE; ++e)
        for (int k = 0; k < nq; ++k) {
            const int64_t r = (int64_t)nq * e + k;
            fface* g = &items[r];
            p3aux* x = &aux[r];
            for (int d = 0; d < 3; ++d) x->l[d] = bary[3 * k + d];
            p3_point(X, F10, e, x->l, g->c, x->xs, x->xt);
            const double J[3] = {x->xs[1] * x->xt[2] - x->xs[2] * x->xt[1], x->xs[2] * x->xt[0] - x->xs[0] * x->xt[2],
                                 x->xs[0] * x->xt[1] - x->xs[1] * x->xt[0]};
            x->Jn = sqrt(J[0] * J[0] + J[1] * J[1] + J[2] * J[2]);
            if (!(x->Jn > 1e-300)) return FF_EDEGEN;
            x->W = w[k];
            g->wn = x->Jn;
            g->a = 0.5 * w[k] * x->Jn;
            for (int d = 0; d < 3; ++d) g->n[d] = J[d] / x->Jn;
        }
    return FF_OK;
}

/* The k-d order of the nE nq records (item r = nq e + k at the rule's point k of element e). */
int tpeo_kd_order_p3(const double* X, int64_t V, const int32_t* F10, int64_t nE, const double* bary, int nq,
                     int leaf, uint32_t* perm) {
    int rc = check_p3(X, V, F10, nE, nq);
    if (rc) return rc;
    if (!bary || !perm || leaf < 1) return FF_EINVAL;
    const int64_t n = nE * nq;
    float (*cen)[3] = malloc(sizeof(float[3]) * (size_t)n);
    if (!cen) return FF_EINVAL;
    for (int64_t e = 0; e < nE; ++e)
        for (int k = 0; k < nq; ++k) {
            double x[3], xs[3], xt[3];
            p3_point(X, F10, e, bary + 3 * k, x, xs, xt);
            for (int d = 0; d < 3; ++d) cen[(int64_t)nq * e + k][d] = (float)x[d];
        }
    rc = kd_core(cen, n, leaf, perm);
    free(cen);
    return rc;
}

static int tree_build_p3(ftree* t, const double* X, int64_t V, const int32_t* F10, int64_t nE, const double* bary,
                         const double* w, int nq, const uint32_t* perm, int leaf, p3aux** aux_out) {
    memset(t, 0, sizeof(*t));
    *aux_out = NULL;
    int rc = check_p3(X, V, F10, nE, nq);
    if (rc) return rc;
    if (!bary || !w || !perm || leaf < 1) return FF_EINVAL;
    const int64_t n = nE * nq;
    fface* items = malloc(sizeof(fface) * (size_t)n);
    p3aux* aux = malloc(sizeof(p3aux) * (size_t)n);
    if (!items || !aux) { free(items); free(aux); return FF_EINVAL; }
    rc = p3_records_of(X, F10, nE, bary, w, nq, items, aux);
    if (!rc) rc = tree_build_items(t, X, V, F10, 10, nq, nE, items, perm, leaf);
    free(items);
    if (rc) { free(aux); return rc; }
    *aux_out = aux;
    return FF_OK;
}

/* Barnes-Hut approximation of E and dE/dX on curved elements (X [V][3], F10 [nE][10]), the rule
 * (bary [nq][3], w [nq]) and the tree perm over its records (tpeo_kd_order_p3).  Outputs as for
 * tpeo_farfield; G_out [V][3]. */
int tpeo_farfield_p3(const double* X, int64_t V, const int32_t* F10, int64_t nE, const double* bary, const double* w,
                     int nq, const uint32_t* perm, int leaf, double theta, double q, double p, double scale,
                     int nthreads, double* E_out, double* G_out, int64_t* stats) {
    if (!(theta >= 0.0) || !(q >= 2.0) || !(p > q)) return FF_EINVAL;
    ftree t;
    p3aux* aux = NULL;
    int rc = tree_build_p3(&t, X, V, F10, nE, bary, w, nq, perm, leaf, &aux);
    if (rc) { tree_free(&t); return rc; }
    const int64_t n = t.nF;
    inner_t* in = calloc((size_t)n, sizeof(inner_t));
    const int64_t nb = (n + BLOCK - 1) / BLOCK;
    walk_stats* bs = calloc((size_t)nb, sizeof(walk_stats));
    if (!in || !bs) { free(in); free(bs); free(aux); tree_free(&t); return FF_EINVAL; }
    const float th = (float)theta;
    int err = FF_OK;
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int64_t b = 0; b < nb; ++b) {
        float tb[4];
        block_ball(&t, b, tb);
        ff_user u = {q, p, in};
        if (walk(&t, b, tb, th, 1, &bs[b], ff_visit, &u)) {
#ifdef _OPENMP
#pragma omp critical
#endif
            err = FF_ENONFIN;
        }
    }
    (void)nthreads;
    if (stats) {
        for (int k = 0; k < 6; ++k) stats[k] = 0;
        for (int64_t b = 0; b < nb; ++b) {
            stats[0] += bs[b].far;
            stats[1] += bs[b].near_cols;
            stats[2] += bs[b].visited;
            stats[3] += 1;
            if (bs[b].near_cols > stats[4]) stats[4] = bs[b].near_cols;
            if (bs[b].far > stats[5]) stats[5] = bs[b].far;
        }
    }
    double E = 0.0;
    if (G_out) memset(G_out, 0, sizeof(double) * 3 * (size_t)V);
    for (int64_t i = 0; i < n && !err; ++i) {
        const fface* g = &t.g[i];
        E += 0.5 * g->a * in[i].K;
        if (!G_out) continue;
        const int64_t r = perm[i], e = r / nq;
        const p3aux* x = &aux[r];
        double gn[3], gx[3], gJ[3], cs[3], ct[3];
        const double ga = scale * in[i].K;
        for (int d = 0; d < 3; ++d) { gn[d] = scale * g->a * in[i].Vn[d]; gx[d] = scale * g->a * in[i].Vc[d]; }
        const double ngn = g->n[0] * gn[0] + g->n[1] * gn[1] + g->n[2] * gn[2];
        for (int d = 0; d < 3; ++d) gJ[d] = ga * 0.5 * x->W * g->n[d] + (gn[d] - ngn * g->n[d]) / x->Jn;
        /* x_t x gJ (the direction of d/dx_s) and gJ x x_s (that of d/dx_t) */
        cs[0] = x->xt[1] * gJ[2] - x->xt[2] * gJ[1]; cs[1] = x->xt[2] * gJ[0] - x->xt[0] * gJ[2];
        cs[2] = x->xt[0] * gJ[1] - x->xt[1] * gJ[0];
        ct[0] = gJ[1] * x->xs[2] - gJ[2] * x->xs[1]; ct[1] = gJ[2] * x->xs[0] - gJ[0] * x->xs[2];
        ct[2] = gJ[0] * x->xs[1] - gJ[1] * x->xs[0];
        double phi[10], ds[10], dt[10];
        tpeo_p3_basis(x->l, phi, ds, dt);
        for (int k = 0; k < 10; ++k) {
            double* o = G_out + 3 * (int64_t)F10[10 * e + k];
            for (int d = 0; d < 3; ++d) o[d] += phi[k] * gx[d] + ds[k] * cs[d] + dt[k] * ct[d];
        }
    }
    if (E_out) *E_out = err ? INFINITY : scale * E;
    free(in); free(bs); free(aux); tree_free(&t);
    return err;
}

/* tpeo_farfield_coverage on the records of curved elements. */
int tpeo_farfield_coverage_p3(const double* X, int64_t V, const int32_t* F10, int64_t nE, const double* bary,
                              const double* w, int nq, const uint32_t* perm, int leaf, double theta, int64_t* out) {
    if (!out || !(theta >= 0.0)) return FF_EINVAL;
    ftree t;
    p3aux* aux = NULL;
    int rc = tree_build_p3(&t, X, V, F10, nE, bary, w, nq, perm, leaf, &aux);
    free(aux);
    if (rc) { tree_free(&t); return rc; }
    rc = coverage_of(&t, theta, out);
    tree_free(&t);
    return rc;
}

/* ---- learned-correction samples ---------------------------------------------------------------------- */

static uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

uint32_t tpeo_sample_hash(uint64_t seed, uint32_t block, uint32_t node) {
    const uint32_t s32 = (uint32_t)(seed ^ (seed >> 32));
    return fmix32(fmix32(fmix32(s32) ^ block) ^ node);
}

/* quadratic form e_a^T M e_b of a symmetric M (xx xy xz yy yz zz) */
static double qform(const double* M, const double* ea, const double* eb) {
    const double Me[3] = {M[0] * eb[0] + M[1] * eb[1] + M[2] * eb[2], M[1] * eb[0] + M[3] * eb[1] + M[4] * eb[2],
                          M[2] * eb[0] + M[4] * eb[1] + M[5] * eb[2]};
    return ea[0] * Me[0] + ea[1] * Me[1] + ea[2] * Me[2];
}

typedef struct {
    double sel_thr;
    uint64_t seed;
    int64_t max_faces, cap, count;
    double q, p;
    int32_t* out_block;
    int32_t* out_node;
    double* feats;   /* [cap][64][19] */
    double* targets; /* [cap][64][8]: 7 targets, weight */
} smp_user;

static int smp_visit(const ftree* t, int64_t b, int64_t node, int far, void* user) {
    smp_user* u = (smp_user*)user;
    if (!far) return FF_OK;
    int64_t p0, p1;
    node_range(t, node, &p0, &p1);
    if (p1 - p0 > u->max_faces) return FF_OK;
    if ((double)tpeo_sample_hash(u->seed, (uint32_t)b, (uint32_t)node) > u->sel_thr) return FF_OK;
    int64_t slot;
#ifdef _OPENMP
#pragma omp atomic capture
#endif
    slot = u->count++;
    if (slot >= u->cap) return FF_OK; /* counted: the caller sees the overflow */
    u->out_block[slot] = (int32_t)b;
    u->out_node[slot] = (int32_t)node;
    const fnode* n = &t->nodes[node];
    const double nn = sqrt(n->N[0] * n->N[0] + n->N[1] * n->N[1] + n->N[2] * n->N[2]);
    const double nu[3] = {n->N[0] / nn, n->N[1] / nn, n->N[2] / nn};
    /* the radius the kernels see: the FP32 decision radius, back in the original frame */
    const double rB = (double)n->rec[3] / t->s;
    const double m2c[6] = {n->m2c[0] / n->A, n->m2c[1] / n->A, n->m2c[2] / n->A,
                           n->m2c[3] / n->A, n->m2c[4] / n->A, n->m2c[5] / n->A};
    const double m2n[6] = {n->m2n[0] / n->A, n->m2n[1] / n->A, n->m2n[2] / n->A,
                           n->m2n[3] / n->A, n->m2n[4] / n->A, n->m2n[5] / n->A};
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int lane = 0; lane < BLOCK; ++lane) {
        double* x = u->feats + ((size_t)slot * BLOCK + lane) * 19;
        double* y = u->targets + ((size_t)slot * BLOCK + lane) * 8;
        memset(x, 0, sizeof(double) * 19);
        memset(y, 0, sizeof(double) * 8);
        const int64_t i = b * BLOCK + lane;
        if (i >= t->nF) continue;
        const fface* S = &t->g[i];
        const double D[3] = {S->c[0] - n->C[0], S->c[1] - n->C[1], S->c[2] - n->C[2]};
        const double rho = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        double e[3][3];
        for (int d = 0; d < 3; ++d) e[0][d] = D[d] / rho;
        const double c1 = S->n[0] * e[0][0] + S->n[1] * e[0][1] + S->n[2] * e[0][2];
        double v[3] = {S->n[0] - c1 * e[0][0], S->n[1] - c1 * e[0][1], S->n[2] - c1 * e[0][2]};
        double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (!(vn > 1e-6)) { /* n_S along e1: any unit vector orthogonal to e1 */
            const double w[3] = {fabs(e[0][0]) < 0.9 ? 1.0 : 0.0, fabs(e[0][0]) < 0.9 ? 0.0 : 1.0, 0.0};
            const double pw = w[0] * e[0][0] + w[1] * e[0][1];
            for (int d = 0; d < 3; ++d) v[d] = w[d] - pw * e[0][d];
            vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        }
        for (int d = 0; d < 3; ++d) e[1][d] = v[d] / vn;
        e[2][0] = e[0][1] * e[1][2] - e[0][2] * e[1][1];
        e[2][1] = e[0][2] * e[1][0] - e[0][0] * e[1][2];
        e[2][2] = e[0][0] * e[1][1] - e[0][1] * e[1][0];
        x[0] = 4.0 * rB / rho;
        x[1] = c1;
        x[2] = S->n[0] * e[1][0] + S->n[1] * e[1][1] + S->n[2] * e[1][2];
        for (int a = 0; a < 3; ++a) x[3 + a] = nu[0] * e[a][0] + nu[1] * e[a][1] + nu[2] * e[a][2];
        x[6] = nn / n->A;
        for (int m = 0; m < 6; ++m) {
            x[7 + m] = qform(m2c, e[pa[m]], e[pb[m]]) / (rB * rB);
            x[13 + m] = qform(m2n, e[pa[m]], e[pb[m]]);
        }
        /* targets: exact sum over the cluster's faces minus the monopole */
        inner_t ex = {0}, mo = {0};
        int bad = 0;
        for (int64_t j = p0; j < p1; ++j) bad |= add_inner(S, t->g[j].c, t->g[j].a, t->g[j].n, u->q, u->p, &ex);
        bad |= add_inner(S, n->C, n->A, nu, u->q, u->p, &mo);
        const double u6 = n->A / ipow(rho, 6), u7 = u6 / rho;
        y[0] = (ex.K - mo.K) / u6;
        for (int a = 0; a < 3; ++a) {
            double dv = 0.0, dc = 0.0;
            for (int d = 0; d < 3; ++d) {
                dv += e[a][d] * (ex.Vn[d] - mo.Vn[d]) / u->q;
                dc += e[a][d] * (ex.Vc[d] - mo.Vc[d]);
            }
            y[1 + a] = dv / u6;
            y[4 + a] = dc / u7;
        }
        y[7] = bad ? 0.0 : 1.0;
    }
    return FF_OK;
}

/* Learned-correction training samples of the walk at theta: for every far cluster selected by
 * tpeo_sample_hash (and holding at most max_faces faces) of every target block, in no particular
 * order: out_block[c], out_node[c] and, per row (face) of the block, feats[c][64][19] and
 * targets[c][64][8] (7 targets, then the weight: 1, or 0 for a row past the last face).  Returns
 * the number of selected (block, cluster) pairs (which may exceed cap: then only cap are written),
 * or a negative error. */
int64_t tpeo_farfield_samples(const double* X, int64_t V, const int32_t* F, int64_t nF, const uint32_t* perm,
                              int leaf, double theta, uint64_t seed, double select_prob, int64_t max_faces,
                              int64_t cap, int32_t* out_block, int32_t* out_node, double* feats, double* targets) {
    if (!(theta > 0.0) || !(select_prob >= 0.0 && select_prob <= 1.0) || cap < 0) return FF_EINVAL;
    ftree t;
    int rc = tree_build(&t, X, V, F, nF, perm, leaf);
    if (rc) { tree_free(&t); return rc; }
    const double thr = select_prob >= 1.0 ? 4294967295.0 : floor(select_prob * 4294967296.0);
    smp_user u = {thr, seed, max_faces, cap, 0, 6.0, 12.0, out_block, out_node, feats, targets};
    const int64_t nb = (nF + BLOCK - 1) / BLOCK;
    const float th = (float)theta;
    for (int64_t b = 0; b < nb; ++b) {
        float tb[4];
        block_ball(&t, b, tb);
        walk_stats st = {0, 0, 0};
        walk(&t, b, tb, th, 1, &st, smp_visit, &u);
    }
    tree_free(&t);
    return u.count;
}

/* ---- dual tree (both integrals clustered) --------------------------------------------------------------- */

typedef struct {
    int Hd;
    int64_t span;
    int64_t* noff;  /* near list of node k: nent[noff[k] .. noff[k] + nnear[k]) */
    int64_t* nnear;
    int64_t* foff;  /* far list: fent[foff[k] .. foff[k] + nfar[k]) */
    int64_t* nfar;
    int64_t* nent;
    int64_t* fent;
    int64_t n_near_ent, n_far_ent;
} dlists;

static void dlists_free(dlists* L) {
    free(L->noff); free(L->nnear); free(L->foff); free(L->nfar); free(L->nent); free(L->fent);
}

static int dual_is_far(const fnode* a, const fnode* b, float theta) {
    const float rmax = fmaxf(a->rec[3], b->rec[3]);
    return 2.0f * rmax < theta * dist_f32(a->rec, b->rec) * (1.0f - 1e-5f);
}

static int push(int64_t** arr, int64_t* n, int64_t* cap, int64_t v) {
    if (*n == *cap) {
        int64_t nc = *cap ? 2 * *cap : 1024;
        int64_t* p = realloc(*arr, sizeof(int64_t) * (size_t)nc);
        if (!p) return FF_EINVAL;
        *arr = p;
        *cap = nc;
    }
    (*arr)[(*n)++] = v;
    return FF_OK;
}

static int dual_lists(const ftree* t, float theta, dlists* L) {
    memset(L, 0, sizeof(*L));
    int Hd = t->H;
    int64_t span = t->leaf;
    while (Hd > 0 && span < DUAL_SPAN) { --Hd; span *= 2; }
    L->Hd = Hd;
    L->span = span;
    const size_t nn = (size_t)2 << Hd;
    L->noff = calloc(nn, sizeof(int64_t)); L->nnear = calloc(nn, sizeof(int64_t));
    L->foff = calloc(nn, sizeof(int64_t)); L->nfar = calloc(nn, sizeof(int64_t));
    if (!L->noff || !L->nnear || !L->foff || !L->nfar) return FF_EINVAL;
    int64_t ncap = 0, fcap = 0;
    if (push(&L->nent, &L->n_near_ent, &ncap, 1)) return FF_EINVAL; /* the root is its own near node */
    L->noff[1] = 0;
    L->nnear[1] = 1;
    for (int l = 1; l <= Hd; ++l)
        for (int64_t A = (int64_t)1 << l; A < ((int64_t)2 << l); ++A) {
            const fnode* a = &t->nodes[A];
            L->noff[A] = L->n_near_ent;
            L->foff[A] = L->n_far_ent;
            if (!(a->af > 0.f)) continue;
            const int64_t P = A >> 1;
            for (int64_t e = 0; e < L->nnear[P]; ++e)
                for (int c = 0; c < 2; ++c) {
                    const int64_t B = 2 * L->nent[L->noff[P] + e] + c;
                    const fnode* bn = &t->nodes[B];
                    if (!(bn->af > 0.f)) continue;
                    if (dual_is_far(a, bn, theta)) {
                        if (push(&L->fent, &L->n_far_ent, &fcap, B)) return FF_EINVAL;
                        L->nfar[A] += 1;
                    } else {
                        if (push(&L->nent, &L->n_near_ent, &ncap, B)) return FF_EINVAL;
                        L->nnear[A] += 1;
                    }
                }
        }
    return FF_OK;
}

/* Nodes of the tree given as the heap index at the tree's own height H; the dual lists use
 * levels 0..Hd of the same numbering (node A at level l covers the same faces either way). */

typedef double complex cplx;

typedef struct { cplx a, n[3], c[3]; } cface;
typedef struct { cplx A, C[3], nu[3]; } cnode;

static void cface_of(const double* X, const int32_t* F, int64_t f, int64_t pv, int pd, double h, cface* o) {
    cplx x[3][3];
    for (int k = 0; k < 3; ++k) {
        const int64_t v = F[3 * f + k];
        for (int d = 0; d < 3; ++d) x[k][d] = X[3 * v + d] + ((v == pv && d == pd) ? I * h : 0.0);
    }
    const cplx e1[3] = {x[1][0] - x[0][0], x[1][1] - x[0][1], x[1][2] - x[0][2]};
    const cplx e2[3] = {x[2][0] - x[0][0], x[2][1] - x[0][1], x[2][2] - x[0][2]};
    const cplx w[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const cplx wn = csqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    o->a = 0.5 * wn;
    for (int d = 0; d < 3; ++d) {
        o->n[d] = w[d] / wn;
        o->c[d] = (x[0][d] + x[1][d] + x[2][d]) / 3.0;
    }
}

/* k(d; n) = (n.d)^q / (d.d)^(p/2) for even integers q and p (analytic: the complex step applies). */
static cplx ckernel(const cplx* d, const cplx* n, int q, int p) {
    const cplx u = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
    const cplx r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    cplx uq = 1.0, rp = 1.0;
    for (int i = 0; i < q; ++i) uq *= u;
    for (int i = 0; i < p / 2; ++i) rp *= r2;
    return uq / rp;
}

static void cnode_of(const ftree* t, const cface* cf, int64_t k, cnode* o) {
    int64_t p0, p1;
    node_range(t, k, &p0, &p1);
    cplx A = 0.0, S[3] = {0, 0, 0}, N[3] = {0, 0, 0};
    for (int64_t i = p0; i < p1; ++i)
        for (int d = 0; d < 3; ++d) {
            if (d == 0) A += cf[i].a;
            S[d] += cf[i].a * cf[i].c[d];
            N[d] += cf[i].a * cf[i].n[d];
        }
    o->A = A;
    const cplx nn = csqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
    for (int d = 0; d < 3; ++d) {
        o->C[d] = S[d] / A;
        o->nu[d] = N[d] / nn;
    }
}

/* The dual energy (without scale) with vertex pv's coordinate pd moved by i h (pv < 0: none), summing
 * only the terms that depend on that vertex when pv >= 0 (the others have no imaginary part).  The
 * dual lists use levels 0..Hd of the tree's own heap numbering (node A covers node_range(A)). */
static cplx dual_energy(const ftree* t, const dlists* L, int q, int p, int64_t pv, int pd, double h) {
    const int64_t nF = t->nF;
    const int64_t nn = (int64_t)2 << L->Hd;
    char* aff_face = calloc((size_t)nF, 1);
    char* aff_node = calloc((size_t)2 << t->H, 1);
    char* have = calloc((size_t)nn, 1);
    cface* cf = malloc(sizeof(cface) * (size_t)nF);
    cnode* cn = calloc((size_t)nn, sizeof(cnode));
    cplx E = 0.0;
    if (!aff_face || !aff_node || !have || !cf || !cn) { E = NAN; goto done; }
    for (int64_t i = 0; i < nF; ++i) {
        const int64_t f = t->perm[i];
        int touched = 0;
        for (int k = 0; k < 3; ++k) touched |= t->F[3 * f + k] == pv;
        aff_face[i] = pv < 0 || touched;
        cface_of(t->X, t->F, f, touched ? pv : -1, pd, h, &cf[i]);
        if (aff_face[i])
            for (int64_t k = ((int64_t)1 << t->H) + i / t->leaf; k >= 1; k >>= 1) aff_node[k] = 1;
    }
    /* far pairs (levels 1..Hd) */
    for (int64_t A = 2; A < nn; ++A)
        for (int64_t e = 0; e < L->nfar[A]; ++e) {
            const int64_t B = L->fent[L->foff[A] + e];
            if (!(aff_node[A] || aff_node[B])) continue;
            if (!have[A]) { cnode_of(t, cf, A, &cn[A]); have[A] = 1; }
            if (!have[B]) { cnode_of(t, cf, B, &cn[B]); have[B] = 1; }
            const cplx d[3] = {cn[A].C[0] - cn[B].C[0], cn[A].C[1] - cn[B].C[1], cn[A].C[2] - cn[B].C[2]};
            E += cn[A].A * cn[B].A * ckernel(d, cn[A].nu, q, p);
        }
    /* near pairs of the dual leaves (level Hd) */
    for (int64_t A = (int64_t)1 << L->Hd; A < nn; ++A) {
        int64_t a0, a1;
        node_range(t, A, &a0, &a1);
        for (int64_t e = 0; e < L->nnear[A]; ++e) {
            const int64_t B = L->nent[L->noff[A] + e];
            if (!(aff_node[A] || aff_node[B])) continue;
            int64_t b0, b1;
            node_range(t, B, &b0, &b1);
            for (int64_t i = a0; i < a1; ++i)
                for (int64_t j = b0; j < b1; ++j) {
                    if (!(aff_face[i] || aff_face[j])) continue;
                    if (shares_vertex(t->F, t->perm[i], t->perm[j])) continue;
                    const cplx d[3] = {cf[i].c[0] - cf[j].c[0], cf[i].c[1] - cf[j].c[1], cf[i].c[2] - cf[j].c[2]};
                    E += cf[i].a * cf[j].a * ckernel(d, cf[i].n, q, p);
                }
        }
    }
done:
    free(aff_face); free(aff_node); free(have); free(cf); free(cn);
    return E;
}

/* Dual-tree approximation: E_out <- its energy; G_out (nullable) [nv][3] <- its exact derivative at
 * the vertices verts[0..nv) (verts NULL: all V vertices, nv = V), by the complex step.
 * stats (nullable, 2 int64): far cluster pairs, face pairs of the near dual leaves (with the
 * excluded ones). */
int tpeo_farfield_dual(const double* X, int64_t V, const int32_t* F, int64_t nF, const uint32_t* perm, int leaf,
                       double theta, double q, double p, double scale, const int32_t* verts, int64_t nv,
                       int nthreads, double* E_out, double* G_out, int64_t* stats) {
    if (!(theta >= 0.0 && theta <= 1.0)) return FF_EINVAL;
    if (q != floor(q) || p != floor(p) || ((int)q % 2) || ((int)p % 2) || !(q >= 2.0) || !(p > q)) return FF_EINVAL;
    if (leaf > DUAL_SPAN || DUAL_SPAN % leaf) return FF_EINVAL;
    ftree t;
    int rc = tree_build(&t, X, V, F, nF, perm, leaf);
    if (rc) { tree_free(&t); return rc; }
    dlists L;
    if ((rc = dual_lists(&t, (float)theta, &L))) { dlists_free(&L); tree_free(&t); return rc; }
    if (stats) {
        stats[0] = L.n_far_ent;
        stats[1] = 0;
        for (int64_t A = (int64_t)1 << L.Hd; A < ((int64_t)2 << L.Hd); ++A) {
            int64_t a0, a1;
            node_range(&t, A, &a0, &a1);
            for (int64_t e = 0; e < L.nnear[A]; ++e) {
                int64_t b0, b1;
                node_range(&t, L.nent[L.noff[A] + e], &b0, &b1);
                stats[1] += (a1 - a0) * (b1 - b0);
            }
        }
    }
    const cplx E = dual_energy(&t, &L, (int)q, (int)p, -1, 0, 0.0);
    if (E_out) *E_out = scale * creal(E);
    rc = isfinite(creal(E)) ? FF_OK : FF_ENONFIN;
    if (G_out && !rc) {
        const int64_t n = verts ? nv : V;
        const double h = 1e-30;
#ifdef _OPENMP
        const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
        for (int64_t m = 0; m < 3 * n; ++m) {
            const int64_t v = verts ? verts[m / 3] : m / 3;
            const cplx Ev = dual_energy(&t, &L, (int)q, (int)p, v, (int)(m % 3), h);
            G_out[m] = scale * cimag(Ev) / h;
        }
    }
    (void)nthreads;
    dlists_free(&L);
    tree_free(&t);
    return rc;
}
