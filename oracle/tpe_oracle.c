/*
 * FP64 CPU oracle for the discrete tangent-point energy and its vertex gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may link, load or call
 * this file: it exists so that tests, the smoke check and the benchmark's CPU-baseline leg
 * can compare the HIP implementation against a plain, slow, obviously correct evaluation of
 * the definition.  It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (paper, Sec. 2.2.2 "Self-avoidance", eq. (TP), with one-point centroid
 * quadrature on flat triangles):
 *
 *   For each face T = (i, j, k):  w_T = (x_j - x_i) x (x_k - x_i),  a_T = |w_T| / 2,
 *                                 n_T = w_T / |w_T|,               c_T = (x_i + x_j + x_k) / 3.
 *
 *   E(X) = scale * sum_S sum_{T : S and T share no vertex}  a_S a_T |n_S . (c_S - c_T)|^q
 *                                                                 / |c_S - c_T|^p
 *
 * over ORDERED face pairs (the double integral over S x S counts both orders).  The paper's
 * energy is q = alpha, p = 2 alpha, scale = rho / alpha (the kernel (1/R)^alpha with the
 * tangent-point radius R = |x-y|^2 / (2 |n(x).(x-y)|) equals 2^alpha |n.(x-y)|^alpha/|x-y|^{2 alpha},
 * and the prefactor 2^-alpha cancels the 2^alpha).
 *
 * The gradient is the exact derivative of that expression with respect to X by the chain
 * rule through c, a and n (the discrete counterpart of the paper's deformation derivative,
 * eq. (dTP)):  with u = n_S . d, d = c_S - c_T, r = |d|,  k(d; n) = |u|^q r^-p,
 *     dk/dd = q |u|^(q-2) u r^-p n  -  p |u|^q r^-(p+2) d,     dk/dn = q |u|^(q-2) u r^-p d.
 * Every pair's derivative is pushed straight to the (up to six) vertices of S and T.  This is
 * deliberately a different organisation from any per-face accumulation scheme.
 *
 * Summation: rows ascending, columns ascending, FP64 with Neumaier compensation; with
 * OpenMP, rows are split statically over threads, each thread keeps its own compensated
 * buffers and the buffers are merged in thread order (deterministic for a fixed thread count).
 *
 * Return codes: 0 ok, -1 invalid argument, -2 degenerate face (area <= 1e-300),
 * -3 non-finite input or a coincident non-adjacent centroid pair (E = +inf there).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OK 0
#define EINVAL_ -1
#define EDEGEN -2
#define ENONFIN -3

typedef struct { double s, c; } nsum; /* Neumaier running sum */

static void nadd(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

/* x^e for a non-negative real exponent; integer exponents by plain repeated multiplication */
static double powr(double x, double e) {
    if (e >= 0.0 && e == floor(e) && e <= 64.0) {
        double r = 1.0;
        for (int i = 0; i < (int)e; ++i) r *= x;
        return r;
    }
    return pow(x, e);
}

typedef struct { double w[3], a, n[3], c[3], wn; } face_t;

static void sub3(const double* a, const double* b, double* o) { o[0]=a[0]-b[0]; o[1]=a[1]-b[1]; o[2]=a[2]-b[2]; }
static double dot3(const double* a, const double* b) { return a[0]*b[0]+a[1]*b[1]+a[2]*b[2]; }
static void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1]*b[2] - a[2]*b[1];
    o[1] = a[2]*b[0] - a[0]*b[2];
    o[2] = a[0]*b[1] - a[1]*b[0];
}

static int face_geom(const double* X, const int32_t* F, int64_t f, face_t* g) {
    const double* xi = X + 3 * (int64_t)F[3*f+0];
    const double* xj = X + 3 * (int64_t)F[3*f+1];
    const double* xk = X + 3 * (int64_t)F[3*f+2];
    double e1[3], e2[3];
    sub3(xj, xi, e1); sub3(xk, xi, e2);
    cross3(e1, e2, g->w);
    g->wn = sqrt(dot3(g->w, g->w));
    g->a = 0.5 * g->wn;
    if (!(g->a > 1e-300)) return EDEGEN;
    for (int d = 0; d < 3; ++d) {
        g->n[d] = g->w[d] / g->wn;
        g->c[d] = (xi[d] + xj[d] + xk[d]) / 3.0;
    }
    return OK;
}

static int share_vertex(const int32_t* F, int64_t s, int64_t t) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (F[3*s+i] == F[3*t+j]) return 1;
    return 0;
}

static int check_inputs(const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p) {
    if (!X || !F || V <= 0 || nF <= 0) return EINVAL_;
    if (!(q >= 2.0) || !(p > q)) return EINVAL_;
    for (int64_t i = 0; i < 3 * nF; ++i)
        if (F[i] < 0 || F[i] >= V) return EINVAL_;
    for (int64_t i = 0; i < 3 * V; ++i)
        if (!isfinite(X[i])) return ENONFIN;
    return OK;
}

static int all_faces(const double* X, const int32_t* F, int64_t nF, face_t* G) {
    for (int64_t f = 0; f < nF; ++f) {
        int rc = face_geom(X, F, f, &G[f]);
        if (rc) return rc;
    }
    return OK;
}

/* Kernel value and its partial derivatives for one ordered pair (S as x, T as y). */
typedef struct { double k, dkdd[3], dkdn[3]; } pairval;

static int pair_eval(const face_t* S, const face_t* T, double q, double p, int want_grad, pairval* o) {
    double d[3];
    sub3(S->c, T->c, d);
    double r2 = dot3(d, d);
    if (!(r2 > 0.0)) return ENONFIN;
    double u = dot3(S->n, d);
    double au = fabs(u);
    double rmp = 1.0 / powr(sqrt(r2), p);       /* r^-p */
    double auq = powr(au, q);                   /* |u|^q */
    o->k = auq * rmp;
    if (want_grad) {
        double uq1 = powr(au, q - 2.0) * u;     /* |u|^(q-2) u */
        double A = q * uq1 * rmp;
        double B = p * auq * rmp / r2;
        for (int i = 0; i < 3; ++i) {
            o->dkdd[i] = A * S->n[i] - B * d[i];
            o->dkdn[i] = A * d[i];
        }
    }
    return OK;
}

/* Push dE/dc, dE/dn, dE/da of face f onto its vertices (chain rule through c, n, a). */
static void face_vjp(const double* X, const int32_t* F, int64_t f, const face_t* g,
                     const double* dc, const double* dn, double da, nsum* GV) {
    int32_t v[3] = {F[3*f+0], F[3*f+1], F[3*f+2]};
    double gw[3];
    double ndn = dn ? dot3(g->n, dn) : 0.0;
    for (int d = 0; d < 3; ++d) {
        gw[d] = 0.5 * da * g->n[d];
        if (dn) gw[d] += (dn[d] - ndn * g->n[d]) / g->wn;
    }
    for (int c = 0; c < 3; ++c) {
        const double* xj = X + 3 * (int64_t)v[(c + 1) % 3];
        const double* xk = X + 3 * (int64_t)v[(c + 2) % 3];
        double e[3], cr[3];
        sub3(xj, xk, e);
        cross3(e, gw, cr);
        for (int d = 0; d < 3; ++d) nadd(&GV[3 * (int64_t)v[c] + d], dc[d] / 3.0 + cr[d]);
    }
}

static int nthreads_of(int req) {
#ifdef _OPENMP
    return req > 0 ? req : omp_get_max_threads();
#else
    (void)req; return 1;
#endif
}

int tpeo_num_threads(int req) { return nthreads_of(req); }

int64_t tpeo_pair_count(const int32_t* F, int64_t nF) {
    int64_t n = 0;
    for (int64_t s = 0; s < nF; ++s)
        for (int64_t t = 0; t < nF; ++t)
            if (!share_vertex(F, s, t)) ++n;
    return n;
}

/* E over the row range [r0, r1) of faces S (full columns).  Used for the full energy and for
 * row-sampled partial energies. */
int tpeo_energy_rows(const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p,
                     double scale, int64_t r0, int64_t r1, int nthreads, double* E_out) {
    int rc = check_inputs(X, V, F, nF, q, p);
    if (rc) return rc;
    if (r0 < 0 || r1 > nF || r0 > r1 || !E_out) return EINVAL_;
    face_t* G = (face_t*)malloc(sizeof(face_t) * (size_t)nF);
    if (!G) return EINVAL_;
    rc = all_faces(X, F, nF, G);
    if (rc) { free(G); return rc; }
    int nt = nthreads_of(nthreads);
    nsum* part = (nsum*)calloc((size_t)nt, sizeof(nsum));
    int err = OK;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        nsum acc = {0.0, 0.0};
        int lerr = OK;
#pragma omp for schedule(static)
        for (int64_t s = r0; s < r1; ++s) {
            for (int64_t t = 0; t < nF; ++t) {
                if (share_vertex(F, s, t)) continue;
                pairval pv;
                if (pair_eval(&G[s], &G[t], q, p, 0, &pv)) { lerr = ENONFIN; continue; }
                nadd(&acc, G[s].a * G[t].a * pv.k);
            }
        }
        part[tid] = acc;
        if (lerr) {
#pragma omp critical
            err = lerr;
        }
    }
    nsum tot = {0.0, 0.0};
    for (int i = 0; i < nt; ++i) { nadd(&tot, part[i].s); nadd(&tot, part[i].c); }
    *E_out = err ? INFINITY : scale * nval(&tot);
    free(part); free(G);
    return err;
}

int tpeo_energy(const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p,
                double scale, int nthreads, double* E_out) {
    return tpeo_energy_rows(X, V, F, nF, q, p, scale, 0, nF, nthreads, E_out);
}

/* The contributions of the ordered pairs (S, T) with row S in [r0, r1) to the energy and to
 * G[V*3] = dE/dX (row-major like X); rows [0, nF) give the full energy and gradient. */
int tpeo_gradient_rows(const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p,
                       double scale, int64_t r0, int64_t r1, int nthreads, double* E_out, double* G_out) {
    int rc = check_inputs(X, V, F, nF, q, p);
    if (rc) return rc;
    if (!G_out || r0 < 0 || r1 > nF || r0 > r1) return EINVAL_;
    face_t* G = (face_t*)malloc(sizeof(face_t) * (size_t)nF);
    if (!G) return EINVAL_;
    rc = all_faces(X, F, nF, G);
    if (rc) { free(G); return rc; }
    int nt = nthreads_of(nthreads);
    nsum* GV = (nsum*)calloc((size_t)nt * (size_t)V * 3, sizeof(nsum));
    nsum* part = (nsum*)calloc((size_t)nt, sizeof(nsum));
    if (!GV || !part) { free(G); free(GV); free(part); return EINVAL_; }
    int err = OK;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        nsum* myG = GV + (size_t)tid * (size_t)V * 3;
        nsum acc = {0.0, 0.0};
        int lerr = OK;
#pragma omp for schedule(static)
        for (int64_t s = r0; s < r1; ++s) {
            for (int64_t t = 0; t < nF; ++t) {
                if (share_vertex(F, s, t)) continue;
                pairval pv;
                if (pair_eval(&G[s], &G[t], q, p, 1, &pv)) { lerr = ENONFIN; continue; }
                double aa = G[s].a * G[t].a;
                nadd(&acc, aa * pv.k);
                double dcS[3], dcT[3], dnS[3];
                for (int i = 0; i < 3; ++i) {
                    dcS[i] = scale * aa * pv.dkdd[i];
                    dcT[i] = -dcS[i];
                    dnS[i] = scale * aa * pv.dkdn[i];
                }
                face_vjp(X, F, s, &G[s], dcS, dnS, scale * G[t].a * pv.k, myG);
                face_vjp(X, F, t, &G[t], dcT, NULL, scale * G[s].a * pv.k, myG);
            }
        }
        part[tid] = acc;
        if (lerr) {
#pragma omp critical
            err = lerr;
        }
    }
    nsum tot = {0.0, 0.0};
    for (int i = 0; i < nt; ++i) { nadd(&tot, part[i].s); nadd(&tot, part[i].c); }
    if (E_out) *E_out = err ? INFINITY : scale * nval(&tot);
    for (int64_t i = 0; i < V * 3; ++i) {
        nsum g = {0.0, 0.0};
        for (int th = 0; th < nt; ++th) {
            nadd(&g, GV[(size_t)th * (size_t)V * 3 + (size_t)i].s);
            nadd(&g, GV[(size_t)th * (size_t)V * 3 + (size_t)i].c);
        }
        G_out[i] = nval(&g);
    }
    free(GV); free(part); free(G);
    return err;
}

/* Full energy and gradient G[V*3] = dE/dX (row-major like X). */
int tpeo_gradient(const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p,
                  double scale, int nthreads, double* E_out, double* G_out) {
    return tpeo_gradient_rows(X, V, F, nF, q, p, scale, 0, nF, nthreads, E_out, G_out);
}

/* Exact gradient at selected vertices only: G_out[nv*3] = dE/dx_v for v = verts[i].
 * Visits, for every face S incident to v, all pairs (S, T) and (T, S); only S depends on x_v
 * (a pair in which both faces contain v is excluded by definition). */
int tpeo_gradient_at(const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p,
                     double scale, const int32_t* verts, int64_t nv, int nthreads, double* G_out) {
    int rc = check_inputs(X, V, F, nF, q, p);
    if (rc) return rc;
    if (!verts || nv < 0 || !G_out) return EINVAL_;
    for (int64_t i = 0; i < nv; ++i) if (verts[i] < 0 || verts[i] >= V) return EINVAL_;
    face_t* G = (face_t*)malloc(sizeof(face_t) * (size_t)nF);
    if (!G) return EINVAL_;
    rc = all_faces(X, F, nF, G);
    if (rc) { free(G); return rc; }
    int nt = nthreads_of(nthreads);
    int err = OK;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t iv = 0; iv < nv; ++iv) {
        int32_t v = verts[iv];
        nsum* GV = (nsum*)calloc((size_t)V * 3, sizeof(nsum)); /* scratch for face_vjp */
        int lerr = OK;
        for (int64_t s = 0; s < nF; ++s) {
            if (F[3*s] != v && F[3*s+1] != v && F[3*s+2] != v) continue;
            for (int64_t t = 0; t < nF; ++t) {
                if (share_vertex(F, s, t)) continue;
                pairval f1, f2;
                if (pair_eval(&G[s], &G[t], q, p, 1, &f1) || pair_eval(&G[t], &G[s], q, p, 1, &f2)) {
                    lerr = ENONFIN; continue;
                }
                double aa = G[s].a * G[t].a;
                double dc[3], dn[3];
                for (int i = 0; i < 3; ++i) {
                    /* (S,T): S is x; (T,S): S is y, d = c_T - c_S so dd/dc_S = -I */
                    dc[i] = scale * aa * (f1.dkdd[i] - f2.dkdd[i]);
                    dn[i] = scale * aa * f1.dkdn[i];
                }
                double da = scale * G[t].a * (f1.k + f2.k);
                face_vjp(X, F, s, &G[s], dc, dn, da, GV);
            }
        }
        for (int d = 0; d < 3; ++d) G_out[3*iv + d] = nval(&GV[3 * (int64_t)v + d]);
        free(GV);
        if (lerr) {
#pragma omp critical
            err = lerr;
        }
    }
    free(G);
    return err;
}

/*
 * Confinement energy (paper Sec. 2.2.3, eq. (TPConf)): the moving surface (X, F) against a fixed
 * confining surface (Y, FY), with the tangent-point kernel built from the moving surface's normal
 * only, one-point centroid quadrature on both:
 *
 *   E_conf(X) = scale * sum_{S in F} sum_{T in FY}  a_S a_T |n_S . (c_S - c_T)|^q / |c_S - c_T|^p
 *
 * (every pair counts once: S always plays x and T always y; no pair is excluded, the meshes being
 * different surfaces).  The gradient is with respect to X only, by the same chain rule as above
 * applied to S alone: dE/dc_S = scale a_S a_T dk/dd, dE/dn_S = scale a_S a_T dk/dn,
 * dE/da_S = scale a_T k.  The paper's prefactor is rho_conf / alpha with rho_conf = 1e-4.
 */
static int conf_common(const double* X, int64_t V, const int32_t* F, int64_t nF, const double* Y, int64_t VY,
                       const int32_t* FY, int64_t nFY, double q, double p, face_t** GS, face_t** GT) {
    int rc = check_inputs(X, V, F, nF, q, p);
    if (rc) return rc;
    rc = check_inputs(Y, VY, FY, nFY, q, p);
    if (rc) return rc;
    *GS = (face_t*)malloc(sizeof(face_t) * (size_t)nF);
    *GT = (face_t*)malloc(sizeof(face_t) * (size_t)nFY);
    if (!*GS || !*GT) return EINVAL_;
    rc = all_faces(X, F, nF, *GS);
    if (!rc) rc = all_faces(Y, FY, nFY, *GT);
    return rc;
}

int tpeo_conf_gradient(const double* X, int64_t V, const int32_t* F, int64_t nF, const double* Y, int64_t VY,
                       const int32_t* FY, int64_t nFY, double q, double p, double scale, int nthreads,
                       double* E_out, double* G_out) {
    face_t *GS = NULL, *GT = NULL;
    int rc = conf_common(X, V, F, nF, Y, VY, FY, nFY, q, p, &GS, &GT);
    if (rc) { free(GS); free(GT); return rc; }
    int nt = nthreads_of(nthreads);
    nsum* GV = G_out ? (nsum*)calloc((size_t)nt * (size_t)V * 3, sizeof(nsum)) : NULL;
    nsum* part = (nsum*)calloc((size_t)nt, sizeof(nsum));
    if ((G_out && !GV) || !part) { free(GS); free(GT); free(GV); free(part); return EINVAL_; }
    int err = OK;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        nsum* myG = GV ? GV + (size_t)tid * (size_t)V * 3 : NULL;
        nsum acc = {0.0, 0.0};
        int lerr = OK;
#pragma omp for schedule(static)
        for (int64_t s = 0; s < nF; ++s) {
            for (int64_t t = 0; t < nFY; ++t) {
                pairval pv;
                if (pair_eval(&GS[s], &GT[t], q, p, myG != NULL, &pv)) { lerr = ENONFIN; continue; }
                double aa = GS[s].a * GT[t].a;
                nadd(&acc, aa * pv.k);
                if (myG) {
                    double dcS[3], dnS[3];
                    for (int i = 0; i < 3; ++i) {
                        dcS[i] = scale * aa * pv.dkdd[i];
                        dnS[i] = scale * aa * pv.dkdn[i];
                    }
                    face_vjp(X, F, s, &GS[s], dcS, dnS, scale * GT[t].a * pv.k, myG);
                }
            }
        }
        part[tid] = acc;
        if (lerr) {
#pragma omp critical
            err = lerr;
        }
    }
    nsum tot = {0.0, 0.0};
    for (int i = 0; i < nt; ++i) { nadd(&tot, part[i].s); nadd(&tot, part[i].c); }
    if (E_out) *E_out = err ? INFINITY : scale * nval(&tot);
    if (G_out)
        for (int64_t i = 0; i < V * 3; ++i) {
            nsum g = {0.0, 0.0};
            for (int th = 0; th < nt; ++th) {
                nadd(&g, GV[(size_t)th * (size_t)V * 3 + (size_t)i].s);
                nadd(&g, GV[(size_t)th * (size_t)V * 3 + (size_t)i].c);
            }
            G_out[i] = nval(&g);
        }
    free(GV); free(part); free(GS); free(GT);
    return err;
}

int tpeo_conf_energy(const double* X, int64_t V, const int32_t* F, int64_t nF, const double* Y, int64_t VY,
                     const int32_t* FY, int64_t nFY, double q, double p, double scale, int nthreads, double* E_out) {
    return tpeo_conf_gradient(X, V, F, nF, Y, VY, FY, nFY, q, p, scale, nthreads, E_out, NULL);
}

/*
 * Multi-point quadrature on each flat triangle (the paper integrates both integrals of eq. (TP)
 * with higher-order rules, Sec. 3.2): face f carries points x_fp = sum_i beta_pi x_(v_i) with weights
 * W_p (sum_p W_p = 1), and
 *
 *   E_Q(X) = scale * sum_S sum_{T : S,T share no vertex} sum_p sum_r W_p W_r a_S a_T
 *                    |n_S . (x_Sp - x_Tr)|^q / |x_Sp - x_Tr|^p .
 *
 * Rules (barycentric points, weights), written out here from their published values:
 *   1: the centroid, weight 1 (the one-point quadrature above);
 *   3: (2/3, 1/6, 1/6) and its permutations, weights 1/3 (exact for degree 2; Strang and Fix);
 *   6: (1 - 2a, a, a) and permutations for a = 0.445948490915965 (weight 0.223381589678011) and
 *      a = 0.091576213509771 (weight 0.109951743655322) (exact for degree 4; Dunavant 1985).
 * The gradient follows the chain rule through the points (dx_fp/dx_(v_i) = beta_pi I), the
 * normal and the area, pushed straight to the vertices as above.
 */
static int quad_rule(int rule, double (*b)[3], double* w) {
    if (rule == 1) {
        b[0][0] = b[0][1] = b[0][2] = 1.0 / 3.0; w[0] = 1.0;
        return 1;
    }
    if (rule == 3) {
        for (int p = 0; p < 3; ++p) {
            for (int i = 0; i < 3; ++i) b[p][i] = (i == p) ? 2.0 / 3.0 : 1.0 / 6.0;
            w[p] = 1.0 / 3.0;
        }
        return 3;
    }
    if (rule == 6) {
        const double a[2] = {0.445948490915965, 0.091576213509771};
        const double wt[2] = {0.223381589678011, 0.109951743655322};
        for (int g = 0; g < 2; ++g)
            for (int p = 0; p < 3; ++p) {
                for (int i = 0; i < 3; ++i) b[3 * g + p][i] = (i == p) ? 1.0 - 2.0 * a[g] : a[g];
                w[3 * g + p] = wt[g];
            }
        return 6;
    }
    return 0;
}

int tpeo_quad_rule(int rule, double* bary_out, double* w_out) {
    double b[6][3], w[6];
    int n = quad_rule(rule, b, w);
    for (int p = 0; p < n; ++p) {
        for (int i = 0; i < 3; ++i) bary_out[3 * p + i] = b[p][i];
        w_out[p] = w[p];
    }
    return n;
}

/* face_vjp with the point's barycentric weights instead of 1/3 for the position term */
static void face_vjp_b(const double* X, const int32_t* F, int64_t f, const face_t* g, const double* dx,
                       const double* beta, const double* dn, double da, nsum* GV) {
    int32_t v[3] = {F[3*f+0], F[3*f+1], F[3*f+2]};
    double gw[3];
    double ndn = dn ? dot3(g->n, dn) : 0.0;
    for (int d = 0; d < 3; ++d) {
        gw[d] = 0.5 * da * g->n[d];
        if (dn) gw[d] += (dn[d] - ndn * g->n[d]) / g->wn;
    }
    for (int c = 0; c < 3; ++c) {
        const double* xj = X + 3 * (int64_t)v[(c + 1) % 3];
        const double* xk = X + 3 * (int64_t)v[(c + 2) % 3];
        double e[3], cr[3];
        sub3(xj, xk, e);
        cross3(e, gw, cr);
        for (int d = 0; d < 3; ++d) nadd(&GV[3 * (int64_t)v[c] + d], beta[c] * dx[d] + cr[d]);
    }
}

int tpeo_gradient_quad(const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p,
                       double scale, int rule, int nthreads, double* E_out, double* G_out) {
    double b[6][3], w[6];
    const int nq = quad_rule(rule, b, w);
    if (!nq) return EINVAL_;
    int rc = check_inputs(X, V, F, nF, q, p);
    if (rc) return rc;
    face_t* G = (face_t*)malloc(sizeof(face_t) * (size_t)nF);
    double* P = (double*)malloc(sizeof(double) * 3 * (size_t)nF * nq);  /* points [f][p][3] */
    if (!G || !P) { free(G); free(P); return EINVAL_; }
    rc = all_faces(X, F, nF, G);
    if (rc) { free(G); free(P); return rc; }
    for (int64_t f = 0; f < nF; ++f)
        for (int k = 0; k < nq; ++k)
            for (int d = 0; d < 3; ++d) {
                double x = 0.0;
                for (int i = 0; i < 3; ++i) x += b[k][i] * X[3 * (int64_t)F[3 * f + i] + d];
                P[(f * nq + k) * 3 + d] = x;
            }
    int nt = nthreads_of(nthreads);
    nsum* GV = G_out ? (nsum*)calloc((size_t)nt * (size_t)V * 3, sizeof(nsum)) : NULL;
    nsum* part = (nsum*)calloc((size_t)nt, sizeof(nsum));
    if ((G_out && !GV) || !part) { free(G); free(P); free(GV); free(part); return EINVAL_; }
    int err = OK;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        nsum* myG = GV ? GV + (size_t)tid * (size_t)V * 3 : NULL;
        nsum acc = {0.0, 0.0};
        int lerr = OK;
#pragma omp for schedule(static)
        for (int64_t s = 0; s < nF; ++s) {
            for (int64_t t = 0; t < nF; ++t) {
                if (share_vertex(F, s, t)) continue;
                for (int ks = 0; ks < nq; ++ks)
                    for (int kt = 0; kt < nq; ++kt) {
                        /* a face record located at the quadrature point, with the face's normal */
                        face_t S = G[s], T = G[t];
                        for (int d = 0; d < 3; ++d) {
                            S.c[d] = P[(s * nq + ks) * 3 + d];
                            T.c[d] = P[(t * nq + kt) * 3 + d];
                        }
                        pairval pv;
                        if (pair_eval(&S, &T, q, p, myG != NULL, &pv)) { lerr = ENONFIN; continue; }
                        const double ww = w[ks] * w[kt];
                        const double aa = ww * G[s].a * G[t].a;
                        nadd(&acc, aa * pv.k);
                        if (myG) {
                            double dxS[3], dxT[3], dnS[3];
                            for (int i = 0; i < 3; ++i) {
                                dxS[i] = scale * aa * pv.dkdd[i];
                                dxT[i] = -dxS[i];
                                dnS[i] = scale * aa * pv.dkdn[i];
                            }
                            face_vjp_b(X, F, s, &G[s], dxS, b[ks], dnS, scale * ww * G[t].a * pv.k, myG);
                            face_vjp_b(X, F, t, &G[t], dxT, b[kt], NULL, scale * ww * G[s].a * pv.k, myG);
                        }
                    }
            }
        }
        part[tid] = acc;
        if (lerr) {
#pragma omp critical
            err = lerr;
        }
    }
    nsum tot = {0.0, 0.0};
    for (int i = 0; i < nt; ++i) { nadd(&tot, part[i].s); nadd(&tot, part[i].c); }
    if (E_out) *E_out = err ? INFINITY : scale * nval(&tot);
    if (G_out)
        for (int64_t i = 0; i < V * 3; ++i) {
            nsum g = {0.0, 0.0};
            for (int th = 0; th < nt; ++th) {
                nadd(&g, GV[(size_t)th * (size_t)V * 3 + (size_t)i].s);
                nadd(&g, GV[(size_t)th * (size_t)V * 3 + (size_t)i].c);
            }
            G_out[i] = nval(&g);
        }
    free(GV); free(part); free(G); free(P);
    return err;
}


/*
 * Curved cubic (P3) triangles (the paper's surface S_h^3, Sec. 3.1; its full integration scheme
 * evaluates positions, area elements and normals at the quadrature points of the curved elements,
 * Sec. 3.2).  Element f has 10 nodes F10[10 f + 0..9] at the barycentric lattice points
 *     0: (1,0,0)      1: (0,1,0)      2: (0,0,1)                      (corners)
 *     3: (2/3,1/3,0)  4: (1/3,2/3,0)                                   (edge 0-1)
 *     5: (0,2/3,1/3)  6: (0,1/3,2/3)                                   (edge 1-2)
 *     7: (1/3,0,2/3)  8: (2/3,0,1/3)                                   (edge 2-0)
 *     9: (1/3,1/3,1/3)                                                 (centre)
 * and the cubic Lagrange basis on barycentric coordinates (l0, l1, l2):
 *     corner i:                   phi = l_i (3 l_i - 1)(3 l_i - 2) / 2
 *     edge node (2/3 on i, 1/3 on j): phi = 9/2 l_i l_j (3 l_i - 1)
 *     centre:                     phi = 27 l0 l1 l2.
 * With reference coordinates (s, t) = (l1, l2), l0 = 1 - s - t, the element maps
 *     x(s, t) = sum_k phi_k X_k,   J = x_s x x_t,   n = J / |J|,
 * and quadrature point p of a rule (barycentric b_p, weight W_p, sum W_p = 1) is a record at
 * x(b_p) with normal n(b_p) and weight alpha_p = W_p |J(b_p)| / 2 (for straight elements:
 * W_p times the area).  The energy is that of the flat multi-point scheme over these records:
 *
 *   E(X) = scale * sum_S sum_{T : S, T share no corner node} sum_p sum_r alpha_Sp alpha_Tr
 *                  |n_Sp . (x_Sp - x_Tr)|^q / |x_Sp - x_Tr|^p .
 *
 * The gradient follows the chain rule through the record: with g = dE/dalpha, gn = dE/dn and
 * gx = dE/dx of a record, gJ = g (W_p / 2) n + (I - n n^T) gn / |J|, and node k receives
 *     phi_k gx + (d phi_k / ds) (x_t x gJ) + (d phi_k / dt) (gJ x x_s).
 */

/* basis values and derivatives with respect to (s, t) at barycentric (l0, l1, l2) */
static void p3_basis(const double* l, double* phi, double* ds, double* dt) {
    static const int EI[6] = {0, 1, 1, 2, 2, 0}, EJ[6] = {1, 0, 2, 1, 0, 2};
    double dl[10][3];
    for (int i = 0; i < 3; ++i) {
        phi[i] = 0.5 * l[i] * (3.0 * l[i] - 1.0) * (3.0 * l[i] - 2.0);
        for (int m = 0; m < 3; ++m) dl[i][m] = 0.0;
        dl[i][i] = 0.5 * (27.0 * l[i] * l[i] - 18.0 * l[i] + 2.0);
    }
    for (int e = 0; e < 6; ++e) {
        const int i = EI[e], j = EJ[e], k = 3 + e;
        phi[k] = 4.5 * l[i] * l[j] * (3.0 * l[i] - 1.0);
        for (int m = 0; m < 3; ++m) dl[k][m] = 0.0;
        dl[k][i] = 4.5 * l[j] * (6.0 * l[i] - 1.0);
        dl[k][j] = 4.5 * l[i] * (3.0 * l[i] - 1.0);
    }
    phi[9] = 27.0 * l[0] * l[1] * l[2];
    dl[9][0] = 27.0 * l[1] * l[2];
    dl[9][1] = 27.0 * l[0] * l[2];
    dl[9][2] = 27.0 * l[0] * l[1];
    /* l0 = 1 - s - t, l1 = s, l2 = t */
    for (int k = 0; k < 10; ++k) {
        ds[k] = dl[k][1] - dl[k][0];
        dt[k] = dl[k][2] - dl[k][0];
    }
}

/* x, x_s, x_t of the element with nodes P (10 x 3) at barycentric l */
static void p3_eval(const double* P, const double* l, double* x, double* xs, double* xt) {
    double phi[10], ds[10], dt[10];
    p3_basis(l, phi, ds, dt);
    for (int d = 0; d < 3; ++d) {
        x[d] = xs[d] = xt[d] = 0.0;
        for (int k = 0; k < 10; ++k) {
            x[d] += phi[k] * P[3 * k + d];
            xs[d] += ds[k] * P[3 * k + d];
            xt[d] += dt[k] * P[3 * k + d];
        }
    }
}

/* The basis at barycentric l (for the far-field oracle's curved records; pinned with the map). */
int tpeo_p3_basis(const double* l, double* phi, double* ds, double* dt) {
    p3_basis(l, phi, ds, dt);
    return OK;
}

int tpeo_p3_map(const double* P, double s, double t, double* x, double* xs, double* xt) {
    const double l[3] = {1.0 - s - t, s, t};
    p3_eval(P, l, x, xs, xt);
    return OK;
}

static int share_corner10(const int32_t* F, int64_t s, int64_t t) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (F[10 * s + i] == F[10 * t + j]) return 1;
    return 0;
}

typedef struct { double x[3], xs[3], xt[3], n[3], Jn, alpha, W; const double* l; } p3rec;

int tpeo_gradient_p3(const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p, double scale,
                     int rule, int nthreads, double* E_out, double* G_out) {
    double b[6][3], w[6];
    const int nq = quad_rule(rule, b, w);
    if (!nq) return EINVAL_;
    if (!X || !F || V <= 0 || nF <= 0 || !(q >= 2.0) || !(p > q)) return EINVAL_;
    for (int64_t i = 0; i < 10 * nF; ++i)
        if (F[i] < 0 || F[i] >= V) return EINVAL_;
    for (int64_t i = 0; i < 3 * V; ++i)
        if (!isfinite(X[i])) return ENONFIN;
    p3rec* R = (p3rec*)malloc(sizeof(p3rec) * (size_t)nF * nq);
    if (!R) return EINVAL_;
    for (int64_t f = 0; f < nF; ++f) {
        double P[30];
        for (int k = 0; k < 10; ++k)
            for (int d = 0; d < 3; ++d) P[3 * k + d] = X[3 * (int64_t)F[10 * f + k] + d];
        for (int k = 0; k < nq; ++k) {
            p3rec* r = &R[f * nq + k];
            p3_eval(P, b[k], r->x, r->xs, r->xt);
            double J[3];
            cross3(r->xs, r->xt, J);
            r->Jn = sqrt(dot3(J, J));
            if (!(r->Jn > 1e-300)) { free(R); return EDEGEN; }
            for (int d = 0; d < 3; ++d) r->n[d] = J[d] / r->Jn;
            r->W = w[k];
            r->alpha = 0.5 * w[k] * r->Jn;
            r->l = b[k];
        }
    }
    int nt = nthreads_of(nthreads);
    nsum* GV = G_out ? (nsum*)calloc((size_t)nt * (size_t)V * 3, sizeof(nsum)) : NULL;
    nsum* part = (nsum*)calloc((size_t)nt, sizeof(nsum));
    if ((G_out && !GV) || !part) { free(R); free(GV); free(part); return EINVAL_; }
    int err = OK;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        nsum* myG = GV ? GV + (size_t)tid * (size_t)V * 3 : NULL;
        nsum acc = {0.0, 0.0};
        int lerr = OK;
#pragma omp for schedule(static)
        for (int64_t s = 0; s < nF; ++s) {
            for (int64_t t = 0; t < nF; ++t) {
                if (share_corner10(F, s, t)) continue;
                for (int ks = 0; ks < nq; ++ks)
                    for (int kt = 0; kt < nq; ++kt) {
                        const p3rec* rs = &R[s * nq + ks];
                        const p3rec* rt = &R[t * nq + kt];
                        face_t S, T;
                        memset(&S, 0, sizeof S);
                        memset(&T, 0, sizeof T);
                        for (int d = 0; d < 3; ++d) {
                            S.c[d] = rs->x[d]; S.n[d] = rs->n[d];
                            T.c[d] = rt->x[d]; T.n[d] = rt->n[d];
                        }
                        pairval pv;
                        if (pair_eval(&S, &T, q, p, myG != NULL, &pv)) { lerr = ENONFIN; continue; }
                        const double aa = rs->alpha * rt->alpha;
                        nadd(&acc, aa * pv.k);
                        if (!myG) continue;
                        /* dE/dx, dE/dn, dE/dalpha of both records, then to their nodes */
                        for (int side = 0; side < 2; ++side) {
                            const p3rec* r = side ? rt : rs;
                            const int64_t f = side ? t : s;
                            double gx[3], gn[3], gJ[3];
                            const double g = scale * (side ? rs->alpha : rt->alpha) * pv.k;
                            for (int i = 0; i < 3; ++i) {
                                gx[i] = (side ? -1.0 : 1.0) * scale * aa * pv.dkdd[i];
                                gn[i] = side ? 0.0 : scale * aa * pv.dkdn[i];
                            }
                            const double ngn = dot3(r->n, gn);
                            for (int i = 0; i < 3; ++i)
                                gJ[i] = g * 0.5 * r->W * r->n[i] + (gn[i] - ngn * r->n[i]) / r->Jn;
                            double phi[10], ds[10], dt[10], cs[3], ct[3];
                            p3_basis(r->l, phi, ds, dt);
                            cross3(r->xt, gJ, cs);   /* x_t x gJ: the d/dx_s direction */
                            cross3(gJ, r->xs, ct);   /* gJ x x_s: the d/dx_t direction */
                            for (int k = 0; k < 10; ++k) {
                                const int64_t v = F[10 * f + k];
                                for (int d = 0; d < 3; ++d)
                                    nadd(&myG[3 * v + d], phi[k] * gx[d] + ds[k] * cs[d] + dt[k] * ct[d]);
                            }
                        }
                    }
            }
        }
        part[tid] = acc;
        if (lerr) {
#pragma omp critical
            err = lerr;
        }
    }
    nsum tot = {0.0, 0.0};
    for (int i = 0; i < nt; ++i) { nadd(&tot, part[i].s); nadd(&tot, part[i].c); }
    if (E_out) *E_out = err ? INFINITY : scale * nval(&tot);
    if (G_out)
        for (int64_t i = 0; i < V * 3; ++i) {
            nsum g = {0.0, 0.0};
            for (int th = 0; th < nt; ++th) {
                nadd(&g, GV[(size_t)th * (size_t)V * 3 + (size_t)i].s);
                nadd(&g, GV[(size_t)th * (size_t)V * 3 + (size_t)i].c);
            }
            G_out[i] = nval(&g);
        }
    free(GV); free(part); free(R);
    return err;
}
