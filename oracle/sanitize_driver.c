/* Test driver that runs every entry point of the oracle once on small meshes read from files, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (oracle.build_sanitized).
 *
 * TEST INFRASTRUCTURE ONLY: built and run by tests/test_oracle_sanitized.py on the CPU.
 *
 * Usage: sanitize_driver <dir>, where <dir> holds
 *   mesh.bin  int64 V, int64 nF, double X[V][3], int32 F[nF][3]   (flat triangles)
 *   conf.bin  the same layout: the fixed confining surface
 *   p3.bin    int64 V, int64 nF, double X[V][3], int32 F[nF][10]  (curved cubic elements)
 * and prints one line per call: name, status, energy, sum of |G| (and counts where there are some),
 * which the test compares with the same calls through the regular build. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

int tpeo_energy(const double*, int64_t, const int32_t*, int64_t, double, double, double, int, double*);
int tpeo_gradient(const double*, int64_t, const int32_t*, int64_t, double, double, double, int, double*, double*);
int tpeo_gradient_rows(const double*, int64_t, const int32_t*, int64_t, double, double, double, int64_t, int64_t,
                       int, double*, double*);
int tpeo_gradient_at(const double*, int64_t, const int32_t*, int64_t, double, double, double, const int32_t*,
                     int64_t, int, double*);
int64_t tpeo_pair_count(const int32_t*, int64_t);
int tpeo_conf_gradient(const double*, int64_t, const int32_t*, int64_t, const double*, int64_t, const int32_t*,
                       int64_t, double, double, double, int, double*, double*);
int tpeo_gradient_quad(const double*, int64_t, const int32_t*, int64_t, double, double, double, int, int, double*,
                       double*);
int tpeo_gradient_p3(const double*, int64_t, const int32_t*, int64_t, double, double, double, int, int, double*,
                     double*);
int tpeo_kd_order(const double*, int64_t, const int32_t*, int64_t, int, uint32_t*);
int tpeo_farfield(const double*, int64_t, const int32_t*, int64_t, const uint32_t*, int, double, double, double,
                  double, int, double*, double*, int64_t*);
int tpeo_farfield_coverage(const double*, int64_t, const int32_t*, int64_t, const uint32_t*, int, double, int64_t*);
int64_t tpeo_farfield_samples(const double*, int64_t, const int32_t*, int64_t, const uint32_t*, int, double,
                              uint64_t, double, int64_t, int64_t, int32_t*, int32_t*, double*, double*);
int tpeo_farfield_dual(const double*, int64_t, const int32_t*, int64_t, const uint32_t*, int, double, double,
                       double, double, const int32_t*, int64_t, int, double*, double*, int64_t*);
int tpeo_quad_rule(int, double*, double*);
int tpeo_kd_order_p3(const double*, int64_t, const int32_t*, int64_t, const double*, int, int, uint32_t*);
int tpeo_farfield_p3(const double*, int64_t, const int32_t*, int64_t, const double*, const double*, int,
                     const uint32_t*, int, double, double, double, double, int, double*, double*, int64_t*);
int tpeo_farfield_coverage_p3(const double*, int64_t, const int32_t*, int64_t, const double*, const double*, int,
                              const uint32_t*, int, double, int64_t*);

typedef struct { int64_t V, nF; double* X; int32_t* F; } mesh;

static int read_mesh(const char* dir, const char* name, int nodes, mesh* m) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE* f = fopen(path, "rb");
    if (!f) return 1;
    int bad = fread(&m->V, 8, 1, f) != 1 || fread(&m->nF, 8, 1, f) != 1 || m->V <= 0 || m->nF <= 0;
    if (!bad) {
        m->X = (double*)malloc(sizeof(double) * 3 * (size_t)m->V);
        m->F = (int32_t*)malloc(sizeof(int32_t) * (size_t)nodes * (size_t)m->nF);
        bad = fread(m->X, sizeof(double), 3 * (size_t)m->V, f) != 3 * (size_t)m->V ||
              fread(m->F, sizeof(int32_t), (size_t)nodes * (size_t)m->nF, f) != (size_t)nodes * (size_t)m->nF;
    }
    fclose(f);
    return bad;
}

static double abs_sum(const double* a, size_t n) {
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += fabs(a[i]);
    return s;
}

int main(int argc, char** argv) {
    if (argc != 2) { fprintf(stderr, "usage: %s <dir>\n", argv[0]); return 2; }
    mesh m = {0}, y = {0}, c = {0};
    if (read_mesh(argv[1], "mesh.bin", 3, &m) || read_mesh(argv[1], "conf.bin", 3, &y) ||
        read_mesh(argv[1], "p3.bin", 10, &c)) {
        fprintf(stderr, "cannot read the input meshes\n");
        return 2;
    }
    const double q = 6.0, p = 12.0, sc = 1.0;
    const int nt = 2, leaf = 32;
    const size_t n3 = 3 * (size_t)m.V;
    double E = 0.0;
    double* G = (double*)calloc(n3, sizeof(double));
    int rc;

    rc = tpeo_energy(m.X, m.V, m.F, m.nF, q, p, sc, nt, &E);
    printf("energy %d %.17g\n", rc, E);
    rc = tpeo_gradient(m.X, m.V, m.F, m.nF, q, p, sc, nt, &E, G);
    printf("gradient %d %.17g %.17g\n", rc, E, abs_sum(G, n3));
    rc = tpeo_gradient_rows(m.X, m.V, m.F, m.nF, q, p, sc, m.nF / 3, m.nF / 2, nt, &E, G);
    printf("gradient_rows %d %.17g %.17g\n", rc, E, abs_sum(G, n3));
    int32_t verts[3] = {0, (int32_t)(m.V / 2), (int32_t)(m.V - 1)};
    double Gv[9];
    rc = tpeo_gradient_at(m.X, m.V, m.F, m.nF, q, p, sc, verts, 3, nt, Gv);
    printf("gradient_at %d %.17g\n", rc, abs_sum(Gv, 9));
    printf("pair_count %lld\n", (long long)tpeo_pair_count(m.F, m.nF));
    rc = tpeo_conf_gradient(m.X, m.V, m.F, m.nF, y.X, y.V, y.F, y.nF, q, p, sc, nt, &E, G);
    printf("conf_gradient %d %.17g %.17g\n", rc, E, abs_sum(G, n3));
    rc = tpeo_gradient_quad(m.X, m.V, m.F, m.nF, q, p, sc, 6, nt, &E, G);
    printf("gradient_quad %d %.17g %.17g\n", rc, E, abs_sum(G, n3));
    double* Gc = (double*)calloc(3 * (size_t)c.V, sizeof(double));
    rc = tpeo_gradient_p3(c.X, c.V, c.F, c.nF, q, p, sc, 3, nt, &E, Gc);
    printf("gradient_p3 %d %.17g %.17g\n", rc, E, abs_sum(Gc, 3 * (size_t)c.V));

    uint32_t* perm = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)m.nF);
    rc = tpeo_kd_order(m.X, m.V, m.F, m.nF, leaf, perm);
    uint64_t h = 1469598103934665603ull;
    for (int64_t i = 0; i < m.nF; ++i) h = (h ^ perm[i]) * 1099511628211ull;
    printf("kd_order %d %llu\n", rc, (unsigned long long)h);
    int64_t st[6] = {0};
    rc = tpeo_farfield(m.X, m.V, m.F, m.nF, perm, leaf, 1.0, q, p, sc, nt, &E, G, st);
    printf("farfield %d %.17g %.17g %lld %lld %lld\n", rc, E, abs_sum(G, n3), (long long)st[0], (long long)st[1],
           (long long)st[2]);
    int64_t cov[2] = {-1, -1};
    rc = tpeo_farfield_coverage(m.X, m.V, m.F, m.nF, perm, leaf, 1.0, cov);
    printf("farfield_coverage %d %lld %lld\n", rc, (long long)cov[0], (long long)cov[1]);
    const int64_t cap = tpeo_farfield_samples(m.X, m.V, m.F, m.nF, perm, leaf, 1.0, 7, 0.5, 1 << 20, 0, NULL, NULL,
                                              NULL, NULL);
    int64_t ns = cap;
    double fs = 0.0, ts = 0.0;
    if (cap > 0) {
        int32_t* blk = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
        int32_t* node = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
        double* feats = (double*)malloc(sizeof(double) * (size_t)cap * 64 * 19);
        double* targ = (double*)malloc(sizeof(double) * (size_t)cap * 64 * 8);
        ns = tpeo_farfield_samples(m.X, m.V, m.F, m.nF, perm, leaf, 1.0, 7, 0.5, 1 << 20, cap, blk, node, feats,
                                   targ);
        fs = abs_sum(feats, (size_t)cap * 64 * 19);
        ts = abs_sum(targ, (size_t)cap * 64 * 8);
        free(blk); free(node); free(feats); free(targ);
    }
    printf("farfield_samples %lld %lld %.17g %.17g\n", (long long)cap, (long long)ns, fs, ts);
    int64_t st2[2] = {0};
    rc = tpeo_farfield_dual(m.X, m.V, m.F, m.nF, perm, leaf, 1.0, q, p, sc, NULL, m.V, nt, &E, G, st2);
    printf("farfield_dual %d %.17g %.17g %lld %lld\n", rc, E, abs_sum(G, n3), (long long)st2[0], (long long)st2[1]);

    double bq[18], wq[6];
    const int nq = tpeo_quad_rule(3, bq, wq);
    uint32_t* perm3 = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)c.nF * (size_t)nq);
    rc = tpeo_kd_order_p3(c.X, c.V, c.F, c.nF, bq, nq, 8, perm3);
    h = 1469598103934665603ull;
    for (int64_t i = 0; i < c.nF * nq; ++i) h = (h ^ perm3[i]) * 1099511628211ull;
    printf("kd_order_p3 %d %llu\n", rc, (unsigned long long)h);
    int64_t st3[6] = {0};
    rc = tpeo_farfield_p3(c.X, c.V, c.F, c.nF, bq, wq, nq, perm3, 8, 1.0, q, p, sc, nt, &E, Gc, st3);
    printf("farfield_p3 %d %.17g %.17g %lld %lld %lld\n", rc, E, abs_sum(Gc, 3 * (size_t)c.V), (long long)st3[0],
           (long long)st3[1], (long long)st3[2]);
    int64_t cov3[2] = {-1, -1};
    rc = tpeo_farfield_coverage_p3(c.X, c.V, c.F, c.nF, bq, wq, nq, perm3, 8, 1.0, cov3);
    printf("farfield_coverage_p3 %d %lld %lld\n", rc, (long long)cov3[0], (long long)cov3[1]);

    free(perm3); free(perm); free(Gc); free(G);
    free(m.X); free(m.F); free(y.X); free(y.F); free(c.X); free(c.F);
    return 0;
}
