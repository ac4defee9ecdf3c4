// Finalize: merge the per-face row sums in FP64 (the pair kernel's compensated partial segments,
// or the far-field walk's FP64 sums), turn them into the gradient contributions of the face's
// three corners, and reduce the energy; then the scatter-free vertex gather.  No floating-point
// atomics anywhere: every sum has a fixed order.
//
// With the row sums of pair.hip (K, S0, Sd, Sdd, Sn) for face S and the kernel k = t^q with
// p = 2q, the partial derivatives of E with respect to the face's own geometry are
//     dE/da_S = K,   dE/dn_S = q a_S Sd,   dE/dc_S = a_S (q (n_S S0 + Sn) - p Sdd),
// which are the paper's inner integrals f_K, f_nu and f (Sec. 3.2, eq. (dTP_reordered)) at the
// face's quadrature point.  They reach the vertices through w = (x_j - x_i) x (x_k - x_i):
//     g_w = (dE/da) n / 2 + (I - n n^T) (dE/dn) / |w|,
//     dE/dx_i = (dE/dc)/3 + (x_j - x_k) x g_w      (and cyclically for j, k).
// The energy is E = (1/2) sum_S a_S K_S (each ordered pair is counted once in the forward and
// once in the reverse part of K).  Everything here is FP64.
#include "common.hpp"

namespace tpe {

__device__ __forceinline__ double wave_sum(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Row sums of face i: from the pair kernel's segments (part != null: the (hi, lo) FP32 pairs of
// every wave whose range covers row i's block, added in FP64 in wave order), else acc64[k][i].
// UNIFORM: the covering waves are the same for the whole wave of threads (consecutive rows, ROWB a
// multiple of 64), so the schedule's divisions run once per wave, on wave-uniform values.
template <int NA, bool UNIFORM = true>
__device__ __forceinline__ void row_sums(const float* __restrict__ part, const Sched& sc,
                                         const double* __restrict__ accs, int64_t Fp, int64_t i, double (&acc)[NA]) {
    if (!part) {
        for (int k = 0; k < NA; ++k) acc[k] = accs[(size_t)k * Fp + i];
        return;
    }
    auto uni = [](int x) { return UNIFORM ? __builtin_amdgcn_readfirstlane(x) : x; };
    const int rr = (int)(i % ROWB);
    const int rb = uni((int)(i / ROWB));
    const int w0 = uni(sc.wave_of((int64_t)rb * sc.upr));
    const int w1 = uni(sc.wave_of((int64_t)(rb + 1) * sc.upr - 1));
    for (int k = 0; k < NA; ++k) acc[k] = 0.0;
    for (int w = w0; w <= w1; ++w) {
        const int seg = uni(rb - (int)(sc.begin(w) / sc.upr));
        const float* ps = part + ((size_t)w * sc.maxseg + seg) * 2 * NA * ROWB + rr;
        for (int k = 0; k < NA; ++k) acc[k] += (double)ps[(size_t)k * ROWB] + (double)ps[(size_t)(NA + k) * ROWB];
    }
}

// Energy of a 256-thread work-group's threads (e per thread): every work-group writes one FP64
// partial, and energy_sum adds the partials in index order after the kernel (the launch boundary
// orders the writes), so the energy is deterministic.  No last-work-group ticket: that needs a
// device-scope release fence in every work-group, which on this chip writes back the L2 (the
// finalize at 327,680 faces took 89 us with it, 26 us without).
__device__ void energy_part(double e, double* __restrict__ epart) {
    __shared__ double ws[4];
    e = wave_sum(e);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) epart[blockIdx.x] = ((ws[0] + ws[1]) + (ws[2] + ws[3]));
}

// E[0] = scale 2^(kexp (p - q - 4)) * (sum of the nb partials), by one work-group of 256 threads:
// thread t adds partials t, t + 256, ... in order, then the waves, then the 4 wave sums.  The row
// sums were taken on positions multiplied by s = 2^kexp, and E(X) = s^(p-q-4) E(sX) exactly.  Runs
// as the extra last work-group of the vertex gather when there is one, else alone (energy_sum).
__device__ void energy_total(const EnergyOut& en) {
    __shared__ double ws[4];
    double t = 0.0;
    for (int b = threadIdx.x; b < en.nb; b += 256) t += en.epart[b];
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0)
        en.E[0] = en.scale * pow2i(norm_exp(en.bbox), en.p - en.q - 4.0) * ((ws[0] + ws[1]) + (ws[2] + ws[3]));
}

__global__ __launch_bounds__(256) void energy_sum(EnergyOut en) { energy_total(en); }

// One thread per sorted face; the energy partials as in energy_part.
template <bool GRAD>
__global__ __launch_bounds__(256) void finalize_kernel(const float* __restrict__ part, Sched sc,
                                                       const double* __restrict__ accs, int64_t Fp, int64_t nF,
                                                       const double* __restrict__ geo,
                                                       const int4* __restrict__ colv,
                                                       const double* __restrict__ X,
                                                       const uint32_t* __restrict__ bbox, double q, double p,
                                                       double scale, double efac, int Q,
                                                       double* __restrict__ corner,
                                                       double* __restrict__ epart, uint32_t* __restrict__ flags) {
    constexpr int NA = GRAD ? NACC : 1;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double e = 0.0;
    // the row sums were taken on positions multiplied by s = 2^k: G(X) = s^(p-q-3) G(sX) and
    // E(X) = s^(p-q-4) E(sX), exactly
    const int kexp = norm_exp(bbox);
    const double s = ldexp(1.0, kexp);
    const double gs = scale * pow2i(kexp, p - q - 3.0);
    if (i < nF) {
        double acc[NA];
        row_sums<NA>(part, sc, accs, Fp, i, acc);
        const double a = geo[5 * i + 0], wn = geo[5 * i + 1];
        const double n[3] = {geo[5 * i + 2], geo[5 * i + 3], geo[5 * i + 4]};
        bool finite = true;
        for (int k = 0; k < NA; ++k) finite &= isfinite(acc[k]);
        if (!GRAD) {
            e = a * acc[0];
        } else {
            e = efac * a * acc[0];
            // the record is quadrature point v.w of its face, with weight wq (Q = 1: the centroid)
            const int4 v = colv[i];
            double bq[3], wq;
            quad_point(Q, v.w, bq, wq);
            const double Ga = gs * wq * acc[0];
            double Gn[3], Gc[3];
            for (int d = 0; d < 3; ++d) {
                Gn[d] = gs * q * a * acc[2 + d];
                Gc[d] = gs * a * (q * (n[d] * acc[1] + acc[8 + d]) - p * acc[5 + d]);
            }
            const double nGn = n[0] * Gn[0] + n[1] * Gn[1] + n[2] * Gn[2];
            double gw[3];
            for (int d = 0; d < 3; ++d) gw[d] = 0.5 * Ga * n[d] + (Gn[d] - nGn * n[d]) / wn;
            const int vv[3] = {v.x, v.y, v.z};
            double x[3][3];
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d) x[c][d] = vv[c] >= 0 ? s * X[3 * (int64_t)vv[c] + d] : 0.0;
            for (int c = 0; c < 3; ++c) {
                const double* xj = x[(c + 1) % 3];
                const double* xk = x[(c + 2) % 3];
                const double ed[3] = {xj[0] - xk[0], xj[1] - xk[1], xj[2] - xk[2]};
                const double cr[3] = {ed[1] * gw[2] - ed[2] * gw[1], ed[2] * gw[0] - ed[0] * gw[2],
                                      ed[0] * gw[1] - ed[1] * gw[0]};
                for (int d = 0; d < 3; ++d) {
                    const double g = (Q == 1 ? Gc[d] / 3.0 : bq[c] * Gc[d]) + cr[d];
                    finite &= isfinite(g);
                    corner[9 * i + 3 * c + d] = g;
                }
            }
        }
        if (!finite) atomicOr(flags, (uint32_t)FLAG_NONFINITE);
    }
    energy_part(e, epart);
}

// G[v] = sum over the (sorted face, corner) slots incident to v, in ascending slot order, so the
// sum is deterministic although the list of v is filled in arbitrary order.  Up to GATHER_REG
// slots (every vertex of a regular mesh): the list is read at once, sorted in registers by an
// odd-even transposition network and the corner loads are issued together, one memory round trip
// instead of one per slot.  Longer lists are walked by repeatedly taking the smallest entry above
// the last one taken (slots are distinct).
constexpr int GATHER_REG = 16;

__global__ __launch_bounds__(256) void vertex_gather(const uint32_t* __restrict__ off,
                                                     const uint32_t* __restrict__ list, int64_t V,
                                                     const double* __restrict__ corner, double* __restrict__ G,
                                                     EnergyOut en) {
    if (en.E && blockIdx.x == gridDim.x - 1) {  // the extra work-group: the energy
        energy_total(en);
        return;
    }
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= V) return;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    const uint32_t b = off[v], e = off[v + 1];
    if (e - b <= (uint32_t)GATHER_REG) {
        const int deg = (int)(e - b);
        uint32_t L[GATHER_REG];
#pragma unroll
        for (int k = 0; k < GATHER_REG; ++k) L[k] = k < deg ? list[b + k] : 0xffffffffu;
#pragma unroll
        for (int r = 0; r < GATHER_REG; ++r)
#pragma unroll
            for (int k = r & 1; k + 1 < GATHER_REG; k += 2) {
                const uint32_t lo = min(L[k], L[k + 1]), hi = max(L[k], L[k + 1]);
                L[k] = lo;
                L[k + 1] = hi;
            }
        double c[GATHER_REG][3];
#pragma unroll
        for (int k = 0; k < GATHER_REG; ++k)
            for (int d = 0; d < 3; ++d) c[k][d] = k < deg ? corner[3 * (size_t)L[k] + d] : 0.0;
#pragma unroll
        for (int k = 0; k < GATHER_REG; ++k)
            if (k < deg) {
                g0 += c[k][0];
                g1 += c[k][1];
                g2 += c[k][2];
            }
    } else {
        uint32_t last = 0;
        for (uint32_t n = b; n < e; ++n) {
            uint32_t m = 0xffffffffu;
            for (uint32_t k = b; k < e; ++k) {
                const uint32_t x = list[k];
                if ((n == b || x > last) && x < m) m = x;
            }
            last = m;
            const double* c = corner + 3 * (size_t)m;
            g0 += c[0];
            g1 += c[1];
            g2 += c[2];
        }
    }
    G[3 * v + 0] = g0;
    G[3 * v + 1] = g1;
    G[3 * v + 2] = g2;
}

// Curved cubic elements: one thread per item e < n of `step` consecutive records, all points of one
// element (record i is point perm[i] % Q of element perm[i] / Q): the Q records of an element in
// the exact path (step = Q, records in point order), one record in the far field (step = 1, the
// tree orders points, not elements).  Each record's row sums give dE/dweight, dE/dn and dE/dx of
// its point as in finalize_kernel; with the element's map recomputed at the point,
//     g_J = (dE/dweight) (w / 2) n + (I - n n^T) (dE/dn) / |J|,
//     node k += phi_k dE/dx + (d phi_k / ds) (x_t x g_J) + (d phi_k / dt) (g_J x x_s),
// summed over the item's records in order and written to corner[e][k] (10 x 3 FP64): the gather's
// slot 10 e + k.
template <bool GRAD>
__global__ __launch_bounds__(256) void p3_finalize_kernel(const float* __restrict__ part, Sched sc,
                                                          const double* __restrict__ accs, int64_t Fp, int64_t n,
                                                          int step, int Q, const uint32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ F10, int64_t V,
                                                          const double* __restrict__ X,
                                                          const uint32_t* __restrict__ bbox, double q, double p,
                                                          double scale, double efac, double* __restrict__ corner,
                                                          double* __restrict__ epart, uint32_t* __restrict__ flags) {
    constexpr int NA = GRAD ? NACC : 1;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double en = 0.0;
    const int kexp = norm_exp(bbox);
    const double s = ldexp(1.0, kexp);
    const double gs = scale * pow2i(kexp, p - q - 3.0);
    if (e < n) {
        const int64_t f = perm[e * step] / Q;
        int32_t id[P3_NODES];
        bool ok = true;
        for (int k = 0; k < P3_NODES; ++k) {
            id[k] = F10[P3_NODES * f + k];
            ok &= id[k] >= 0 && id[k] < V;  // (bad ids were reported by the record kernel)
        }
        double g[P3_NODES][3];
        for (int k = 0; k < P3_NODES; ++k) g[k][0] = g[k][1] = g[k][2] = 0.0;
        bool finite = true;
        for (int j = 0; j < step; ++j) {
            const int64_t i = e * step + j;
            const int pt = (int)(perm[i] % Q);
            double acc[NA];
            row_sums<NA, false>(part, sc, accs, Fp, i, acc);
            double b[3], wq;
            quad_point(Q, pt, b, wq);
            double phi[P3_NODES], ds[P3_NODES], dt[P3_NODES];
            p3_shape(b, phi, ds, dt);
            double xs[3] = {0.0, 0.0, 0.0}, xt[3] = {0.0, 0.0, 0.0};
            if (ok)
                for (int k = 0; k < P3_NODES; ++k)
                    for (int d = 0; d < 3; ++d) {
                        const double x = s * X[3 * (int64_t)id[k] + d];
                        xs[d] += ds[k] * x;
                        xt[d] += dt[k] * x;
                    }
            const double J[3] = {xs[1] * xt[2] - xs[2] * xt[1], xs[2] * xt[0] - xs[0] * xt[2],
                                 xs[0] * xt[1] - xs[1] * xt[0]};
            double wn = sqrt(J[0] * J[0] + J[1] * J[1] + J[2] * J[2]);
            if (!(wn > 0.0)) wn = 1.0;  // degenerate: reported by the record kernel
            const double n[3] = {J[0] / wn, J[1] / wn, J[2] / wn};
            const double a = 0.5 * wq * wn;
            for (int k = 0; k < NA; ++k) finite &= isfinite(acc[k]);
            en += (GRAD ? efac : 1.0) * a * acc[0];  // the energy-only row sums hold each pair once
            if (GRAD) {
                const double Ga = gs * wq * acc[0];
                double Gn[3], Gc[3];
                for (int d = 0; d < 3; ++d) {
                    Gn[d] = gs * q * a * acc[2 + d];
                    Gc[d] = gs * a * (q * (n[d] * acc[1] + acc[8 + d]) - p * acc[5 + d]);
                }
                const double nGn = n[0] * Gn[0] + n[1] * Gn[1] + n[2] * Gn[2];
                double gJ[3];
                for (int d = 0; d < 3; ++d) gJ[d] = 0.5 * Ga * n[d] + (Gn[d] - nGn * n[d]) / wn;
                const double cs[3] = {xt[1] * gJ[2] - xt[2] * gJ[1], xt[2] * gJ[0] - xt[0] * gJ[2],
                                      xt[0] * gJ[1] - xt[1] * gJ[0]};
                const double ct[3] = {gJ[1] * xs[2] - gJ[2] * xs[1], gJ[2] * xs[0] - gJ[0] * xs[2],
                                      gJ[0] * xs[1] - gJ[1] * xs[0]};
                for (int k = 0; k < P3_NODES; ++k)
                    for (int d = 0; d < 3; ++d) g[k][d] += phi[k] * Gc[d] + ds[k] * cs[d] + dt[k] * ct[d];
            }
        }
        if (GRAD)
            for (int k = 0; k < P3_NODES; ++k)
                for (int d = 0; d < 3; ++d) {
                    finite &= isfinite(g[k][d]);
                    corner[(size_t)P3_NODES * 3 * e + 3 * k + d] = g[k][d];
                }
        if (!finite) atomicOr(flags, (uint32_t)FLAG_NONFINITE);
    }
    energy_part(en, epart);
}

int finalize_blocks(int64_t nF) { return (int)((nF + 255) / 256); }

// Row sums of the symmetric pair kernel, one thread per (face i, sum k): acc64[k][i] <- the
// segments of the work-groups that cover i's super block (work-group order), then the column
// partials of the symmetric units (I', i's columns) of the earlier super blocks I' (ascending), all
// added in FP64.  Each wave's 64 faces lie in one row block, so the covering work-groups are
// wave-uniform.  With the gradient the kernel's 8 sums K, S0, Sd, V = Sn - 2 Sdd become the 11 of
// the finalize as Sn = V and Sdd = 0 (the finalize uses Sn and Sdd only as q Sn - p Sdd, p = 2q).
template <int NA>
__global__ __launch_bounds__(256) void sym_merge_kernel(const float* __restrict__ part,
                                                        const float* __restrict__ colpart,
                                                        const int* __restrict__ first, SymSched sc, int64_t nR,
                                                        int64_t Fp, double* __restrict__ acc64) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= nR) return;
    int ks = k;  // the kernel's sum that feeds finalize sum k
    if constexpr (NA == NSYM) {
        if (k >= 5 && k < 8) {
            acc64[(size_t)k * Fp + i] = 0.0;
            return;
        }
        ks = k < 5 ? k : k - 3;
    }
    const int rr = (int)(i % ROWB);
    const int rb = __builtin_amdgcn_readfirstlane((int)(i / ROWB));
    const int I = rb / sc.nw, wv = rb % sc.nw;
    const int w0 = __builtin_amdgcn_readfirstlane(sc.wave_of(sc.base(I)));
    const int w1 = __builtin_amdgcn_readfirstlane(sc.wave_of(sc.base(I + 1) - 1));
    // The loops are unrolled so that the loads of several terms are in flight together; the adds
    // stay in order.  Slot w + I of an empty work-group is in bounds but unrelated: its value is
    // dropped.
    double acc = 0.0;
#pragma unroll 8
    for (int w = w0; w <= w1; ++w) {
        const int f = first[w];
        const float v = part[(((size_t)(w + I) * sc.nw + wv) * NA + ks) * ROWB + rr];
        acc += f <= I ? (double)v : 0.0;
    }
    const int J = (int)(i / SYM_COLS), jj = (int)(i % SYM_COLS);
#pragma unroll 8
    for (int Ip = 0; Ip < I; ++Ip)
        acc += (double)colpart[((size_t)(sc.base_sym(Ip) + J - SUB * sc.sbc * (Ip + 1)) * NA + ks) * SYM_COLS + jj];
    acc64[(size_t)k * Fp + i] = acc;
}

hipError_t launch_sym_merge(bool grad, const float* part, const float* colpart, const int* first,
                            const SymSched& sc, int64_t nR, int64_t Fp, double* acc64, hipStream_t st) {
    const dim3 grid((unsigned)((nR + 255) / 256), grad ? NACC : 1);
    if (grad)
        hipLaunchKernelGGL((sym_merge_kernel<NSYM>), grid, dim3(256), 0, st, part, colpart, first, sc, nR, Fp, acc64);
    else
        hipLaunchKernelGGL((sym_merge_kernel<1>), grid, dim3(256), 0, st, part, colpart, first, sc, nR, Fp, acc64);
    return hipGetLastError();
}

// The energy of a finalize (nothing when E is null): summed by its own one-work-group launch, or
// left to the vertex gather that follows (in_gather; the caller passes the same EnergyOut there).
static hipError_t finish_energy(const double* epart, int nb, const uint32_t* bbox, double q, double p, double scale,
                                double* E, EnergyOut* in_gather, hipStream_t st) {
    const EnergyOut en = {epart, nb, bbox, q, p, scale, E};
    if (in_gather) *in_gather = en;
    else if (E) hipLaunchKernelGGL(energy_sum, dim3(1), dim3(256), 0, st, en);
    return hipGetLastError();
}

// Row sums: the pair kernel's segments (part, sc) or, with part null, acc64 (NA x Fp FP64);
// efac: E = efac sum_S a_S K_S with the gradient's row sums (1/2 for the self energy, whose K
// holds both orders of every pair; 1 for the confinement).  epart: finalize_blocks(nF) FP64.
// in_gather: see finish_energy.
hipError_t launch_finalize(bool grad, const float* part, const Sched& sc, int64_t Fp, int64_t nF, const double* acc64,
                           const double* geo, const int4* colv, const double* X, const uint32_t* bbox, double q,
                           double p, double scale, double efac, int Q, double* corner, double* epart,
                           uint32_t* flags, double* E, EnergyOut* in_gather, hipStream_t st) {
    const int nb = finalize_blocks(nF);
    if (grad)
        hipLaunchKernelGGL((finalize_kernel<true>), dim3(nb), dim3(256), 0, st, part, sc, acc64, Fp, nF, geo, colv, X,
                           bbox, q, p, scale, efac, Q, corner, epart, flags);
    else
        hipLaunchKernelGGL((finalize_kernel<false>), dim3(nb), dim3(256), 0, st, part, sc, acc64, Fp, nF, geo, colv, X,
                           bbox, q, p, scale, efac, Q, corner, epart, flags);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : finish_energy(epart, nb, bbox, q, p, scale, E, in_gather, st);
}

// n items of `step` records (see p3_finalize_kernel)
hipError_t launch_p3_finalize(bool grad, const float* part, const Sched& sc, int64_t Fp, int64_t n, int step, int Q,
                              const double* acc64, const uint32_t* perm, const int32_t* F10, int64_t V,
                              const double* X, const uint32_t* bbox, double q, double p, double scale, double efac,
                              double* corner, double* epart, uint32_t* flags, double* E, EnergyOut* in_gather,
                              hipStream_t st) {
    const int nb = finalize_blocks(n);
    if (grad)
        hipLaunchKernelGGL((p3_finalize_kernel<true>), dim3(nb), dim3(256), 0, st, part, sc, acc64, Fp, n, step, Q,
                           perm, F10, V, X, bbox, q, p, scale, efac, corner, epart, flags);
    else
        hipLaunchKernelGGL((p3_finalize_kernel<false>), dim3(nb), dim3(256), 0, st, part, sc, acc64, Fp, n, step, Q,
                           perm, F10, V, X, bbox, q, p, scale, efac, corner, epart, flags);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : finish_energy(epart, nb, bbox, q, p, scale, E, in_gather, st);
}

// en: the energy left to the gather by the finalize (E null: none)
hipError_t launch_gather(const uint32_t* off, const uint32_t* list, int64_t V, const double* corner, double* G,
                         const EnergyOut& en, hipStream_t st) {
    const int nb = (int)((V + 255) / 256) + (en.E ? 1 : 0);
    hipLaunchKernelGGL(vertex_gather, dim3(nb), dim3(256), 0, st, off, list, V, corner, G, en);
    return hipGetLastError();
}

}  // namespace tpe
