// Exact all-pairs triangle-pair kernel for the tangent-point energy and its per-face adjoint sums.
//
// Definition (paper Sec. 2.2.2, eq. (TP), one-point centroid quadrature on flat triangles): for an
// ordered pair of faces (S, T) sharing no vertex, with d = c_S - c_T, w = 1/|d|^2,
//     k(S,T) = |n_S . d|^q / |d|^p = t^q,   t = (n_S . d) w       (the fast path has p = 2q).
// The reordered derivative (paper Sec. 3.2, eq. (dTP_reordered)) evaluates the inner integrals as
// functions of the outer point only, so every row face S can collect everything its own gradient
// needs from a loop over columns T, with no writes to other faces.  With tau = (n_T . d) w,
// s = a_T t^(q-1) w,  s' = a_T tau^(q-1) w  the row sums are
//     K   = sum a_T (t^q + tau^q)            -> dE/da_S   (f_K: forward + reverse kernel)
//     S0  = sum s                            -> forward d/dc_S, along n_S
//     Sd  = sum s d                          -> dE/dn_S   (f_nu)
//     Sdd = sum a_T w (t^q + tau^q) d        -> forward + reverse d/dc_S, along d
//     Sn  = sum s' n_T                       -> reverse d/dc_S, along n_T
// (11 scalars).  The finalize pass turns them into corner gradients in FP64.
//
// MI355X mapping: every wave64 holds a row block of ROWB = 128 row faces (2 per lane) in VGPRs.
// The launch is persistent and balanced (see Sched in common.hpp) over work-groups of PAIR_NW
// waves: the waves of a work-group take contiguous quarters of the same row block's column range
// and hand their compensated sums to wave 0 through LDS, which folds them into its own and writes
// one partial-sum segment for the work-group (a quarter of the segment traffic of one-wave groups).
// All lanes visit the same column at the same time, so column records are wave-uniform and are
// fetched with scalar loads into SGPRs (one 32-byte record per column); every VALU instruction
// takes the column operand straight from an SGPR.  Columns come in chunks of 64 faces stored
// relative to an FP64 origin at the centre of the chunk's centroid box; each row re-expresses its
// centroid relative to that origin once per chunk, so nearby pairs see small, accurately rounded
// coordinates (what limits the accuracy of nearly touching pairs).  FP32 sums
// run over CHUNK columns and are folded into Kahan-compensated (hi, lo) FP32 pairs.  (Row block,
// chunk) pairs in which some row shares a vertex with some column (a few percent, faces being in
// Morton order) take a masked variant that compares vertex indices; all others run with no
// exclusion test.
#include <algorithm>

#include "common.hpp"

namespace tpe {

template <int Q>
__device__ __forceinline__ void powq(float t, float& tq1, float& tq) {
    if constexpr (Q == 6) {
        float t2 = t * t;
        float t4 = t2 * t2;
        tq1 = t4 * t;
        tq = tq1 * t;
    } else {
        float r = 1.f;
#pragma unroll
        for (int i = 0; i < Q - 1; ++i) r *= t;
        tq1 = r;
        tq = r * t;
    }
}

template <int Q>
__device__ __forceinline__ float powq_only(float t) {
    if constexpr (Q == 6) {
        float t2 = t * t;
        float t3 = t2 * t;
        return t3 * t3;
    } else {
        float r = 1.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) r *= t;
        return r;
    }
}

__device__ __forceinline__ void kahan_fold(float x, float& hi, float& c) {
    float y = x - c;
    float t = hi + y;
    c = (t - hi) - y;
    hi = t;
}

// CONF: the column is a face of a fixed confining surface (paper Sec. 2.2.3, eq. (TPConf)): only
// the row's normal enters and the pair counts once, so only the forward terms are summed (K, S0,
// Sd, and Sdd with t^q alone; Sn stays 0).
template <int Q, bool GRAD, bool MASK, bool CONF = false>
__device__ __forceinline__ void pair_update(const ColRec& cr, int4 cv, float rx, float ry, float rz,
                                            float nx, float ny, float nz, int v0, int v1, int v2,
                                            float* acc) {
    float dx = rx - cr.cx, dy = ry - cr.cy, dz = rz - cr.cz;
    float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    float w = __builtin_amdgcn_rcpf(r2);
    if constexpr (MASK) {
        bool ex = (v0 == cv.x) | (v0 == cv.y) | (v0 == cv.z) | (v1 == cv.x) | (v1 == cv.y) |
                  (v1 == cv.z) | (v2 == cv.x) | (v2 == cv.y) | (v2 == cv.z);
        w = ex ? 0.f : w;
    }
    float u = fmaf(nz, dz, fmaf(ny, dy, nx * dx));
    float t = u * w;
    if constexpr (!GRAD) {
        acc[0] = fmaf(cr.a, powq_only<Q>(t), acc[0]);
    } else if constexpr (CONF) {
        float t5, t6;
        powq<Q>(t, t5, t6);
        float aw = cr.a * w;
        float s = aw * t5;
        float m = aw * t6;
        acc[0] = fmaf(cr.a, t6, acc[0]);
        acc[1] += s;
        acc[2] = fmaf(s, dx, acc[2]);
        acc[3] = fmaf(s, dy, acc[3]);
        acc[4] = fmaf(s, dz, acc[4]);
        acc[5] = fmaf(m, dx, acc[5]);
        acc[6] = fmaf(m, dy, acc[6]);
        acc[7] = fmaf(m, dz, acc[7]);
    } else {
        float v = fmaf(cr.nz, dz, fmaf(cr.ny, dy, cr.nx * dx));
        float tau = v * w;
        float t5, t6, s5, s6;
        powq<Q>(t, t5, t6);
        powq<Q>(tau, s5, s6);
        float aw = cr.a * w;
        float s = aw * t5;
        float sp = aw * s5;
        float e = t6 + s6;
        float m = aw * e;
        acc[0] = fmaf(cr.a, e, acc[0]);
        acc[1] += s;
        acc[2] = fmaf(s, dx, acc[2]);
        acc[3] = fmaf(s, dy, acc[3]);
        acc[4] = fmaf(s, dz, acc[4]);
        acc[5] = fmaf(m, dx, acc[5]);
        acc[6] = fmaf(m, dy, acc[6]);
        acc[7] = fmaf(m, dz, acc[7]);
        acc[8] = fmaf(sp, cr.nx, acc[8]);
        acc[9] = fmaf(sp, cr.ny, acc[9]);
        acc[10] = fmaf(sp, cr.nz, acc[10]);
    }
}

// Other exponents (the generic path): even q = Q and even p with q < p <= 2q.  With t = u w and
// m = p/2 - q <= 0 the kernel is k = t^q w^m and s = a t^(q-1) w^(m+1): the fast path's sums with
// w^m = (|d|^2)^(-m) folded in (mneg = -m multiplications per pair).
template <int Q, bool GRAD, bool MASK>
__device__ __forceinline__ void pair_update_gen(const ColRec& cr, int4 cv, float rx, float ry, float rz, float nx,
                                                float ny, float nz, int v0, int v1, int v2, int mneg, float* acc) {
    float dx = rx - cr.cx, dy = ry - cr.cy, dz = rz - cr.cz;
    float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    float w = __builtin_amdgcn_rcpf(r2);
    if constexpr (MASK) {
        bool ex = (v0 == cv.x) | (v0 == cv.y) | (v0 == cv.z) | (v1 == cv.x) | (v1 == cv.y) |
                  (v1 == cv.z) | (v2 == cv.x) | (v2 == cv.y) | (v2 == cv.z);
        w = ex ? 0.f : w;
    }
    float wm = 1.f;
    for (int j = 0; j < mneg; ++j) wm *= r2;
    if constexpr (MASK) wm = w == 0.f ? 0.f : wm;
    float u = fmaf(nz, dz, fmaf(ny, dy, nx * dx));
    float t = u * w;
    float tq1, tq;
    powq<Q>(t, tq1, tq);
    if constexpr (!GRAD) {
        acc[0] = fmaf(cr.a, tq * wm, acc[0]);
    } else {
        float v = fmaf(cr.nz, dz, fmaf(cr.ny, dy, cr.nx * dx));
        float tau = v * w;
        float sq1, sq;
        powq<Q>(tau, sq1, sq);
        float aw = cr.a * w * wm;
        float s = aw * tq1;
        float sp = aw * sq1;
        float e = tq + sq;
        float m = aw * e;
        acc[0] = fmaf(cr.a * wm, e, acc[0]);
        acc[1] += s;
        acc[2] = fmaf(s, dx, acc[2]);
        acc[3] = fmaf(s, dy, acc[3]);
        acc[4] = fmaf(s, dz, acc[4]);
        acc[5] = fmaf(m, dx, acc[5]);
        acc[6] = fmaf(m, dy, acc[6]);
        acc[7] = fmaf(m, dz, acc[7]);
        acc[8] = fmaf(sp, cr.nx, acc[8]);
        acc[9] = fmaf(sp, cr.ny, acc[9]);
        acc[10] = fmaf(sp, cr.nz, acc[10]);
    }
}

// One chunk of CHUNK columns for the wave's RPL x 64 rows: plain FP32 sums over the chunk, then a
// Kahan fold into the rows' (hi, lo) accumulators.
template <int Q, bool GRAD, bool MASK, bool CONF = false, bool GEN = false>
__device__ __forceinline__ void chunk_pass(int mneg, const ColRec* __restrict__ tc, const int4* __restrict__ tv,
                                           const float (&rx)[RPL], const float (&ry)[RPL],
                                           const float (&rz)[RPL], const float (&nx)[RPL],
                                           const float (&ny)[RPL], const float (&nz)[RPL],
                                           const int (&rv)[RPL][3], float (&hi)[RPL][NACC],
                                           float (&lo)[RPL][NACC]) {
    constexpr int NA = GRAD ? NACC : 1;
    float acc[RPL][NA];
#pragma unroll
    for (int r = 0; r < RPL; ++r)
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[r][k] = 0.f;
#pragma unroll 4
    for (int j = 0; j < CHUNK; ++j) {
        const ColRec cr = tc[j];
        int4 cv = make_int4(0, 0, 0, 0);
        if constexpr (MASK) cv = tv[j];
#pragma unroll
        for (int r = 0; r < RPL; ++r)
            if constexpr (GEN)
                pair_update_gen<Q, GRAD, MASK>(cr, cv, rx[r], ry[r], rz[r], nx[r], ny[r], nz[r], rv[r][0], rv[r][1],
                                               rv[r][2], mneg, acc[r]);
            else
                pair_update<Q, GRAD, MASK, CONF>(cr, cv, rx[r], ry[r], rz[r], nx[r], ny[r], nz[r], rv[r][0],
                                                 rv[r][1], rv[r][2], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r)
#pragma unroll
        for (int k = 0; k < NA; ++k) kahan_fold(acc[r][k], hi[r][k], lo[r][k]);
}

// grid: W work-groups of PAIR_NW waves.  part layout: [W * maxseg segments][2 * NA][ROWB] FP32;
// the first NA rows of a segment hold hi, the next NA the compensation to add (the work-group's
// waves' compensated sums folded into wave 0's).
// Rows come from (rcols, rc64, rcolv), columns from (ccols, ccolv, corg): the same arrays for the
// self energy, the confining surface's for CONF (no exclusion map then).
template <int Q, bool GRAD, bool CONF = false, bool GEN = false>
__global__ __launch_bounds__(WAVE * PAIR_NW) void pair_kernel(const ColRec* __restrict__ rcols,
                                                              const double* __restrict__ rc64,
                                                              const int4* __restrict__ rcolv,
                                                              const ColRec* __restrict__ ccols,
                                                              const int4* __restrict__ ccolv,
                                                              const double* __restrict__ corg,
                                                              const uint32_t* __restrict__ touch, int touch_words,
                                                              Sched sc, float* __restrict__ part, int mneg) {
    constexpr int NA = GRAD ? NACC : 1;
    constexpr int CPT = CTILE / CHUNK;  // chunks per tile
    // waves 1.. hand their (hi, -c) to wave 0: [PAIR_NW - 1][2 NA][ROWB] floats of dynamic LDS (static
    // LDS of this size makes the compiler give up on occupancy and spend registers)
    extern __shared__ float red_lds[];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);  // wave-uniform (SGPR)
    const int g = blockIdx.x;
    int64_t u = sc.begin(g);
    const int64_t u1 = sc.begin(g + 1);
    int seg = 0;
    while (u < u1) {  // uniform over the work-group
        const int rb = (int)(u / sc.upr);
        const int64_t uend = min(u1, (int64_t)(rb + 1) * sc.upr);
        const int64_t len = uend - u;
        const int64_t my0 = u + len * wave / PAIR_NW, my1 = u + len * (wave + 1) / PAIR_NW;
        double cxd[RPL], cyd[RPL], czd[RPL];
        float nx[RPL], ny[RPL], nz[RPL];
        int rv[RPL][3];
        float hi[RPL][NACC], lo[RPL][NACC];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = rb * ROWB + r * WAVE + lane;
            cxd[r] = rc64[3 * (size_t)i + 0];
            cyd[r] = rc64[3 * (size_t)i + 1];
            czd[r] = rc64[3 * (size_t)i + 2];
            const ColRec me = rcols[i];
            nx[r] = me.nx; ny[r] = me.ny; nz[r] = me.nz;
            const int4 v = rcolv[i];
            rv[r][0] = v.x; rv[r][1] = v.y; rv[r][2] = v.z;
#pragma unroll
            for (int k = 0; k < NACC; ++k) { hi[r][k] = 0.f; lo[r][k] = 0.f; }
        }
        const uint32_t* my_touch = CONF ? nullptr : touch + (size_t)rb * touch_words;
        int cur_t = -1;
        float rx[RPL], ry[RPL], rz[RPL];
        for (int64_t x = my0; x < my1; ++x) {
            const int cu = (int)(x - (int64_t)rb * sc.upr);
            const int t = cu / CPT;
            if (t != cur_t) {
                // rows relative to this tile's FP64 origin (columns are stored relative to it)
                const double ox = corg[3 * t + 0], oy = corg[3 * t + 1], oz = corg[3 * t + 2];
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    rx[r] = (float)(cxd[r] - ox);
                    ry[r] = (float)(cyd[r] - oy);
                    rz[r] = (float)(czd[r] - oz);
                }
                cur_t = t;
            }
            const ColRec* tc = ccols + (size_t)cu * CHUNK;
            const int4* tv = ccolv + (size_t)cu * CHUNK;
            if constexpr (CONF) {
                chunk_pass<Q, GRAD, false, true>(mneg, tc, tv, rx, ry, rz, nx, ny, nz, rv, hi, lo);
            } else {
                const bool masked = (my_touch[cu >> 5] >> (cu & 31)) & 1u;
                if (masked)
                    chunk_pass<Q, GRAD, true, false, GEN>(mneg, tc, tv, rx, ry, rz, nx, ny, nz, rv, hi, lo);
                else
                    chunk_pass<Q, GRAD, false, false, GEN>(mneg, tc, tv, rx, ry, rz, nx, ny, nz, rv, hi, lo);
            }
        }
        if (wave > 0) {
            float* mine = red_lds + (size_t)(wave - 1) * 2 * NA * ROWB + lane;
#pragma unroll
            for (int r = 0; r < RPL; ++r)
#pragma unroll
                for (int k = 0; k < NA; ++k) {
                    mine[k * ROWB + r * WAVE] = hi[r][k];
                    mine[(NA + k) * ROWB + r * WAVE] = -lo[r][k];
                }
        }
        __syncthreads();
        if (wave == 0) {
            // compensated FP32 sum of the four waves' (hi, -c) pairs, in wave order
            const float* theirs = red_lds + lane;
            float* out = part + ((size_t)g * sc.maxseg + seg) * 2 * NA * ROWB + lane;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
#pragma unroll
                for (int k = 0; k < NA; ++k) {
#pragma unroll
                    for (int j = 0; j < PAIR_NW - 1; ++j) {
                        kahan_fold(theirs[(j * 2 * NA + k) * ROWB + r * WAVE], hi[r][k], lo[r][k]);
                        kahan_fold(theirs[(j * 2 * NA + NA + k) * ROWB + r * WAVE], hi[r][k], lo[r][k]);
                    }
                    out[(size_t)k * ROWB + r * WAVE] = hi[r][k];
                    out[(size_t)(NA + k) * ROWB + r * WAVE] = -lo[r][k];
                }
                // one row's LDS loads in flight at a time (keeps the register count at the loop's)
                asm volatile("" ::: "memory");
            }
        }
        __syncthreads();
        u = uend;
        ++seg;
    }
}

static size_t pair_lds_bytes(bool grad) { return sizeof(float) * (PAIR_NW - 1) * 2 * (grad ? NACC : 1) * ROWB; }

int pair_blocks_per_cu(bool grad) {
    int nb = 0;
    hipError_t e = grad ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pair_kernel<6, true>, WAVE * PAIR_NW,
                                                                       pair_lds_bytes(true))
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pair_kernel<6, false>, WAVE * PAIR_NW,
                                                                       pair_lds_bytes(false));
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

// rows_p padded rows (multiple of ROWB) against cols_p padded columns (multiple of CHUNK)
Sched make_sched(int64_t rows_p, int64_t cols_p, int waves) {
    Sched sc;
    const int nrb = (int)(rows_p / ROWB);
    sc.upr = (int)(cols_p / CHUNK);
    sc.U = (int64_t)nrb * sc.upr;
    sc.W = (int)std::max<int64_t>(1, std::min<int64_t>(waves, sc.U));
    const int64_t per = (sc.U + sc.W - 1) / sc.W;
    sc.maxseg = (int)((per + sc.upr - 1) / sc.upr) + 1;
    return sc;
}

int64_t pair_part_floats(const Sched& sc, bool grad) {
    return (int64_t)sc.W * sc.maxseg * 2 * (grad ? NACC : 1) * ROWB;
}

template <int Q, bool GEN>
static void launch_pair_q(bool grad, const ColRec* cols, const int4* colv, const double* c64, const double* org,
                          const uint32_t* touch, int touch_words, const Sched& sc, float* part, int mneg,
                          hipStream_t st) {
    if (grad)
        hipLaunchKernelGGL((pair_kernel<Q, true, false, GEN>), dim3(sc.W), dim3(WAVE * PAIR_NW), pair_lds_bytes(true),
                           st, cols, c64, colv, cols, colv, org, touch, touch_words, sc, part, mneg);
    else
        hipLaunchKernelGGL((pair_kernel<Q, false, false, GEN>), dim3(sc.W), dim3(WAVE * PAIR_NW),
                           pair_lds_bytes(false), st, cols, c64, colv, cols, colv, org, touch, touch_words, sc, part,
                           mneg);
}

// (q, p) = (6, 12) runs the fast kernel; other supported exponents (see pair_exponents_ok) the
// generic one.
bool pair_exponents_ok(int q, int p) { return (q == 2 || q == 4 || q == 6 || q == 8) && p % 2 == 0 && p > q && p <= 2 * q; }

hipError_t launch_pair(bool grad, int q, int p, const ColRec* cols, const int4* colv, const double* c64,
                       const double* org, const uint32_t* touch, int touch_words, const Sched& sc, float* part,
                       hipStream_t st) {
    const int mneg = q - p / 2;
    if (q == 6 && p == 12) launch_pair_q<6, false>(grad, cols, colv, c64, org, touch, touch_words, sc, part, 0, st);
    else if (q == 2) launch_pair_q<2, true>(grad, cols, colv, c64, org, touch, touch_words, sc, part, mneg, st);
    else if (q == 4) launch_pair_q<4, true>(grad, cols, colv, c64, org, touch, touch_words, sc, part, mneg, st);
    else if (q == 6) launch_pair_q<6, true>(grad, cols, colv, c64, org, touch, touch_words, sc, part, mneg, st);
    else if (q == 8) launch_pair_q<8, true>(grad, cols, colv, c64, org, touch, touch_words, sc, part, mneg, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// Confinement: rows (moving surface) against the confining surface's columns; the energy-only
// kernel is the self kernel's (forward term only) without exclusion.
hipError_t launch_pair_conf(bool grad, const ColRec* rcols, const double* rc64, const int4* rcolv,
                            const ColRec* ccols, const int4* ccolv, const double* corg, const Sched& sc, float* part,
                            hipStream_t st) {
    if (grad)
        hipLaunchKernelGGL((pair_kernel<6, true, true>), dim3(sc.W), dim3(WAVE * PAIR_NW), pair_lds_bytes(true), st,
                           rcols, rc64, rcolv, ccols, ccolv, corg, nullptr, 0, sc, part, 0);
    else
        hipLaunchKernelGGL((pair_kernel<6, false, true>), dim3(sc.W), dim3(WAVE * PAIR_NW), pair_lds_bytes(false),
                           st, rcols, rc64, rcolv, ccols, ccolv, corg, nullptr, 0, sc, part, 0);
    return hipGetLastError();
}

}  // namespace tpe
