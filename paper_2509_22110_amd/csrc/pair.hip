// Exact all-pairs triangle-pair kernel for the tangent-point energy and its per-face adjoint sums.
//
// Definition (paper Sec. 2, eq. (TP), one-point centroid quadrature on flat triangles): for an
// ordered pair of faces (S, T) sharing no vertex, with d = c_S - c_T, w = 1/|d|^2,
//     k(S,T) = |n_S . d|^q / |d|^p = t^q,   t = (n_S . d) w       (the fast path has p = 2q).
// The reordered derivative (paper Sec. 3.3, eq. (dTP_reordered)) evaluates the inner integrals as
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
// MI355X mapping: one wave64 per work-group holds ROWB = 128 row faces (2 per lane) in VGPRs.
// All lanes visit the same column at the same time, so column records are wave-uniform and are
// fetched with scalar loads into SGPRs (one 32-byte record per column); no LDS is needed and every
// VALU instruction takes the column operand straight from an SGPR.  Columns come in tiles of 256
// faces stored relative to an FP64 tile origin; each row re-expresses its centroid relative to
// that origin once per tile, so nearby pairs see small, accurately rounded coordinates.  FP32 sums
// run over CHUNK columns and are folded into Kahan-compensated (hi, lo) FP32 pairs.  Tile pairs in
// which some row shares a vertex with some column (a few percent, faces being in Morton order)
// take a masked variant that compares vertex indices; all other tiles run with no exclusion test.
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

template <int Q, bool GRAD, bool MASK>
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

template <int Q, bool GRAD, bool MASK>
__device__ __forceinline__ void tile_pass(const ColRec* __restrict__ tc, const int4* __restrict__ tv,
                                          const float (&rx)[RPL], const float (&ry)[RPL],
                                          const float (&rz)[RPL], const float (&nx)[RPL],
                                          const float (&ny)[RPL], const float (&nz)[RPL],
                                          const int (&rv)[RPL][3], float (&hi)[RPL][NACC],
                                          float (&lo)[RPL][NACC]) {
    constexpr int NA = GRAD ? NACC : 1;
    for (int c0 = 0; c0 < CTILE; c0 += CHUNK) {
        float acc[RPL][NA];
#pragma unroll
        for (int r = 0; r < RPL; ++r)
#pragma unroll
            for (int k = 0; k < NA; ++k) acc[r][k] = 0.f;
#pragma unroll 4
        for (int j = c0; j < c0 + CHUNK; ++j) {
            const ColRec cr = tc[j];
            int4 cv = make_int4(0, 0, 0, 0);
            if constexpr (MASK) cv = tv[j];
#pragma unroll
            for (int r = 0; r < RPL; ++r)
                pair_update<Q, GRAD, MASK>(cr, cv, rx[r], ry[r], rz[r], nx[r], ny[r], nz[r],
                                           rv[r][0], rv[r][1], rv[r][2], acc[r]);
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r)
#pragma unroll
            for (int k = 0; k < NA; ++k) kahan_fold(acc[r][k], hi[r][k], lo[r][k]);
    }
}

// grid: (n_rowblocks, n_splits); block: one wave.  part layout: [split][2*NA][Fp] FP32, first NA
// rows hold hi, next NA rows hold the compensation to ADD (i.e. -c of Kahan's running error).
template <int Q, bool GRAD>
__global__ __launch_bounds__(WAVE) void pair_kernel(const ColRec* __restrict__ cols,
                                                    const int4* __restrict__ colv,
                                                    const double* __restrict__ c64,
                                                    const double* __restrict__ org,
                                                    const uint32_t* __restrict__ touch, int touch_words,
                                                    int Fp, int ntiles, int tiles_per_split,
                                                    float* __restrict__ part) {
    constexpr int NA = GRAD ? NACC : 1;
    const int lane = threadIdx.x;
    const int rb = blockIdx.x;
    const int split = blockIdx.y;
    const int t0 = split * tiles_per_split;
    const int t1 = min(ntiles, t0 + tiles_per_split);

    double cxd[RPL], cyd[RPL], czd[RPL];
    float nx[RPL], ny[RPL], nz[RPL];
    int rv[RPL][3];
    float hi[RPL][NACC], lo[RPL][NACC];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = rb * ROWB + r * WAVE + lane;
        cxd[r] = c64[3 * (size_t)i + 0];
        cyd[r] = c64[3 * (size_t)i + 1];
        czd[r] = c64[3 * (size_t)i + 2];
        const ColRec me = cols[i];
        nx[r] = me.nx; ny[r] = me.ny; nz[r] = me.nz;
        const int4 v = colv[i];
        rv[r][0] = v.x; rv[r][1] = v.y; rv[r][2] = v.z;
#pragma unroll
        for (int k = 0; k < NACC; ++k) { hi[r][k] = 0.f; lo[r][k] = 0.f; }
    }
    const uint32_t* my_touch = touch + (size_t)rb * touch_words;
    for (int t = t0; t < t1; ++t) {
        const double ox = org[3 * t + 0], oy = org[3 * t + 1], oz = org[3 * t + 2];
        float rx[RPL], ry[RPL], rz[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            rx[r] = (float)(cxd[r] - ox);
            ry[r] = (float)(cyd[r] - oy);
            rz[r] = (float)(czd[r] - oz);
        }
        const bool masked = (my_touch[t >> 5] >> (t & 31)) & 1u;
        const ColRec* tc = cols + (size_t)t * CTILE;
        const int4* tv = colv + (size_t)t * CTILE;
        if (masked)
            tile_pass<Q, GRAD, true>(tc, tv, rx, ry, rz, nx, ny, nz, rv, hi, lo);
        else
            tile_pass<Q, GRAD, false>(tc, tv, rx, ry, rz, nx, ny, nz, rv, hi, lo);
    }
    float* out = part + (size_t)split * 2 * NA * Fp;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = rb * ROWB + r * WAVE + lane;
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            out[(size_t)k * Fp + i] = hi[r][k];
            out[(size_t)(NA + k) * Fp + i] = -lo[r][k];
        }
    }
}

// Host-side launchers (declared in kernels.hpp).
hipError_t launch_pair(bool grad, const ColRec* cols, const int4* colv, const double* c64,
                       const double* org, const uint32_t* touch, int touch_words, int Fp, int ntiles,
                       int tiles_per_split, int nsplits, float* part, hipStream_t st) {
    dim3 grid(Fp / ROWB, nsplits);
    if (grad)
        hipLaunchKernelGGL((pair_kernel<6, true>), grid, dim3(WAVE), 0, st, cols, colv, c64, org,
                           touch, touch_words, Fp, ntiles, tiles_per_split, part);
    else
        hipLaunchKernelGGL((pair_kernel<6, false>), grid, dim3(WAVE), 0, st, cols, colv, c64, org,
                           touch, touch_words, Fp, ntiles, tiles_per_split, part);
    return hipGetLastError();
}

}  // namespace tpe
