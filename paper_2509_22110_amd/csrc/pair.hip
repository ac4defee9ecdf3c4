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
// All lanes visit the same column at the same time, so column records are wave-uniform: each
// chunk's 64 records (32 bytes each) are loaded once, one per lane, into the wave's LDS slots and
// read back column by column as broadcasts (the same bits as scalar loads into SGPRs, and faster:
// 93.8 against 101.0 ms at 327,680 faces).  Columns come in chunks of 64 faces stored
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
// FOLDV (gradient only): fold the chunk's sums into the symmetric kernel's 8-sum layout K, S0,
// Sd, V = Sn - 2 Sdd (see pair_sym_kernel) instead of the 11 row sums; with GEN, V = Sn + vcoef
// Sdd, vcoef = -p/q.
template <int Q, bool GRAD, bool MASK, bool CONF = false, bool GEN = false, bool FOLDV = false, int UNR = 4, int NH>
__device__ __forceinline__ void chunk_pass(int mneg, const ColRec* __restrict__ tc, const int4* __restrict__ tv,
                                           const float (&rx)[RPL], const float (&ry)[RPL],
                                           const float (&rz)[RPL], const float (&nx)[RPL],
                                           const float (&ny)[RPL], const float (&nz)[RPL],
                                           const int (&rv)[RPL][3], float (&hi)[RPL][NH],
                                           float (&lo)[RPL][NH], float vcoef = -2.f) {
    static_assert(NH == ((FOLDV && GRAD) ? 8 : NACC) || !GRAD, "row sum layout");
    constexpr int NA = GRAD ? NACC : 1;
    float acc[RPL][NA];
#pragma unroll
    for (int r = 0; r < RPL; ++r)
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[r][k] = 0.f;
#pragma unroll UNR
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
    for (int r = 0; r < RPL; ++r) {
        if constexpr (FOLDV && GRAD) {
#pragma unroll
            for (int k = 0; k < 5; ++k) kahan_fold(acc[r][k], hi[r][k], lo[r][k]);
#pragma unroll
            for (int d = 0; d < 3; ++d)
                kahan_fold(fmaf(GEN ? vcoef : -2.f, acc[r][5 + d], acc[r][8 + d]), hi[r][5 + d], lo[r][5 + d]);
        } else {
#pragma unroll
            for (int k = 0; k < NA; ++k) kahan_fold(acc[r][k], hi[r][k], lo[r][k]);
        }
    }
}

// grid: W work-groups of PAIR_NW waves.  part layout: [W * maxseg segments][2 * NA][ROWB] FP32;
// the first NA rows of a segment hold hi, the next NA the compensation to add (the work-group's
// waves' compensated sums folded into wave 0's).
// Rows come from (rcols, rc64, rcolv), columns from (ccols, ccolv, corg): the same arrays for the
// self energy, the confining surface's for CONF (no exclusion map then).
// LDS floats of one wave's column slots: CHUNK records and their vertex ids
constexpr int PAIR_STAGE_FLOATS = CHUNK * (int)((sizeof(ColRec) + sizeof(int4)) / sizeof(float));
static_assert(CHUNK == WAVE, "one column record per lane");
// columns per unrolled step of the row kernel: the columns now come from LDS into VGPRs
constexpr int PAIR_UNR = 2;
static_assert(PAIR_STAGE_FLOATS <= 2 * NACC * ROWB, "slots inside a wave's hand-over area");

template <int Q, bool GRAD, bool CONF = false, bool GEN = false>
// at least 4 waves per SIMD (128 VGPRs): the few values the generic kernel then keeps in scratch are
// touched once per chunk, outside the column loop
__global__ __launch_bounds__(WAVE * PAIR_NW) __attribute__((amdgpu_waves_per_eu(4))) void pair_kernel(const ColRec* __restrict__ rcols,
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
    // the wave's column slots: with the gradient wave w > 0 uses its own hand-over area (written
    // only after its last chunk of a segment, read by wave 0 between the segment's two barriers) and
    // wave 0 the space after them; without it every wave's slots follow the hand-over areas
    float* stg = red_lds + (size_t)(PAIR_NW - 1) * 2 * NA * ROWB;
    if constexpr (GRAD) stg = wave == 0 ? stg : red_lds + (size_t)(wave - 1) * 2 * NA * ROWB;
    else stg += (size_t)wave * PAIR_STAGE_FLOATS;
    ColRec* scol = reinterpret_cast<ColRec*>(stg);
    int4* sver = reinterpret_cast<int4*>(stg + CHUNK * (sizeof(ColRec) / sizeof(float)));
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
            const bool masked = !CONF && ((my_touch[cu >> 5] >> (cu & 31)) & 1u);
            {
                // the chunk's records (one per lane; the column arrays are padded to whole chunks)
                // through the wave's LDS slots, read back column by column as broadcasts
                const float4* src = reinterpret_cast<const float4*>(ccols + (size_t)cu * CHUNK + lane);
                const float4 c0 = src[0], c1 = src[1];
                int4 v = make_int4(0, 0, 0, 0);
                if (masked) v = ccolv[(size_t)cu * CHUNK + lane];
                asm volatile("" ::: "memory");  // the previous chunk's reads of the slots come first
                float4* dst = reinterpret_cast<float4*>(scol + lane);
                dst[0] = c0;
                dst[1] = c1;
                if (masked) sver[lane] = v;
                asm volatile("" ::: "memory");  // the reads below see every lane's record
            }
            if constexpr (CONF) {
                chunk_pass<Q, GRAD, false, true, false, false, PAIR_UNR>(mneg, scol, sver, rx, ry, rz, nx, ny, nz, rv, hi, lo);
            } else {
                if (masked)
                    chunk_pass<Q, GRAD, true, false, GEN, false, PAIR_UNR>(mneg, scol, sver, rx, ry, rz, nx, ny, nz, rv, hi, lo);
                else
                    chunk_pass<Q, GRAD, false, false, GEN, false, PAIR_UNR>(mneg, scol, sver, rx, ry, rz, nx, ny, nz, rv, hi, lo);
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

// ---------------------------------------------------------------------------------------------
// Symmetric kernel (self energy, (q, p) = (6, 12)): every unordered pair {S, T} of faces in
// different super blocks is evaluated once, by the wave that holds S as a row, and credited to both
// faces.  The reversed ordered pair (T, S) has d -> -d and t <-> -tau, so with
//     T1 = w t^(q-1),  U1 = w tau^(q-1),  e = t^q + tau^q   (q - 1 odd)
// the row face S collects, with weight a_T,
//     K += a_T e, S0 += a_T T1, Sd += a_T T1 d, Sdd += a_T w e d, Sn += a_T U1 n_T,
// and the column face T, with weight a_S,
//     K += a_S e, S0 -= a_S U1, Sd += a_S U1 d, Sdd -= a_S w e d, Sn -= a_S T1 n_S,
// i.e. exactly what T's own row pass over S would add.  The energy-only kernel credits a_T t^q to
// S and a_S tau^q to T (each ordered pair's forward kernel, as the row-only energy kernel sums).
// The shared part of a pair (d, w, t, tau and their powers) is computed once instead of twice.
// Sn and Sdd only reach the gradient through dE/dc = a (q (n S0 + Sn) - p Sdd), so each face keeps
// 8 sums, K, S0, Sd and V = Sn - (p/q) Sdd = Sn - 2 Sdd, and the merge hands the finalize
// Sn = V, Sdd = 0: three fewer column sums to carry through the wave per step.
//
// Layout of a symmetric unit on one wave: the 128 rows stay in the lanes (2 per lane) as in the
// row-only kernel; the unit's SYM_COLS columns are held one per lane too (SYM_COLS = 64: one per
// lane of the wave; 16: one per lane of each row of 16 lanes), lane l taking column
// (l + j) mod SYM_COLS at step j from LDS.  A column's sums travel with it: after every step they
// move one lane down (a DPP wave or row rotation fused into the add of the step's contributions), so
// after the SYM_COLS steps every lane holds the sums of one column over the rows of its group of
// lanes, and the work-group adds the (64 / SYM_COLS) x NW partial sums of each column in LDS,
// without any cross-lane reduction.

// Shared part of the pair (row face, column face) for the symmetric kernel.  Energy only: e = t^q
// (the row face's kernel) and we = tau^q (the column face's), since the energy-only row sums hold
// the forward kernel alone.
struct SymPair {
    float dx, dy, dz, e, we, T1, U1;
};

// Other even exponents (GEN; q = Q, p even with q < p <= 2q): with m = p/2 - q <= 0 the pair's
// factor |d|^(-2m) = (|d|^2)^mneg, mneg = -m, multiplies every term (as in pair_update_gen), and
// the column record's wv = -2 a weighs the Sdd part of V = Sn - (p/q) Sdd once `we` carries the
// factor wscale = p / (2q); the chunk passes of the diagonal units fold V with vcoef = -p/q.
struct SymExp {
    int mneg;
    float wscale, vcoef;
};

template <bool GRAD, bool MASK, int Q = 6, bool GEN = false, int MNEG = 0>
__device__ __forceinline__ SymPair sym_pair(const ColRec& cr, int4 cv, float rx, float ry, float rz, float nx,
                                            float ny, float nz, int v0, int v1, int v2, const SymExp& ex) {
    SymPair P;
    P.dx = rx - cr.cx; P.dy = ry - cr.cy; P.dz = rz - cr.cz;
    float r2 = fmaf(P.dz, P.dz, fmaf(P.dy, P.dy, P.dx * P.dx));
    float w = __builtin_amdgcn_rcpf(r2);
    if constexpr (MASK) {
        bool ex = (v0 == cv.x) | (v0 == cv.y) | (v0 == cv.z) | (v1 == cv.x) | (v1 == cv.y) |
                  (v1 == cv.z) | (v2 == cv.x) | (v2 == cv.y) | (v2 == cv.z);
        w = ex ? 0.f : w;
    }
    float u = fmaf(nz, P.dz, fmaf(ny, P.dy, nx * P.dx));
    float v = fmaf(cr.nz, P.dz, fmaf(cr.ny, P.dy, cr.nx * P.dx));
    float t = u * w, tau = v * w;
    if constexpr (GEN) {
        // a masked pair has w = 0, hence t = tau = 0 and every term 0 whatever wm is
        float wm = 1.f;
#pragma unroll
        for (int j = 0; j < MNEG; ++j) wm *= r2;
        float tq1, tq, sq1, sq;
        powq<Q>(t, tq1, tq);
        powq<Q>(tau, sq1, sq);
        if constexpr (!GRAD) {
            P.e = wm * tq;
            P.we = wm * sq;
        } else {
            const float ww = w * wm, es = tq + sq;
            P.T1 = ww * tq1;
            P.U1 = ww * sq1;
            P.e = wm * es;
            P.we = ex.wscale * ww * es;
        }
    } else if constexpr (!GRAD) {
        float t3 = t * t * t, s3 = tau * tau * tau;
        P.e = t3 * t3;
        P.we = s3 * s3;
    } else {
        float t2 = t * t, t4 = t2 * t2, t5 = t4 * t;
        float s2 = tau * tau, s4 = s2 * s2, s5 = s4 * tau;
        P.T1 = w * t5;
        P.U1 = w * s5;
        P.e = fmaf(t5, t, s5 * tau);
        P.we = w * P.e;
    }
    return P;
}

// the row face's share, weight a_T = cr.a (cr.wv = -2 a_T for the Sdd part of V)
template <bool GRAD>
__device__ __forceinline__ void sym_row(const ColRec& cr, const SymPair& P, float* acc) {
    acc[0] = fmaf(cr.a, P.e, acc[0]);
    if constexpr (GRAD) {
        float s = cr.a * P.T1;
        acc[1] += s;
        acc[2] = fmaf(s, P.dx, acc[2]);
        acc[3] = fmaf(s, P.dy, acc[3]);
        acc[4] = fmaf(s, P.dz, acc[4]);
        float m2 = cr.wv * P.we;
        float sp = cr.a * P.U1;
        acc[5] = fmaf(sp, cr.nx, fmaf(m2, P.dx, acc[5]));
        acc[6] = fmaf(sp, cr.ny, fmaf(m2, P.dy, acc[6]));
        acc[7] = fmaf(sp, cr.nz, fmaf(m2, P.dz, acc[7]));
    }
}

// x moved down by one lane within each group of SYM_COLS lanes, the group's last lane taking its
// first lane's value (DPP wave_rol:1 for 64, row_ror:15 for 16), plus y
__device__ __forceinline__ float rot_add(float x, float y) {
    static_assert(SYM_COLS == 64 || SYM_COLS == 16, "rotation over the wave or over rows of 16 lanes");
    constexpr int ctrl = SYM_COLS == 64 ? 0x134 : 0x12F;
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xf, 0xf, false)) + y;
}

// The column face's share of the step's two pairs (rows 0 and 1 of the lane, weights a_S; aS2 =
// 2 a_S), added to the column sums after moving them one lane down (ROT; the first step has
// nothing to move).  For the column, Sn -= a_S T1 n_S and Sdd -= a_S w e d, so V gains
// -a_S T1 n_S + 2 a_S w e d.
template <bool GRAD, bool ROT>
__device__ __forceinline__ void sym_col(const SymPair& P0, const SymPair& P1, float aS0, float aS1, float aS20,
                                        float aS21, float nx0, float ny0, float nz0, float nx1, float ny1, float nz1,
                                        float* ca) {
    float c[GRAD ? NSYM : 1];
    if constexpr (!GRAD) {
        c[0] = fmaf(aS1, P1.we, aS0 * P0.we);
    } else {
        c[0] = fmaf(aS1, P1.e, aS0 * P0.e);
        const float y0 = aS0 * P0.U1, y1 = aS1 * P1.U1;
        const float z0 = aS20 * P0.we, z1 = aS21 * P1.we;
        const float x0 = aS0 * P0.T1, x1 = aS1 * P1.T1;
        c[1] = -y0 - y1;
        c[2] = fmaf(y1, P1.dx, y0 * P0.dx);
        c[3] = fmaf(y1, P1.dy, y0 * P0.dy);
        c[4] = fmaf(y1, P1.dz, y0 * P0.dz);
        c[5] = fmaf(-x1, nx1, fmaf(z1, P1.dx, fmaf(-x0, nx0, z0 * P0.dx)));
        c[6] = fmaf(-x1, ny1, fmaf(z1, P1.dy, fmaf(-x0, ny0, z0 * P0.dy)));
        c[7] = fmaf(-x1, nz1, fmaf(z1, P1.dz, fmaf(-x0, nz0, z0 * P0.dz)));
    }
#pragma unroll
    for (int k = 0; k < (GRAD ? NSYM : 1); ++k) ca[k] = ROT ? rot_add(ca[k], c[k]) : c[k];
}

template <bool GRAD, bool MASK, bool ROT, int Q = 6, bool GEN = false, int MNEG = 0>
__device__ __forceinline__ void sym_step(const ColRec& cr, int4 cv, const float (&rx)[RPL], const float (&ry)[RPL],
                                         const float (&rz)[RPL], const float (&nx)[RPL], const float (&ny)[RPL],
                                         const float (&nz)[RPL], const float (&aS)[RPL], const float (&aS2)[RPL],
                                         const int (&rv)[RPL][3], float (&acc)[RPL][GRAD ? NSYM : 1], float* ca,
                                         const SymExp& ex) {
    static_assert(RPL == 2, "the column share is written for two rows per lane");
    const SymPair P0 = sym_pair<GRAD, MASK, Q, GEN, MNEG>(cr, cv, rx[0], ry[0], rz[0], nx[0], ny[0], nz[0], rv[0][0],
                                                    rv[0][1], rv[0][2], ex);
    const SymPair P1 = sym_pair<GRAD, MASK, Q, GEN, MNEG>(cr, cv, rx[1], ry[1], rz[1], nx[1], ny[1], nz[1], rv[1][0],
                                                    rv[1][1], rv[1][2], ex);
    sym_row<GRAD>(cr, P0, acc[0]);
    sym_row<GRAD>(cr, P1, acc[1]);
    sym_col<GRAD, ROT>(P0, P1, aS[0], aS[1], aS2[0], aS2[1], nx[0], ny[0], nz[0], nx[1], ny[1], nz[1], ca);
}

// One symmetric unit for the wave: its rows against the SYM_COLS columns staged in LDS (lcol, lv).
// Row sums are folded into (hi, lo) as in chunk_pass; on return lane l holds in ca the sums of
// column (l + SYM_COLS - 1) mod SYM_COLS over the rows of its group of SYM_COLS lanes.
template <bool GRAD, bool MASK, int Q = 6, bool GEN = false, int MNEG = 0>
__device__ __forceinline__ void sym_chunk_pass(const ColRec* lcol, const int4* lv, const float (&rx)[RPL],
                                               const float (&ry)[RPL], const float (&rz)[RPL],
                                               const float (&nx)[RPL], const float (&ny)[RPL],
                                               const float (&nz)[RPL], const float (&aS)[RPL],
                                               const float (&aS2)[RPL], const int (&rv)[RPL][3],
                                               float (&hi)[RPL][NSYM], float (&lo)[RPL][NSYM], float* ca,
                                               const SymExp& ex = SymExp{0, 1.f, -2.f}) {
    constexpr int NA = GRAD ? NSYM : 1;
    const int sl = threadIdx.x & (SYM_COLS - 1);
    float acc[RPL][NA];
#pragma unroll
    for (int r = 0; r < RPL; ++r)
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[r][k] = 0.f;
    {
        const ColRec cr = lcol[sl];
        const int4 cv = MASK ? lv[sl] : make_int4(0, 0, 0, 0);
        sym_step<GRAD, MASK, false, Q, GEN, MNEG>(cr, cv, rx, ry, rz, nx, ny, nz, aS, aS2, rv, acc, ca, ex);
    }
    // steps 1 .. SYM_COLS - 1, two per iteration (SYM_COLS - 1 is odd: the last one after the loop)
#pragma unroll 1
    for (int j = 1; j < SYM_COLS - 1; j += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int col = (sl + j + h) & (SYM_COLS - 1);
            const ColRec cr = lcol[col];
            const int4 cv = MASK ? lv[col] : make_int4(0, 0, 0, 0);
            sym_step<GRAD, MASK, true, Q, GEN, MNEG>(cr, cv, rx, ry, rz, nx, ny, nz, aS, aS2, rv, acc, ca, ex);
        }
    }
    {
        const int col = (sl + SYM_COLS - 1) & (SYM_COLS - 1);
        const ColRec cr = lcol[col];
        const int4 cv = MASK ? lv[col] : make_int4(0, 0, 0, 0);
        sym_step<GRAD, MASK, true, Q, GEN, MNEG>(cr, cv, rx, ry, rz, nx, ny, nz, aS, aS2, rv, acc, ca, ex);
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r)
#pragma unroll
        for (int k = 0; k < NA; ++k) kahan_fold(acc[r][k], hi[r][k], lo[r][k]);
}

// LDS of the symmetric kernel's work-group: two column buffers (records, vertex ids) and two column
// reduction buffers [NW][WAVE / SYM_COLS][SYM_COLS][CS] (CS = NSYM with the gradient).
template <bool GRAD>
constexpr int sym_cs() { return GRAD ? NSYM : 1; }
template <bool GRAD, int NW>
constexpr size_t sym_lds_floats() {
    return 2 * (size_t)SYM_COLS * (8 + 4) + 2 * (size_t)NW * WAVE * sym_cs<GRAD>();
}

// grid: W work-groups of NW = sc.nw waves (see SymSched).  part: [W + nsb][NW][NA][ROWB] FP32, one
// segment per (work-group g, super block I it touches) at slot g + I (the slots of consecutive
// work-groups do not overlap: each super block after a work-group's first adds one slot), each wave
// writing its own row block's compensated sums rounded to FP32 (hi minus the compensation).  colpart:
// [symmetric unit][NA][SYM_COLS] FP32, the sums of the unit's NW * ROWB rows for each of its columns, added
// over the waves and rows of lanes in a fixed order.
// first[w]: the first super block of work-group w (INT32_MAX if its range is empty).
template <bool GRAD, int NW>
// At least 4 waves per SIMD (128 VGPRs, against 165 unconstrained): the compiler then keeps a few
// long-lived values (FP64 row centroids, vertex ids) in scratch, reloaded once per super block,
// and the column loop is unchanged.
__global__ __launch_bounds__(WAVE * NW) __attribute__((amdgpu_waves_per_eu(4))) void pair_sym_kernel(const ColRec* __restrict__ cols,
                                                                 const double* __restrict__ c64,
                                                                 const int4* __restrict__ colv,
                                                                 const double* __restrict__ corg,
                                                                 const uint32_t* __restrict__ touch, int touch_words,
                                                                 SymSched sc, float* __restrict__ part,
                                                                 float* __restrict__ colpart, int* __restrict__ first) {
    constexpr int NA = GRAD ? NSYM : 1;
    constexpr int CS = sym_cs<GRAD>();
    constexpr int SBC = NW * ROWB / CHUNK;  // equals sc.sbc
    extern __shared__ float lds[];
    ColRec* lcol = reinterpret_cast<ColRec*>(lds);                 // [2][SYM_COLS]
    int4* lvid = reinterpret_cast<int4*>(lds + 2 * SYM_COLS * 8);  // [2][SYM_COLS]
    float* red = lds + 2 * SYM_COLS * 12;                          // [2][NW][WAVE][CS]
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int g = blockIdx.x;
    int64_t u = sc.begin(g);
    const int64_t u1 = sc.begin(g + 1);
    if (u >= u1) {  // uniform over the work-group; an empty range (more work-groups than units)
        if (threadIdx.x == 0) first[g] = INT32_MAX;
        return;
    }
    int I = sc.block_of(u);
    if (threadIdx.x == 0) first[g] = I;
    int64_t k = u - sc.base(I);
    // staging of a unit's columns: SYM_COLS columns x 12 dwords (record, vertex ids); thread t
    // moves SPT consecutive dwords of column t / TPC (TPC threads per column)
    constexpr int NT = WAVE * NW;
    constexpr int TPC = NT / SYM_COLS < 12 ? NT / SYM_COLS : 12;
    constexpr int SPT = 12 / TPC;
    static_assert(TPC * SPT == 12 && SYM_COLS * TPC <= NT, "staging layout");
    const bool stager = threadIdx.x < SYM_COLS * TPC;
    const int sc_col = threadIdx.x / TPC, sc_d0 = SPT * (threadIdx.x % TPC);
    auto stage_load = [&](int slice, float (&reg)[SPT]) {
        if (!stager) return;
        const size_t c = (size_t)slice * SYM_COLS + sc_col;
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int d = sc_d0 + q;
            reg[q] = d < 8 ? reinterpret_cast<const float*>(cols + c)[d]
                           : reinterpret_cast<const float*>(colv + c)[d - 8];
        }
    };
    auto stage_store = [&](int b, const float (&reg)[SPT]) {
        if (!stager) return;
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int d = sc_d0 + q;
            if (d < 8) reinterpret_cast<float*>(lcol + b * SYM_COLS + sc_col)[d] = reg[q];
            else reinterpret_cast<float*>(lvid + b * SYM_COLS + sc_col)[d - 8] = reg[q];
        }
    };
    int nsym = 0;  // symmetric units done by this work-group
    float pre[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) pre[q] = 0.f;
    // the SYM_COLS-column slice of symmetric unit k >= SBC of super block I
    auto slice_of = [&](int I_, int64_t k_) { return SUB * SBC * (I_ + 1) + (int)(k_ - SBC); };
    if (k >= SBC) {  // the range starts on a symmetric unit: stage it now
        stage_load(slice_of(I, k), pre);
        stage_store(0, pre);
        __syncthreads();
    }
    while (u < u1) {  // uniform over the work-group
        const int rb = I * NW + wave;
        double cxd[RPL], cyd[RPL], czd[RPL];
        float nx[RPL], ny[RPL], nz[RPL], aS[RPL], aS2[RPL];
        int rv[RPL][3];
        float hi[RPL][NSYM], lo[RPL][NSYM];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = rb * ROWB + r * WAVE + lane;
            cxd[r] = c64[3 * (size_t)i + 0];
            cyd[r] = c64[3 * (size_t)i + 1];
            czd[r] = c64[3 * (size_t)i + 2];
            const ColRec me = cols[i];
            nx[r] = me.nx; ny[r] = me.ny; nz[r] = me.nz; aS[r] = me.a; aS2[r] = -me.wv;
            const int4 v = colv[i];
            rv[r][0] = v.x; rv[r][1] = v.y; rv[r][2] = v.z;
#pragma unroll
            for (int a = 0; a < NSYM; ++a) { hi[r][a] = 0.f; lo[r][a] = 0.f; }
        }
        const uint32_t* my_touch = touch + (size_t)rb * touch_words;
        const int64_t kn = sc.ua() - sc.ud() * I;  // units of super block I
        const int64_t kend = min(kn, k + (u1 - u));
        for (; k < kend; ++k, ++u) {
            // chunk of the unit (diagonal: the unit's columns; symmetric: the chunk of its slice)
            const int J = k < SBC ? SBC * I + (int)k : slice_of(I, k) / SUB;
            // the next unit of the range, if symmetric (a super block starts with diagonal units)
            const bool next_sym = u + 1 < u1 && k + 1 < kn && k + 1 >= SBC;
            if (next_sym) stage_load(slice_of(I, k + 1), pre);
            // rows relative to the chunk's FP64 origin (its columns are stored relative to it)
            const double ox = corg[3 * J + 0], oy = corg[3 * J + 1], oz = corg[3 * J + 2];
            float rx[RPL], ry[RPL], rz[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                rx[r] = (float)(cxd[r] - ox);
                ry[r] = (float)(cyd[r] - oy);
                rz[r] = (float)(czd[r] - oz);
            }
            const bool masked = (my_touch[J >> 5] >> (J & 31)) & 1u;
            if (k < SBC) {
                const ColRec* tc = cols + (size_t)J * CHUNK;
                const int4* tv = colv + (size_t)J * CHUNK;
                if (masked) chunk_pass<6, GRAD, true, false, false, true>(0, tc, tv, rx, ry, rz, nx, ny, nz, rv, hi, lo);
                else chunk_pass<6, GRAD, false, false, false, true>(0, tc, tv, rx, ry, rz, nx, ny, nz, rv, hi, lo);
                if (next_sym) {
                    stage_store(nsym & 1, pre);
                    __syncthreads();
                }
            } else {
                const int b = nsym & 1;
                float ca[NA];
                if (masked)
                    sym_chunk_pass<GRAD, true>(lcol + b * SYM_COLS, lvid + b * SYM_COLS, rx, ry, rz, nx, ny, nz, aS,
                                               aS2, rv, hi, lo, ca);
                else
                    sym_chunk_pass<GRAD, false>(lcol + b * SYM_COLS, lvid + b * SYM_COLS, rx, ry, rz, nx, ny, nz,
                                                aS, aS2, rv, hi, lo, ca);
                // lane l holds column (l + SYM_COLS - 1) mod SYM_COLS of its group of lanes l / SYM_COLS
                const int mycol = (lane + SYM_COLS - 1) & (SYM_COLS - 1);
                float* mine = red + (((size_t)(b * NW + wave) * (WAVE / SYM_COLS) + lane / SYM_COLS) * SYM_COLS +
                                     mycol) * CS;
#pragma unroll
                for (int a = 0; a < NA; ++a) mine[a] = ca[a];
                if (next_sym) stage_store(b ^ 1, pre);
                // Buffers: unit s reads chunk buffer s & 1 and writes reduction buffer s & 1; the
                // next symmetric unit's chunk goes to the other buffer, whose last reader (unit s - 1)
                // finished before the previous barrier, and reduction buffer s & 1 is written again
                // by unit s + 2 only after the barrier of unit s + 1, which every wave reaches after
                // its reads below.
                __syncthreads();
                const float* rbuf = red + (size_t)b * NW * WAVE * CS;
                float* out = colpart + (size_t)(sc.base_sym(I) + k - SBC) * NA * SYM_COLS;
                for (int e = threadIdx.x; e < NA * SYM_COLS; e += NT) {
                    const int a = e / SYM_COLS, j = e % SYM_COLS;
                    float sum = 0.f;
#pragma unroll
                    for (int w = 0; w < NW * (WAVE / SYM_COLS); ++w) sum += rbuf[(w * SYM_COLS + j) * CS + a];
                    out[e] = sum;
                }
                ++nsym;
            }
        }
        float* o = part + ((size_t)(g + I) * NW + wave) * NA * ROWB + lane;
#pragma unroll
        for (int r = 0; r < RPL; ++r)
#pragma unroll
            for (int a = 0; a < NA; ++a) o[(size_t)a * ROWB + r * WAVE] = hi[r][a] - lo[r][a];
        ++I;
        k = 0;
    }
}

// The same kernel without work-group barriers (NW >= 2).  With barriers every wave waits at each
// unit for the slowest one, and the waves of a SIMD progress at different rates (the oldest
// first): 70.3 ms at 327,680 faces with 4 waves against 64.8 with 1.  Here each wave stages its
// own copy of a unit's columns (LDS [NW][SYM_COLS], 48 B a column) and the work-group's column
// partial goes through a ring of SYM_RING slots: every wave writes its column sums into the
// unit's slot and counts itself in (an LDS atomic after its writes), and the wave that arrives
// last adds the NW contributions in wave order (the bits of the barrier kernel) and writes the
// partial, then frees the slot (count reset, then the slot's use counter advanced).  A wave
// waits only before reusing a slot whose previous unit is not yet reduced, i.e. when it is
// SYM_RING units ahead of the slowest wave of its work-group; the slowest wave never waits, so
// every wait ends.  The wait is bounded all the same (FLAG_SYNC and a wrong result beyond it).
constexpr int SYM_RING = 3;
constexpr uint32_t SYM_SPIN_LIMIT = 1u << 22;  // sleeps of 2 x 64 cycles, about 0.2 s

template <bool GRAD, int NW>
constexpr size_t sym_free_lds_floats() {
    return (size_t)NW * SYM_COLS * (8 + 4) + (size_t)SYM_RING * NW * WAVE * sym_cs<GRAD>() + 2 * SYM_RING;
}

template <bool GRAD, int NW, int Q, bool GEN, int MNEG>
__device__ __forceinline__ void sym_free_body(const ColRec* __restrict__ cols, const double* __restrict__ c64,
                                              const int4* __restrict__ colv, const double* __restrict__ corg,
                                              const uint32_t* __restrict__ touch, int touch_words, const SymSched& sc,
                                              float* __restrict__ part, float* __restrict__ colpart,
                                              int* __restrict__ first, uint32_t* __restrict__ flags,
                                              const SymExp& ex) {
    static_assert(NW >= 2 && WAVE == SYM_COLS, "one column per lane, several waves");
    constexpr int NA = GRAD ? NSYM : 1;
    constexpr int CS = sym_cs<GRAD>();
    constexpr int SBC = NW * ROWB / CHUNK;  // equals sc.sbc
    extern __shared__ float lds[];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    ColRec* lcol = reinterpret_cast<ColRec*>(lds) + wave * SYM_COLS;                  // [NW][SYM_COLS]
    int4* lvid = reinterpret_cast<int4*>(lds + NW * SYM_COLS * 8) + wave * SYM_COLS;  // [NW][SYM_COLS]
    float* ring = lds + NW * SYM_COLS * 12;                                           // [SYM_RING][NW][WAVE][CS]
    uint32_t* arrived = reinterpret_cast<uint32_t*>(ring + SYM_RING * NW * WAVE * CS);  // [SYM_RING]
    uint32_t* done = arrived + SYM_RING;                                                // [SYM_RING] uses completed
    const int g = blockIdx.x;
    int64_t u = sc.begin(g);
    const int64_t u1 = sc.begin(g + 1);
    if (u >= u1) {  // uniform over the work-group; an empty range (more work-groups than units)
        if (threadIdx.x == 0) first[g] = INT32_MAX;
        return;
    }
    if (threadIdx.x < 2 * SYM_RING) arrived[threadIdx.x] = 0u;  // arrived and done
    __syncthreads();  // the only barrier
    int I = sc.block_of(u);
    if (threadIdx.x == 0) first[g] = I;
    int64_t k = u - sc.base(I);
    auto slice_of = [&](int I_, int64_t k_) { return SUB * SBC * (I_ + 1) + (int)(k_ - SBC); };
    uint32_t nsym = 0;  // symmetric units done by this wave (the same sequence in every wave)
    bool timed_out = false;
    while (u < u1) {
        const int rb = I * NW + wave;
        double cxd[RPL], cyd[RPL], czd[RPL];
        float nx[RPL], ny[RPL], nz[RPL], aS[RPL], aS2[RPL];
        int rv[RPL][3];
        float hi[RPL][NSYM], lo[RPL][NSYM];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = rb * ROWB + r * WAVE + lane;
            cxd[r] = c64[3 * (size_t)i + 0];
            cyd[r] = c64[3 * (size_t)i + 1];
            czd[r] = c64[3 * (size_t)i + 2];
            const ColRec me = cols[i];
            nx[r] = me.nx; ny[r] = me.ny; nz[r] = me.nz; aS[r] = me.a; aS2[r] = -me.wv;
            const int4 v = colv[i];
            rv[r][0] = v.x; rv[r][1] = v.y; rv[r][2] = v.z;
#pragma unroll
            for (int a = 0; a < NSYM; ++a) { hi[r][a] = 0.f; lo[r][a] = 0.f; }
        }
        const uint32_t* my_touch = touch + (size_t)rb * touch_words;
        const int64_t kn = sc.ua() - sc.ud() * I;  // units of super block I
        const int64_t kend = min(kn, k + (u1 - u));
        for (; k < kend; ++k, ++u) {
            const int J = k < SBC ? SBC * I + (int)k : slice_of(I, k) / SUB;
            const double ox = corg[3 * J + 0], oy = corg[3 * J + 1], oz = corg[3 * J + 2];
            float rx[RPL], ry[RPL], rz[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                rx[r] = (float)(cxd[r] - ox);
                ry[r] = (float)(cyd[r] - oy);
                rz[r] = (float)(czd[r] - oz);
            }
            const bool masked = (my_touch[J >> 5] >> (J & 31)) & 1u;
            if (k < SBC) {
                const ColRec* tc = cols + (size_t)J * CHUNK;
                const int4* tv = colv + (size_t)J * CHUNK;
                if (masked)
                    chunk_pass<Q, GRAD, true, false, GEN, true>(ex.mneg, tc, tv, rx, ry, rz, nx, ny, nz, rv, hi, lo,
                                                                ex.vcoef);
                else
                    chunk_pass<Q, GRAD, false, false, GEN, true>(ex.mneg, tc, tv, rx, ry, rz, nx, ny, nz, rv, hi, lo,
                                                                 ex.vcoef);
                continue;
            }
            // this wave's copy of the unit's columns (lane l: column l); the compiler fences keep
            // the previous unit's reads of the copy before these writes and these writes before the
            // reads below (LDS operations of one wave complete in order)
            {
                const size_t c = (size_t)slice_of(I, k) * SYM_COLS + lane;
                const ColRec cr = cols[c];
                const int4 cv = colv[c];
                asm volatile("" ::: "memory");
                lcol[lane] = cr;
                lvid[lane] = cv;
                asm volatile("" ::: "memory");
            }
            float ca[NA];
            if (masked)
                sym_chunk_pass<GRAD, true, Q, GEN, MNEG>(lcol, lvid, rx, ry, rz, nx, ny, nz, aS, aS2, rv, hi, lo, ca, ex);
            else
                sym_chunk_pass<GRAD, false, Q, GEN, MNEG>(lcol, lvid, rx, ry, rz, nx, ny, nz, aS, aS2, rv, hi, lo, ca, ex);
            // the unit's slot: wait until its previous use (unit nsym - SYM_RING) has been reduced
            const uint32_t slot = nsym % SYM_RING, use = nsym / SYM_RING;
            for (uint32_t it = 0; !timed_out; ++it) {
                if (__hip_atomic_load(&done[slot], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == use) break;
                if (it >= SYM_SPIN_LIMIT) timed_out = true;
                __builtin_amdgcn_s_sleep(2);
            }
            float* mine = ring + (((size_t)slot * NW + wave) * WAVE + ((lane + SYM_COLS - 1) & (SYM_COLS - 1))) * CS;
#pragma unroll
            for (int a = 0; a < NA; ++a) mine[a] = ca[a];
            uint32_t before = 0u;
            if (lane == 0)  // after the wave's writes (release), counted once per wave
                before = __hip_atomic_fetch_add(&arrived[slot], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            before = __builtin_amdgcn_readfirstlane(before);
            if (before == (uint32_t)(NW - 1)) {  // the last wave: reduce in wave order, free the slot
                const float* rbuf = ring + (size_t)slot * NW * WAVE * CS;
                float* out = colpart + (size_t)(sc.base_sym(I) + k - SBC) * NA * SYM_COLS;
                for (int e = lane; e < NA * SYM_COLS; e += WAVE) {
                    const int a = e / SYM_COLS, j = e % SYM_COLS;
                    float sum = 0.f;
#pragma unroll
                    for (int w = 0; w < NW; ++w) sum += rbuf[(w * SYM_COLS + j) * CS + a];
                    out[e] = sum;
                }
                if (lane == 0) {
                    __hip_atomic_store(&arrived[slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_store(&done[slot], use + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
            ++nsym;
        }
        float* o = part + ((size_t)(g + I) * NW + wave) * NA * ROWB + lane;
#pragma unroll
        for (int r = 0; r < RPL; ++r)
#pragma unroll
            for (int a = 0; a < NA; ++a) o[(size_t)a * ROWB + r * WAVE] = hi[r][a] - lo[r][a];
        ++I;
        k = 0;
    }
    if (timed_out && lane == 0) atomicOr(flags, (uint32_t)FLAG_SYNC);
}

template <bool GRAD, int NW>
__global__ __launch_bounds__(WAVE * NW) __attribute__((amdgpu_waves_per_eu(4))) void pair_sym_free_kernel(
    const ColRec* __restrict__ cols, const double* __restrict__ c64, const int4* __restrict__ colv,
    const double* __restrict__ corg, const uint32_t* __restrict__ touch, int touch_words, SymSched sc,
    float* __restrict__ part, float* __restrict__ colpart, int* __restrict__ first, uint32_t* __restrict__ flags) {
    sym_free_body<GRAD, NW, 6, false, 0>(cols, c64, colv, corg, touch, touch_words, sc, part, colpart, first, flags,
                                      SymExp{0, 1.f, -2.f});
}

// The same kernel for the other even exponents (q = Q, p = 2 (Q - MNEG) with q < p <= 2q; ex
// from launch_pair_sym): the pair terms of pair_update_gen, every unordered pair once.
template <bool GRAD, int NW, int Q, int MNEG>
__global__ __launch_bounds__(WAVE * NW) __attribute__((amdgpu_waves_per_eu(4))) void pair_sym_free_gen_kernel(
    const ColRec* __restrict__ cols, const double* __restrict__ c64, const int4* __restrict__ colv,
    const double* __restrict__ corg, const uint32_t* __restrict__ touch, int touch_words, SymSched sc,
    float* __restrict__ part, float* __restrict__ colpart, int* __restrict__ first, uint32_t* __restrict__ flags,
    SymExp ex) {
    sym_free_body<GRAD, NW, Q, true, MNEG>(cols, c64, colv, corg, touch, touch_words, sc, part, colpart, first, flags,
                                           ex);
}

template <int NW>
static size_t pair_sym_lds_bytes(bool grad) {
    return sizeof(float) * (grad ? sym_lds_floats<true, NW>() : sym_lds_floats<false, NW>());
}

template <int NW>
static int sym_blocks_per_cu(bool grad) {
    int nb = 0;
    hipError_t e = grad ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pair_sym_kernel<true, NW>, WAVE * NW,
                                                                       pair_sym_lds_bytes<NW>(true))
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pair_sym_kernel<false, NW>, WAVE * NW,
                                                                       pair_sym_lds_bytes<NW>(false));
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

template <int NW>
static size_t pair_sym_free_lds_bytes(bool grad) {
    return sizeof(float) * (grad ? sym_free_lds_floats<true, NW>() : sym_free_lds_floats<false, NW>());
}

template <int NW>
static int sym_free_blocks_per_cu(bool grad) {
    int nb = 0;
    hipError_t e = grad ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pair_sym_free_kernel<true, NW>,
                                                                       WAVE * NW, pair_sym_free_lds_bytes<NW>(true))
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pair_sym_free_kernel<false, NW>,
                                                                       WAVE * NW, pair_sym_free_lds_bytes<NW>(false));
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

// resident work-groups per CU of the symmetric kernel with nw waves per work-group (1, 2, 4; 8
// without barriers), with barriers or without (decoupled, nw >= 2)
int pair_sym_blocks_per_cu(bool grad, int nw, bool decoupled) {
    if (decoupled && nw == 2) return sym_free_blocks_per_cu<2>(grad);
    if (decoupled && nw == 4) return sym_free_blocks_per_cu<4>(grad);
    if (decoupled && nw == 8) return sym_free_blocks_per_cu<8>(grad);
    if (nw == 8) return 0;  // 8 waves only without barriers
    return nw == 1 ? sym_blocks_per_cu<1>(grad) : nw == 2 ? sym_blocks_per_cu<2>(grad) : sym_blocks_per_cu<4>(grad);
}

// Fp padded faces (a multiple of nw * ROWB); W work-groups of nw waves in equal parts, plus `tail`
// work-groups of about one unit each at the end (dropped when that would be more than half the cost)
SymSched make_sym_sched(int64_t Fp, int W, int tail, int nw) {
    SymSched sc;
    sc.nw = nw;
    sc.sbc = nw * ROWB / CHUNK;
    sc.nsb = (int)(Fp / ((int64_t)nw * ROWB));
    sc.nch = (int)(Fp / CHUNK);
    sc.U = sc.base(sc.nsb);
    sc.C = (int64_t)SYM_COST * sc.U + (int64_t)(DIAG_COST - SYM_COST) * sc.sbc * sc.nsb;
    const int64_t Ct = (int64_t)SYM_COST * std::max(tail, 0);
    if (tail > 0 && 2 * Ct <= sc.C && (int64_t)W + tail <= sc.U) {
        sc.W1 = std::max(W, 1);
        sc.W = sc.W1 + tail;
        sc.C1 = sc.C - Ct;
    } else {
        sc.W = (int)std::max<int64_t>(1, std::min<int64_t>(W, sc.U));
        sc.W1 = sc.W;
        sc.C1 = sc.C;
    }
    return sc;
}

int64_t sym_part_floats(const SymSched& sc, bool grad) {
    return ((int64_t)sc.W + sc.nsb) * sc.nw * (grad ? NSYM : 1) * ROWB;
}
int64_t sym_colpart_floats(const SymSched& sc, bool grad) {
    return sc.base_sym(sc.nsb) * (grad ? NSYM : 1) * SYM_COLS;
}

template <int NW>
static void launch_sym_nw(bool grad, const ColRec* cols, const int4* colv, const double* c64, const double* org,
                          const uint32_t* touch, int touch_words, const SymSched& sc, float* part, float* colpart,
                          int* first, hipStream_t st) {
    if (grad)
        hipLaunchKernelGGL((pair_sym_kernel<true, NW>), dim3(sc.W), dim3(WAVE * NW), pair_sym_lds_bytes<NW>(true), st,
                           cols, c64, colv, org, touch, touch_words, sc, part, colpart, first);
    else
        hipLaunchKernelGGL((pair_sym_kernel<false, NW>), dim3(sc.W), dim3(WAVE * NW), pair_sym_lds_bytes<NW>(false),
                           st, cols, c64, colv, org, touch, touch_words, sc, part, colpart, first);
}

template <int NW>
static void launch_sym_free_nw(bool grad, const ColRec* cols, const int4* colv, const double* c64, const double* org,
                               const uint32_t* touch, int touch_words, const SymSched& sc, float* part, float* colpart,
                               int* first, uint32_t* flags, hipStream_t st) {
    if (grad)
        hipLaunchKernelGGL((pair_sym_free_kernel<true, NW>), dim3(sc.W), dim3(WAVE * NW), pair_sym_free_lds_bytes<NW>(true),
                           st, cols, c64, colv, org, touch, touch_words, sc, part, colpart, first, flags);
    else
        hipLaunchKernelGGL((pair_sym_free_kernel<false, NW>), dim3(sc.W), dim3(WAVE * NW),
                           pair_sym_free_lds_bytes<NW>(false), st, cols, c64, colv, org, touch, touch_words, sc, part,
                           colpart, first, flags);
}

template <int NW, int Q, int MNEG>
static void launch_sym_free_gen(bool grad, const ColRec* cols, const int4* colv, const double* c64, const double* org,
                                const uint32_t* touch, int touch_words, const SymSched& sc, float* part,
                                float* colpart, int* first, uint32_t* flags, const SymExp& ex, hipStream_t st) {
    if (grad)
        hipLaunchKernelGGL((pair_sym_free_gen_kernel<true, NW, Q, MNEG>), dim3(sc.W), dim3(WAVE * NW),
                           pair_sym_free_lds_bytes<NW>(true), st, cols, c64, colv, org, touch, touch_words, sc, part,
                           colpart, first, flags, ex);
    else
        hipLaunchKernelGGL((pair_sym_free_gen_kernel<false, NW, Q, MNEG>), dim3(sc.W), dim3(WAVE * NW),
                           pair_sym_free_lds_bytes<NW>(false), st, cols, c64, colv, org, touch, touch_words, sc, part,
                           colpart, first, flags, ex);
}

// (q, mneg) of the even exponents other than (6, 12): q in {2, 4, 6, 8}, 0 <= mneg < q / 2
template <int NW>
static hipError_t launch_sym_free_q(bool grad, int q, int mneg, const ColRec* cols, const int4* colv,
                                    const double* c64, const double* org, const uint32_t* touch, int touch_words,
                                    const SymSched& sc, float* part, float* colpart, int* first, uint32_t* flags,
                                    const SymExp& ex, hipStream_t st) {
#define TPE_SYM_GEN(QQ, MM)                                                                                         \
    if (q == QQ && mneg == MM) {                                                                                   \
        launch_sym_free_gen<NW, QQ, MM>(grad, cols, colv, c64, org, touch, touch_words, sc, part, colpart, first, \
                                        flags, ex, st);                                                          \
        return hipSuccess;                                                                                       \
    }
    TPE_SYM_GEN(2, 0)
    TPE_SYM_GEN(4, 0)
    TPE_SYM_GEN(4, 1)
    TPE_SYM_GEN(6, 1)
    TPE_SYM_GEN(6, 2)
    TPE_SYM_GEN(8, 0)
    TPE_SYM_GEN(8, 1)
    TPE_SYM_GEN(8, 2)
    TPE_SYM_GEN(8, 3)
#undef TPE_SYM_GEN
    return hipErrorInvalidValue;
}

// The symmetric kernel of the other even exponents runs without barriers, with 4 or 8 waves.
bool pair_sym_gen_ok(int nw, bool decoupled) { return decoupled && (nw == 4 || nw == 8); }

// decoupled: the kernel without work-group barriers (nw >= 2; the same bits).  (q, p) other than
// (6, 12): pair_sym_free_gen_kernel (pair_sym_gen_ok must hold).
hipError_t launch_pair_sym(bool grad, int q, int p, const ColRec* cols, const int4* colv, const double* c64,
                           const double* org, const uint32_t* touch, int touch_words, const SymSched& sc, float* part,
                           float* colpart, int* first, bool decoupled, uint32_t* flags, hipStream_t st) {
    if (q != 6 || p != 12) {
        if (!pair_sym_gen_ok(sc.nw, decoupled)) return hipErrorInvalidValue;
        const SymExp ex = {q - p / 2, (float)p / (float)(2 * q), -(float)p / (float)q};
        const hipError_t e = sc.nw == 4 ? launch_sym_free_q<4>(grad, q, ex.mneg, cols, colv, c64, org, touch,
                                                               touch_words, sc, part, colpart, first, flags, ex, st)
                                        : launch_sym_free_q<8>(grad, q, ex.mneg, cols, colv, c64, org, touch,
                                                               touch_words, sc, part, colpart, first, flags, ex, st);
        return e != hipSuccess ? e : hipGetLastError();
    }
    if (decoupled && sc.nw == 2)
        launch_sym_free_nw<2>(grad, cols, colv, c64, org, touch, touch_words, sc, part, colpart, first, flags, st);
    else if (decoupled && sc.nw == 4)
        launch_sym_free_nw<4>(grad, cols, colv, c64, org, touch, touch_words, sc, part, colpart, first, flags, st);
    else if (decoupled && sc.nw == 8)
        launch_sym_free_nw<8>(grad, cols, colv, c64, org, touch, touch_words, sc, part, colpart, first, flags, st);
    else if (sc.nw == 1) launch_sym_nw<1>(grad, cols, colv, c64, org, touch, touch_words, sc, part, colpart, first, st);
    else if (sc.nw == 2) launch_sym_nw<2>(grad, cols, colv, c64, org, touch, touch_words, sc, part, colpart, first, st);
    else if (sc.nw == 4) launch_sym_nw<4>(grad, cols, colv, c64, org, touch, touch_words, sc, part, colpart, first, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

static size_t pair_lds_bytes(bool grad) {
    return sizeof(float) * ((PAIR_NW - 1) * 2 * (grad ? NACC : 1) * ROWB + (grad ? 1 : PAIR_NW) * PAIR_STAGE_FLOATS);
}

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
