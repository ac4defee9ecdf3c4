// Cluster-tree records and the pair arithmetic shared by the far-field walks (tree.hip: clusters
// of the inner integrals; dual.hip: clusters of both integrals).
#pragma once
#include <algorithm>

#include "common.hpp"

namespace tpe {

// FP64 node moments (combine pass) and the FP32 record the traversal reads.
struct NodeF64 {
    double A, cx, cy, cz, nx, ny, nz, r;
    double m2c[6];  // sum a (c - C)(c - C)^T: xx, xy, xz, yy, yz, zz
    double m2n[6];  // sum a n n^T
};

struct __align__(32) NodeRec {
    float cx, cy, cz, r;  // centroid (normalised frame), radius bound
    float a, nx, ny, nz;  // area, unit mean normal
};

// FP32 moments for the learned correction's features: second moments of (c - C_B) and of n,
// both divided by A_B, and the coherence |N_B| / A_B.
struct __align__(16) NodeMom {
    float m2c[6];
    float m2n[6];
    float coh, pad0, pad1, pad2;
};

// pair arithmetic shared with the exact kernel.  MASK: 0 no exclusion; 1 the pair is excluded when
// the row face (v0, v1, v2) and the column face cv share a vertex; 2 when cv.x != 0 (the caller's
// precomputed exclusion bit).
template <int Q, bool GRAD, int MASK>
__device__ __forceinline__ void ff_pair(const ColRec& cr, int4 cv, float rx, float ry, float rz, float nx, float ny,
                                        float nz, int v0, int v1, int v2, float* acc) {
    float dx = rx - cr.cx, dy = ry - cr.cy, dz = rz - cr.cz;
    float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    float w = __builtin_amdgcn_rcpf(r2);
    if constexpr (MASK == 1) {
        bool ex = (v0 == cv.x) | (v0 == cv.y) | (v0 == cv.z) | (v1 == cv.x) | (v1 == cv.y) | (v1 == cv.z) |
                  (v2 == cv.x) | (v2 == cv.y) | (v2 == cv.z);
        w = ex ? 0.f : w;
    } else if constexpr (MASK == 2) {
        w = cv.x ? 0.f : w;
    }
    float u = fmaf(nz, dz, fmaf(ny, dy, nx * dx));
    float t = u * w;
    float v = fmaf(cr.nz, dz, fmaf(cr.ny, dy, cr.nx * dx));
    float tau = v * w;
    float t2 = t * t, t4 = t2 * t2, t5 = t4 * t, t6 = t5 * t;
    float s2 = tau * tau, s4 = s2 * s2, s5 = s4 * tau, s6 = s5 * tau;
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

__device__ __forceinline__ void ff_fold(float (&acc)[NACC], float (&hi)[NACC], float (&lo)[NACC]) {
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
        float y = acc[k] - lo[k];
        float t = hi[k] + y;
        lo[k] = (t - hi[k]) - y;
        hi[k] = t;
        acc[k] = 0.f;
    }
}

// The same fold with the compensation terms in LDS (LOL): slot k * 64 + lane of the wave's own
// area lol, touched only here, once per 64 columns, so the registers lo stay free.  The same values
// and operations, so the same bits.
template <bool LOL>
__device__ __forceinline__ void ff_fold_at(float (&acc)[NACC], float (&hi)[NACC], float (&lo)[NACC], float* lol,
                                           int lane) {
    if constexpr (!LOL) {
        ff_fold(acc, hi, lo);
    } else {
#pragma unroll
        for (int k = 0; k < NACC; ++k) {
            const float l = lol[k * 64 + lane];
            float y = acc[k] - l;
            float t = hi[k] + y;
            lol[k * 64 + lane] = (t - hi[k]) - y;
            hi[k] = t;
            acc[k] = 0.f;
        }
    }
}

// The pairs of the block's rows with m <= 64 column records already staged in the wave's slots,
// SU independent pair chains per step; LOL: compensation terms in the wave's LDS slots lol.
template <bool MASK, int SU, bool LOL = false>
__device__ __forceinline__ void ff_staged_pairs(const ColRec* st, const int4* sv, int m, float rx, float ry, float rz,
                                                const ColRec& me, const int4& mv, float (&acc)[NACC],
                                                float (&hi)[NACC], float (&lo)[NACC], float* lol, int lane,
                                                int& cnt) {
    const int4 nov = make_int4(0, 0, 0, 0);
    int k = 0;
    for (; k + SU <= m; k += SU) {
#pragma unroll
        for (int u = 0; u < SU; ++u)
            ff_pair<6, true, MASK>(st[k + u], MASK ? sv[k + u] : nov, rx, ry, rz, me.nx, me.ny, me.nz, mv.x, mv.y,
                                   mv.z, acc);
        cnt += SU;
        if (cnt >= 64) { ff_fold_at<LOL>(acc, hi, lo, lol, lane); cnt = 0; }
    }
    for (; k < m; ++k) {
        ff_pair<6, true, MASK>(st[k], MASK ? sv[k] : nov, rx, ry, rz, me.nx, me.ny, me.nz, mv.x, mv.y, mv.z, acc);
        if (++cnt >= 64) { ff_fold_at<LOL>(acc, hi, lo, lol, lane); cnt = 0; }
    }
}

// Exact pairs of the block's rows with the faces [f0, f1) (a near node), with the shared-vertex
// exclusion when MASK (a node whose vertices cannot reach the block's needs none); rows are
// re-expressed relative to each tile's FP64 origin.  The column records go through the wave's own
// LDS slots st[64] / sv[64]: every piece of at most 64 faces within one origin tile is fetched with
// one coalesced load per lane and read back column by column at a wave-uniform address (a
// broadcast), SU columns per step.  At 327,680 faces the monopole far field took 0.95 ms per call
// this way with 2 columns per step against 1.12 ms with the columns read by scalar loads four at a
// time (the same pairs in the same order; loading the next piece into registers while evaluating
// this one: 0.97 ms).  With LOL the compensation terms live in LDS (ff_fold_at) and the registers
// allow 8 columns per step: 0.92 ms.
template <bool MASK, int SU, bool LOL = false>
__device__ __forceinline__ void ff_near_staged(const ColRec* __restrict__ cols, const int4* __restrict__ colv,
                                               const double* __restrict__ org, int64_t f0, int64_t f1, double cxd,
                                               double cyd, double czd, const ColRec& me, const int4& mv,
                                               ColRec* st, int4* sv, int lane, float (&acc)[NACC],
                                               float (&hi)[NACC], float (&lo)[NACC], int& cnt,
                                               float* lol = nullptr) {
    static_assert(CTILE <= 64, "a piece must fit the wave's 64 slots");
    const int4 nov = make_int4(0, 0, 0, 0);
    int64_t f = f0;
    while (f < f1) {
        const int64_t t = f / CTILE;
        const int64_t fend = std::min<int64_t>(f1, (t + 1) * CTILE);
        const int m = (int)(fend - f);
        // the record as two float4 halves (a whole-struct copy under the condition went through
        // scratch memory)
        float4 c0 = make_float4(0.f, 0.f, 0.f, 0.f), c1 = c0;
        int4 v = nov;
        if (lane < m) {
            const float4* src = reinterpret_cast<const float4*>(cols + f + lane);
            c0 = src[0];
            c1 = src[1];
            if constexpr (MASK) v = colv[f + lane];
        }
        const float rx = (float)(cxd - org[3 * t]), ry = (float)(cyd - org[3 * t + 1]), rz = (float)(czd - org[3 * t + 2]);
        asm volatile("" ::: "memory");  // the previous piece's reads of the slots come first
        float4* dst = reinterpret_cast<float4*>(st + lane);
        dst[0] = c0;
        dst[1] = c1;
        if constexpr (MASK) sv[lane] = v;
        asm volatile("" ::: "memory");  // the reads below see every lane's record
        ff_staged_pairs<MASK, SU, LOL>(st, sv, m, rx, ry, rz, me, mv, acc, hi, lo, lol, lane, cnt);
        f = fend;
    }
}

__device__ __forceinline__ float lane_f(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

}  // namespace tpe
