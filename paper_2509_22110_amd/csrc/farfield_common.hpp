// Cluster-tree records and the pair arithmetic shared by the far-field walks (tree.hip: clusters
// of the inner integrals; dual.hip: clusters of both integrals).
#pragma once
#include <algorithm>

#include "common.hpp"

namespace tpe {

// FP64 node moments (combine pass) and the FP32 record the traversal reads with scalar loads.
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

// pair arithmetic shared with the exact kernel
template <int Q, bool GRAD, bool MASK>
__device__ __forceinline__ void ff_pair(const ColRec& cr, int4 cv, float rx, float ry, float rz, float nx, float ny,
                                        float nz, int v0, int v1, int v2, float* acc) {
    float dx = rx - cr.cx, dy = ry - cr.cy, dz = rz - cr.cz;
    float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    float w = __builtin_amdgcn_rcpf(r2);
    if constexpr (MASK) {
        bool ex = (v0 == cv.x) | (v0 == cv.y) | (v0 == cv.z) | (v1 == cv.x) | (v1 == cv.y) | (v1 == cv.z) |
                  (v2 == cv.x) | (v2 == cv.y) | (v2 == cv.z);
        w = ex ? 0.f : w;
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

// Exact pairs of the block's rows with the faces [f0, f1) (a near node), with the shared-vertex
// exclusion when MASK (a node whose vertices cannot reach the block's needs none); columns are
// read with scalar loads, four at a time, rows re-expressed relative to each chunk's FP64 origin.
template <bool MASK>
__device__ __forceinline__ void ff_near_range(const ColRec* __restrict__ cols, const int4* __restrict__ colv,
                                              const double* __restrict__ org, int64_t f0, int64_t f1, double cxd,
                                              double cyd, double czd, const ColRec& me, const int4& mv,
                                              float (&acc)[NACC], float (&hi)[NACC], float (&lo)[NACC], int& cnt) {
    const int4 nov = make_int4(0, 0, 0, 0);
    int64_t f = f0;
    while (f < f1) {
        const int64_t t = f / CTILE;
        const int64_t fend = std::min<int64_t>(f1, (t + 1) * CTILE);
        const float rx = (float)(cxd - org[3 * t]), ry = (float)(cyd - org[3 * t + 1]), rz = (float)(czd - org[3 * t + 2]);
        for (; f + 4 <= fend; f += 4) {
            const ColRec c0 = cols[f], c1 = cols[f + 1], c2 = cols[f + 2], c3 = cols[f + 3];
            int4 v0 = nov, v1 = nov, v2 = nov, v3 = nov;
            if constexpr (MASK) { v0 = colv[f]; v1 = colv[f + 1]; v2 = colv[f + 2]; v3 = colv[f + 3]; }
            ff_pair<6, true, MASK>(c0, v0, rx, ry, rz, me.nx, me.ny, me.nz, mv.x, mv.y, mv.z, acc);
            ff_pair<6, true, MASK>(c1, v1, rx, ry, rz, me.nx, me.ny, me.nz, mv.x, mv.y, mv.z, acc);
            ff_pair<6, true, MASK>(c2, v2, rx, ry, rz, me.nx, me.ny, me.nz, mv.x, mv.y, mv.z, acc);
            ff_pair<6, true, MASK>(c3, v3, rx, ry, rz, me.nx, me.ny, me.nz, mv.x, mv.y, mv.z, acc);
            cnt += 4;
            if (cnt >= 64) { ff_fold(acc, hi, lo); cnt = 0; }
        }
        for (; f < fend; ++f) {
            ff_pair<6, true, MASK>(cols[f], MASK ? colv[f] : nov, rx, ry, rz, me.nx, me.ny, me.nz, mv.x, mv.y, mv.z,
                                   acc);
            if (++cnt >= 64) { ff_fold(acc, hi, lo); cnt = 0; }
        }
    }
}

__device__ __forceinline__ float lane_f(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

}  // namespace tpe
