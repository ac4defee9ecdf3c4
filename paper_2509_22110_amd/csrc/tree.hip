// Cluster tree over Morton-ordered faces and the Barnes-Hut far field of the inner integrals.
//
// The paper clusters only the inner integrals f_K, f_nu, f of eq. (dTP_reordered) (Sec. 3.2): for
// an outer point x, the contribution of a patch of faces far enough from x is replaced by one
// evaluation with precomputed averages over the patch, and no derivative has to be propagated
// back to the patch because the test function only appears in the outer integral.  Here:
//   - the tree is an implicit complete binary tree over leaves of `leaf` consecutive faces in k-d
//     order (node k has children 2k, 2k+1; leaves are nodes 2^H .. 2^H + nleaf - 1);
//   - per node: area A_B = sum a, area-weighted centroid C_B, area-weighted normal sum N_B,
//     second moments of (c - C_B) and of n weighted by area, and a radius r_B that bounds the
//     distance from C_B to every vertex of every member face (exact at leaves, propagated up as
//     max over children of |C_child - C_B| + r_child);
//   - a target block of 64 consecutive faces (one wave) is enclosed by a ball (C_T, r_T) that
//     bounds its faces' vertices; a cluster B is far when 2 r_B < theta (|C_T - C_B| - r_T);
//   - a far cluster acts on every face S of the block as one pseudo-face (monopole): centroid C_B,
//     area A_B, unit normal N_B/|N_B|, through exactly the same pair arithmetic as the exact
//     kernel (forward term with n_S, reverse term with N_B/|N_B|);
//   - a cluster that is not far is opened; a leaf that is not far is evaluated exactly, pair by
//     pair, with the shared-vertex exclusion.  Because r_T and r_B bound vertices, a far cluster
//     never contains a face sharing a vertex with a target face.
// The output is the exact kernel's per-face row-sum layout, so the FP64 finalize and the vertex
// gather are shared with the exact path.
#include <algorithm>

#include "common.hpp"
#include "farfield_common.hpp"
#include "mlp.hpp"
#include "mlp_infer.hpp"

namespace tpe {

__device__ __forceinline__ void sym_add_outer(double* m, double w, double x, double y, double z) {
    m[0] += w * x * x; m[1] += w * x * y; m[2] += w * x * z;
    m[3] += w * y * y; m[4] += w * y * z; m[5] += w * z * z;
}

__device__ __forceinline__ float round_up_f(double v) {
    float f = (float)v;
    return (double)f >= v ? f : nextafterf(f, INFINITY);
}

__device__ __forceinline__ void write_mom(const NodeF64& n, NodeMom* mom) {
    NodeMom m = {};
    if (n.A > 0.0) {
        for (int k = 0; k < 6; ++k) {
            m.m2c[k] = (float)(n.m2c[k] / n.A);
            m.m2n[k] = (float)(n.m2n[k] / n.A);
        }
        m.coh = (float)(sqrt(n.nx * n.nx + n.ny * n.ny + n.nz * n.nz) / n.A);
    }
    *mom = m;
}

// FP32 record of a node: centre relative to the origin o (norm_origin), radius rounded up.
__device__ __forceinline__ void write_rec(const NodeF64& n, const double* o, NodeRec* rec) {
    NodeRec r;
    const double cx = n.cx - o[0], cy = n.cy - o[1], cz = n.cz - o[2];
    r.cx = (float)cx; r.cy = (float)cy; r.cz = (float)cz;
    // the FP32 centroid moves by at most ~|C| 2^-24; fold that into the radius bound
    const double slack = 1e-6 * (1.0 + fabs(cx) + fabs(cy) + fabs(cz));
    r.r = n.A > 0.0 ? round_up_f(n.r + slack) : 0.f;
    r.a = (float)n.A;
    const double nn = sqrt(n.nx * n.nx + n.ny * n.ny + n.nz * n.nz);
    r.nx = nn > 0.0 ? (float)(n.nx / nn) : 0.f;
    r.ny = nn > 0.0 ? (float)(n.ny / nn) : 0.f;
    r.nz = nn > 0.0 ? (float)(n.nz / nn) : 0.f;
    *rec = r;
}

__device__ __forceinline__ double wave_sum_d(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}
__device__ __forceinline__ double wave_max_d(double x) {
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
    return x;
}

// The ball of target block b (its faces 64 b + lane, one per lane of the calling wave): centre the
// mean of the faces' centres, radius the largest distance from it to a vertex of the faces, in the
// FP32 record frame with the slack of write_rec; lane 0 writes balls[b].  Every lane of the wave
// calls it (the sums run over the whole wave).
__device__ __forceinline__ void block_ball_wave(const double* __restrict__ c64, const int4* __restrict__ colv,
                                                const double* __restrict__ X, const uint32_t* __restrict__ bbox,
                                                int64_t nF, int64_t b, int lane, float4* __restrict__ balls) {
    const int64_t i = b * 64 + lane;
    const bool act = i < nF;
    const double s = norm_scale(bbox);
    const double nact = wave_sum_d(act ? 1.0 : 0.0);
    const double cx = wave_sum_d(act ? c64[3 * i] : 0.0) / fmax(nact, 1.0);
    const double cy = wave_sum_d(act ? c64[3 * i + 1] : 0.0) / fmax(nact, 1.0);
    const double cz = wave_sum_d(act ? c64[3 * i + 2] : 0.0) / fmax(nact, 1.0);
    double r = 0.0;
    if (act) {
        const int4 v = colv[i];
        const int vv[3] = {v.x, v.y, v.z};
        for (int k = 0; k < 3; ++k) {
            if (vv[k] < 0) continue;
            const double dx = s * X[3 * (int64_t)vv[k]] - cx, dy = s * X[3 * (int64_t)vv[k] + 1] - cy,
                         dz = s * X[3 * (int64_t)vv[k] + 2] - cz;
            r = fmax(r, sqrt(dx * dx + dy * dy + dz * dz));
        }
    }
    r = wave_max_d(r);
    if (lane == 0) {
        double o[3];
        norm_origin(bbox, o);
        const double rx = cx - o[0], ry = cy - o[1], rz = cz - o[2];  // relative to the records' origin
        const double slack = 1e-6 * (1.0 + fabs(rx) + fabs(ry) + fabs(rz));
        balls[b] = make_float4((float)rx, (float)ry, (float)rz, round_up_f(r + slack));
    }
}

// G lanes per leaf slot j in [0, 2^H) (G = the leaf size rounded up to a power of two, at most 64;
// 64 / G slots per wave): faces [j*leaf, min((j+1)*leaf, nF)) in sorted order, the group's lanes
// striding over them; the FP64 sums are reduced across the group in a fixed order (every lane of
// the group ends with the same bits: each butterfly step adds the same two values).  MOM2: also the
// second moments (the learned correction's features); the monopole needs A, C, N and r only.
constexpr int MOM_LEAF_WAVES = 4;

__device__ __forceinline__ double group_sum_d(double x, int G) {
    for (int off = G >> 1; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}
__device__ __forceinline__ double group_max_d(double x, int G) {
    for (int off = G >> 1; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
    return x;
}

template <bool MOM2>
__device__ __forceinline__ void store_node(NodeF64* __restrict__ d, const NodeF64& n);

template <bool MOM2>
__global__ __launch_bounds__(64 * MOM_LEAF_WAVES) void leaf_moments(const double* __restrict__ c64,
                                                                    const double* __restrict__ geo,
                                                                    const int4* __restrict__ colv,
                                                                    const double* __restrict__ X,
                                                                    const uint32_t* __restrict__ bbox, int64_t nF,
                                                                    int leaf, int H, int G, NodeF64* __restrict__ nodes,
                                                                    NodeRec* __restrict__ recs,
                                                                    NodeMom* __restrict__ moms,
                                                                    float4* __restrict__ balls) {
    const int lane = threadIdx.x & 63;
    const int64_t nslot = (int64_t)1 << H;
    const int64_t j = (blockIdx.x * (int64_t)MOM_LEAF_WAVES + (threadIdx.x >> 6)) * (64 / G) + lane / G;
    const int t = lane & (G - 1);
    if (__builtin_amdgcn_readfirstlane((int)(j - lane / G >= nslot))) return;  // uniform over the wave
    // leaves of 32 (balls given): the wave's two leaves are target block j0 / 2, whose ball it
    // writes as target_balls would (the same wave sums, the same bits)
    const int64_t bb = __builtin_amdgcn_readfirstlane((int)((j - lane / G) / 2));
    if (balls && bb * 64 < nF) block_ball_wave(c64, colv, X, bbox, nF, bb, lane, balls);
    const double s = norm_scale(bbox);
    const int64_t f0 = j < nslot ? j * leaf : 0, f1 = j < nslot ? std::min<int64_t>(nF, f0 + leaf) : 0;
    double A = 0, sx = 0, sy = 0, sz = 0, nx = 0, ny = 0, nz = 0;
    for (int64_t i = f0 + t; i < f1; i += G) {
        const double a = geo[5 * i];
        A += a;
        sx += a * c64[3 * i]; sy += a * c64[3 * i + 1]; sz += a * c64[3 * i + 2];
        nx += a * geo[5 * i + 2]; ny += a * geo[5 * i + 3]; nz += a * geo[5 * i + 4];
    }
    NodeF64 n = {};
    n.A = group_sum_d(A, G);
    sx = group_sum_d(sx, G); sy = group_sum_d(sy, G); sz = group_sum_d(sz, G);
    n.nx = group_sum_d(nx, G); n.ny = group_sum_d(ny, G); n.nz = group_sum_d(nz, G);
    const bool has = n.A > 0.0;  // uniform over the group
    n.cx = has ? sx / n.A : 0.0; n.cy = has ? sy / n.A : 0.0; n.cz = has ? sz / n.A : 0.0;
    double m2c[6] = {0, 0, 0, 0, 0, 0}, m2n[6] = {0, 0, 0, 0, 0, 0}, r = 0.0;
    for (int64_t i = has ? f0 + t : f1; i < f1; i += G) {
        if constexpr (MOM2) {
            const double a = geo[5 * i];
            sym_add_outer(m2c, a, c64[3 * i] - n.cx, c64[3 * i + 1] - n.cy, c64[3 * i + 2] - n.cz);
            sym_add_outer(m2n, a, geo[5 * i + 2], geo[5 * i + 3], geo[5 * i + 4]);
        }
        const int4 v = colv[i];
        const int vv[3] = {v.x, v.y, v.z};
        for (int k = 0; k < 3; ++k) {
            if (vv[k] < 0) continue;
            const double dx = s * X[3 * (int64_t)vv[k]] - n.cx, dy = s * X[3 * (int64_t)vv[k] + 1] - n.cy,
                         dz = s * X[3 * (int64_t)vv[k] + 2] - n.cz;
            r = fmax(r, sqrt(dx * dx + dy * dy + dz * dz));
        }
    }
    if constexpr (MOM2)
        for (int k = 0; k < 6; ++k) {
            n.m2c[k] = group_sum_d(m2c[k], G);
            n.m2n[k] = group_sum_d(m2n[k], G);
        }
    n.r = group_max_d(r, G);  // a group without area keeps all zeros: no face added to any sum
    if (t == 0 && j < nslot) {
        double o[3];
        norm_origin(bbox, o);
        store_node<MOM2>(&nodes[nslot + j], n);
        write_rec(n, o, &recs[nslot + j]);
        if constexpr (MOM2) write_mom(n, &moms[nslot + j]);
    }
}

// FP64 node records in global memory, field by field (without MOM2 the second moments are neither
// read nor written: no reader of such a call looks at them)
template <bool MOM2>
__device__ __forceinline__ void store_node(NodeF64* __restrict__ d, const NodeF64& n) {
    d->A = n.A; d->cx = n.cx; d->cy = n.cy; d->cz = n.cz; d->nx = n.nx; d->ny = n.ny; d->nz = n.nz; d->r = n.r;
    if constexpr (MOM2)
        for (int c = 0; c < 6; ++c) { d->m2c[c] = n.m2c[c]; d->m2n[c] = n.m2n[c]; }
}
template <bool MOM2>
__device__ __forceinline__ NodeF64 load_node(const NodeF64* __restrict__ d) {
    NodeF64 n = {};
    n.A = d->A; n.cx = d->cx; n.cy = d->cy; n.cz = d->cz; n.nx = d->nx; n.ny = d->ny; n.nz = d->nz; n.r = d->r;
    if constexpr (MOM2)
        for (int c = 0; c < 6; ++c) { n.m2c[c] = d->m2c[c]; n.m2n[c] = d->m2n[c]; }
    return n;
}

// A node from its two children (MOM2: with the second moments).
template <bool MOM2>
__device__ __forceinline__ NodeF64 combine_nodes(const NodeF64& a, const NodeF64& b) {
    NodeF64 n = {};
    n.A = a.A + b.A;
    if (n.A > 0.0) {
        n.cx = (a.A * a.cx + b.A * b.cx) / n.A;
        n.cy = (a.A * a.cy + b.A * b.cy) / n.A;
        n.cz = (a.A * a.cz + b.A * b.cz) / n.A;
        n.nx = a.nx + b.nx; n.ny = a.ny + b.ny; n.nz = a.nz + b.nz;
        auto child = [&](const NodeF64& q) {  // the first child, then the second
            if (!(q.A > 0.0)) return;
            const double dx = q.cx - n.cx, dy = q.cy - n.cy, dz = q.cz - n.cz;
            n.r = fmax(n.r, sqrt(dx * dx + dy * dy + dz * dz) + q.r);
            if constexpr (MOM2) {
                for (int m = 0; m < 6; ++m) { n.m2c[m] += q.m2c[m]; n.m2n[m] += q.m2n[m]; }
                sym_add_outer(n.m2c, q.A, dx, dy, dz);  // parallel-axis shift to the new centroid
            }
        };
        child(a);
        child(b);
    }
    return n;
}

// Levels L - 1, ..., L - nl from the nodes of level L, in one launch: work-group g loads the
// 2^nl nodes [2^L + g 2^nl, 2^L + (g + 1) 2^nl) of level L into LDS (blockDim.x = 2^nl) and
// combines them level by level up to their common ancestor at level L - nl, writing every node.
// The tree's internal levels take ceil(H / MOM_SUB) launches instead of H.  LDS holds the nodes
// field-major (one array per field: a lane's reads of its two children fall in distinct banks,
// where whole records would put every other lane on the same bank).
constexpr int MOM_SUB = 8;

template <bool MOM2>
__global__ __launch_bounds__(1 << MOM_SUB) void subtree_moments(int L, int nl, const uint32_t* __restrict__ bbox,
                                                                NodeF64* __restrict__ nodes,
                                                                NodeRec* __restrict__ recs,
                                                                NodeMom* __restrict__ moms) {
    constexpr int NF = MOM2 ? 20 : 8;  // fields: A, C (3), N (3), r, then m2c (6), m2n (6)
    __shared__ double buf[NF][1 << MOM_SUB];
    const int t = threadIdx.x, cnt = 1 << nl;
    const int64_t g = blockIdx.x;
    auto get = [&](int idx) {
        NodeF64 n = {};
        n.A = buf[0][idx]; n.cx = buf[1][idx]; n.cy = buf[2][idx]; n.cz = buf[3][idx];
        n.nx = buf[4][idx]; n.ny = buf[5][idx]; n.nz = buf[6][idx]; n.r = buf[7][idx];
        if constexpr (MOM2) {
#pragma unroll
            for (int c = 0; c < 6; ++c) { n.m2c[c] = buf[8 + c][idx]; n.m2n[c] = buf[14 + c][idx]; }
        }
        return n;
    };
    auto put = [&](int idx, const NodeF64& n) {
        buf[0][idx] = n.A; buf[1][idx] = n.cx; buf[2][idx] = n.cy; buf[3][idx] = n.cz;
        buf[4][idx] = n.nx; buf[5][idx] = n.ny; buf[6][idx] = n.nz; buf[7][idx] = n.r;
        if constexpr (MOM2) {
#pragma unroll
            for (int c = 0; c < 6; ++c) { buf[8 + c][idx] = n.m2c[c]; buf[14 + c][idx] = n.m2n[c]; }
        }
    };
    put(t, load_node<MOM2>(&nodes[((int64_t)1 << L) + g * cnt + t]));
    __syncthreads();
    double o[3];
    norm_origin(bbox, o);
    for (int st = 1; st <= nl; ++st) {
        const int m = cnt >> st;
        NodeF64 par = {};
        if (t < m) par = combine_nodes<MOM2>(get(2 * t), get(2 * t + 1));
        __syncthreads();
        if (t < m) {
            put(t, par);
            const int64_t k = ((int64_t)1 << (L - st)) + g * m + t;
            store_node<MOM2>(&nodes[k], par);
            write_rec(par, o, &recs[k]);
            if constexpr (MOM2) write_mom(par, &moms[k]);
        }
        __syncthreads();
    }
}

// Ball (C_T, r_T) of each target block of 64 sorted faces: C_T = mean of the centroids, r_T bounds
// the distance to every vertex of the block's faces (plus FP32 rounding slack).  One wave each.
__global__ __launch_bounds__(64) void target_balls(const double* __restrict__ c64, const int4* __restrict__ colv,
                                                   const double* __restrict__ X, const uint32_t* __restrict__ bbox,
                                                   int64_t nF, float4* __restrict__ balls) {
    block_ball_wave(c64, colv, X, bbox, nF, blockIdx.x, threadIdx.x, balls);
}

// ---- learned correction: features and training samples -----------------------------------------
// For a target face S (centroid c_S, normal n_S) and a far cluster B, with D = c_S - C_B, rho = |D|:
// local frame e1 = D / rho, e2 = unit part of n_S orthogonal to e1 (any orthogonal unit vector if
// none), e3 = e1 x e2.  Features (dimensionless, rotation-invariant by construction):
//   0: 4 r_B / rho            1, 2: n_S . e1, n_S . e2
//   3-5: unit mean normal of B in the frame       6: coherence |N_B| / A_B
//   7-12: M2c / (A_B r_B^2) in the frame (xx, xy, xz, yy, yz, zz)
//   13-18: M2n / A_B in the frame                 19-31: 0
// Outputs (7 used): the correction (exact sum over B minus monopole) of the quantities the face's
// gradient is made of -- K (for dE/da and E), Sd (for dE/dn) and the net C = q (n_S S0 + Sn) - p Sdd
// (for dE/dc) -- vectors in the frame, divided by their units u = A_B rho^-6 for K and Sd, and
// A_B rho^-7 for C.  Predicting C itself (not S0, Sn, Sdd separately) keeps the near
// cancellation between its terms out of the network's errors.
struct Frame {
    float e1[3], e2[3], e3[3];
    float rho, s2;  // s2 = (r_B / rho)^2
};

__device__ __forceinline__ void quad_frame(const float* m, const Frame& f, float scale, float* out) {
    // out = scale * (e_a . M e_b) for (a,b) in (11, 12, 13, 22, 23, 33); M symmetric (xx xy xz yy yz zz)
    const float* E[3] = {f.e1, f.e2, f.e3};
    float Me[3][3];
    for (int a = 0; a < 3; ++a) {
        const float* e = E[a];
        Me[a][0] = m[0] * e[0] + m[1] * e[1] + m[2] * e[2];
        Me[a][1] = m[1] * e[0] + m[3] * e[1] + m[4] * e[2];
        Me[a][2] = m[2] * e[0] + m[4] * e[1] + m[5] * e[2];
    }
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int q = 0; q < 6; ++q) {
        const float* e = E[pa[q]];
        out[q] = scale * (e[0] * Me[pb[q]][0] + e[1] * Me[pb[q]][1] + e[2] * Me[pb[q]][2]);
    }
}

__device__ __forceinline__ void ff_features(float ax, float ay, float az, float nx, float ny, float nz,
                                            const NodeRec& nd, const NodeMom& mm, Frame& fr, float* x) {
    float dx = ax - nd.cx, dy = ay - nd.cy, dz = az - nd.cz;
    const float rho = sqrtf(dx * dx + dy * dy + dz * dz);
    const float ir = 1.f / rho;
    fr.e1[0] = dx * ir; fr.e1[1] = dy * ir; fr.e1[2] = dz * ir;
    const float c1 = nx * fr.e1[0] + ny * fr.e1[1] + nz * fr.e1[2];
    float vx = nx - c1 * fr.e1[0], vy = ny - c1 * fr.e1[1], vz = nz - c1 * fr.e1[2];
    float vn = sqrtf(vx * vx + vy * vy + vz * vz);
    if (!(vn > 1e-6f)) {
        // any unit vector orthogonal to e1
        const float ux = fabsf(fr.e1[0]) < 0.9f ? 1.f : 0.f, uy = 1.f - ux;
        const float pu = ux * fr.e1[0] + uy * fr.e1[1];
        vx = ux - pu * fr.e1[0]; vy = uy - pu * fr.e1[1]; vz = -pu * fr.e1[2];
        vn = sqrtf(vx * vx + vy * vy + vz * vz);
    }
    fr.e2[0] = vx / vn; fr.e2[1] = vy / vn; fr.e2[2] = vz / vn;
    fr.e3[0] = fr.e1[1] * fr.e2[2] - fr.e1[2] * fr.e2[1];
    fr.e3[1] = fr.e1[2] * fr.e2[0] - fr.e1[0] * fr.e2[2];
    fr.e3[2] = fr.e1[0] * fr.e2[1] - fr.e1[1] * fr.e2[0];
    fr.rho = rho;
    const float s = nd.r * ir;
    fr.s2 = s * s;
    x[0] = 4.f * s;
    x[1] = c1;
    x[2] = nx * fr.e2[0] + ny * fr.e2[1] + nz * fr.e2[2];
    x[3] = nd.nx * fr.e1[0] + nd.ny * fr.e1[1] + nd.nz * fr.e1[2];
    x[4] = nd.nx * fr.e2[0] + nd.ny * fr.e2[1] + nd.nz * fr.e2[2];
    x[5] = nd.nx * fr.e3[0] + nd.ny * fr.e3[1] + nd.nz * fr.e3[2];
    x[6] = mm.coh;
    quad_frame(mm.m2c, fr, nd.r > 0.f ? 1.f / (nd.r * nd.r) : 0.f, x + 7);
    quad_frame(mm.m2n, fr, 1.f, x + 13);
    for (int k = 19; k < 32; ++k) x[k] = 0.f;
}

// units of the outputs: u6 = A_B rho^-6 for K and Sd, u7 = u6 / rho for C (the magnitude of the
// monopole's own contribution, so the loss measures error relative to it)
__device__ __forceinline__ void out_units(float A, const Frame& fr, float& u6, float& u7) {
    const float ir = 1.f / fr.rho;
    const float r2 = ir * ir, r6 = r2 * r2 * r2;
    u6 = A * r6;
    u7 = u6 * ir;
}

// net dE/dc combination of the row sums, C = q (n_S S0 + Sn) - p Sdd  (q = 6, p = 12)
__device__ __forceinline__ void net_c(const float* acc, float nx, float ny, float nz, float* c) {
    c[0] = 6.f * (nx * acc[1] + acc[8]) - 12.f * acc[5];
    c[1] = 6.f * (ny * acc[1] + acc[9]) - 12.f * acc[6];
    c[2] = 6.f * (nz * acc[1] + acc[10]) - 12.f * acc[7];
}

// accumulator-space vector (global frame) -> frame components
__device__ __forceinline__ void to_frame(const float* v, const Frame& fr, float* o) {
    o[0] = v[0] * fr.e1[0] + v[1] * fr.e1[1] + v[2] * fr.e1[2];
    o[1] = v[0] * fr.e2[0] + v[1] * fr.e2[1] + v[2] * fr.e2[2];
    o[2] = v[0] * fr.e3[0] + v[1] * fr.e3[1] + v[2] * fr.e3[2];
}

// Learned correction of one far cluster for the wave's 64 rows: features per row, the MLP on the
// 64 x 32 feature block (MFMA, LDS scratch), and the corrections added to the row sums.
// The correction's gate, r_B / rho >= min_s for the row at (ax, ay, az), in one fixed evaluation
// (explicit FMAs): ff_correct's batch filter and mlp_correction take the same decision.
__device__ __forceinline__ bool mlp_gate(const MlpPacked* __restrict__ W, const NodeRec& cn, float ax, float ay,
                                         float az) {
    const float gx = ax - cn.cx, gy = ay - cn.cy, gz = az - cn.cz;
    const float d2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
    const float s2 = W->min_s * W->min_s;
    return cn.r * cn.r >= s2 * d2;
}

__device__ __forceinline__ void mlp_correction(const MlpPacked* __restrict__ W, const NodeRec& cn, const NodeMom& mm,
                                               float ax, float ay, float az, float nx, float ny, float nz,
                                               MlpScratch& ms, float (&acc)[NACC]) {
    // the gate, checked before the features: the wave skips the network when no row needs it
    const bool gate = mlp_gate(W, cn, ax, ay, az);
    if (!__any(gate)) return;
    Frame fr;
    float x[32], y[16];
    ff_features(ax, ay, az, nx, ny, nz, cn, mm, fr, x);
    mlp_infer64(W, x, ms, y);
    if (!gate) return;
    float u6, u7;
    out_units(cn.a, fr, u6, u7);
    acc[0] += u6 * y[0];
    // dC enters through Sn: q * dSn = dC leaves S0 and Sdd untouched
    const float u7q = u7 * (1.f / 6.f);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        acc[2 + d] += u6 * (y[1] * fr.e1[d] + y[2] * fr.e2[d] + y[3] * fr.e3[d]);
        acc[8 + d] += u7q * (y[4] * fr.e1[d] + y[5] * fr.e2[d] + y[6] * fr.e3[d]);
    }
}

// |C_T - C_B| for the admissibility test, with the products in a fixed order (the decision is an
// integer outcome of FP32 arithmetic, reproduced exactly by an independent evaluation).
__device__ __forceinline__ float ball_dist(const float4& tb, const NodeRec& nd) {
    const float dx = tb.x - nd.cx, dy = tb.y - nd.cy, dz = tb.z - nd.cz;
    return sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
}

constexpr int FF_STACK = 1024;  // LDS node stack per wave (overflow falls back to exact evaluation)
constexpr int FF_NW = 4;          // waves per target block, monopole far field
constexpr int FF_NW_LEARNED = 4;  // waves per target block with the learned correction

// ---- the walk as lists: classify once per target block, then evaluate ---------------------------
// ff_classify walks the tree for each target block once, one wave per block, batched depth first:
// up to 64 nodes are popped at once (one per lane) and tested in parallel; far clusters are listed,
// near nodes (leaves, or nodes the LDS stack could not open -- evaluating such a node exactly is
// always correct) are listed, other nodes push their two children (right below left, so the left
// is popped first).  The stack holds at most 128 + 64 (H - 1) + 1 entries (entries are ordered by
// depth from the bottom, at most 64 of each depth stay behind a deeper one and the top depth has at
// most 128), within FF_STACK for trees of height <= 14 (458,752 faces with leaves of 32).  It writes the block's near nodes (faces evaluated exactly:
// leaves, or nodes the stack could not open; only non-empty ones) and far clusters, each in walk
// order, into ent[b * cap ...]: near nodes from the front, far clusters from the back.  The far and
// near nodes of a block are disjoint subtrees holding every non-empty leaf once, so a block has at
// most ceil(nF / leaf) entries; cap below that sets FLAG_LISTS when a block outgrows it.
// lst[b] = (near count, far count, near columns, visited nodes).
constexpr int FFC_NW = 4;  // blocks (waves) per classify work-group

__global__ __launch_bounds__(64 * FFC_NW) void ff_classify(const NodeRec* __restrict__ nodes, int H, int leaf,
                                                           int64_t nF, const float4* __restrict__ balls, float theta,
                                                           int64_t cap, uint32_t* __restrict__ ent,
                                                           uint4* __restrict__ lst, uint32_t* __restrict__ work,
                                                           uint32_t* __restrict__ flags) {
    __shared__ int stacks[FFC_NW][FF_STACK];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int64_t nb = (nF + 63) / 64;
    const int64_t b = blockIdx.x * (int64_t)FFC_NW + wave;
    if (b >= nb) return;  // uniform over the wave
    int* stack = stacks[wave];
    const float4 tb = balls[b];
    const int64_t leaf0 = (int64_t)1 << H;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t* e = ent + (size_t)b * cap;
    uint32_t n_far = 0, n_near = 0, n_near_cols = 0, n_visit = 0;
    bool over = false;
    if (lane == 0) stack[0] = 1;
    int sz = 1;
    while (sz > 0) {
        lds_phase();  // the pops below read entries other lanes pushed
        const int n = sz < 64 ? sz : 64;
        sz -= n;
        const bool act = lane < n;
        const int k = act ? stack[sz + lane] : 0;
        NodeRec nd = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (act) nd = nodes[k];
        n_visit += n;
        const bool valid = act && nd.a > 0.f;
        const float dist = ball_dist(tb, nd);
        const bool far = valid && (2.f * nd.r < theta * (dist - tb.w));
        const bool isleaf = (int64_t)k >= leaf0;
        bool open = valid && !far && !isleaf;
        const int nopen = __popcll(__ballot(open));
        const bool overflow = sz + 2 * nopen > FF_STACK;
        if (overflow) open = false;
        // a near node's face range [f0, f1) (empty ranges of padding leaves are skipped)
        int64_t f0 = 0, f1 = 0;
        const bool near0 = valid && !far && !open;
        if (near0) {
            const int lev = 63 - __builtin_clzll((unsigned long long)k);
            const int64_t span = (int64_t)1 << (H - lev);
            f0 = ((int64_t)k - ((int64_t)1 << lev)) * span * leaf;
            f1 = f0 + span * leaf < nF ? f0 + span * leaf : nF;
        }
        const bool near = near0 && f0 < f1;
        if (!overflow) {
            const uint64_t om = __ballot(open);
            if (open) {
                const int pos = sz + 2 * (int)__popcll(om & lt);
                stack[pos] = 2 * k + 1;
                stack[pos + 1] = 2 * k;
            }
            sz += 2 * nopen;
        }
        const uint64_t fm = __ballot(far), nm = __ballot(near);
        const uint32_t fi = n_far + (uint32_t)__popcll(fm & lt), ni = n_near + (uint32_t)__popcll(nm & lt);
        if (far) {
            if ((int64_t)fi + n_near + __popcll(nm) < cap) e[cap - 1 - fi] = (uint32_t)k;
            else over = true;
        }
        if (near) {
            if ((int64_t)ni + n_far + __popcll(fm) < cap) e[ni] = (uint32_t)k;
            else over = true;
        }
        n_far += (uint32_t)__popcll(fm);
        n_near += (uint32_t)__popcll(nm);
        uint32_t cols = near ? (uint32_t)(f1 - f0) : 0u;
        for (int off = 32; off > 0; off >>= 1) cols += __shfl_xor(cols, off);
        n_near_cols += cols;
    }
    if (__any(over)) {
        if (lane == 0) atomicOr(flags, (uint32_t)FLAG_LISTS);
        n_far = n_near = 0;  // nothing of this block is evaluated; the call reports the error
    }
    if (lane == 0) {
        lst[b] = make_uint4(n_near, n_far, n_near_cols, n_visit);
        if (work) work[b] = n_near_cols + n_visit + n_far;
    }
}

// Tiles (CTILE = 64 consecutive sorted faces, the unit the near loop stages) holding a face that
// shares a vertex with a target block (the block's own tile among them), per block of 64 faces:
// nbl[b * NBL_STRIDE] = their count (NBL_OVERFLOW if more than NBL_MAX), then the tile ids in
// ascending order; and per (block, listed tile s, row lane) the 64-bit exclusion mask
// xm[(b * NBL_MAX + s) * 64 + lane], bit j set when the block's face 64 b + lane shares a vertex
// with the tile's face 64 t + j (itself included).  A piece of a near node needs the exclusion
// exactly when its tile is listed, and then tests one bit per pair instead of comparing nine vertex
// ids; the unmasked and masked loops give the same bits wherever no pair is excluded.  Both depend
// on the faces and the order only (built once per tree).  One wave per block: every lane walks its
// face's three vertex lists and inserts the tiles into an LDS hash set.
constexpr int NBL_MAX = 16;
constexpr int NBL_STRIDE = NBL_MAX + 1;
constexpr uint32_t NBL_OVERFLOW = 0xffffffffu;

__global__ __launch_bounds__(64) void block_neighbour_tiles(const int4* __restrict__ colv,
                                                            const uint32_t* __restrict__ voff,
                                                            const uint32_t* __restrict__ vlist, int64_t nF,
                                                            int64_t V, uint32_t* __restrict__ nbl) {
    constexpr int HS = 256;  // hash slots (a block touches a few dozen tiles at most on a manifold)
    __shared__ uint32_t set[HS];
    __shared__ uint32_t nset;
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    for (int k = lane; k < HS; k += 64) set[k] = 0xffffffffu;
    if (lane == 0) nset = 0u;
    __syncthreads();
    const int64_t i = b * 64 + lane;
    bool full = false;
    if (i < nF) {
        const int4 v = colv[i];
        const int vv[3] = {v.x, v.y, v.z};
        for (int k = 0; k < 3 && !full; ++k) {
            if (vv[k] < 0 || vv[k] >= V) continue;
            for (uint32_t s = voff[vv[k]]; s < voff[vv[k] + 1] && !full; ++s) {
                const uint32_t lf = (uint32_t)((vlist[s] / 3) / (uint32_t)CTILE);
                uint32_t h = (lf * 0x9e3779b9u) >> 24;  // HS = 256 slots
                for (int probe = 0; probe < HS; ++probe, h = (h + 1) & (HS - 1)) {
                    const uint32_t old = atomicCAS(&set[h], 0xffffffffu, lf);
                    if (old == 0xffffffffu) {
                        if (atomicAdd(&nset, 1u) >= (uint32_t)NBL_MAX) full = true;
                        break;
                    }
                    if (old == lf) break;
                }
            }
        }
    }
    __syncthreads();
    if (lane == 0) {
        uint32_t* out = nbl + (size_t)b * NBL_STRIDE;
        if (nset > (uint32_t)NBL_MAX) {
            out[0] = NBL_OVERFLOW;
        } else {
            uint32_t m = 0, L[NBL_MAX];
            for (int k = 0; k < HS; ++k) {
                const uint32_t x = set[k];
                if (x == 0xffffffffu) continue;
                int p = (int)m++;  // insertion into the sorted prefix
                while (p > 0 && L[p - 1] > x) { L[p] = L[p - 1]; --p; }
                L[p] = x;
            }
            out[0] = m;
            for (uint32_t k = 0; k < m; ++k) out[1 + k] = L[k];
        }
    }
}

// One wave per (block, listed tile): the rows' exclusion masks of that tile.
__global__ __launch_bounds__(64) void block_exclusion_masks(const int4* __restrict__ colv, int64_t nF,
                                                            const uint32_t* __restrict__ nbl, uint2* __restrict__ xm) {
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    const uint32_t s = blockIdx.y;
    const uint32_t n = nbl[(size_t)b * NBL_STRIDE];
    if (n > (uint32_t)NBL_MAX || s >= n) return;
    const int64_t t = nbl[(size_t)b * NBL_STRIDE + 1 + s];
    const int64_t i = b * 64 + lane;
    uint32_t lo = 0u, hi = 0u;
    if (i < nF) {
        const int4 r = colv[i];
        for (int j = 0; j < CTILE && t * CTILE + j < nF; ++j) {
            const int4 v = colv[t * CTILE + j];
            const bool shared = (r.x == v.x) | (r.x == v.y) | (r.x == v.z) | (r.y == v.x) | (r.y == v.y) |
                                (r.y == v.z) | (r.z == v.x) | (r.z == v.y) | (r.z == v.z);
            if (shared) {
                if (j < 32) lo |= 1u << j;
                else hi |= 1u << (j - 32);
            }
        }
    }
    xm[((size_t)b * NBL_MAX + s) * 64 + lane] = make_uint2(lo, hi);
}

hipError_t launch_block_neighbours(const int4* colv, const uint32_t* voff, const uint32_t* vlist, int64_t nF,
                                   int64_t V, uint32_t* nbl, uint2* xm, hipStream_t st) {
    const unsigned nb = (unsigned)((nF + 63) / 64);
    hipLaunchKernelGGL(block_neighbour_tiles, dim3(nb), dim3(64), 0, st, colv, voff, vlist, nF, V, nbl);
    hipLaunchKernelGGL(block_exclusion_masks, dim3(nb, NBL_MAX), dim3(64), 0, st, colv, nF, nbl, xm);
    return hipGetLastError();
}
int64_t block_neighbour_words(int64_t n) { return ((n + 63) / 64) * NBL_STRIDE; }
int64_t block_exclusion_mask_words(int64_t n) { return ((n + 63) / 64) * NBL_MAX * 64; }

// One work-group of NW waves per target block (launch order `order`, else tree order): the block's
// far clusters and near nodes from ff_classify's lists, entry j of each list to wave j mod NW, far
// clusters first; the waves' compensated sums are folded into wave 0's through LDS and written as
// the block's FP64 row sums acc64[k][i].  (Splitting the heaviest blocks over several work-groups
// was measured slower: the launch is bound by the total pair work, not by its last block.  At
// least 3 waves per SIMD: the monopole walk at 327,680 faces takes 1.19 ms of call time at 3, 1.20
// at 4 (128 VGPRs with spills), 1.28 at 5.)
template <int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3))) void ff_eval(
    const ColRec* __restrict__ cols, const int4* __restrict__ colv, const double* __restrict__ c64,
    const double* __restrict__ org, const NodeRec* __restrict__ nodes, int H, int leaf, int64_t nF,
    const uint32_t* __restrict__ bbox, const float4* __restrict__ balls, int64_t Fp, double* __restrict__ acc64,
    const uint32_t* __restrict__ order, int64_t cap, const uint32_t* __restrict__ ent, const uint4* __restrict__ lst,
    const uint32_t* __restrict__ nbl, const uint2* __restrict__ xm) {
    constexpr int NRED = NW > 1 ? NW - 1 : 1;
    __shared__ float red[NRED][2 * NACC][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int64_t b = order ? (int64_t)order[blockIdx.x] : (int64_t)blockIdx.x;
    const int64_t i = b * 64 + lane;
    const double cxd = c64[3 * i], cyd = c64[3 * i + 1], czd = c64[3 * i + 2];
    const ColRec me = cols[i];
    const int4 mv = colv[i];
    double o[3];
    norm_origin(bbox, o);
    const float ax = (float)(cxd - o[0]), ay = (float)(cyd - o[1]), az = (float)(czd - o[2]);
    const float4 tb = balls[b];
    const uint4 L = lst[b];
    const uint32_t* e = ent + (size_t)b * cap;
    float hi[NACC], lo[NACC], acc[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) { hi[k] = 0.f; lo[k] = 0.f; acc[k] = 0.f; }
    // the monopole evaluation keeps its compensation terms in the fold area during the walk (LOL,
    // each wave its own slots, touched once per 64 columns): the registers go to more columns per
    // step below
    constexpr bool LOL = NW > 1;
    static_assert(!LOL || NW * NACC <= NRED * 2 * NACC, "the waves' compensation terms fit the fold area");
    float* lol = LOL ? &red[0][0][0] + (size_t)wave * NACC * 64 : nullptr;
    if constexpr (LOL) {
#pragma unroll
        for (int k = 0; k < NACC; ++k) lol[k * 64 + lane] = 0.f;
    }
    int cnt = 0;
    const int4 nov = make_int4(0, 0, 0, 0);
    // near nodes: exact pairs over their faces.  With the block's neighbour tiles listed, each piece
    // of a node (its faces within one tile) tests its tile against the list (one compare and a
    // ballot) and reads the rows' exclusion bits where it is listed; without the list (curved
    // elements, or more than NBL_MAX such tiles) the vertex ids are compared wherever the node's
    // and the block's vertex balls can meet (conservative margin for FP32)
    __shared__ ColRec nst[NW][64];
    __shared__ int4 nsv[NW][64];
    // the block's neighbour tiles: lane m holds listed tile m
    const uint32_t nn = nbl ? nbl[(size_t)b * NBL_STRIDE] : NBL_OVERFLOW;
    const bool listed = nn <= (uint32_t)NBL_MAX;
    const uint32_t my_tile = listed && (uint32_t)lane < nn ? nbl[(size_t)b * NBL_STRIDE + 1 + lane] : 0xffffffffu;
    const uint2* xmb = xm ? xm + (size_t)b * NBL_MAX * 64 : nullptr;
    // columns per step: 32 independent pair chains (96 VGPRs with the compensation terms in LDS and
    // one inner loop; the level-7 call took 0.943 ms with 2, 0.922 with 4 and 0.915 with 8 in four
    // separate loops, then 0.913 / 0.901 / 0.897 ms with 8 / 16 / 32 in one)
    constexpr int SU = 32;
    {
        // One inner loop for every batch of up to 64 columns: the wave's far clusters (entries
        // j = wave, wave + NW, ... of the far list), 64 at a time as pseudo-faces, then the pieces
        // of its near nodes.  Every lane fetches one column's record (independent loads in flight
        // together); the records are staged in the wave's LDS slots and read back column by column
        // at a wave-uniform address (a broadcast).  A single loop keeps one register assignment for
        // the sums (four inlined loops had the compiler copying 22 of them at every switch between
        // loops).  The exclusion mode is uniform per batch: none, the tile's mask bits, or the
        // vertex compares of the fall-back.  The same pairs in the same order as separate loops.
        const uint32_t nfw = L.y > (uint32_t)wave ? (L.y - 1 - (uint32_t)wave) / NW + 1 : 0u;
        uint32_t fb = 0;          // far clusters staged so far
        uint32_t jn = wave;       // next near entry
        int64_t f = 0, f1 = 0;    // the current near node's remaining faces
        bool cmp_node = false;    // fall-back: the current node compares vertex ids
        ColRec* st = nst[wave];
        int4* sv = nsv[wave];
        for (;;) {
            int m, mode = 0, pos0 = 0;  // mode 0: no exclusion, 1: mask bits, 2: vertex compares
            float px, py, pz;
            float4 c0 = make_float4(0.f, 0.f, 0.f, 0.f), c1 = c0;
            int4 v = nov;
            uint2 mk = make_uint2(0u, 0u);
            if (fb < nfw) {
                m = (int)(nfw - fb < 64u ? nfw - fb : 64u);
                if (lane < m) {
                    // NodeRec (cx, cy, cz, r | a, nx, ny, nz) as a column record (cx, cy, cz, a | nx, ny, nz, 0),
                    // two float4 halves (a whole-struct copy under the condition went through scratch)
                    const float4* src = reinterpret_cast<const float4*>(
                        nodes + e[cap - 1 - ((uint32_t)wave + NW * (fb + (uint32_t)lane))]);
                    const float4 n0 = src[0], n1 = src[1];
                    c0 = make_float4(n0.x, n0.y, n0.z, n1.x);
                    c1 = make_float4(n1.y, n1.z, n1.w, 0.f);
                }
                px = ax;
                py = ay;
                pz = az;
                fb += (uint32_t)m;
            } else {
                if (f >= f1) {  // the next near node
                    if (jn >= L.x) break;
                    const int64_t kk = (int64_t)e[jn];
                    jn += NW;
                    const int lev = 63 - __builtin_clzll((unsigned long long)kk);
                    const int64_t span = (int64_t)1 << (H - lev);
                    f = (kk - ((int64_t)1 << lev)) * span * leaf;
                    f1 = std::min<int64_t>(nF, f + span * leaf);
                    if (!listed) {
                        const NodeRec nd = nodes[kk];
                        cmp_node = !(ball_dist(tb, nd) * (1.f - 1e-5f) > tb.w + nd.r);
                    }
                    continue;
                }
                const int64_t t = f / CTILE;
                const int64_t fend = std::min<int64_t>(f1, (t + 1) * CTILE);
                m = (int)(fend - f);
                if (lane < m) {
                    const float4* src = reinterpret_cast<const float4*>(cols + f + lane);
                    c0 = src[0];
                    c1 = src[1];
                    if (!listed && cmp_node) v = colv[f + lane];
                }
                px = (float)(cxd - org[3 * t]);
                py = (float)(cyd - org[3 * t + 1]);
                pz = (float)(czd - org[3 * t + 2]);
                if (listed) {
                    const uint64_t hit = __ballot(my_tile == (uint32_t)t);
                    if (hit) {
                        mode = 1;
                        mk = xmb[(size_t)(__ffsll((unsigned long long)hit) - 1) * 64 + lane];
                        pos0 = (int)(f - t * CTILE);
                    }
                } else if (cmp_node) {
                    mode = 2;
                }
                f = fend;
            }
            lds_phase();  // the previous batch's reads of the slots come first
            float4* dst = reinterpret_cast<float4*>(st + lane);
            dst[0] = c0;
            dst[1] = c1;
            if (mode == 2) sv[lane] = v;
            lds_phase();  // the reads below see every lane's record
            const uint64_t m64 = ((((uint64_t)mk.y) << 32) | (uint64_t)mk.x) >> pos0;  // bit k: column k
            const uint32_t mlo = (uint32_t)m64, mhi = (uint32_t)(m64 >> 32);
            static_assert(32 % SU == 0, "a step's columns read one 32-bit word of the mask");
            int k = 0;
            for (; k + SU <= m; k += SU) {
                if (mode == 1) {
                    const uint32_t wd = k < 32 ? mlo : mhi;
#pragma unroll
                    for (int u = 0; u < SU; ++u)
                        ff_pair<6, true, 2>(st[k + u], make_int4((int)((wd >> ((k & 31) + u)) & 1u), 0, 0, 0), px, py,
                                            pz, me.nx, me.ny, me.nz, 0, 0, 0, acc);
                } else if (mode == 2) {
#pragma unroll
                    for (int u = 0; u < SU; ++u)
                        ff_pair<6, true, 1>(st[k + u], sv[k + u], px, py, pz, me.nx, me.ny, me.nz, mv.x, mv.y, mv.z,
                                            acc);
                } else {
#pragma unroll
                    for (int u = 0; u < SU; ++u)
                        ff_pair<6, true, 0>(st[k + u], nov, px, py, pz, me.nx, me.ny, me.nz, 0, 0, 0, acc);
                }
                cnt += SU;
                if (cnt >= 64) { ff_fold_at<LOL>(acc, hi, lo, lol, lane); cnt = 0; }
            }
            for (; k < m; ++k) {
                const uint32_t wd = k < 32 ? mlo : mhi;
                if (mode == 1)
                    ff_pair<6, true, 2>(st[k], make_int4((int)((wd >> (k & 31)) & 1u), 0, 0, 0), px, py, pz, me.nx,
                                        me.ny, me.nz, 0, 0, 0, acc);
                else if (mode == 2)
                    ff_pair<6, true, 1>(st[k], sv[k], px, py, pz, me.nx, me.ny, me.nz, mv.x, mv.y, mv.z, acc);
                else
                    ff_pair<6, true, 0>(st[k], nov, px, py, pz, me.nx, me.ny, me.nz, 0, 0, 0, acc);
                if (++cnt >= 64) { ff_fold_at<LOL>(acc, hi, lo, lol, lane); cnt = 0; }
            }
        }
    }
    ff_fold_at<LOL>(acc, hi, lo, lol, lane);
    if constexpr (LOL) {
#pragma unroll
        for (int k = 0; k < NACC; ++k) lo[k] = lol[k * 64 + lane];
        __syncthreads();  // every wave has its terms back before the fold area is reused below
    }
    if constexpr (NW > 1) {
        if (wave > 0) {
#pragma unroll
            for (int kk = 0; kk < NACC; ++kk) {
                red[wave - 1][kk][lane] = hi[kk];
                red[wave - 1][NACC + kk][lane] = lo[kk];
            }
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int j = 0; j < NW - 1; ++j)
#pragma unroll
                for (int kk = 0; kk < NACC; ++kk) {
                    float y = red[j][kk][lane] - lo[kk];
                    float t = hi[kk] + y;
                    lo[kk] = (t - hi[kk]) - y;
                    hi[kk] = t;
                    y = -red[j][NACC + kk][lane] - lo[kk];
                    t = hi[kk] + y;
                    lo[kk] = (t - hi[kk]) - y;
                    hi[kk] = t;
                }
        }
    }
    if (wave == 0) {
#pragma unroll
        for (int kk = 0; kk < NACC; ++kk) acc64[(size_t)kk * Fp + i] = (double)hi[kk] - (double)lo[kk];
    }
}

// The learned correction of the far field: one work-group of NW waves per target block (tree
// order), after ff_eval has written the block's exact near pairs and monopole far pairs to acc64.
// Entry j of the block's far list goes to wave j mod NW; mlp_correction gates each cluster (the
// wave skips the network when no row qualifies) and adds the network's predicted corrections to the
// wave's FP32 sums, folded every 64 clusters as in ff_eval and across the waves through the MLP
// scratch; wave 0 adds them to acc64.  Keeping the network out of ff_eval lets the pairs run at
// that kernel's occupancy (the level-7 learned call took 2.06 ms in one kernel, whose pairs alone,
// with the gate closed, took 0.98 ms against the monopole kernel's 0.72 ms).
template <int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3))) void ff_correct(
    const ColRec* __restrict__ cols, const double* __restrict__ c64, const NodeRec* __restrict__ nodes,
    const NodeMom* __restrict__ moms, const MlpPacked* __restrict__ W, const uint32_t* __restrict__ bbox,
    int64_t Fp, double* __restrict__ acc64, int64_t cap, const uint32_t* __restrict__ ent,
    const uint4* __restrict__ lst) {
    constexpr int NRED = NW > 1 ? NW - 1 : 1;
    __shared__ MlpScratch ms[NW];
    static_assert(sizeof(MlpScratch) * NW >= sizeof(float) * NRED * 2 * NACC * 64, "fold space");
    float (*red)[2 * NACC][64] = reinterpret_cast<float (*)[2 * NACC][64]>(&ms[0]);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int64_t b = blockIdx.x;
    const int64_t i = b * 64 + lane;
    const double cxd = c64[3 * i], cyd = c64[3 * i + 1], czd = c64[3 * i + 2];
    const ColRec me = cols[i];
    double o[3];
    norm_origin(bbox, o);
    const float ax = (float)(cxd - o[0]), ay = (float)(cyd - o[1]), az = (float)(czd - o[2]);
    const uint4 L = lst[b];
    const uint32_t* e = ent + (size_t)b * cap;
    float hi[NACC], lo[NACC], acc[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) { hi[k] = 0.f; lo[k] = 0.f; acc[k] = 0.f; }
    int cnt = 0;
    // the wave's clusters 64 at a time: every lane fetches one record (independent loads in flight
    // together), staged in LDS and read back one by one at a wave-uniform address, so that the gate
    // of a cluster the network skips costs no dependent load
    __shared__ NodeRec cst[NW][64];
    __shared__ uint32_t cix[NW][64];
    const uint32_t nfw = L.y > (uint32_t)wave ? (L.y - 1 - (uint32_t)wave) / NW + 1 : 0u;
    for (uint32_t base = 0; base < nfw; base += 64) {
        const uint32_t m = nfw - base < 64u ? nfw - base : 64u;
        float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0;
        uint32_t kx = 0u;
        if ((uint32_t)lane < m) {
            kx = e[cap - 1 - ((uint32_t)wave + NW * (base + (uint32_t)lane))];
            const float4* src = reinterpret_cast<const float4*>(nodes + kx);
            n0 = src[0];
            n1 = src[1];
        }
        lds_phase();  // the previous batch's reads of the slots come first
        float4* dst = reinterpret_cast<float4*>(&cst[wave][lane]);
        dst[0] = n0;
        dst[1] = n1;
        cix[wave][lane] = kx;
        lds_phase();  // the reads below see every lane's record
        // the batch's gates first (a few instructions per cluster, no branch), then the network on
        // the clusters some row needs, in order
        uint64_t need = 0ull;
        for (uint32_t k = 0; k < m; ++k) {
            const NodeRec nd = cst[wave][k];
            if (__any(mlp_gate(W, nd, ax, ay, az))) need |= 1ull << k;
        }
        while (need) {
            const uint32_t k = (uint32_t)(__ffsll((unsigned long long)need) - 1);
            need &= need - 1ull;
            const NodeRec nd = cst[wave][k];
            mlp_correction(W, nd, moms[cix[wave][k]], ax, ay, az, me.nx, me.ny, me.nz, ms[wave], acc);
            if (++cnt >= 64) { ff_fold(acc, hi, lo); cnt = 0; }
        }
    }
    ff_fold(acc, hi, lo);
    if constexpr (NW > 1) {
        __syncthreads();  // the MLP scratch is reused below
        if (wave > 0) {
#pragma unroll
            for (int kk = 0; kk < NACC; ++kk) {
                red[wave - 1][kk][lane] = hi[kk];
                red[wave - 1][NACC + kk][lane] = lo[kk];
            }
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int j = 0; j < NW - 1; ++j)
#pragma unroll
                for (int kk = 0; kk < NACC; ++kk) {
                    float y = red[j][kk][lane] - lo[kk];
                    float t = hi[kk] + y;
                    lo[kk] = (t - hi[kk]) - y;
                    hi[kk] = t;
                    y = -red[j][NACC + kk][lane] - lo[kk];
                    t = hi[kk] + y;
                    lo[kk] = (t - hi[kk]) - y;
                    hi[kk] = t;
                }
        }
    }
    if (wave == 0) {
#pragma unroll
        for (int kk = 0; kk < NACC; ++kk) acc64[(size_t)kk * Fp + i] += (double)hi[kk] - (double)lo[kk];
    }
}

// MurmurHash3's 32-bit finaliser (Appleby): a bijective avalanche mix.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// Deterministic sample selection: u(seed, block, node) = fmix32(fmix32(fmix32(seed) ^ block) ^ node).
__device__ __forceinline__ uint32_t sample_hash(uint32_t seed, uint32_t block, uint32_t node) {
    return fmix32(fmix32(fmix32(seed) ^ block) ^ node);
}

// Training samples: the walk and decisions of ff_classify; for far clusters with at most max_faces
// faces, selected with probability ~ sel (hash of seed, block, node), up to `quota` per block, every
// row of the block yields one sample: features and the (exact - monopole) correction in units.
// Output rows [(b * quota + c) * 64 + lane]; rows not filled keep weight 0 (targets[.][15]).
__global__ __launch_bounds__(64) void farfield_samples(const ColRec* __restrict__ cols, const int4* __restrict__ colv,
                                                       const double* __restrict__ c64,
                                                       const NodeRec* __restrict__ nodes,
                                                       const NodeMom* __restrict__ moms, int H, int leaf, int64_t nF,
                                                       const uint32_t* __restrict__ bbox,
                                                       const float4* __restrict__ balls, float theta, uint32_t seed,
                                                       uint32_t sel, int quota, int64_t max_faces,
                                                       float* __restrict__ feats, float* __restrict__ targets,
                                                       const MlpPacked* __restrict__ W, float* __restrict__ pred) {
    __shared__ int stack[FF_STACK];
    __shared__ MlpScratch ms;
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t i = b * 64 + lane;
    const bool rowok = i < nF;
    double o[3];
    norm_origin(bbox, o);
    const float ax = (float)(c64[3 * i] - o[0]), ay = (float)(c64[3 * i + 1] - o[1]), az = (float)(c64[3 * i + 2] - o[2]);
    const ColRec me = cols[i];
    const float4 tb = balls[b];
    const int4 nov = make_int4(0, 0, 0, 0);
    const int64_t leaf0 = (int64_t)1 << H;
    int taken = 0;
    // clear this block's output rows
    for (int c = 0; c < quota; ++c) {
        const int64_t row = (b * quota + c) * 64 + lane;
        for (int k = 0; k < 32; ++k) feats[row * 32 + k] = 0.f;
        for (int k = 0; k < 16; ++k) targets[row * 16 + k] = 0.f;
    }
    if (lane == 0) stack[0] = 1;
    int sz = 1;
    while (sz > 0 && taken < quota) {
        lds_phase();  // the pops below read entries other lanes pushed
        const int n = sz < 64 ? sz : 64;
        sz -= n;
        const bool act = lane < n;
        const int k = act ? stack[sz + lane] : 0;
        NodeRec nd = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (act) nd = nodes[k];
        const bool valid = act && nd.a > 0.f;
        const float dist = ball_dist(tb, nd);
        const bool far = valid && (2.f * nd.r < theta * (dist - tb.w));
        const bool isleaf = (int64_t)k >= leaf0;
        bool open = valid && !far && !isleaf;
        const int nopen = __popcll(__ballot(open));
        if (sz + 2 * nopen <= FF_STACK) {
            const uint64_t om = __ballot(open);
            const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
            if (open) {
                const int pos = sz + 2 * (int)__popcll(om & lt);
                stack[pos] = 2 * k + 1;
                stack[pos + 1] = 2 * k;
            }
            sz += 2 * nopen;
        }
        uint64_t fm = __ballot(far);
        while (fm && taken < quota) {
            const int l = (int)__builtin_ctzll(fm);
            fm &= fm - 1;
            const int kk = __builtin_amdgcn_readlane(k, l);
            const int lev = 31 - __builtin_clz((unsigned)kk);
            const int64_t span = (int64_t)1 << (H - lev);
            const int64_t f0 = ((int64_t)kk - ((int64_t)1 << lev)) * span * leaf;
            const int64_t f1 = std::min<int64_t>(nF, f0 + span * leaf);
            if (f1 - f0 > max_faces || sample_hash(seed, (uint32_t)b, (uint32_t)kk) > sel) continue;
            NodeRec cn;
            cn.cx = lane_f(nd.cx, l); cn.cy = lane_f(nd.cy, l); cn.cz = lane_f(nd.cz, l); cn.r = lane_f(nd.r, l);
            cn.a = lane_f(nd.a, l); cn.nx = lane_f(nd.nx, l); cn.ny = lane_f(nd.ny, l); cn.nz = lane_f(nd.nz, l);
            const NodeMom mm = moms[kk];
            // exact contribution of the cluster's faces, in absolute (normalised) coordinates
            float ex[NACC], mo[NACC];
            for (int q = 0; q < NACC; ++q) { ex[q] = 0.f; mo[q] = 0.f; }
            for (int64_t f = f0; f < f1; ++f) {
                ColRec cr = cols[f];
                // columns are stored relative to their tile origin; use absolute (normalised) ones here
                cr.cx = (float)(c64[3 * f] - o[0]);
                cr.cy = (float)(c64[3 * f + 1] - o[1]);
                cr.cz = (float)(c64[3 * f + 2] - o[2]);
                ff_pair<6, true, false>(cr, nov, ax, ay, az, me.nx, me.ny, me.nz, 0, 0, 0, ex);
            }
            const ColRec mc = {cn.cx, cn.cy, cn.cz, cn.a, cn.nx, cn.ny, cn.nz, 0.f};
            ff_pair<6, true, false>(mc, nov, ax, ay, az, me.nx, me.ny, me.nz, 0, 0, 0, mo);
            Frame fr;
            float x[32];
            ff_features(ax, ay, az, me.nx, me.ny, me.nz, cn, mm, fr, x);
            float u6, u7;
            out_units(cn.a, fr, u6, u7);
            float cex[3], cmo[3], dsd[3], dc[3];
            net_c(ex, me.nx, me.ny, me.nz, cex);
            net_c(mo, me.nx, me.ny, me.nz, cmo);
            for (int q = 0; q < 3; ++q) { dsd[q] = ex[2 + q] - mo[2 + q]; dc[q] = cex[q] - cmo[q]; }
            float y[16];
            y[0] = (ex[0] - mo[0]) / u6;
            to_frame(dsd, fr, y + 1);
            to_frame(dc, fr, y + 4);
            for (int q = 1; q < 4; ++q) y[q] /= u6;
            for (int q = 4; q < 7; ++q) y[q] /= u7;
            for (int q = 7; q < 16; ++q) y[q] = 0.f;
            y[14] = (float)kk;  // the cluster's node (exact below 2^24): which cluster the sample is of
            bool fin = rowok;
            for (int q = 0; q < 7; ++q) fin &= isfinite(y[q]);
            y[15] = fin ? 1.f : 0.f;
            const int64_t row = (b * quota + taken) * 64 + lane;
            if (pred) {
                // the in-walk inference on exactly these features (parity hook for the fused path)
                float yp[16];
                mlp_infer64(W, x, ms, yp);
                for (int q = 0; q < 16; ++q) pred[row * 16 + q] = yp[q];
            }
            for (int q = 0; q < 32; ++q) feats[row * 32 + q] = x[q];
            for (int q = 0; q < 16; ++q) targets[row * 16 + q] = fin ? y[q] : 0.f;
            ++taken;
        }
    }
}

// ---- k-d ordering of the faces (tree build) -------------------------------------------------------
// The faces are ordered so that every node of the implicit complete binary tree is a compact
// piece of the surface: level by level, the faces of each node are sorted along the longest axis
// of the node's centroid bounding box; the node's first child then takes the lower part (its leaf
// capacity) and the second child the rest.  This is a balanced k-d (median-like) split on face
// centroids, done with one stable radix sort per level on (node index, quantised coordinate).

__global__ void kd_centroids(const double* __restrict__ X, int64_t V, const int32_t* __restrict__ F, int64_t nF,
                             float4* __restrict__ cen, uint32_t* __restrict__ perm) {
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f >= nF) return;
    const int32_t a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
    if (a >= 0 && a < V && b >= 0 && b < V && c >= 0 && c < V) {
        const double x = (X[3 * (int64_t)a] + X[3 * (int64_t)b] + X[3 * (int64_t)c]) / 3.0;
        const double y = (X[3 * (int64_t)a + 1] + X[3 * (int64_t)b + 1] + X[3 * (int64_t)c + 1]) / 3.0;
        const double z = (X[3 * (int64_t)a + 2] + X[3 * (int64_t)b + 2] + X[3 * (int64_t)c + 2]) / 3.0;
        if (isfinite(x + y + z)) r = make_float4((float)x, (float)y, (float)z, 0.f);
    }
    cen[f] = r;
    perm[f] = (uint32_t)f;
}

// Curved cubic elements: item r = quadrature point r % Q of element r / Q (nodes F10[10 (r / Q) ..]),
// at x(b) of the element's cubic map; the tree is built over these points.
__global__ void kd_centroids_p3(const double* __restrict__ X, int64_t V, const int32_t* __restrict__ F10, int64_t nF,
                                int Q, float4* __restrict__ cen, uint32_t* __restrict__ perm) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= nF * Q) return;
    const int64_t f = r / Q;
    double b[3], wq;
    quad_point(Q, (int)(r % Q), b, wq);
    double phi[P3_NODES], ds[P3_NODES], dt[P3_NODES];
    p3_shape(b, phi, ds, dt);
    double x[3] = {0.0, 0.0, 0.0};
    bool ok = true;
    for (int k = 0; k < P3_NODES; ++k) {
        const int32_t v = F10[P3_NODES * f + k];
        if (v < 0 || v >= V) { ok = false; break; }
        for (int d = 0; d < 3; ++d) x[d] += phi[k] * X[3 * (int64_t)v + d];
    }
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ok && isfinite(x[0] + x[1] + x[2])) c = make_float4((float)x[0], (float)x[1], (float)x[2], 0.f);
    cen[r] = c;
    perm[r] = (uint32_t)r;
}

__device__ __forceinline__ uint32_t f2o(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ void kd_box_init(uint32_t* __restrict__ nb, int64_t nnodes) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < nnodes * 6) nb[t] = (t % 6) < 3 ? 0xffffffffu : 0u;
}

// Centroid bounding box of every node of `level` (min xyz, max xyz in the order-preserving encoding).
__global__ void kd_node_bbox(const uint32_t* __restrict__ perm, const float4* __restrict__ cen, int64_t nF,
                             int64_t node_faces, uint32_t* __restrict__ nb) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool act = i < nF;
    const int64_t j = act ? i / node_faces : -1;
    float4 c = act ? cen[perm[i]] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t j0 = __shfl(j, __builtin_ctzll(__ballot(act) | (1ull << 63)));
    const bool uniform = __ballot(act && j != j0) == 0ull;
    if (uniform) {
        float mn[3] = {act ? c.x : INFINITY, act ? c.y : INFINITY, act ? c.z : INFINITY};
        float mx[3] = {act ? c.x : -INFINITY, act ? c.y : -INFINITY, act ? c.z : -INFINITY};
        for (int d = 0; d < 3; ++d)
            for (int off = 32; off > 0; off >>= 1) {
                mn[d] = fminf(mn[d], __shfl_xor(mn[d], off));
                mx[d] = fmaxf(mx[d], __shfl_xor(mx[d], off));
            }
        if ((threadIdx.x & 63) == 0 && j0 >= 0)
            for (int d = 0; d < 3; ++d) {
                atomicMin(&nb[6 * j0 + d], f2o(mn[d]));
                atomicMax(&nb[6 * j0 + 3 + d], f2o(mx[d]));
            }
    } else if (act) {
        const float v[3] = {c.x, c.y, c.z};
        for (int d = 0; d < 3; ++d) {
            atomicMin(&nb[6 * j + d], f2o(v[d]));
            atomicMax(&nb[6 * j + 3 + d], f2o(v[d]));
        }
    }
}

// The same boxes at the levels whose nodes hold at least KD_BIG faces: a work-group covers KD_BIG
// consecutive sorted faces (KD_PER per thread), which meet at most two nodes (A, the node of the
// first face, and A + 1); the two boxes are reduced over the work-group and each gets one set of
// atomics per work-group.  With one thread per face, every wave of the launch sent its atomics to
// the same six words at the top level (350 us at 327,680 faces).  Min and max are exact, so the
// boxes are the same bits either way.
constexpr int KD_PER = 8;
constexpr int KD_BIG = 256 * KD_PER;

__global__ __launch_bounds__(256) void kd_node_bbox_big(const uint32_t* __restrict__ perm,
                                                        const float4* __restrict__ cen, int64_t nF,
                                                        int64_t node_faces, uint32_t* __restrict__ nb) {
    __shared__ float red[4][12];
    const int64_t base = blockIdx.x * (int64_t)KD_BIG;
    const int64_t jA = base / node_faces, bound = (jA + 1) * node_faces;
    // [0..2] min, [3..5] max of node A; [6..11] the same for node A + 1
    float r[12];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r[d] = r[6 + d] = INFINITY;
        r[3 + d] = r[9 + d] = -INFINITY;
    }
#pragma unroll
    for (int k = 0; k < KD_PER; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        if (i < nF) {
            const float4 c = cen[perm[i]];
            const float v[3] = {c.x, c.y, c.z};
            const bool a = i < bound;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                r[d] = a ? fminf(r[d], v[d]) : r[d];
                r[3 + d] = a ? fmaxf(r[3 + d], v[d]) : r[3 + d];
                r[6 + d] = a ? r[6 + d] : fminf(r[6 + d], v[d]);
                r[9 + d] = a ? r[9 + d] : fmaxf(r[9 + d], v[d]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 12; ++q)
        for (int off = 32; off > 0; off >>= 1) {
            const float o = __shfl_xor(r[q], off);
            r[q] = (q % 6) < 3 ? fminf(r[q], o) : fmaxf(r[q], o);
        }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < 12; ++q) red[threadIdx.x >> 6][q] = r[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < 12; ++q)
            for (int w = 1; w < 4; ++w) r[q] = (q % 6) < 3 ? fminf(r[q], red[w][q]) : fmaxf(r[q], red[w][q]);
        for (int h = 0; h < 2; ++h) {
            const float* b = r + 6 * h;
            if (!(b[0] <= b[3])) continue;  // no face of this node here
            const int64_t j = jA + h;
            for (int d = 0; d < 3; ++d) {
                atomicMin(&nb[6 * j + d], f2o(b[d]));
                atomicMax(&nb[6 * j + 3 + d], f2o(b[3 + d]));
            }
        }
    }
}

// key = (node index << qbits) | coordinate along the node's longest axis quantised to qbits.
__global__ void kd_keys(const uint32_t* __restrict__ perm, const float4* __restrict__ cen, int64_t nF,
                        int64_t node_faces, const uint32_t* __restrict__ nb, int qbits, uint32_t* __restrict__ keys) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nF) return;
    const int64_t j = i / node_faces;
    const float4 c = cen[perm[i]];
    float lo[3], ext[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = ordered_to_float(nb[6 * j + d]);
        ext[d] = ordered_to_float(nb[6 * j + 3 + d]) - lo[d];
    }
    int ax = 0;
    if (ext[1] > ext[ax]) ax = 1;
    if (ext[2] > ext[ax]) ax = 2;
    const float v = ax == 0 ? c.x : (ax == 1 ? c.y : c.z);
    const float maxq = (float)((1u << qbits) - 1u);
    float s = ext[ax] > 0.f ? (v - lo[ax]) / ext[ax] * maxq : 0.f;
    s = fminf(fmaxf(s, 0.f), maxq);
    const uint32_t q = isfinite(s) ? (uint32_t)s : 0u;
    keys[i] = ((uint32_t)j << qbits) | q;
}

hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* ktmp, uint32_t* vtmp, int64_t n, int bits,
                      uint32_t* hist, uint32_t* off, hipStream_t st);

// perm (n entries) <- k-d order of the items for a tree of height H over leaves of `leaf` items.
// Items: the nF faces (Q = 0: F holds 3 vertex ids per face), or the Q quadrature points of each
// of the nF curved cubic elements (Q >= 1: F holds 10 node ids per element), n = nF Q.
// Scratch: cen (n float4), nb (6 * 2^max(H-1,0) words), keys/ktmp/vtmp (n words), hist/off.
hipError_t build_kd_order(const double* X, int64_t V, const int32_t* F, int64_t nF, int Q, int leaf, int H,
                          float4* cen, uint32_t* nb, uint32_t* perm, uint32_t* keys, uint32_t* ktmp, uint32_t* vtmp,
                          uint32_t* hist, uint32_t* off, hipStream_t st) {
    if (Q > 0) {
        hipLaunchKernelGGL(kd_centroids_p3, dim3((unsigned)((nF * Q + 255) / 256)), dim3(256), 0, st, X, V, F, nF, Q,
                           cen, perm);
        nF *= Q;
    } else {
        hipLaunchKernelGGL(kd_centroids, dim3((unsigned)((nF + 255) / 256)), dim3(256), 0, st, X, V, F, nF, cen, perm);
    }
    const unsigned g = (unsigned)((nF + 255) / 256);
    for (int level = 0; level < H; ++level) {
        const int64_t nnodes = (int64_t)1 << level;
        const int64_t node_faces = ((int64_t)1 << (H - level)) * leaf;
        hipLaunchKernelGGL(kd_box_init, dim3((unsigned)((nnodes * 6 + 255) / 256)), dim3(256), 0, st, nb, nnodes);
        if (node_faces >= KD_BIG)
            hipLaunchKernelGGL(kd_node_bbox_big, dim3((unsigned)((nF + KD_BIG - 1) / KD_BIG)), dim3(256), 0, st, perm,
                               cen, nF, node_faces, nb);
        else
            hipLaunchKernelGGL(kd_node_bbox, dim3(g), dim3(256), 0, st, perm, cen, nF, node_faces, nb);
        const int qbits = std::min(16, 32 - level);
        hipLaunchKernelGGL(kd_keys, dim3(g), dim3(256), 0, st, perm, cen, nF, node_faces, nb, qbits, keys);
        hipError_t e = radix_sort(keys, perm, ktmp, vtmp, nF, level + qbits, hist, off, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// ---- host side ----------------------------------------------------------------------------------

int tree_height(int64_t nF, int leaf) {
    const int64_t nleaf = (nF + leaf - 1) / leaf;
    int H = 0;
    while (((int64_t)1 << H) < nleaf) ++H;
    return H;
}

size_t tree_node_bytes(int H) { return ((size_t)2 << H) * sizeof(NodeF64); }
size_t tree_rec_bytes(int H) { return ((size_t)2 << H) * (sizeof(NodeRec) + sizeof(NodeMom)); }

// Node moments (leaves, then the subtrees) and, with balls given, the target blocks' balls: with
// leaves of 32 faces inside the leaf pass (a wave's two leaves are one block), else by target_balls.
hipError_t launch_tree_moments(const double* c64, const double* geo, const int4* colv, const double* X,
                               const uint32_t* bbox, int64_t nF, int leaf, int H, void* nodes64, void* recs, bool mom2,
                               float4* balls, hipStream_t st) {
    NodeF64* n = (NodeF64*)nodes64;
    NodeRec* r = (NodeRec*)recs;
    NodeMom* m = (NodeMom*)(r + ((size_t)2 << H));
    const int64_t nslot = (int64_t)1 << H;
    int G = 1;
    while (G < leaf && G < 64) G *= 2;
    const int64_t per_wg = (int64_t)MOM_LEAF_WAVES * (64 / G);  // leaf slots per work-group
    const dim3 lg((unsigned)((nslot + per_wg - 1) / per_wg)), lb(64 * MOM_LEAF_WAVES);
    float4* fused = leaf == 32 ? balls : nullptr;
    if (mom2)
        hipLaunchKernelGGL(leaf_moments<true>, lg, lb, 0, st, c64, geo, colv, X, bbox, nF, leaf, H, G, n, r, m, fused);
    else
        hipLaunchKernelGGL(leaf_moments<false>, lg, lb, 0, st, c64, geo, colv, X, bbox, nF, leaf, H, G, n, r, m, fused);
    if (balls && !fused)
        hipLaunchKernelGGL(target_balls, dim3((unsigned)((nF + 63) / 64)), dim3(64), 0, st, c64, colv, X, bbox, nF,
                           balls);
    for (int L = H; L > 0;) {
        const int nl = std::min(L, MOM_SUB);
        const dim3 sg((unsigned)(((int64_t)1 << L) >> nl)), sb(1 << nl);
        if (mom2) hipLaunchKernelGGL(subtree_moments<true>, sg, sb, 0, st, L, nl, bbox, n, r, m);
        else hipLaunchKernelGGL(subtree_moments<false>, sg, sb, 0, st, L, nl, bbox, n, r, m);
        L -= nl;
    }
    return hipGetLastError();
}

hipError_t launch_farfield_samples(const ColRec* cols, const int4* colv, const double* c64, const double* X,
                                  const uint32_t* bbox, const void* recs, int H, int leaf, int64_t nF, float theta,
                                  uint32_t seed, uint32_t sel, int quota, int64_t max_faces, float4* balls,
                                  float* feats, float* targets, const void* mlp_packed, float* pred, hipStream_t st) {
    const int64_t nb = (nF + 63) / 64;
    const NodeRec* r = (const NodeRec*)recs;
    const NodeMom* m = (const NodeMom*)(r + ((size_t)2 << H));
    hipLaunchKernelGGL(target_balls, dim3((unsigned)nb), dim3(64), 0, st, c64, colv, X, bbox, nF, balls);
    hipLaunchKernelGGL(farfield_samples, dim3((unsigned)nb), dim3(64), 0, st, cols, colv, c64, r, m, H, leaf, nF, bbox, balls,
                       theta, seed, sel, quota, max_faces, feats, targets, (const MlpPacked*)mlp_packed, pred);
    return hipGetLastError();
}

// Launch order of the walk's target blocks: heaviest first, by the work each block's lists hold in
// this call (work-groups start in launch order, so the few blocks with several times the average
// near work no longer start late and set the end of the launch); equal keys keep tree order, and
// all-zero work gives the identity.  Used for the monopole walk (1.76 -> 1.55 ms at 327,680 faces
// when introduced); the walk with the learned correction runs in tree order, which it prefers (2.76
// against 2.83 ms ordered: its heavy part, the network on far clusters, is spread more evenly, and
// neighbouring blocks share near leaves in the caches).  The key is a monotone 8-bit code of the
// work (exponent and three mantissa bits).  The order changes only when blocks run, never what
// they compute.
__device__ __forceinline__ uint32_t work_key(uint32_t w) {
    uint32_t code = w;
    if (w >= 8u) {
        const int e = 31 - __clz((int)w);
        code = ((uint32_t)(e - 2) << 3) | ((w >> (e - 3)) & 7u);
    }
    return 255u - code;
}

// One work-group: a stable counting sort of the nb keys into `order` (null: none), chunk by chunk
// of FO_NT blocks (ranks among equal keys from wave ballots, then across the waves in LDS), and,
// with lst and stats, the call's interaction counts from the blocks' list records (far clusters,
// near columns and visited nodes summed, blocks, the largest near-column and far-cluster counts of
// a block) in the same pass.  Replaces a key kernel, a radix pass, two copies and a reduction.
constexpr int FO_NT = 1024;
constexpr int FO_KEYS = 32768;  // blocks whose 8-bit keys the sort keeps in LDS (beyond: re-read)

__global__ __launch_bounds__(FO_NT) void ff_order_sort(const uint32_t* __restrict__ work, int64_t nb,
                                                       uint32_t* __restrict__ order, const uint4* __restrict__ lst,
                                                       unsigned long long* __restrict__ stats) {
    constexpr int NWV = FO_NT / 64;
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[NWV][256];
    __shared__ unsigned long long red[NWV][5];
    __shared__ uint8_t kc[FO_KEYS];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int k = tid; k < 256; k += FO_NT) base[k] = 0u;
    unsigned long long far = 0, cols = 0, vis = 0, mcols = 0, mfar = 0;
    // the keys and counts first: independent loads (several in flight), keys kept in LDS
#pragma unroll 4
    for (int64_t c0 = 0; c0 < nb; c0 += FO_NT) {
        const int64_t b = c0 + tid;
        if (b < nb) {
            if (order && b < FO_KEYS) kc[b] = (uint8_t)work_key(work[b]);
            if (lst) {
                const uint4 L = lst[b];
                far += L.y; cols += L.z; vis += L.w;
                mcols = L.z > mcols ? L.z : mcols;
                mfar = L.y > mfar ? L.y : mfar;
            }
        }
    }
    __syncthreads();
    auto key_of = [&](int64_t b) { return b < FO_KEYS ? (uint32_t)kc[b] : work_key(work[b]); };
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // lanes of this wave holding the same key as this lane (valid lanes only)
    auto same_key = [&](bool valid, uint32_t k) {
        uint64_t same = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t m = __ballot(valid && ((k >> bit) & 1u));
            same &= ((k >> bit) & 1u) ? m : ~m;
        }
        return same;
    };
    if (order)
        for (int64_t c0 = 0; c0 < nb; c0 += FO_NT) {
            // counts, one LDS add per key and wave (per-element adds on the few distinct keys
            // serialised); the order of the adds is immaterial
            const int64_t b = c0 + tid;
            const bool valid = b < nb;
            const uint32_t k = valid ? key_of(b) : 0u;
            const uint64_t same = same_key(valid, k);
            if (valid && (same & lt) == 0ull) atomicAdd(&base[k], (uint32_t)__popcll(same));
        }
    if (lst && stats) {
        for (int off = 32; off > 0; off >>= 1) {
            far += __shfl_xor(far, off);
            cols += __shfl_xor(cols, off);
            vis += __shfl_xor(vis, off);
            const unsigned long long a = __shfl_xor(mcols, off), c = __shfl_xor(mfar, off);
            mcols = a > mcols ? a : mcols;
            mfar = c > mfar ? c : mfar;
        }
        if (lane == 0) { red[w][0] = far; red[w][1] = cols; red[w][2] = vis; red[w][3] = mcols; red[w][4] = mfar; }
    }
    __syncthreads();
    if (lst && stats && tid == 0) {
        for (int k = 1; k < NWV; ++k) {
            far += red[k][0]; cols += red[k][1]; vis += red[k][2];
            mcols = red[k][3] > mcols ? red[k][3] : mcols;
            mfar = red[k][4] > mfar ? red[k][4] : mfar;
        }
        stats[0] = far; stats[1] = cols; stats[2] = vis; stats[3] = (unsigned long long)nb;
        stats[4] = mcols; stats[5] = mfar;
    }
    if (!order) return;  // uniform
    if (w == 0) {  // exclusive scan of the 256 counts, 4 per lane
        uint32_t v[4];
        for (int q = 0; q < 4; ++q) v[q] = base[4 * lane + q];
        const uint32_t s = v[0] + v[1] + v[2] + v[3];
        uint32_t x = s;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        uint32_t e = x - s;
        for (int q = 0; q < 4; ++q) { base[4 * lane + q] = e; e += v[q]; }
    }
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += FO_NT) {
        for (int k = tid; k < NWV * 256; k += FO_NT) wcnt[k >> 8][k & 255] = 0u;
        __syncthreads();
        const int64_t b = c0 + tid;
        const bool valid = b < nb;
        const uint32_t k = valid ? key_of(b) : 0u;
        const uint64_t same = same_key(valid, k);
        const uint32_t rank = (uint32_t)__popcll(same & lt);
        if (valid && rank == 0u) wcnt[w][k] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[k] + rank;
            for (int v = 0; v < w; ++v) pos += wcnt[v][k];
            order[pos] = (uint32_t)b;
        }
        __syncthreads();
        for (int kk = tid; kk < 256; kk += FO_NT) {
            uint32_t t = 0u;
            for (int v = 0; v < NWV; ++v) t += wcnt[v][kk];
            base[kk] += t;
        }
        __syncthreads();
    }
}

// order (null: none): heaviest first by work; lst and stats (nullable): the walk's counts
hipError_t launch_ff_order(const uint32_t* work, int64_t nb, uint32_t* order, const uint4* lst,
                           unsigned long long* stats, hipStream_t st) {
    hipLaunchKernelGGL(ff_order_sort, dim3(1), dim3(FO_NT), 0, st, work, nb, order, lst, stats);
    return hipGetLastError();
}

// Entries per block of the walk's lists: every non-empty leaf at most once, within 8 GiB in all.
int64_t ff_list_cap(int64_t n, int leaf) {
    const int64_t nb = (n + 63) / 64, nleaf = (n + leaf - 1) / leaf;
    const int64_t budget = ((int64_t)2 << 30) / std::max<int64_t>(nb, 1);
    return std::max<int64_t>(1, std::min(nleaf, budget));
}

// The far field of the tree's target blocks (their balls written by launch_tree_moments): the
// classify pass (lists, the blocks' work, interaction counts), the launch order (monopole: heaviest blocks first by this call's work; with
// the correction: tree order, which it prefers), the evaluation.  sort: keys, vals, ktmp, vtmp,
// hist, hoff of a radix sort of ceil(nF / 64) entries.  ev0 / ev1 (nullable): HIP events recorded
// around the evaluation launch alone.
hipError_t launch_farfield(const ColRec* cols, const int4* colv, const double* c64, const double* org,
                           const double* X, const uint32_t* bbox, const void* recs, int H, int leaf, int64_t nF,
                           int64_t Fp, float theta, const void* mlp_packed, float4* balls, double* acc64,
                           unsigned long long* stats, uint32_t* work, uint32_t* ent, uint4* lst, int64_t cap,
                           uint32_t* flags, uint32_t* const sort[6], const uint32_t* nbl, const uint2* xm,
                           hipEvent_t ev0, hipEvent_t ev1, hipStream_t st) {
    const int64_t nb = (nF + 63) / 64;  // padding rows past nF ride along in the last block only
    const NodeRec* r = (const NodeRec*)recs;
    const NodeMom* m = (const NodeMom*)(r + ((size_t)2 << H));
    hipLaunchKernelGGL(ff_classify, dim3((unsigned)((nb + FFC_NW - 1) / FFC_NW)), dim3(64 * FFC_NW), 0, st, r, H, leaf,
                       nF, balls, theta, cap, ent, lst, work, flags);
    // launch order (heaviest blocks first) and the interaction counts, in one work-group
    const uint32_t* order = sort[1];
    hipError_t e = launch_ff_order(work, nb, sort[1], lst, stats, st);
    if (e != hipSuccess) return e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;  // timing: the evaluation alone
    hipLaunchKernelGGL((ff_eval<FF_NW>), dim3((unsigned)nb), dim3(64 * FF_NW), 0, st, cols, colv, c64, org, r, H, leaf,
                       nF, bbox, balls, Fp, acc64, order, cap, ent, lst, nbl, xm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (mlp_packed)  // the learned correction, added to the row sums
        hipLaunchKernelGGL((ff_correct<FF_NW_LEARNED>), dim3((unsigned)nb), dim3(64 * FF_NW_LEARNED), 0, st, cols, c64,
                           r, m, (const MlpPacked*)mlp_packed, bbox, Fp, acc64, cap, ent, lst);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return ev1 ? hipEventRecord(ev1, st) : hipSuccess;
}

}  // namespace tpe
