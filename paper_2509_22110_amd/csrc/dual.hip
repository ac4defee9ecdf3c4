// Dual-tree (cluster-cluster) far field: both integrals clustered.
//
// The paper clusters only the inner integrals (tree.hip); the clustering it compares against
// (Sec. 3.2) clusters both and then has to carry derivatives back from the clusters to the faces.
// That scheme, on the same implicit k-d tree:
//   - Approximate energy.  Every ordered pair of faces (S, T) is covered exactly once by a pair of
//     same-level clusters (A, B), A containing S and B containing T: either a far pair, replaced by
//     one interaction of two pseudo-faces (area A_A, centroid C_A, unit mean normal nu_A = N_A/|N_A|
//     with N_A = sum_{S in A} a_S n_S, and likewise for B), or a pair of near dual leaves, summed
//     exactly face by face with the shared-vertex exclusion.  (A, B) is far when
//     2 max(r_A, r_B) < theta |C_A - C_B| (theta <= 1, so the vertex balls are disjoint and no far
//     pair holds two faces sharing a vertex).
//   - Lists.  The tree is complete, so the pairs are found level by level as in a fast multipole
//     method: the candidates of node A are the children of its parent's near list; each is far
//     (an interaction of A) or near (kept for A's children).  Dual leaves are the nodes of 64
//     faces (one wave of rows); their near lists are summed exactly.
//   - Gradient.  The approximate energy is differentiated exactly.  For a far pair the pseudo-face
//     A collects the exact kernel's 11 row sums (K, S0, Sd, Sdd, Sn) against the pseudo-face B,
//     giving dE/dA_A = K, dE/dC_A = A_A (q (nu_A S0 + Sn) - p Sdd) and dE/dnu_A = q A_A Sd (over
//     all ordered far pairs (A, .); the summand is symmetric in A and B, so each ordered pair
//     carries the full derivative of its own cluster).  Through nu_A = N_A / |N_A|,
//     dE/dN_A = (I - nu_A nu_A^T) dE/dnu_A / |N_A|.  Down the tree, a face S of A receives
//       dE/da_S += dE/dA_A + (dE/dC_A / A_A) . (c_S - C_A) + dE/dN_A . n_S,
//       dE/dc_S += a_S dE/dC_A / A_A,          dE/dn_S += a_S dE/dN_A,
//     written as the equivalent row sums K += dE/da_S, Sd += dE/dN_A / q, Sn += dE/dC_A / (q A_A)
//     (with S0 and Sdd untouched) so that the exact path's FP64 finalize turns them into corner
//     gradients; the energy E = (1/2) sum_S a_S K_S comes out as (1/2) sum of the far pairs'
//     A_A K_A plus the near field, because the extra terms sum to zero over a cluster's faces.
#include "farfield_common.hpp"

namespace tpe {

// faces of a dual leaf (a row wave); the dual leaves are the nodes of level dual_level(H, leaf)
constexpr int DUAL_SPAN = 64;

__device__ __forceinline__ bool dual_far(const NodeRec& a, const NodeRec& b, float theta) {
    const float dx = a.cx - b.cx, dy = a.cy - b.cy, dz = a.cz - b.cz;
    const float d = sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));  // fixed order: an exact FP32 decision
    // FP32 slack on the distance; theta <= 1 makes the vertex balls disjoint
    return 2.f * fmaxf(a.r, b.r) < theta * d * (1.f - 1e-5f);
}

// The root is its own only near pair.  Entries of node A: ent[off[A] .. off[A] + nnear[A]) near,
// then nfar[A] far, so one scan per level places both.
__global__ void dual_init(uint32_t* __restrict__ off, uint32_t* __restrict__ nnear, uint32_t* __restrict__ nfar,
                          uint32_t* __restrict__ ent) {
    off[1] = 0;
    nnear[1] = 1;
    nfar[1] = 0;
    ent[0] = 1;
}

// Level l >= 1, one wave per node A in [2^l, 2^(l+1)): the candidates (children of the parent's
// near list, in list order) are classified 64 at a time, one per lane, and compacted by ballot, so
// the near and far entries keep the candidates' order.  FILL = false: count them into cnt[A -
// 2^l] (their sum, for the scan) and nnear / nfar.  FILL = true: write them at base + rel[A - 2^l],
// base = end of the previous level's entries.
template <bool FILL>
__global__ __launch_bounds__(256) void dual_level(int level, const NodeRec* __restrict__ recs, float theta,
                                                  uint32_t* __restrict__ off, uint32_t* __restrict__ nnear,
                                                  uint32_t* __restrict__ nfar, uint32_t* __restrict__ cnt,
                                                  const uint32_t* __restrict__ rel, uint32_t* __restrict__ ent,
                                                  uint32_t cap, uint32_t* __restrict__ flags) {
    const int lane = threadIdx.x & 63;
    const int64_t t = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
    const int64_t first = (int64_t)1 << level;
    if (t >= first) return;  // uniform over the wave
    const int64_t A = first + t;
    const NodeRec a = recs[A];
    uint32_t pos = 0, fpos = 0;
    if (FILL) {
        const int64_t last = first - 1;  // last node of the previous level
        const uint32_t base = off[last] + nnear[last] + nfar[last];
        pos = base + rel[t];
        fpos = pos + nnear[A];
        if (lane == 0) off[A] = pos;
    }
    uint32_t nn = 0, nf = 0;
    if (a.a > 0.f) {
        const int64_t P = A >> 1;
        const uint32_t o = off[P];
        uint32_t c = nnear[P];
        if ((uint64_t)o + c > cap) {  // the parent's list overflowed: nothing valid to read
            c = 0;
            if (FILL && lane == 0) atomicOr(flags, (uint32_t)FLAG_LISTS);
        }
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        for (uint32_t e0 = 0; e0 < 2 * c; e0 += 64) {
            const uint32_t e = e0 + lane;
            bool valid = false, far = false;
            uint32_t B = 0;
            if (e < 2 * c) {
                B = 2 * ent[o + e / 2] + (e & 1);
                const NodeRec b = recs[B];
                valid = b.a > 0.f;
                far = valid && dual_far(a, b, theta);
            }
            const uint64_t fm = __ballot(far), nm = __ballot(valid && !far);
            if (FILL) {
                if (far) {
                    const uint64_t at = (uint64_t)fpos + nf + __popcll(fm & lt);
                    if (at < cap) ent[at] = B;
                    else atomicOr(flags, (uint32_t)FLAG_LISTS);
                } else if (valid) {
                    const uint64_t at = (uint64_t)pos + nn + __popcll(nm & lt);
                    if (at < cap) ent[at] = B;
                    else atomicOr(flags, (uint32_t)FLAG_LISTS);
                }
            }
            nf += (uint32_t)__popcll(fm);
            nn += (uint32_t)__popcll(nm);
        }
    }
    if (!FILL && lane == 0) {
        nnear[A] = nn;
        nfar[A] = nf;
        cnt[t] = nn + nf;
    }
}

__device__ __forceinline__ double wave_sum_f64(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// One wave per node A (levels 1 .. Hd): the 11 row sums of the pseudo-face A against its far
// clusters (lanes over the list, FP64 sums of the FP32 pair terms, then a fixed-order butterfly),
// turned into the cluster's adjoint adj[A] = {dE/dA_A, dE/dC_A / A_A (3), dE/dN_A (3), 0}.
__global__ __launch_bounds__(256) void dual_far_eval(int Hd, const NodeRec* __restrict__ recs,
                                                     const NodeF64* __restrict__ nodes,
                                                     const uint32_t* __restrict__ off,
                                                     const uint32_t* __restrict__ nnear,
                                                     const uint32_t* __restrict__ nfar,
                                                     const uint32_t* __restrict__ ent, uint32_t cap, double q,
                                                     double p, double* __restrict__ adj,
                                                     unsigned long long* __restrict__ stats) {
    const int lane = threadIdx.x & 63;
    const int64_t A = 2 + blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
    if (A >= ((int64_t)2 << Hd)) return;  // uniform over the wave
    double* o = adj + 8 * A;
    const uint32_t nf = nfar[A];
    const NodeRec a = recs[A];
    const uint32_t f0 = off[A] + nnear[A];
    if (nf == 0 || !(a.a > 0.f) || (uint64_t)f0 + nf > cap) {
        if (lane < 8) o[lane] = 0.0;
        return;
    }
    double R[NACC];
    for (int k = 0; k < NACC; ++k) R[k] = 0.0;
    const int4 nov = make_int4(0, 0, 0, 0);
    for (uint32_t e = lane; e < nf; e += 64) {
        const NodeRec b = recs[ent[f0 + e]];
        const ColRec cr = {b.cx, b.cy, b.cz, b.a, b.nx, b.ny, b.nz, 0.f};
        float acc[NACC];
        for (int k = 0; k < NACC; ++k) acc[k] = 0.f;
        ff_pair<6, true, false>(cr, nov, a.cx, a.cy, a.cz, a.nx, a.ny, a.nz, 0, 0, 0, acc);
        for (int k = 0; k < NACC; ++k) R[k] += (double)acc[k];
    }
    for (int k = 0; k < NACC; ++k) R[k] = wave_sum_f64(R[k]);
    if (lane == 0) {
        const NodeF64 n = nodes[A];
        const double Nn = sqrt(n.nx * n.nx + n.ny * n.ny + n.nz * n.nz);
        const double nu[3] = {Nn > 0.0 ? n.nx / Nn : 0.0, Nn > 0.0 ? n.ny / Nn : 0.0, Nn > 0.0 ? n.nz / Nn : 0.0};
        o[0] = R[0];
        double gnu[3];
        for (int d = 0; d < 3; ++d) {
            o[1 + d] = q * (nu[d] * R[1] + R[8 + d]) - p * R[5 + d];
            gnu[d] = q * n.A * R[2 + d];
        }
        const double ng = nu[0] * gnu[0] + nu[1] * gnu[1] + nu[2] * gnu[2];
        for (int d = 0; d < 3; ++d) o[4 + d] = Nn > 0.0 ? (gnu[d] - ng * nu[d]) / Nn : 0.0;
        o[7] = 0.0;
        if (stats && nf) atomicAdd(&stats[0], (unsigned long long)nf);  // same word for every node
    }
}

// DUAL_SPLIT work-groups of DUAL_NW waves per dual leaf (its faces one per lane): the exact pairs
// with the faces of the leaf's near list.  Near lists are heavy-tailed (a few leaves have tens of
// times the mean), so each leaf's entries are dealt round-robin over the DUAL_SPLIT x DUAL_NW waves
// of its work-groups; a work-group folds its waves through LDS in wave order and writes one FP32
// partial per (row, sum), and dual_near_merge adds a leaf's partials in work-group order.
constexpr int DUAL_NW = 4;
constexpr int DUAL_SPLIT = 8;

__global__ __launch_bounds__(64 * DUAL_NW) void dual_near_eval(
    int Hd, int64_t span, const ColRec* __restrict__ cols, const int4* __restrict__ colv,
    const double* __restrict__ c64, const double* __restrict__ org, const NodeRec* __restrict__ recs,
    const uint32_t* __restrict__ off, const uint32_t* __restrict__ nnear, const uint32_t* __restrict__ ent,
    uint32_t cap, int64_t nF, int64_t Fp, float* __restrict__ part, unsigned long long* __restrict__ stats,
    const uint32_t* __restrict__ order) {
    __shared__ float red[DUAL_NW - 1][2 * NACC][64];
    __shared__ unsigned long long wpairs[DUAL_NW];
    __shared__ ColRec nst[DUAL_NW][64];
    __shared__ int4 nsv[DUAL_NW][64];
    const int split = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int64_t x = order ? (int64_t)order[blockIdx.x] : (int64_t)blockIdx.x;  // the leaf
    const int64_t A = ((int64_t)1 << Hd) + x;
    const int64_t i0 = x * span;
    const bool row = lane < span && i0 + lane < Fp;
    const int64_t i = row ? i0 + lane : 0;  // lanes without a row read row 0 and write nothing
    const double cxd = c64[3 * i], cyd = c64[3 * i + 1], czd = c64[3 * i + 2];
    const ColRec me = cols[i];
    const int4 mv = colv[i];
    const NodeRec a = recs[A];
    float hi[NACC], lo[NACC], acc[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) { hi[k] = 0.f; lo[k] = 0.f; acc[k] = 0.f; }
    int cnt = 0;
    const uint32_t o = off[A];
    const uint32_t nn = a.a > 0.f && (uint64_t)o + nnear[A] <= cap ? nnear[A] : 0u;
    uint64_t pairs = 0;
    for (uint32_t e = (uint32_t)(split * DUAL_NW + wave); e < nn; e += DUAL_SPLIT * DUAL_NW) {
        const int64_t B = ent[o + e];
        const int64_t f0 = (B - ((int64_t)1 << Hd)) * span, f1 = std::min<int64_t>(nF, f0 + span);
        if (f0 >= f1) continue;
        pairs += (uint64_t)(f1 - f0);
        const NodeRec b = recs[B];
        const float dx = a.cx - b.cx, dy = a.cy - b.cy, dz = a.cz - b.cz;
        // vertex balls apart (with FP32 slack): no face of B shares a vertex with a face of A
        const bool disjoint = sqrtf(dx * dx + dy * dy + dz * dz) * (1.f - 1e-5f) > a.r + b.r;
        if (disjoint)
            ff_near_staged<false, 2>(cols, colv, org, f0, f1, cxd, cyd, czd, me, mv, nst[wave], nsv[wave], lane, acc,
                                     hi, lo, cnt);
        else
            ff_near_staged<true, 2>(cols, colv, org, f0, f1, cxd, cyd, czd, me, mv, nst[wave], nsv[wave], lane, acc,
                                    hi, lo, cnt);
    }
    ff_fold(acc, hi, lo);
    if (wave > 0) {
#pragma unroll
        for (int k = 0; k < NACC; ++k) {
            red[wave - 1][k][lane] = hi[k];
            red[wave - 1][NACC + k][lane] = lo[k];
        }
    }
    if (lane == 0) wpairs[wave] = pairs;
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int j = 0; j < DUAL_NW - 1; ++j)
#pragma unroll
            for (int k = 0; k < NACC; ++k) {
                float y = red[j][k][lane] - lo[k];
                float t = hi[k] + y;
                lo[k] = (t - hi[k]) - y;
                hi[k] = t;
                y = -red[j][NACC + k][lane] - lo[k];
                t = hi[k] + y;
                lo[k] = (t - hi[k]) - y;
                hi[k] = t;
            }
        float* o = part + ((size_t)x * DUAL_SPLIT + split) * NACC * 64 + lane;
#pragma unroll
        for (int k = 0; k < NACC; ++k) o[(size_t)k * 64] = hi[k] - lo[k];
    }
    // one counter update per work-group (the same word for all of them)
    if (stats && threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < DUAL_NW; ++w) t += wpairs[w];
        if (t) atomicAdd(&stats[1], t * (unsigned long long)std::min<int64_t>(span, nF - i0));
    }
}

// acc64[k][i] <- the partials of face i's leaf, added in FP64 in work-group order (one thread per
// (face, sum)).
__global__ void dual_near_merge(int64_t span, const float* __restrict__ part, int64_t nF, int64_t Fp,
                                double* __restrict__ acc64) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= nF) return;
    const int64_t leaf = i / span;
    const float* pp = part + ((size_t)leaf * DUAL_SPLIT * NACC + k) * 64 + (i - leaf * span);
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < DUAL_SPLIT; ++w) s += (double)pp[(size_t)w * NACC * 64];
    acc64[(size_t)k * Fp + i] = s;
}

// One thread per face i: the far-field adjoints of the clusters that contain it (levels 1 .. Hd),
// added to its row sums as equivalent K, Sd and Sn (see the top of the file).
__global__ void dual_down(int Hd, int64_t span, const NodeF64* __restrict__ nodes, const double* __restrict__ adj,
                          const double* __restrict__ c64, const double* __restrict__ geo, int64_t nF, int64_t Fp,
                          double q, double* __restrict__ acc64) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nF) return;
    const int64_t leafnode = ((int64_t)1 << Hd) + i / span;
    const double cs[3] = {c64[3 * i], c64[3 * i + 1], c64[3 * i + 2]};
    const double ns[3] = {geo[5 * i + 2], geo[5 * i + 3], geo[5 * i + 4]};
    double K = 0.0, Sd[3] = {0.0, 0.0, 0.0}, Sn[3] = {0.0, 0.0, 0.0};
    for (int l = Hd; l >= 1; --l) {
        const int64_t A = leafnode >> (Hd - l);
        const double* o = adj + 8 * A;
        if (o[0] == 0.0 && o[1] == 0.0 && o[2] == 0.0 && o[3] == 0.0 && o[4] == 0.0 && o[5] == 0.0 && o[6] == 0.0)
            continue;
        const NodeF64 n = nodes[A];
        const double C[3] = {n.cx, n.cy, n.cz};
        K += o[0];
        for (int d = 0; d < 3; ++d) {
            K += o[1 + d] * (cs[d] - C[d]) + o[4 + d] * ns[d];
            Sd[d] += o[4 + d] / q;
            Sn[d] += o[1 + d] / q;
        }
    }
    acc64[i] += K;
    for (int d = 0; d < 3; ++d) {
        acc64[(size_t)(2 + d) * Fp + i] += Sd[d];
        acc64[(size_t)(8 + d) * Fp + i] += Sn[d];
    }
}

// dual leaves: the level whose nodes hold DUAL_SPAN faces (or the root, for smaller meshes)
int dual_level(int H, int leaf) {
    int l = H;
    int64_t span = leaf;
    while (l > 0 && span < DUAL_SPAN) {
        --l;
        span *= 2;
    }
    return l;
}
int64_t dual_span(int H, int leaf) { return (int64_t)leaf << (H - dual_level(H, leaf)); }
// FP32 floats of the near partials: DUAL_SPLIT x NACC x 64 per dual leaf
int64_t dual_part_floats(int H, int leaf) { return ((int64_t)1 << dual_level(H, leaf)) * DUAL_SPLIT * NACC * 64; }
// entry capacity of the lists (near + far over all levels); an overflow sets FLAG_LISTS, which the
// caller reports as an error (no list entry beyond the capacity is ever read)
int64_t dual_entry_cap(int H, int leaf) {
    const int Hd = dual_level(H, leaf);
    return std::max<int64_t>((int64_t)1 << 16, ((int64_t)2 << Hd) * 384);
}

int64_t scan_ws_words(int64_t n);
hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* ws, hipStream_t st);
hipError_t launch_ff_order(const uint32_t* work, int64_t nb, uint32_t* order, const uint4* lst,
                           unsigned long long* stats, hipStream_t st);

// The whole dual-tree evaluation after the records and tree moments: lists, far clusters, near
// leaves, downward pass; leaves FP64 row sums in acc64 for the finalize.
hipError_t launch_dual(int H, int leaf, float theta, const ColRec* cols, const int4* colv, const double* c64,
                       const double* geo, const double* org, const void* nodes64, const void* recs_, int64_t nF,
                       int64_t Fp, double q, double p, uint32_t* off, uint32_t* nnear, uint32_t* nfar, uint32_t* cnt,
                       uint32_t* rel, uint32_t* ent, uint32_t* scanws, double* adj, float* part, double* acc64,
                       uint32_t* flags, unsigned long long* stats, uint32_t* const sort[6], hipStream_t st) {
    const NodeF64* nodes = (const NodeF64*)nodes64;
    const NodeRec* recs = (const NodeRec*)recs_;
    const int Hd = dual_level(H, leaf);
    const int64_t span = dual_span(H, leaf);
    const uint32_t cap = (uint32_t)dual_entry_cap(H, leaf);
    hipLaunchKernelGGL(dual_init, dim3(1), dim3(1), 0, st, off, nnear, nfar, ent);
    for (int l = 1; l <= Hd; ++l) {
        const int64_t n = (int64_t)1 << l;
        const dim3 g((unsigned)((n + 3) / 4));  // 4 nodes (waves) per work-group
        hipLaunchKernelGGL((dual_level<false>), g, dim3(256), 0, st, l, recs, theta, off, nnear, nfar, cnt, rel, ent,
                           cap, flags);
        hipError_t e = launch_exclusive_scan(cnt, n, rel, scanws, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((dual_level<true>), g, dim3(256), 0, st, l, recs, theta, off, nnear, nfar, cnt, rel, ent,
                           cap, flags);
    }
    const int64_t nn = ((int64_t)2 << Hd) - 2;
    if (nn > 0)
        hipLaunchKernelGGL(dual_far_eval, dim3((unsigned)((nn + 3) / 4)), dim3(256), 0, st, Hd, recs, nodes, off,
                           nnear, nfar, ent, cap, q, p, adj, stats);
    // leaves with the longest near lists first (work-groups start in launch order), into sort[1]
    const int64_t nleaf = (int64_t)1 << Hd;
    hipError_t e = launch_ff_order(nnear + nleaf, nleaf, sort[1], nullptr, nullptr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dual_near_eval, dim3((unsigned)nleaf, DUAL_SPLIT), dim3(64 * DUAL_NW), 0, st, Hd, span, cols,
                       colv, c64, org, recs, off, nnear, ent, cap, nF, Fp, part, stats, (const uint32_t*)sort[1]);
    hipLaunchKernelGGL(dual_near_merge, dim3((unsigned)((nF + 255) / 256), NACC), dim3(256), 0, st, span, part, nF, Fp,
                       acc64);
    hipLaunchKernelGGL(dual_down, dim3((unsigned)((nF + 255) / 256)), dim3(256), 0, st, Hd, span, nodes, adj, c64, geo,
                       nF, Fp, q, acc64);
    return hipGetLastError();
}

}  // namespace tpe
