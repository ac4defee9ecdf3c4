// Internal helpers shared by the HIP sources of libtpe (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpe {

// Device-side error flags, OR-ed into one word by the kernels and read back by the host.
enum : uint32_t {
    FLAG_BAD_INDEX = 1u,   // a face refers to a vertex outside [0, V)
    FLAG_DEGENERATE = 2u,  // a face with area <= 1e-300
    FLAG_NONFINITE = 4u,   // non-finite coordinate, or a non-finite accumulated result
    FLAG_LISTS = 8u,       // the dual-tree interaction lists outgrew their scratch
    FLAG_TREE_FACES = 16u, // the face list differs from the one the tree was built with
    FLAG_SYNC = 32u,       // a wave of the symmetric kernel gave up waiting for its work-group
};

// Geometry of the exact all-pairs kernel.
constexpr int WAVE = 64;
constexpr int RPL = 2;                  // rows (target faces) per lane
constexpr int ROWB = WAVE * RPL;        // rows of a row block (held by each wave of a work-group)
constexpr int PAIR_NW = 4;              // waves per pair-kernel work-group (split a row block's columns)
constexpr int CTILE = 64;               // columns per tile (one FP64 origin per tile = per chunk)
constexpr int CHUNK = 64;               // columns summed in plain FP32 before a compensated fold
constexpr int NACC = 11;                // accumulators per row face (see pair.hip)

// Triangle quadrature rules: point p of the Q-point rule as barycentric weights b on the face's
// vertices (in the order of F) and its weight w (the weights sum to 1).
//   Q = 1: the centroid.
//   Q = 3: (2/3, 1/6, 1/6) and its permutations, weights 1/3 (exact for degree 2; Strang and Fix).
//   Q = 6: (1 - 2a, a, a) and its permutations for a = 0.445948490915965, weight 0.223381589678011,
//          and for a = 0.091576213509771, weight 0.109951743655322 (exact for degree 4; Dunavant).
__host__ __device__ inline bool quad_rule_ok(int Q) { return Q == 1 || Q == 3 || Q == 6; }
__host__ __device__ inline void quad_point(int Q, int p, double* b, double& w) {
    if (Q == 3) {
        for (int i = 0; i < 3; ++i) b[i] = i == p ? 2.0 / 3.0 : 1.0 / 6.0;
        w = 1.0 / 3.0;
    } else if (Q == 6) {
        const int g = p / 3, k = p % 3;
        const double a = g == 0 ? 0.445948490915965 : 0.091576213509771;
        for (int i = 0; i < 3; ++i) b[i] = i == k ? 1.0 - 2.0 * a : a;
        w = g == 0 ? 0.223381589678011 : 0.109951743655322;
    } else {
        b[0] = b[1] = b[2] = 1.0 / 3.0;
        w = 1.0;
    }
}

// Curved cubic element (the paper's S_h^3): 10 nodes at the barycentric lattice points
// m / 3, m = (m0, m1, m2) with m0 + m1 + m2 = 3, in the order of P3_M below (corners, the two
// nodes of edges 0-1, 1-2, 2-0 starting at the edge's first corner, centre).  The Lagrange basis
// function of node m is the product over the three barycentric coordinates of
//     L_k(x) = prod_{j<k} (3x - j) / (j + 1)      (k = m_c, x = l_c),
// which is 1 at its own node and 0 at the other nine.  With reference coordinates (s, t) =
// (l1, l2), d/ds = d/dl1 - d/dl0 and d/dt = d/dl2 - d/dl0.
constexpr int P3_NODES = 10;
__host__ __device__ constexpr int p3_m(int node, int c) {
    // m_c of each node, three base-4 digits per node: corners, edges 0-1, 1-2, 2-0, centre
    constexpr int M[P3_NODES] = {0x300, 0x030, 0x003, 0x210, 0x120, 0x021, 0x012, 0x102, 0x201, 0x111};
    return (M[node] >> (4 * (2 - c))) & 0xf;
}

__device__ __forceinline__ void p3_lk(int k, double x, double& v, double& dv) {
    // L_k and its derivative for k = 0..3
    const double y = 3.0 * x;
    if (k == 0) { v = 1.0; dv = 0.0; }
    else if (k == 1) { v = y; dv = 3.0; }
    else if (k == 2) { v = 0.5 * y * (y - 1.0); dv = 1.5 * (2.0 * y - 1.0); }
    else { v = y * (y - 1.0) * (y - 2.0) / 6.0; dv = 0.5 * (3.0 * y * y - 6.0 * y + 2.0); }
}

// basis values and (s, t) derivatives at barycentric l
__device__ __forceinline__ void p3_shape(const double* l, double* phi, double* ds, double* dt) {
#pragma unroll
    for (int k = 0; k < P3_NODES; ++k) {
        double v[3], dv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) p3_lk(p3_m(k, c), l[c], v[c], dv[c]);
        phi[k] = v[0] * v[1] * v[2];
        const double d0 = dv[0] * v[1] * v[2], d1 = v[0] * dv[1] * v[2], d2 = v[0] * v[1] * dv[2];
        ds[k] = d1 - d0;
        dt[k] = d2 - d0;
    }
}

// Column record of the pair kernels and the far field: centroid relative to its tile origin,
// area, normal, and wv = -2 a, the weight of a column's Sdd term in the symmetric kernel's
// combined sum V = Sn - (p/q) Sdd for (q, p) = (6, 12).
struct __align__(32) ColRec {
    float cx, cy, cz, a;
    float nx, ny, nz, wv;
};

// Balanced persistent schedule.  The work is U = nrb * upr units, a unit being one chunk of CHUNK
// columns for one row block of ROWB rows (upr = Fp / CHUNK units per row block, in column order).
// Work-group w of W takes the contiguous units [floor(w U / W), floor((w+1) U / W)), so every
// work-group does the same work to within one unit and, with W equal to the number of resident
// work-groups, the launch has no tail.  A range may cover the end of one row block and the start
// of the next: the work-group writes one partial-sum segment per row block it touches (at most
// maxseg), and the finalize pass adds, for each row block, the segments of the work-groups that
// cover it, in work-group order.
struct Sched {
    int64_t U;
    int W, upr, maxseg;
    __host__ __device__ int64_t begin(int w) const { return (int64_t)w * U / W; }
    // the work-group whose range contains unit x
    __host__ __device__ int wave_of(int64_t x) const { return (int)(((x + 1) * (int64_t)W - 1) / U); }
};

// Symmetric schedule of the self energy's pair kernel.  A work-group of nw waves (1, 2 or 4) holds
// a super block of nw * ROWB rows (one row block per wave).  Super block I owns first its sbc =
// nw * ROWB / CHUNK diagonal units, the CHUNK-column chunks J = sbc I, ..., sbc I + sbc - 1 of its
// own faces (pairs inside the super block, evaluated from both sides as ordered pairs), then its
// symmetric units, the SYM_COLS-column slices of all later chunks (every unordered pair once,
// credited to both faces; the columns' share goes to one column partial per symmetric unit).
// Units are numbered super block by super block; work-group w takes the contiguous range
// [begin(w), begin(w+1)), a diagonal unit costing DIAG_COST and a symmetric one SYM_COST.  The
// first W1 work-groups share the cost C1 in equal parts; the other W - W1 share the rest, about
// one unit each, so that the end of the launch is made of short ranges the hardware hands to
// whichever slots free up first (W1 = W: equal parts for all).  Fewer waves per work-group wait
// less at the work-group's barriers but write more column partials (one per unit: the partial
// volume is inversely proportional to nw).
// sums per face in the symmetric kernel: K, S0, Sd (3), V = Sn - 2 Sdd (3)
constexpr int NSYM = 8;
constexpr int SYM_COLS = 64;              // columns of a symmetric unit (64: the wave; 16: a row of lanes)
constexpr int SUB = CHUNK / SYM_COLS;     // symmetric units per chunk
// relative costs, measured: a diagonal unit (the row-only pass over CHUNK columns, nearly always
// with vertex comparisons, and the first unit of a super block with its row loads) takes about
// 1.7 times a symmetric unit of 64 columns, which itself takes about 122 VALU instructions per
// column and lane
constexpr int SYM_COST = 12 * SYM_COLS / 64, DIAG_COST = 20;

struct SymSched {
    int64_t U, C;  // units, total cost
    int W, nsb, nch;
    int W1;        // work-groups sharing the cost C1 (the rest share C - C1)
    int64_t C1;
    int nw;        // waves (row blocks) per work-group: 1, 2 or 4
    int sbc;       // chunks per super block, nw * ROWB / CHUNK
    // units of super block I: sbc + SUB (nch - sbc (I + 1)) = A - D I
    __host__ __device__ int64_t ua() const { return sbc + (int64_t)SUB * (nch - sbc); }
    __host__ __device__ int64_t ud() const { return (int64_t)SUB * sbc; }
    // first unit of super block I
    __host__ __device__ int64_t base(int64_t I) const { return I * ua() - ud() * I * (I - 1) / 2; }
    // symmetric units of the super blocks before I
    __host__ __device__ int64_t base_sym(int64_t I) const {
        return (int64_t)SUB * (I * (nch - sbc) - (int64_t)sbc * I * (I - 1) / 2);
    }
    // super block of unit u (0 <= u < U): the root of base(I) = u, then corrected to be exact
    __host__ __device__ int block_of(int64_t u) const {
        const double h = 0.5 * (double)ud(), b = (double)ua() + h;
        const double disc = b * b - 4.0 * h * (double)u;
        int I = (int)((b - sqrt(disc > 0.0 ? disc : 0.0)) / (2.0 * h));
        I = I < 0 ? 0 : (I > nsb - 1 ? nsb - 1 : I);
        while (I > 0 && base(I) > u) --I;
        while (I < nsb - 1 && base(I + 1) <= u) ++I;
        return I;
    }
    // cost of the units [0, u)
    __host__ __device__ int64_t cost(int64_t u) const {
        if (u >= U) return C;
        const int I = block_of(u);
        const int64_t k = u - base(I);
        const int64_t ndiag = (int64_t)sbc * I + (k < sbc ? k : sbc);
        return SYM_COST * u + (int64_t)(DIAG_COST - SYM_COST) * ndiag;
    }
    // does the range of work-group w start at or before a unit whose preceding cost is c?
    __host__ __device__ bool reached(int64_t c, int w) const {
        if (w <= W1) return c * W1 >= (int64_t)w * C1;
        return c >= C1 && (c - C1) * (W - W1) >= (int64_t)(w - W1) * (C - C1);
    }
    // first unit of work-group w: the smallest u with reached(cost(u), w)
    __host__ __device__ int64_t begin(int w) const {
        if (w <= 0) return 0;
        if (w >= W) return U;
        int64_t lo = 0, hi = U;
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (reached(cost(mid), w)) hi = mid;
            else lo = mid + 1;
        }
        return lo;
    }
    // the work-group whose range contains unit x (the largest w with reached(cost(x), w))
    __host__ __device__ int wave_of(int64_t x) const {
        const int64_t c = cost(x);
        int w;
        if (c < C1) w = (int)(c * W1 / C1);
        else if (W == W1) w = W - 1;
        else w = W1 + (int)((c - C1) * (W - W1) / (C - C1));
        return w < W - 1 ? w : W - 1;
    }
};

// The energy of a finalize: E[0] = scale 2^(kexp (p - q - 4)) (sum of the nb FP64 work-group
// partials epart), kexp from the bounding box; E null: no energy.
struct EnergyOut {
    const double* epart;
    int nb;
    const uint32_t* bbox;
    double q, p, scale;
    double* E;
};

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
inline int64_t ceil_div(int64_t x, int64_t m) { return (x + m - 1) / m; }

// The centroid bounding box's words: bbox[0..5] the box, bbox[BBOX_TICKET] the reduction's ticket,
// bbox[BBOX_FSUM] the checksum of the face list, bbox[BBOX_PART + 8 g ...] the slot of work-group g
// (BBOX_SLOTS of them)
constexpr int BBOX_SLOTS = 256;
constexpr int BBOX_TICKET = 6;
constexpr int BBOX_FSUM = 7;
constexpr int BBOX_PART = 8;
constexpr int BBOX_WORDS = BBOX_PART + 8 * BBOX_SLOTS;

__device__ __forceinline__ float ordered_to_float(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// Exponent k of the power of two s = 2^k with (largest centroid-bounding-box extent) * s in
// [0.5, 1); 0 if the box is empty or degenerate.  bbox holds order-preserving encodings of
// (min xyz, max xyz).
__device__ __forceinline__ int norm_exp(const uint32_t* bbox) {
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double e = (double)ordered_to_float(bbox[3 + d]) - (double)ordered_to_float(bbox[d]);
        if (e > ext && isfinite(e)) ext = e;
    }
    if (!(ext > 0.0) || !isfinite(ext)) return 0;
    int ex;
    (void)frexp(ext, &ex);
    return -ex;
}
__device__ __forceinline__ double norm_scale(const uint32_t* bbox) { return ldexp(1.0, norm_exp(bbox)); }

// Centre of the centroid bounding box in the normalised frame (0 for an empty box): the origin of
// the far field's FP32 cluster records and rows, so that their coordinates stay small wherever the
// mesh sits (FP32 positions of a mesh translated by 1e4 would carry errors of 1e-3).
__device__ __forceinline__ void norm_origin(const uint32_t* bbox, double* o) {
    const double s = norm_scale(bbox);
    for (int d = 0; d < 3; ++d) {
        const double lo = (double)ordered_to_float(bbox[d]), hi = (double)ordered_to_float(bbox[3 + d]);
        o[d] = lo <= hi && isfinite(lo) && isfinite(hi) ? s * (0.5 * (lo + hi)) : 0.0;
    }
}

// s^m for s = 2^k and an integer-valued m, exactly.
__device__ __forceinline__ double pow2i(int k, double m) { return ldexp(1.0, (int)llrint(k * m)); }

// Far-away padding for rows/columns past the last face (area 0, so they contribute exactly 0).
constexpr float PAD_COORD = 1.0e4f;

}  // namespace tpe
