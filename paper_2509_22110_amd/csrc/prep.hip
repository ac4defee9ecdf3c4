// Geometry preparation, spatial (Morton) ordering, vertex->corner adjacency and the tile-pair
// exclusion map.
//
// Per face T = (i, j, k) (paper Sec. 3.2: positions, area elements and normals are cached per
// quadrature point, contiguously, and iterated in memory order):
//     w = (x_j - x_i) x (x_k - x_i),  a = |w|/2,  n = w/|w|,  c = (x_i + x_j + x_k)/3   (FP64)
// Faces are reordered along a 30-bit Morton curve of their centroids so that a tile of 256
// consecutive faces is spatially compact: that keeps tile-relative FP32 coordinates small and
// confines faces sharing a vertex (the excluded pairs) to few tile pairs.
#include "common.hpp"

namespace tpe {

__device__ __forceinline__ uint32_t float_to_ordered(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ void fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// One launch that prepares the scratch state of a call: zero [zero, zero+nzero), bbox to
// (+max x3, 0 x3) in the order-preserving encoding with its ticket word at 0, and optionally the
// error word.
__global__ void init_scratch(uint32_t* __restrict__ zero, int64_t nzero, uint32_t* __restrict__ bbox,
                             uint32_t* __restrict__ flags) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < 6) bbox[i] = i < 3 ? 0xffffffffu : 0u;
    if (i == 6) bbox[BBOX_TICKET] = 0u;
    if (i == 7 && flags) flags[0] = 0u;
    for (; i < nzero; i += (int64_t)gridDim.x * blockDim.x) zero[i] = 0u;
}

// Checksum term of face-list entry j (value v): a bijective 32-bit mix (MurmurHash3's finaliser)
// of v and its position; the checksum is the sum of the terms modulo 2^32, whatever the order.
__device__ __forceinline__ uint32_t face_entry_hash(uint32_t v, uint32_t j) {
    uint32_t h = v ^ (j * 0x9e3779b9u);
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// bbox[0..2] = ordered(min), bbox[3..5] = ordered(max) of face centroids (FP32), merged into what
// bbox holds (it starts at (0xffffffff x3, 0 x3); a second launch adds a second surface), and
// bbox[BBOX_FSUM] = the checksum of the face list (its three corners per face); with `expect`, a
// checksum that differs from *expect sets FLAG_TREE_FACES.  Also validates indices / coordinates
// and flags errors.  Grid-stride loop and a reduction over the
// work-group, whose result goes to its slot of bbox[BBOX_PART...]; the work-group that takes the
// last ticket (bbox[BBOX_TICKET]) reduces the slots in slot order, writes the box and resets the
// ticket.  (Six same-address atomics per work-group cost about 11 ns each: with 1,024 work-groups
// they took 70 us.)  Face f's corners are F[fs f + 0..2] (fs = 3 for triangles, 10 for curved
// cubic elements, whose centroid here is that of their corners).
static_assert(BBOX_SLOTS <= 256, "one slot per thread of the last work-group");
__global__ __launch_bounds__(256) void face_bbox(const double* __restrict__ X, int64_t V,
                                                  const int32_t* __restrict__ F, int fs, int64_t nF,
                                                  uint32_t* __restrict__ bbox, uint32_t* __restrict__ flags,
                                                  const uint32_t* __restrict__ expect) {
    __shared__ float smn[4][3], smx[4][3];
    __shared__ uint32_t sfl[4], ssum[4];
    __shared__ bool last;
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    uint32_t fl = 0, sum = 0;
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < nF; f += (int64_t)gridDim.x * blockDim.x) {
        int32_t v[3] = {F[fs * f], F[fs * f + 1], F[fs * f + 2]};
        for (int k = 0; k < 3; ++k) sum += face_entry_hash((uint32_t)v[k], (uint32_t)(3 * f + k));
        double c[3] = {0, 0, 0};
        bool ok = true;
        for (int k = 0; k < 3; ++k) {
            if (v[k] < 0 || v[k] >= V) { ok = false; fl |= FLAG_BAD_INDEX; }
        }
        if (!ok) continue;
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) {
                double x = X[3 * (int64_t)v[k] + d];
                if (!isfinite(x)) fl |= FLAG_NONFINITE;
                c[d] += x;
            }
        for (int d = 0; d < 3; ++d) {
            float cf = (float)(c[d] / 3.0);
            if (isfinite(cf)) { mn[d] = fminf(mn[d], cf); mx[d] = fmaxf(mx[d], cf); }
        }
    }
    for (int d = 0; d < 3; ++d) {
        float a = mn[d], b = mx[d];
        for (int off = 32; off > 0; off >>= 1) {
            a = fminf(a, __shfl_xor(a, off));
            b = fmaxf(b, __shfl_xor(b, off));
        }
        mn[d] = a; mx[d] = b;
    }
    for (int off = 32; off > 0; off >>= 1) {
        fl |= __shfl_xor(fl, off);
        sum += __shfl_xor(sum, off);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        for (int d = 0; d < 3; ++d) { smn[w][d] = mn[d]; smx[w][d] = mx[d]; }
        sfl[w] = fl;
        ssum[w] = sum;
    }
    __syncthreads();
    uint32_t* part = bbox + BBOX_PART;
    if (threadIdx.x == 0) {
        uint32_t* my = part + 8 * (size_t)blockIdx.x;
        for (int d = 0; d < 3; ++d) {
            const float a = fminf(fminf(smn[0][d], smn[1][d]), fminf(smn[2][d], smn[3][d]));
            const float b = fmaxf(fmaxf(smx[0][d], smx[1][d]), fmaxf(smx[2][d], smx[3][d]));
            my[d] = a <= b ? float_to_ordered(a) : 0xffffffffu;  // empty: the identities of min / max
            my[3 + d] = a <= b ? float_to_ordered(b) : 0u;
        }
        my[6] = sfl[0] | sfl[1] | sfl[2] | sfl[3];
        my[7] = ssum[0] + ssum[1] + ssum[2] + ssum[3];
        __threadfence();  // the slot is visible before the ticket is taken
        last = atomicAdd(&bbox[BBOX_TICKET], 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;  // uniform over the work-group
    __threadfence();
    // the slots, one per thread (gridDim.x <= BBOX_SLOTS <= blockDim.x), reduced over the work-group
    uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u}, f = 0u, cs = 0u;
    if (threadIdx.x < gridDim.x) {
        const uint32_t* q = part + 8 * (size_t)threadIdx.x;
        for (int d = 0; d < 3; ++d) {
            lo[d] = __hip_atomic_load(q + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            hi[d] = __hip_atomic_load(q + 3 + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        f = __hip_atomic_load(q + 6, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        cs = __hip_atomic_load(q + 7, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int off = 32; off > 0; off >>= 1) {
        for (int d = 0; d < 3; ++d) {
            const uint32_t a = __shfl_xor(lo[d], off), b = __shfl_xor(hi[d], off);
            lo[d] = a < lo[d] ? a : lo[d];
            hi[d] = b > hi[d] ? b : hi[d];
        }
        f |= __shfl_xor(f, off);
        cs += __shfl_xor(cs, off);
    }
    __shared__ uint32_t rlo[4][3], rhi[4][3], rfl[4], rcs[4];
    if ((threadIdx.x & 63) == 0) {
        for (int d = 0; d < 3; ++d) { rlo[w][d] = lo[d]; rhi[w][d] = hi[d]; }
        rfl[w] = f;
        rcs[w] = cs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int d = 0; d < 3; ++d) {
            uint32_t a = bbox[d], b = bbox[3 + d];  // what an earlier launch left (or the initial box)
            for (int k = 0; k < 4; ++k) {
                a = rlo[k][d] < a ? rlo[k][d] : a;
                b = rhi[k][d] > b ? rhi[k][d] : b;
            }
            bbox[d] = a;
            bbox[3 + d] = b;
        }
        uint32_t ff = rfl[0] | rfl[1] | rfl[2] | rfl[3];
        const uint32_t total = rcs[0] + rcs[1] + rcs[2] + rcs[3];
        bbox[BBOX_FSUM] = total;
        if (expect && total != *expect) ff |= FLAG_TREE_FACES;
        bbox[BBOX_TICKET] = 0u;  // for a second launch on the same box
        if (ff) atomicOr(flags, ff);
    }
}

__device__ __forceinline__ uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;  // interleave the low 10 bits with two zero bits each
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// 3*bits-bit Morton key (bits <= 10 per axis) of each face centroid inside the centroid bounding
// box; value = face id.
// One key per record r < Q nF (the Q quadrature points of face r / Q share the face centroid's key,
// so a stable sort keeps a face's records together, in point order).
__global__ void morton_keys(const double* __restrict__ X, int64_t V, const int32_t* __restrict__ F, int fs,
                            int64_t nF, int Q, const uint32_t* __restrict__ bbox, int bits,
                            uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= nF * Q) return;
    const int64_t f = r / Q;
    float lo[3], ext[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = ordered_to_float(bbox[d]);
        float hi = ordered_to_float(bbox[3 + d]);
        ext[d] = hi - lo[d];
        if (!(ext[d] > 0.f) || !isfinite(ext[d])) ext[d] = 1.f;
        if (!isfinite(lo[d])) lo[d] = 0.f;
    }
    uint32_t q[3] = {0, 0, 0};
    int32_t v[3] = {F[fs * f], F[fs * f + 1], F[fs * f + 2]};
    bool ok = v[0] >= 0 && v[0] < V && v[1] >= 0 && v[1] < V && v[2] >= 0 && v[2] < V;
    if (ok) {
        for (int d = 0; d < 3; ++d) {
            double c = (X[3 * (int64_t)v[0] + d] + X[3 * (int64_t)v[1] + d] + X[3 * (int64_t)v[2] + d]) / 3.0;
            const float cells = (float)(1u << bits);
            float s = ((float)c - lo[d]) / ext[d];
            s = fminf(fmaxf(s * cells, 0.f), cells - 1.f);
            q[d] = isfinite(s) ? (uint32_t)s : 0u;
        }
    }
    keys[r] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    vals[r] = (uint32_t)r;
}

// Sorted face records.  For sorted position i < nF: face f = perm[i].  Positions in [nF, Fp) are
// padding: far away, zero area, vertex ids -1 (never equal to a real id; padded rows are never
// read back, padded columns contribute exactly zero).  All positions are multiplied by the exact
// power of two s = norm_scale(bbox) that brings the mesh extent into [0.5, 1), so the FP32 pair
// arithmetic stays in range at any physical scale; the finalize pass undoes s exactly.
//   cols[i]  : centroid relative to the FP64 origin of tile i/CTILE, area, unit normal (FP32)
//   colv[i]  : vertex ids (for the exclusion test)
//   c64[i]   : centroid (FP64)
//   org[t]   : FP64 origin of tile t = centroid of its first face
//   geo[i]   : FP64 {a, |w|, n.x, n.y, n.z} for the finalize pass
__device__ __forceinline__ double wave_min(double x) {
    for (int off = 32; off > 0; off >>= 1) x = fmin(x, __shfl_xor(x, off));
    return x;
}
__device__ __forceinline__ double wave_max(double x) {
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
    return x;
}

// One thread per sorted position i < Fp (whole waves: Fp is a multiple of 128).  Record perm[i] = r
// is quadrature point r % Q of face r / Q (Q = 1: the centroid): position sum_k b_k x_(v_k),
// weight w a, the face's normal, vertex ids and the point index (colv.w).  A wave covers one
// chunk of CTILE = 64 positions; the chunk's FP64 origin is the centre of its points' bounding
// box, so the FP32 record coordinates relative to it are at most half the chunk's extent (their
// rounding error sets the accuracy of the closest pairs).
__device__ void store_record(int64_t i, bool real, bool ok, uint32_t fl, const double* c, const double* n,
                             double a, double wn, const int32_t* v, int pt, double* __restrict__ org,
                             ColRec* __restrict__ cols, int4* __restrict__ colv, double* __restrict__ c64,
                             double* __restrict__ geo, uint32_t* __restrict__ cnt, uint32_t* __restrict__ flags);

__global__ void face_records(const double* __restrict__ X, int64_t V, const int32_t* __restrict__ F,
                             int64_t nF, int Q, int64_t Fp, const uint32_t* __restrict__ perm,
                             const uint32_t* __restrict__ bbox, double* __restrict__ org,
                             ColRec* __restrict__ cols, int4* __restrict__ colv, double* __restrict__ c64,
                             double* __restrict__ geo, uint32_t* __restrict__ cnt,
                             uint32_t* __restrict__ flags) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= Fp) return;
    const double s = norm_scale(bbox);
    bool real = i < nF * Q, ok = false;
    int32_t v[3] = {-1, -1, -1};
    int pt = 0;
    double a = 0.0, wn = 1.0, n[3] = {0.0, 0.0, 0.0}, c[3] = {0.0, 0.0, 0.0};
    uint32_t fl = 0;
    if (real) {
        const int64_t rec = perm[i];
        const int64_t f = rec / Q;
        pt = (int)(rec % Q);
        v[0] = F[3 * f]; v[1] = F[3 * f + 1]; v[2] = F[3 * f + 2];
        ok = v[0] >= 0 && v[0] < V && v[1] >= 0 && v[1] < V && v[2] >= 0 && v[2] < V;
        double xi[3] = {0, 0, 0}, xj[3] = {1, 0, 0}, xk[3] = {0, 1, 0};
        if (ok)
            for (int d = 0; d < 3; ++d) {
                xi[d] = s * X[3 * (int64_t)v[0] + d];
                xj[d] = s * X[3 * (int64_t)v[1] + d];
                xk[d] = s * X[3 * (int64_t)v[2] + d];
            }
        bool fin = true;
        for (int d = 0; d < 3; ++d) fin &= isfinite(xi[d]) && isfinite(xj[d]) && isfinite(xk[d]);
        if (!fin) {  // reported as non-finite input, not as a degenerate face
            fl |= FLAG_NONFINITE;
            for (int d = 0; d < 3; ++d) { xi[d] = 0.0; xj[d] = d == 0 ? 1.0 : 0.0; xk[d] = d == 1 ? 1.0 : 0.0; }
        }
        const double e1[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
        const double e2[3] = {xk[0] - xi[0], xk[1] - xi[1], xk[2] - xi[2]};
        const double w[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        a = 0.5 * wn;
        if (!(a > 1e-300 * s * s)) { fl |= FLAG_DEGENERATE; wn = 1.0; a = 0.0; }
        for (int d = 0; d < 3; ++d) n[d] = w[d] / wn;
        if (Q == 1) {
            for (int d = 0; d < 3; ++d) c[d] = (xi[d] + xj[d] + xk[d]) / 3.0;
        } else {
            double b[3], wq;
            quad_point(Q, pt, b, wq);
            for (int d = 0; d < 3; ++d) c[d] = b[0] * xi[d] + b[1] * xj[d] + b[2] * xk[d];
            a *= wq;  // the record's weight in place of the face's area
        }
        if (!isfinite(c[0] + c[1] + c[2] + n[0] + n[1] + n[2])) {
            fl |= FLAG_NONFINITE;
            c[0] = c[1] = c[2] = 0.0; n[0] = n[1] = n[2] = 0.0; a = 0.0;
        }
    }
    store_record(i, real, ok, fl, c, n, a, wn, v, pt, org, cols, colv, c64, geo, cnt, flags);
}

// The common tail of the record kernels (all lanes of the wave take part): the chunk origin, the
// FP32 record, vertex ids and point index, the FP64 position and {a, |w|, n}, the corner counts of
// the vertex CSR, and the error flags.
__device__ void store_record(int64_t i, bool real, bool ok, uint32_t fl, const double* c, const double* n,
                             double a, double wn, const int32_t* v, int pt, double* __restrict__ org,
                             ColRec* __restrict__ cols, int4* __restrict__ colv, double* __restrict__ c64,
                             double* __restrict__ geo, uint32_t* __restrict__ cnt, uint32_t* __restrict__ flags) {
    // chunk origin: centre of the bounding box of the chunk's real centroids (0 if none)
    const bool inbox = real && ok && !(fl & FLAG_NONFINITE);
    double o[3];
    const bool any = __ballot(inbox) != 0ull;
    for (int d = 0; d < 3; ++d) {
        const double lo = wave_min(inbox ? c[d] : INFINITY);
        const double hi = wave_max(inbox ? c[d] : -INFINITY);
        o[d] = any ? 0.5 * (lo + hi) : 0.0;
    }
    if ((i % CTILE) == 0)
        for (int d = 0; d < 3; ++d) org[3 * (i / CTILE) + d] = o[d];
    ColRec r;
    if (real) {
        if (fl) atomicOr(flags, fl);
        r.cx = (float)(c[0] - o[0]);
        r.cy = (float)(c[1] - o[1]);
        r.cz = (float)(c[2] - o[2]);
        if (ok && cnt)
            for (int k = 0; k < 3; ++k) atomicAdd(&cnt[v[k]], 1u);
        r.a = (float)a;
        r.nx = (float)n[0]; r.ny = (float)n[1]; r.nz = (float)n[2];
        r.wv = -2.f * r.a;
        colv[i] = ok ? make_int4(v[0], v[1], v[2], pt) : make_int4(-3, -3, -3, 0);
        c64[3 * i + 0] = c[0]; c64[3 * i + 1] = c[1]; c64[3 * i + 2] = c[2];
        geo[5 * i + 0] = a; geo[5 * i + 1] = wn;
        geo[5 * i + 2] = n[0]; geo[5 * i + 3] = n[1]; geo[5 * i + 4] = n[2];
    } else {
        // padding: far from everything, zero area; row padding ids differ from column ids
        r.cx = PAD_COORD; r.cy = PAD_COORD; r.cz = PAD_COORD; r.a = 0.f;
        r.nx = 0.f; r.ny = 0.f; r.nz = 0.f; r.wv = 0.f;
        colv[i] = make_int4(-1, -1, -1, 0);
        c64[3 * i + 0] = o[0] + PAD_COORD;
        c64[3 * i + 1] = o[1] + PAD_COORD;
        c64[3 * i + 2] = o[2] + PAD_COORD;
        for (int k = 0; k < 5; ++k) geo[5 * i + k] = 0.0;
    }
    cols[i] = r;
}

// Curved cubic elements: one thread per sorted position i < Fp.  Record perm[i] = r is quadrature
// point r % Q of element r / Q, whose nodes are F10[10 (r / Q) + 0..9] (corners first): with the
// element's cubic map x(s, t), the record sits at x(b) for the rule's barycentric point b, with
// normal J / |J| and weight w |J| / 2, J = x_s x x_t (for a straight element: w times the area,
// the flat record).  The vertex ids of the record are the element's corner nodes, so records of
// elements sharing a corner are excluded from each other, as for flat faces.  geo holds
// {weight, |J|, n}.
__global__ void p3_records(const double* __restrict__ X, int64_t V, const int32_t* __restrict__ F10, int64_t nF,
                           int Q, int64_t Fp, const uint32_t* __restrict__ perm, const uint32_t* __restrict__ bbox,
                           double* __restrict__ org, ColRec* __restrict__ cols, int4* __restrict__ colv,
                           double* __restrict__ c64, double* __restrict__ geo, uint32_t* __restrict__ cnt,
                           uint32_t* __restrict__ flags) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= Fp) return;
    const double s = norm_scale(bbox);
    bool real = i < nF * Q, ok = false;
    int32_t v[3] = {-1, -1, -1};
    int pt = 0;
    double a = 0.0, wn = 1.0, n[3] = {0.0, 0.0, 0.0}, c[3] = {0.0, 0.0, 0.0};
    uint32_t fl = 0;
    if (real) {
        const int64_t rec = perm[i];
        const int64_t f = rec / Q;
        pt = (int)(rec % Q);
        int32_t id[P3_NODES];
        ok = true;
        for (int k = 0; k < P3_NODES; ++k) {
            id[k] = F10[P3_NODES * f + k];
            ok &= id[k] >= 0 && id[k] < V;
        }
        if (!ok) fl |= FLAG_BAD_INDEX;
        for (int k = 0; k < 3; ++k) v[k] = id[k];
        double b[3], wq;
        quad_point(Q, pt, b, wq);
        double phi[P3_NODES], ds[P3_NODES], dt[P3_NODES];
        p3_shape(b, phi, ds, dt);
        double xs[3] = {0.0, 0.0, 0.0}, xt[3] = {0.0, 0.0, 0.0};
        bool fin = true;
        if (ok)
            for (int k = 0; k < P3_NODES; ++k)
                for (int d = 0; d < 3; ++d) {
                    const double x = s * X[3 * (int64_t)id[k] + d];
                    fin &= isfinite(x);
                    c[d] += phi[k] * x;
                    xs[d] += ds[k] * x;
                    xt[d] += dt[k] * x;
                }
        if (!fin) fl |= FLAG_NONFINITE;
        const double J[3] = {xs[1] * xt[2] - xs[2] * xt[1], xs[2] * xt[0] - xs[0] * xt[2],
                             xs[0] * xt[1] - xs[1] * xt[0]};
        wn = sqrt(J[0] * J[0] + J[1] * J[1] + J[2] * J[2]);
        a = 0.5 * wq * wn;
        if (ok && fin && !(wn > 1e-300 * s * s)) fl |= FLAG_DEGENERATE;
        if (!(wn > 1e-300 * s * s) || !ok || !fin) { wn = 1.0; a = 0.0; }
        for (int d = 0; d < 3; ++d) n[d] = J[d] / wn;
        if (!isfinite(c[0] + c[1] + c[2] + n[0] + n[1] + n[2])) {
            fl |= FLAG_NONFINITE;
            c[0] = c[1] = c[2] = 0.0; n[0] = n[1] = n[2] = 0.0; a = 0.0;
        }
    }
    store_record(i, real, ok, fl, c, n, a, wn, v, pt, org, cols, colv, c64, geo, cnt, flags);
}

// node -> (item, node slot) adjacency of curved cubic elements, for the vertex gather: item e of
// `step` records (records e step .. e step + step - 1, see p3_finalize_kernel) belongs to element
// perm[e step] / Q; slot 10 e + k is that element's node k.  p3_node_count adds the per-node
// counts (cnt zero on entry); p3_node_fill writes the lists (cursor zero on entry; order within a
// list arbitrary, the gather orders it).
__global__ void p3_node_count(const int32_t* __restrict__ F10, int64_t n, int step, int Q, int64_t V,
                              const uint32_t* __restrict__ perm, uint32_t* __restrict__ cnt) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int64_t f = perm[e * step] / Q;
    for (int k = 0; k < P3_NODES; ++k) {
        const int32_t v = F10[P3_NODES * f + k];
        if (v >= 0 && v < V) atomicAdd(&cnt[v], 1u);
    }
}

__global__ void p3_node_fill(const int32_t* __restrict__ F10, int64_t n, int step, int Q, int64_t V,
                             const uint32_t* __restrict__ perm, const uint32_t* __restrict__ off,
                             uint32_t* __restrict__ cursor, uint32_t* __restrict__ list) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int64_t f = perm[e * step] / Q;
    for (int k = 0; k < P3_NODES; ++k) {
        const int32_t v = F10[P3_NODES * f + k];
        if (v >= 0 && v < V) {
            const uint32_t pos = atomicAdd(&cursor[v], 1u);
            list[off[v] + pos] = (uint32_t)(P3_NODES * e + k);
        }
    }
}

// ---- vertex -> (sorted face, corner) adjacency, CSR, deterministic order ----------------------
// (per-vertex counts are accumulated by face_records)

__global__ void corner_fill(const int4* __restrict__ colv, int64_t nF, int64_t V,
                            const uint32_t* __restrict__ off, uint32_t* __restrict__ cursor,
                            uint32_t* __restrict__ list) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nF) return;
    int4 v = colv[i];
    int vv[3] = {v.x, v.y, v.z};
    for (int k = 0; k < 3; ++k)
        if (vv[k] >= 0 && vv[k] < V) {
            uint32_t pos = atomicAdd(&cursor[vv[k]], 1u);
            list[off[vv[k]] + pos] = (uint32_t)(3 * i + k);
        }
}

// Exclusion map: bit (rb, c) set iff some row of row block rb shares a vertex with some column of
// the c-th chunk of CHUNK columns.  Rows/columns are sorted positions.  One work-group per row block builds its
// row of the map in LDS (dynamic shared memory, touch_words words) and stores it: no global
// atomics and no prior zeroing.
__global__ __launch_bounds__(256) void touch_map(const int4* __restrict__ colv, int64_t nF, int64_t V,
                                                  const uint32_t* __restrict__ off,
                                                  const uint32_t* __restrict__ list, int touch_words,
                                                  uint32_t* __restrict__ touch) {
    extern __shared__ uint32_t bits[];
    const int64_t rb = blockIdx.x;
    for (int w = threadIdx.x; w < touch_words; w += blockDim.x) bits[w] = 0u;
    __syncthreads();
    // ROWB rows x 3 corners, one (row, corner) per thread
    for (int e = threadIdx.x; e < ROWB * 3; e += blockDim.x) {
        const int64_t i = rb * ROWB + e / 3;
        if (i >= nF) continue;
        const int4 v = colv[i];
        const int vk = (e % 3 == 0) ? v.x : (e % 3 == 1) ? v.y : v.z;
        if (vk < 0 || vk >= V) continue;
        for (uint32_t q = off[vk]; q < off[vk + 1]; ++q) {
            const uint32_t t = (list[q] / 3) / CHUNK;
            atomicOr(&bits[t >> 5], 1u << (t & 31));
        }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < touch_words; w += blockDim.x) touch[rb * touch_words + w] = bits[w];
}

// ---- host launchers ----------------------------------------------------------------------------

hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* off, uint32_t* ws, hipStream_t st);

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

hipError_t launch_fill(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int g = (int)std::min<int64_t>(nblk(n, 256), 4096);
    hipLaunchKernelGGL(fill_u32, dim3(g), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_init(uint32_t* zero, int64_t nzero, uint32_t* bbox, uint32_t* flags, hipStream_t st) {
    int g = (int)std::min<int64_t>(std::max<int64_t>(nblk(nzero, 256), 1), 2048);
    hipLaunchKernelGGL(init_scratch, dim3(g), dim3(256), 0, st, zero, nzero, bbox, flags);
    return hipGetLastError();
}

// fs: ints per face in F (3 for triangles; 10 for curved cubic elements, corners first)
// expect (nullable, device): the checksum the face list must have (FLAG_TREE_FACES otherwise)
hipError_t launch_bbox(const double* X, int64_t V, const int32_t* F, int fs, int64_t nF, uint32_t* bbox,
                       uint32_t* flags, hipStream_t st, const uint32_t* expect) {
    // up to BBOX_SLOTS work-groups (a few faces per thread): the loads of a face's corners are
    // dependent gathers, so the pass is bound by latency, not by its few bytes
    int g = (int)std::max<int64_t>(1, std::min<int64_t>(nblk(nF, 256), BBOX_SLOTS));
    hipLaunchKernelGGL(face_bbox, dim3(g), dim3(256), 0, st, X, V, F, fs, nF, bbox, flags, expect);
    return hipGetLastError();
}

hipError_t launch_morton(const double* X, int64_t V, const int32_t* F, int fs, int64_t nF, int Q,
                         const uint32_t* bbox, int bits, uint32_t* keys, uint32_t* vals, hipStream_t st) {
    hipLaunchKernelGGL(morton_keys, dim3(nblk(nF * Q, 256)), dim3(256), 0, st, X, V, F, fs, nF, Q, bbox, bits, keys,
                       vals);
    return hipGetLastError();
}

hipError_t launch_p3_records(const double* X, int64_t V, const int32_t* F10, int64_t nF, int Q, int64_t Fp,
                             const uint32_t* perm, const uint32_t* bbox, double* org, ColRec* cols, int4* colv,
                             double* c64, double* geo, uint32_t* cnt, uint32_t* flags, hipStream_t st) {
    hipLaunchKernelGGL(p3_records, dim3(nblk(Fp, 256)), dim3(256), 0, st, X, V, F10, nF, Q, Fp, perm, bbox, org,
                       cols, colv, c64, geo, cnt, flags);
    return hipGetLastError();
}

// node CSR of the gather over n items of `step` records: cnt and cursor (V entries each) zero on
// entry; ws: scan workspace (scan_ws_words(V) words); list: 10 n entries
hipError_t launch_p3_nodes(const int32_t* F10, int64_t n, int step, int Q, int64_t V, const uint32_t* perm,
                           uint32_t* cnt, uint32_t* off, uint32_t* cursor, uint32_t* list, uint32_t* ws,
                           hipStream_t st) {
    hipLaunchKernelGGL(p3_node_count, dim3(nblk(n, 256)), dim3(256), 0, st, F10, n, step, Q, V, perm, cnt);
    hipError_t e = launch_exclusive_scan(cnt, V, off, ws, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(p3_node_fill, dim3(nblk(n, 256)), dim3(256), 0, st, F10, n, step, Q, V, perm, off, cursor,
                       list);
    return hipGetLastError();
}

// cnt (V entries) must be zero on entry; face_records accumulates the per-vertex corner counts.
hipError_t launch_records(const double* X, int64_t V, const int32_t* F, int64_t nF, int Q, int64_t Fp,
                          const uint32_t* perm, const uint32_t* bbox, double* org, ColRec* cols, int4* colv,
                          double* c64, double* geo, uint32_t* cnt, uint32_t* flags, hipStream_t st) {
    hipLaunchKernelGGL(face_records, dim3(nblk(Fp, 256)), dim3(256), 0, st, X, V, F, nF, Q, Fp, perm, bbox, org,
                       cols, colv, c64, geo, cnt, flags);
    return hipGetLastError();
}

// cnt holds the per-vertex corner counts; cursor must be zero (V entries); ws: scan workspace
// (scan_ws_words(V) words).
hipError_t launch_adjacency(const int4* colv, int64_t nF, int64_t V, uint32_t* cnt, uint32_t* off,
                            uint32_t* cursor, uint32_t* list, uint32_t* ws, hipStream_t st) {
    hipError_t e = launch_exclusive_scan(cnt, V, off, ws, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(corner_fill, dim3(nblk(nF, 256)), dim3(256), 0, st, colv, nF, V, off, cursor, list);
    return hipGetLastError();
}

hipError_t launch_touch(const int4* colv, int64_t nF, int64_t V, const uint32_t* off, const uint32_t* list,
                        int nrb, int touch_words, uint32_t* touch, hipStream_t st) {
    hipLaunchKernelGGL(touch_map, dim3(nrb), dim3(256), touch_words * sizeof(uint32_t), st, colv, nF, V, off, list,
                       touch_words, touch);
    return hipGetLastError();
}

}  // namespace tpe
