// C ABI of libtpe: context, scratch arena, validation and the exact energy / gradient pipeline.
//
// Pipeline of one tpe_gradient call (all on the context's stream, no host synchronisation
// unless sync checks are on):
//   init_scratch -> face_bbox -> morton_keys -> radix sort (2 or 3 passes) -> face_records
//   (+ per-vertex corner counts) -> vertex->corner CSR (scan, fill)
//   -> tile-pair exclusion map -> pair_kernel (exact all-pairs row sums, compensated segments)
//   -> finalize (FP64 merge of the segments, adjoint, energy) -> vertex_gather (ascending order).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tpe.h"
#include "common.hpp"
#include "mlp.hpp"

namespace tpe {
hipError_t launch_fill(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
hipError_t launch_init(uint32_t* zero, int64_t nzero, uint32_t* bbox, uint32_t* flags, hipStream_t st);
hipError_t launch_bbox(const double* X, int64_t V, const int32_t* F, int fs, int64_t nF, uint32_t* bbox,
                       uint32_t* flags, hipStream_t st, const uint32_t* expect = nullptr);
hipError_t launch_morton(const double* X, int64_t V, const int32_t* F, int fs, int64_t nF, int Q, const uint32_t* bbox,
                         int bits, uint32_t* keys, uint32_t* vals, hipStream_t st);
hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* ktmp, uint32_t* vtmp, int64_t n, int bits,
                      uint32_t* hist, uint32_t* off, hipStream_t st);
int64_t radix_hist_words(int64_t n);
int64_t scan_ws_words(int64_t n);
hipError_t launch_records(const double* X, int64_t V, const int32_t* F, int64_t nF, int Q, int64_t Fp,
                          const uint32_t* perm, const uint32_t* bbox, double* org, ColRec* cols, int4* colv,
                          double* c64, double* geo, uint32_t* cnt, uint32_t* flags, hipStream_t st);
hipError_t launch_adjacency(const int4* colv, int64_t nF, int64_t V, uint32_t* cnt, uint32_t* off, uint32_t* cursor,
                            uint32_t* list, uint32_t* ws, hipStream_t st);
hipError_t launch_p3_records(const double* X, int64_t V, const int32_t* F10, int64_t nF, int Q, int64_t Fp,
                             const uint32_t* perm, const uint32_t* bbox, double* org, ColRec* cols, int4* colv,
                             double* c64, double* geo, uint32_t* cnt, uint32_t* flags, hipStream_t st);
hipError_t launch_p3_nodes(const int32_t* F10, int64_t n, int step, int Q, int64_t V, const uint32_t* perm,
                           uint32_t* cnt, uint32_t* off, uint32_t* cursor, uint32_t* list, uint32_t* ws,
                           hipStream_t st);
hipError_t launch_p3_finalize(bool grad, const float* part, const Sched& sc, int64_t Fp, int64_t n, int step, int Q,
                              const double* acc64, const uint32_t* perm, const int32_t* F10, int64_t V,
                              const double* X, const uint32_t* bbox, double q, double p, double scale, double efac,
                              double* corner, double* epart, uint32_t* flags, double* E, EnergyOut* in_gather,
                              hipStream_t st);
hipError_t launch_touch(const int4* colv, int64_t nF, int64_t V, const uint32_t* off, const uint32_t* list,
                        int nrb, int touch_words, uint32_t* touch, hipStream_t st);
int pair_blocks_per_cu(bool grad);
Sched make_sched(int64_t rows_p, int64_t cols_p, int waves);
int64_t pair_part_floats(const Sched& sc, bool grad);
hipError_t launch_pair(bool grad, int q, int p, const ColRec* cols, const int4* colv, const double* c64,
                       const double* org, const uint32_t* touch, int touch_words, const Sched& sc, float* part,
                       hipStream_t st);
bool pair_exponents_ok(int q, int p);
hipError_t launch_finalize(bool grad, const float* part, const Sched& sc, int64_t Fp, int64_t nF, const double* acc64,
                           const double* geo, const int4* colv, const double* X, const uint32_t* bbox, double q,
                           double p, double scale, double efac, int Q, double* corner, double* epart,
                           uint32_t* flags, double* E, EnergyOut* in_gather, hipStream_t st);
hipError_t launch_sym_merge(bool grad, const float* part, const float* colpart, const int* first,
                            const SymSched& sc, int64_t nR, int64_t Fp, double* acc64, hipStream_t st);
int pair_sym_blocks_per_cu(bool grad, int nw, bool decoupled);
SymSched make_sym_sched(int64_t Fp, int W, int tail, int nw);
int64_t sym_part_floats(const SymSched& sc, bool grad);
int64_t sym_colpart_floats(const SymSched& sc, bool grad);
hipError_t launch_pair_sym(bool grad, int q, int p, const ColRec* cols, const int4* colv, const double* c64,
                           const double* org, const uint32_t* touch, int touch_words, const SymSched& sc, float* part,
                           float* colpart, int* first, bool decoupled, uint32_t* flags, hipStream_t st);
bool pair_sym_gen_ok(int nw, bool decoupled);
int dual_level(int H, int leaf);
int64_t dual_entry_cap(int H, int leaf);
int64_t dual_part_floats(int H, int leaf);
hipError_t launch_dual(int H, int leaf, float theta, const ColRec* cols, const int4* colv, const double* c64,
                       const double* geo, const double* org, const void* nodes64, const void* recs_, int64_t nF,
                       int64_t Fp, double q, double p, uint32_t* off, uint32_t* nnear, uint32_t* nfar, uint32_t* cnt,
                       uint32_t* rel, uint32_t* ent, uint32_t* scanws, double* adj, float* part, double* acc64,
                       uint32_t* flags, unsigned long long* stats, uint32_t* const sort[6], hipStream_t st);
// the symmetric kernel is used while its column partials (32 B per face and earlier super block)
// fit in this many bytes (of the GPU's 288 GB of HBM): about 1,480,000 faces with super blocks of 512
// faces, about 2,100,000 with 1,024; if the allocation fails the call runs the row-only kernel instead
constexpr int64_t SYM_MAX_COLPART_BYTES = (int64_t)64 << 30;
// With work-group barriers (TPE_OPT_SYM_BARRIERS = 1), work-groups of 1 or 2 waves (super blocks of
// 128 or 256 faces) run the symmetric kernel faster than 4 (each wave waits less at the barriers:
// 64.3 / 64.6 / 70.2 ms at 327,680 faces) but write 4 or 2 times the column partials, which the
// merge reads back (the whole step: 67.1 / 66.2 / 71.2 ms); the fewest waves whose partials fit in
// this budget are then taken (20,480 faces: 1 wave; 327,680 faces: 2, 6.2 GiB), else 4.  Without
// barriers (the default) 4 waves run fastest at every size: 61.9 ms, step 62.9 ms (8 waves, with
// half the partials: 63.7 ms; taken only where 4 would exceed SYM_MAX_COLPART_BYTES).
constexpr int64_t SYM_FAST_COLPART_BYTES = (int64_t)8 << 30;
hipError_t launch_pair_conf(bool grad, const ColRec* rcols, const double* rc64, const int4* rcolv,
                            const ColRec* ccols, const int4* ccolv, const double* corg, const Sched& sc, float* part,
                            hipStream_t st);
hipError_t launch_gather(const uint32_t* off, const uint32_t* list, int64_t V, const double* corner, double* G,
                         const EnergyOut& en, hipStream_t st);
int finalize_blocks(int64_t nF);
int tree_height(int64_t nF, int leaf);
hipError_t build_kd_order(const double* X, int64_t V, const int32_t* F, int64_t nF, int Q, int leaf, int H, float4* cen,
                          uint32_t* nb, uint32_t* perm, uint32_t* keys, uint32_t* ktmp, uint32_t* vtmp,
                          uint32_t* hist, uint32_t* off, hipStream_t st);
size_t tree_node_bytes(int H);
size_t tree_rec_bytes(int H);
hipError_t launch_tree_moments(const double* c64, const double* geo, const int4* colv, const double* X,
                               const uint32_t* bbox, int64_t nF, int leaf, int H, void* nodes64, void* recs, bool mom2,
                               float4* balls, hipStream_t st);
hipError_t launch_farfield_samples(const ColRec* cols, const int4* colv, const double* c64, const double* X,
                                  const uint32_t* bbox, const void* recs, int H, int leaf, int64_t nF, float theta,
                                  uint32_t seed, uint32_t sel, int quota, int64_t max_faces, float4* balls,
                                  float* feats, float* targets, const void* mlp_packed, float* pred, hipStream_t st);
hipError_t launch_farfield(const ColRec* cols, const int4* colv, const double* c64, const double* org,
                           const double* X, const uint32_t* bbox, const void* recs, int H, int leaf, int64_t nF,
                           int64_t Fp, float theta, const void* mlp_packed, float4* balls, double* acc64,
                           unsigned long long* stats, uint32_t* work, uint32_t* ent, uint4* lst, int64_t cap,
                           uint32_t* flags, uint32_t* const sort[6], const uint32_t* nbl, const uint2* xm,
                           hipEvent_t ev0, hipEvent_t ev1, hipStream_t st);
int64_t ff_list_cap(int64_t n, int leaf);
hipError_t launch_block_neighbours(const int4* colv, const uint32_t* voff, const uint32_t* vlist, int64_t nF,
                                   int64_t V, uint32_t* nbl, uint2* xm, hipStream_t st);
int64_t block_neighbour_words(int64_t n);
int64_t block_exclusion_mask_words(int64_t n);

// Per sorted face: number of faces (itself included) that share at least one vertex with it.
__global__ void excluded_count(const int4* __restrict__ colv, int64_t nF, int64_t V, const uint32_t* __restrict__ off,
                               const uint32_t* __restrict__ list, unsigned long long* __restrict__ total) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    unsigned long long c = 0;
    if (i < nF) {
        const int4 v = colv[i];
        const int vv[3] = {v.x, v.y, v.z};
        for (int k = 0; k < 3; ++k) {
            if (vv[k] < 0 || vv[k] >= V) continue;
            for (uint32_t e = off[vv[k]]; e < off[vv[k] + 1]; ++e) {
                const uint32_t j = list[e] / 3;
                // count j once: only at the first of i's vertices whose list contains j
                bool seen = false;
                for (int k2 = 0; k2 < k && !seen; ++k2) {
                    if (vv[k2] < 0 || vv[k2] >= V) continue;
                    for (uint32_t e2 = off[vv[k2]]; e2 < off[vv[k2] + 1]; ++e2)
                        if (list[e2] / 3 == j) { seen = true; break; }
                }
                if (!seen) ++c;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(total, c);
}

// Vertex ids of each face in input order (used where no sorting is needed).
__global__ void face_ids(const int32_t* __restrict__ F, int64_t nF, int64_t V, int4* __restrict__ colv,
                         uint32_t* __restrict__ cnt, uint32_t* __restrict__ flags) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nF) return;
    const int a = F[3 * i], b = F[3 * i + 1], c = F[3 * i + 2];
    const bool ok = a >= 0 && a < V && b >= 0 && b < V && c >= 0 && c < V;
    if (!ok) atomicOr(flags, (uint32_t)FLAG_BAD_INDEX);
    colv[i] = ok ? make_int4(a, b, c, 0) : make_int4(-3, -3, -3, 0);
    if (ok) {
        atomicAdd(&cnt[a], 1u);
        atomicAdd(&cnt[b], 1u);
        atomicAdd(&cnt[c], 1u);
    }
}
}  // namespace tpe

using namespace tpe;

// ---- scratch of the entry point that allocates nothing (tpe_gradient_noalloc) -------------------
// One file-scope device array, which every GPU the library runs on holds for the process's life.
// In host code `noalloc_scratch` names a host-side stand-in, not device memory: its device address
// is looked up once per device (tpe_create, with the device current) and only that address is
// handed to kernels.  Every tpe_gradient_noalloc call on a device uses that device's copy.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) char noalloc_scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_noalloc_mu;
std::vector<void*> g_noalloc_ptr;  // device address of noalloc_scratch per device (null: not looked up)

// With `device` current: look up its copy of the array, once.
void noalloc_setup(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if ((int)g_noalloc_ptr.size() <= device) g_noalloc_ptr.resize((size_t)device + 1, nullptr);
    if (g_noalloc_ptr[device]) return;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch)) == hipSuccess && ptr)
        g_noalloc_ptr[device] = ptr;
    else
        (void)hipGetLastError();  // tpe_gradient_noalloc then reports TPE_ERR_HIP
}

void* noalloc_ptr(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    return device >= 0 && device < (int)g_noalloc_ptr.size() ? g_noalloc_ptr[device] : nullptr;
}
}  // namespace

struct tpe_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    bool sync_checks = true;
    int64_t target_waves = 0;     // 0: resident-wave capacity of the pair kernel
    int quad = 1;                 // quadrature points per face of the exact path (1, 3 or 6)
    int resident[2] = {0, 0};     // pair-kernel work-groups resident on the device (energy, gradient)
    int resident_sym[4][2] = {};  // the same for the symmetric pair kernel, work-groups of 1, 2, 4 waves
    int resident_symf[4][2] = {}; // the same for its barrier-free form (2, 4 and 8 waves)
    int sym_waves = 0;            // waves per work-group of the symmetric kernel (0: by size)
    bool sym_barriers = false;    // the symmetric kernel with work-group barriers (else barrier-free)
    bool symmetric = true;        // exact self energy (6, 12): symmetric pair kernel where it fits
    char* arena = nullptr;
    size_t arena_bytes = 0;
    uint32_t* dflags = nullptr;   // device error word
    uint32_t* hflags = nullptr;   // pinned host mirror
    unsigned long long* dstats = nullptr;  // far-field interaction counters of the last call
    int kernel_timing = 0;        // 1: the dominant kernel, 2: finalize + vertex gather
    std::vector<hipEvent_t> ev_pool;  // pairs (start, stop), reused
    size_t ev_used = 0;               // events recorded since the last tpe_kernel_time
    // second stream (default priority) for the far field's vertex CSR, which only the final gather
    // reads: it runs beside the moments and the walk, forked from and joined back into `stream`
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // end of the last call that enqueued work: recorded on that call's stream, waited for by the
    // next call when it runs on another stream (see Ordered)
    hipEvent_t done = nullptr;
    hipStream_t done_stream = nullptr;
    bool done_valid = false;
};

struct tpe_mlp {
    int device = 0;
    int64_t step = 0;
    float* P = nullptr;  // FP32 master parameters (device)
    float* M = nullptr;  // Adam first moments
    float* V = nullptr;  // Adam second moments
    void* packed = nullptr;  // BF16 fragments + biases for inference (kept in sync with P)
    float min_s = 0.f;       // apply the correction only to clusters with r_B / rho >= min_s
    float lam = 0.f;         // weight of the neighbouring-row difference term of the training loss
    float* gpart = nullptr;  // per-tile gradient partials (grow-only)
    float* lpart = nullptr;
    int64_t cap_tiles = 0;
};

struct tpe_tree {
    int device = 0;
    int64_t nF = 0, V = 0;
    int leaf = 32, H = 0;
    int Q = 0;                 // 0: a tree over faces; >= 1: over the Q quadrature points of each curved element
    int64_t n = 0;             // items: nF faces, or nF Q points
    uint32_t* perm = nullptr;  // sorted position -> input item (face f, or point r = Q f + point) (device, n entries)
    uint32_t* work = nullptr;  // work of each 64-item target block in the last far-field walk (device, (n + 63) / 64)
    // flat trees: the vertex -> (sorted face, corner) lists of the gather (3 nF slots, V + 1
    // offsets), which depend only on F and the order, and the checksum of F they were built from
    uint32_t* voff = nullptr;
    uint32_t* vlist = nullptr;
    uint32_t* fsum = nullptr;
    uint32_t* nbl = nullptr;   // flat trees: per target block, the tiles holding a face that shares a vertex with it
    uint2* xm = nullptr;       // flat trees: per (target block, listed tile, row) the 64-bit exclusion mask
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int fail(tpe_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(tpe_ctx* c, hipError_t e, const char* where) {
    return fail(c, TPE_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                                              \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr);    \
    } while (0)

// Stream order of the calls of one context.  Every call enqueues on ctx->stream; if the previous
// call ran on another stream (tpe_set_stream in between, as the Python binding does for torch's
// current stream), the new stream first waits for the event recorded at the end of that call.  On
// leaving, the call records the event on its own stream.  So calls never overlap on the context's
// scratch arena, flags or counters whatever streams they run on, and a stream the caller has
// switched away from may be destroyed afterwards (the event was recorded on it already).
struct Ordered {
    tpe_ctx* ctx;
    int rc = TPE_OK;
    explicit Ordered(tpe_ctx* c) : ctx(c) {
        if (ctx->done_valid && ctx->done_stream != ctx->stream) {
            const hipError_t e = hipStreamWaitEvent(ctx->stream, ctx->done, 0);
            if (e != hipSuccess) rc = hip_fail(ctx, e, "hipStreamWaitEvent");
        }
    }
    ~Ordered() {
        if (hipEventRecord(ctx->done, ctx->stream) == hipSuccess) {
            ctx->done_stream = ctx->stream;
            ctx->done_valid = true;
        } else {
            (void)hipGetLastError();
        }
    }
    Ordered(const Ordered&) = delete;
    Ordered& operator=(const Ordered&) = delete;
};

#define ORDERED(ctx)                    \
    Ordered ordered_call_(ctx);         \
    if (ordered_call_.rc) return ordered_call_.rc

// Bump allocator over the arena; 256-byte aligned slices.
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(char* b) : base(b) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
};

struct Plan {
    int64_t nF, V, Fp;
    int Q = 1;        // quadrature points per face (records per face)
    bool p3 = false;  // curved cubic elements: F holds 10 node ids per element, V counts all nodes
    int fs = 3;       // ints per face in F
    uint32_t *ncnt = nullptr, *ncursor = nullptr, *noff = nullptr, *nlist = nullptr;  // node CSR (p3)
    int64_t nR = 0;   // records = Q nF
    int ntiles, nrb, touch_words, sort_blocks, fin_blocks;
    Sched sc;
    // symmetric pair kernel (exact self energy)
    bool sym = false;
    SymSched ssc{};
    bool sym_free = false;  // the symmetric kernel without work-group barriers
    float* colpart = nullptr;
    int* first = nullptr;
    // buffers
    uint32_t *keys, *vals, *ktmp, *vtmp, *hist, *hoff, *bbox;
    uint32_t *zero_begin, *cnt, *cursor, *touch, *zero_end;
    uint32_t *voff, *list, *scanws;
    double *org, *c64, *geo, *corner, *epart, *acc64;
    int morton_bits;
    ColRec* cols;
    int4* colv;
    float* part;
    unsigned long long* counter;
    // confinement: the fixed confining surface (columns)
    int64_t nFY = 0, VY = 0, FpY = 0;
    int morton_bits_y = 0;
    ColRec* colsY = nullptr;
    int4* colvY = nullptr;
    double *c64Y = nullptr, *geoY = nullptr, *orgY = nullptr;
    // far field
    int treeH = -1;
    void *nodes64 = nullptr, *recs = nullptr;
    float4* balls = nullptr;
    float4* cen4 = nullptr;
    uint32_t* nbox = nullptr;
    // lists of the far-field walk (leaf size of the tree; 0: not used)
    int ff_leaf = 0;
    int64_t ff_cap = 0;
    uint32_t* ff_ent = nullptr;
    uint4* ff_lst = nullptr;
    // dual-tree far field (leaf size of the tree; -1: not used)
    int dual_leaf = -1;
    uint32_t *doff = nullptr, *dnear = nullptr, *dfar = nullptr, *dcnt = nullptr, *drel = nullptr;
    uint32_t *dent = nullptr, *dscan = nullptr;
    double* dadj = nullptr;
    float* dpart = nullptr;
    size_t bytes;
};

void layout(Plan& P, char* base, bool grad) {
    Carve c(base);
    const int64_t nF = P.nF, V = P.V, Fp = P.Fp;
    const int64_t nR = P.nR;
    const int64_t ns = std::max(nR, P.nFY);  // the sort buffers serve both surfaces in turn
    P.keys = c.take<uint32_t>(ns);
    P.vals = c.take<uint32_t>(ns);
    P.ktmp = c.take<uint32_t>(ns);
    P.vtmp = c.take<uint32_t>(ns);
    P.hist = c.take<uint32_t>((size_t)radix_hist_words(ns));
    P.hoff = c.take<uint32_t>((size_t)radix_hist_words(ns));
    P.bbox = c.take<uint32_t>(BBOX_WORDS);
    P.counter = c.take<unsigned long long>(1);
    // one contiguous zero-initialised region
    P.zero_begin = c.take<uint32_t>(0);
    P.cnt = c.take<uint32_t>(V);
    P.cursor = c.take<uint32_t>(V);
    if (P.p3 && grad) {
        P.ncnt = c.take<uint32_t>(V);
        P.ncursor = c.take<uint32_t>(V);
    }
    P.zero_end = c.take<uint32_t>(0);
    // the exact path's P3 finalize works per element, the far field's per point record
    const int64_t p3_items = P.treeH >= 0 ? nR : nF;
    if (P.p3 && grad) {
        P.noff = c.take<uint32_t>(V + 1);
        P.nlist = c.take<uint32_t>((size_t)P3_NODES * p3_items);
    }
    P.touch = c.take<uint32_t>((size_t)P.nrb * P.touch_words);
    P.voff = c.take<uint32_t>(V + 1);
    P.scanws = c.take<uint32_t>((size_t)scan_ws_words(V) + 1);
    P.list = c.take<uint32_t>(3 * nR);
    P.org = c.take<double>(3 * (size_t)P.ntiles);
    P.cols = c.take<ColRec>(Fp);
    P.colv = c.take<int4>(Fp);
    P.c64 = c.take<double>(3 * Fp);
    P.geo = c.take<double>(5 * Fp);
    P.part = c.take<float>((size_t)(P.sym ? sym_part_floats(P.ssc, grad) : pair_part_floats(P.sc, grad)));
    if (P.sym) {
        P.colpart = c.take<float>((size_t)sym_colpart_floats(P.ssc, grad));
        P.first = c.take<int>((size_t)P.ssc.W);
    }
    P.corner = c.take<double>(grad ? std::max<int64_t>(9 * nR, P.p3 ? 3 * P3_NODES * p3_items : 0) : 1);
    P.acc64 = c.take<double>((size_t)(grad ? NACC : 1) * Fp);
    P.epart = c.take<double>(P.fin_blocks);
    if (P.FpY > 0) {
        P.colsY = c.take<ColRec>(P.FpY);
        P.colvY = c.take<int4>(P.FpY);
        P.c64Y = c.take<double>(3 * P.FpY);
        P.geoY = c.take<double>(5 * P.FpY);
        P.orgY = c.take<double>(3 * (P.FpY / CTILE));
    }
    if (P.treeH >= 0) {
        P.nodes64 = c.take<char>(tree_node_bytes(P.treeH));
        P.recs = c.take<char>(tree_rec_bytes(P.treeH));
        P.balls = c.take<float4>(Fp / 64);
        P.cen4 = c.take<float4>(nR);
        P.nbox = c.take<uint32_t>((size_t)6 << std::max(P.treeH - 1, 0));
        if (P.ff_leaf > 0) {
            const int64_t nb = (nR + 63) / 64;
            P.ff_cap = ff_list_cap(nR, P.ff_leaf);
            P.ff_ent = c.take<uint32_t>((size_t)(nb * P.ff_cap));
            P.ff_lst = c.take<uint4>((size_t)nb);
        }
        if (P.dual_leaf > 0) {
            const int Hd = dual_level(P.treeH, P.dual_leaf);
            const size_t nn = (size_t)2 << Hd, nl = (size_t)1 << Hd;
            P.doff = c.take<uint32_t>(nn);
            P.dnear = c.take<uint32_t>(nn);
            P.dfar = c.take<uint32_t>(nn);
            P.dcnt = c.take<uint32_t>(nl);
            P.drel = c.take<uint32_t>(nl);
            P.dscan = c.take<uint32_t>((size_t)scan_ws_words((int64_t)nl) + 1);
            P.dent = c.take<uint32_t>((size_t)dual_entry_cap(P.treeH, P.dual_leaf));
            P.dadj = c.take<double>(8 * nn);
            P.dpart = c.take<float>((size_t)dual_part_floats(P.treeH, P.dual_leaf));
        }
    }
    P.bytes = c.off + 256;
}

// sym: the exact self energy asks for the symmetric kernel (taken if its buffers fit)
void plan(Plan& P, const tpe_ctx* ctx, int64_t nF, int64_t V, bool grad, int treeH = -1, int64_t nFY = 0,
          int64_t VY = 0, int Q = 1, bool sym = false, bool p3 = false) {
    P.treeH = treeH;
    P.p3 = p3;
    P.fs = p3 ? P3_NODES : 3;
    P.Q = Q;
    P.nR = nF * Q;
    P.nFY = nFY;
    P.VY = VY;
    P.FpY = nFY > 0 ? round_up(nFY, std::max(ROWB, CTILE)) : 0;
    P.morton_bits_y = nFY <= (int64_t)1 << 18 ? 6 : 10;
    P.nF = nF;
    P.V = V;
    P.Fp = round_up(P.nR, std::max(ROWB, CTILE));
    P.sym = false;
    if (sym) {
        // waves per work-group: forced by TPE_OPT_SYM_WAVES; else 4 without barriers (the fastest
        // at every size, and the fewest column partials); with barriers the fewest waves whose
        // column partials fit in SYM_FAST_COLPART_BYTES
        int nw = ctx->sym_waves;
        if (nw == 0 && !ctx->sym_barriers) {
            // 8 waves only where 4 would exceed the partials' cap (half the partials, 4% slower)
            const int64_t Fs4 = round_up(P.nR, (int64_t)4 * ROWB);
            nw = sym_colpart_floats(make_sym_sched(Fs4, 1, 0, 4), grad) * (int64_t)sizeof(float) <=
                         SYM_MAX_COLPART_BYTES
                     ? 4
                     : 8;
        }
        if (nw == 0) {
            nw = 4;
            for (int cand = 1; cand < 4; cand *= 2) {
                const SymSched t = make_sym_sched(round_up(P.nR, (int64_t)cand * ROWB), 1, 0, cand);
                if (sym_colpart_floats(t, grad) * (int64_t)sizeof(float) <= SYM_FAST_COLPART_BYTES) {
                    nw = cand;
                    break;
                }
            }
        }
        const int64_t Fs = round_up(P.nR, (int64_t)nw * ROWB);
        // work-groups: 1 to 8 times the resident count, one step per 16 units a resident slot
        // would get (the hardware refills the slots of early finishers, which evens out the
        // finish times; more work-groups add row segments for the merge to read), then one
        // single-unit work-group per resident slot for the end of the launch
        if (nw == 8 && ctx->sym_barriers) nw = 4;  // 8 waves only without barriers
        const bool decoupled = nw >= 2 && !ctx->sym_barriers;
        const int resident = std::max(1, (decoupled ? ctx->resident_symf : ctx->resident_sym)
                                             [nw == 1 ? 0 : nw == 2 ? 1 : nw == 4 ? 2 : 3][grad ? 1 : 0]);
        int W = resident, tail = 0;
        if (ctx->target_waves > 0) {
            W = (int)ctx->target_waves;
        } else {
            const int64_t units = make_sym_sched(Fs, 1, 0, nw).U;
            W *= (int)std::max<int64_t>(1, std::min<int64_t>(8, units / ((int64_t)W * 16)));
            tail = resident;
        }
        const SymSched t = make_sym_sched(Fs, W, tail, nw);
        if (sym_colpart_floats(t, grad) * (int64_t)sizeof(float) <= SYM_MAX_COLPART_BYTES) {
            P.sym = true;
            P.sym_free = decoupled;
            P.ssc = t;
            P.Fp = Fs;
        }
    }
    P.ntiles = (int)(P.Fp / CTILE);
    P.nrb = (int)(P.Fp / ROWB);
    P.touch_words = (int)((P.Fp / CHUNK + 31) / 32);
    P.sc = make_sched(P.Fp, P.FpY > 0 ? P.FpY : P.Fp,
                      ctx->target_waves > 0 ? (int)ctx->target_waves : ctx->resident[grad ? 1 : 0]);
    P.sort_blocks = (int)ceil_div(P.nR, 4096);
    // Morton resolution: 6 bits per axis (2 radix passes of 9 bits) up to 2^18 faces, 10 above
    // (3 passes of 10 bits)
    P.morton_bits = nF <= (int64_t)1 << 18 ? 6 : 10;
    P.fin_blocks = finalize_blocks(P.nR);
    layout(P, nullptr, grad);
}

int ensure_arena(tpe_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->arena_bytes) return TPE_OK;
    if (ctx->arena) {
        // every earlier user of the arena: the calls before this one (ended by ctx->done, on
        // whichever stream), the side stream, and what this call has enqueued so far
        hipError_t e = ctx->done_valid ? hipEventSynchronize(ctx->done) : hipSuccess;
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->side);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
        (void)hipFree(ctx->arena);
        ctx->arena = nullptr;
        ctx->arena_bytes = 0;
    }
    size_t want = bytes + bytes / 8;
    if (hipMalloc(&ctx->arena, want) != hipSuccess) {
        ctx->arena = nullptr;
        (void)hipGetLastError();
        return fail(ctx, TPE_ERR_OOM, "hipMalloc of " + std::to_string(want) + " bytes failed");
    }
    ctx->arena_bytes = want;
    return TPE_OK;
}

// generic: the exact energy / gradient also take the other exponents of pair_exponents_ok;
// everything else (far field, learned correction, confinement) is (6, 12) only.
int check_common(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p,
                 bool generic = false) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!X || !F) return fail(ctx, TPE_ERR_INVALID_ARG, "null X or F");
    if (V < 1 || nF < 1) return fail(ctx, TPE_ERR_INVALID_ARG, "V and nF must be >= 1");
    if (nF > (int64_t)1 << 24 || V > (int64_t)1 << 26)
        return fail(ctx, TPE_ERR_INVALID_ARG, "mesh too large (nF <= 2^24, V <= 2^26)");
    if (!(q >= 2.0) || !(p > q) || !std::isfinite(q) || !std::isfinite(p))
        return fail(ctx, TPE_ERR_INVALID_ARG, "exponents must satisfy 2 <= q < p");
    const bool fast = q == 6.0 && p == 12.0;
    const bool other = generic && q == (int)q && p == (int)p && pair_exponents_ok((int)q, (int)p);
    if (!fast && !other)
        return fail(ctx, TPE_ERR_UNSUPPORTED,
                    generic ? "exponents: (6, 12), or even q in {2, 4, 6, 8} with even p, q < p <= 2q"
                            : "only (q, p) = (6, 12) is implemented here");
    return TPE_OK;
}

int report_flags(tpe_ctx* ctx) {
    HIPCHK(hipMemcpyAsync(ctx->hflags, ctx->dflags, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const uint32_t f = *ctx->hflags;
    if (f & FLAG_BAD_INDEX) return fail(ctx, TPE_ERR_INVALID_ARG, "face vertex index out of range");
    if (f & FLAG_NONFINITE)
        return fail(ctx, TPE_ERR_NONFINITE, "non-finite input or result (coincident non-adjacent centroids?)");
    if (f & FLAG_DEGENERATE) return fail(ctx, TPE_ERR_DEGENERATE, "degenerate face (area <= 1e-300)");
    if (f & FLAG_SYNC)
        return fail(ctx, TPE_ERR_HIP, "symmetric pair kernel: a wave gave up waiting for its work-group");
    if (f & FLAG_TREE_FACES)
        return fail(ctx, TPE_ERR_INVALID_ARG, "the faces differ from those the tree was built with");
    if (f & FLAG_LISTS)
        return fail(ctx, TPE_ERR_OOM,
                    "far-field interaction lists exceed their scratch (theta too small for this mesh)");
    return TPE_OK;
}

// Next (start, stop) event pair for kernel timing; the pool grows on demand.
int timing_events(tpe_ctx* ctx, hipEvent_t* a, hipEvent_t* b) {
    while (ctx->ev_pool.size() < ctx->ev_used + 2) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ctx->ev_pool.push_back(e);
    }
    *a = ctx->ev_pool[ctx->ev_used];
    *b = ctx->ev_pool[ctx->ev_used + 1];
    ctx->ev_used += 2;
    return TPE_OK;
}

// Shared front half: sort faces, build records, adjacency and exclusion map.
int prepare(tpe_ctx* ctx, Plan& P, const double* X, const int32_t* F) {
    hipStream_t st = ctx->stream;
    HIPCHK(launch_init(P.zero_begin, P.zero_end - P.zero_begin, P.bbox, ctx->sync_checks ? ctx->dflags : nullptr, st));
    HIPCHK(launch_bbox(X, P.V, F, P.fs, P.nF, P.bbox, ctx->dflags, st));
    HIPCHK(launch_morton(X, P.V, F, P.fs, P.nF, P.Q, P.bbox, P.morton_bits, P.keys, P.vals, st));
    HIPCHK(radix_sort(P.keys, P.vals, P.ktmp, P.vtmp, P.nR, 3 * P.morton_bits, P.hist, P.hoff, st));
    if (P.p3)
        HIPCHK(launch_p3_records(X, P.V, F, P.nF, P.Q, P.Fp, P.vals, P.bbox, P.org, P.cols, P.colv, P.c64, P.geo,
                                 P.cnt, ctx->dflags, st));
    else
        HIPCHK(launch_records(X, P.V, F, P.nF, P.Q, P.Fp, P.vals, P.bbox, P.org, P.cols, P.colv, P.c64, P.geo, P.cnt,
                              ctx->dflags, st));
    HIPCHK(launch_adjacency(P.colv, P.nR, P.V, P.cnt, P.voff, P.cursor, P.list, P.scanws, st));
    HIPCHK(launch_touch(P.colv, P.nR, P.V, P.voff, P.list, P.nrb, P.touch_words, P.touch, st));
    return TPE_OK;
}

// p3: curved cubic elements (F: 10 node ids per element, corners first; V: all nodes)
// noalloc: carve the scratch from the device's static array instead of the context's arena (no
// allocation of any kind; the row-only pair kernel, whose scratch is linear in the faces)
int run_exact(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p,
              double scale, double* E, double* G, bool p3 = false, bool noalloc = false) {
    int rc = check_common(ctx, X, V, F, nF, q, p, true);
    if (rc) return rc;
    if (!std::isfinite(scale)) return fail(ctx, TPE_ERR_INVALID_ARG, "scale must be finite");
    const bool grad = G != nullptr;
    if (nF * ctx->quad > (int64_t)1 << 26) return fail(ctx, TPE_ERR_INVALID_ARG, "too many quadrature points (> 2^26)");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    Plan P;
    char* base = nullptr;
    if (noalloc) {
        plan(P, ctx, nF, V, grad, -1, 0, 0, ctx->quad, false, p3);
        base = static_cast<char*>(noalloc_ptr(ctx->device));
        if (!base) return fail(ctx, TPE_ERR_HIP, "the no-allocation scratch has no device address");
        if (P.bytes > NOALLOC_SCRATCH_BYTES)
            return fail(ctx, TPE_ERR_INVALID_ARG,
                        "mesh too large for the no-allocation scratch: " + std::to_string(P.bytes) +
                            " bytes needed, " + std::to_string(NOALLOC_SCRATCH_BYTES) + " available");
    } else {
        // the symmetric kernel: (6, 12), and the other even exponents without barriers (4 or 8
        // waves per work-group; else the row-only kernel)
        const bool fast = q == 6.0 && p == 12.0;
        plan(P, ctx, nF, V, grad, -1, 0, 0, ctx->quad, ctx->symmetric && (fast || !ctx->sym_barriers), p3);
        if (P.sym && !fast && !pair_sym_gen_ok(P.ssc.nw, P.sym_free)) {
            P = Plan();
            plan(P, ctx, nF, V, grad, -1, 0, 0, ctx->quad, false, p3);
        }
        rc = ensure_arena(ctx, P.bytes);
        if (rc == TPE_ERR_OOM && P.sym) {  // no room for the column partials: the row-only kernel
            P = Plan();
            plan(P, ctx, nF, V, grad, -1, 0, 0, ctx->quad, false, p3);
            ctx->err.clear();
            rc = ensure_arena(ctx, P.bytes);
        }
        if (rc) return rc;
        base = ctx->arena;
    }
    layout(P, base, grad);
    hipStream_t st = ctx->stream;
    if ((rc = prepare(ctx, P, X, F))) return rc;
    if (p3 && grad)
        HIPCHK(launch_p3_nodes(F, nF, P.Q, P.Q, V, P.vals, P.ncnt, P.noff, P.ncursor, P.nlist, P.scanws, st));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const int timing = noalloc ? 0 : ctx->kernel_timing;  // timing events are created on demand: not here
    if (timing) {
        if ((rc = timing_events(ctx, &ev0, &ev1))) return rc;
    }
    if (timing == 1) HIPCHK(hipEventRecord(ev0, st));
    if (P.sym) {
        HIPCHK(launch_pair_sym(grad, (int)q, (int)p, P.cols, P.colv, P.c64, P.org, P.touch, P.touch_words, P.ssc,
                               P.part, P.colpart, P.first, P.sym_free, ctx->dflags, st));
    } else {
        HIPCHK(launch_pair(grad, (int)q, (int)p, P.cols, P.colv, P.c64, P.org, P.touch, P.touch_words, P.sc, P.part,
                           st));
    }
    if (timing == 1) HIPCHK(hipEventRecord(ev1, st));
    if (timing == 2) HIPCHK(hipEventRecord(ev0, st));
    if (P.sym) HIPCHK(launch_sym_merge(grad, P.part, P.colpart, P.first, P.ssc, P.nR, P.Fp, P.acc64, st));
    EnergyOut en = {};  // with the gradient, the energy is summed by the gather's extra work-group
    if (p3) {
        HIPCHK(launch_p3_finalize(grad, P.sym ? nullptr : P.part, P.sc, P.Fp, nF, P.Q, P.Q, P.sym ? P.acc64 : nullptr,
                                  P.vals, F, V, X, P.bbox, q, p, scale, 0.5, P.corner, P.epart, ctx->dflags,
                                  E, grad ? &en : nullptr, st));
        if (grad) HIPCHK(launch_gather(P.noff, P.nlist, V, P.corner, G, en, st));
    } else {
        HIPCHK(launch_finalize(grad, P.sym ? nullptr : P.part, P.sc, P.Fp, P.nR, P.sym ? P.acc64 : nullptr, P.geo,
                               P.colv, X, P.bbox, q, p, scale, 0.5, P.Q, P.corner, P.epart, ctx->dflags, E,
                               grad ? &en : nullptr, st));
        if (grad) HIPCHK(launch_gather(P.voff, P.list, V, P.corner, G, en, st));
    }
    if (timing == 2) HIPCHK(hipEventRecord(ev1, st));
    if (ctx->sync_checks) return report_flags(ctx);
    return TPE_OK;
}

// Confinement energy / gradient: rows = the moving surface (X, F) in Morton order with its CSR for
// the gather; columns = the confining surface (Y, FY) in Morton order, records only.  Both are
// normalised by one power of two from their common bounding box.
int run_conf(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF, const double* Y, int64_t VY,
             const int32_t* FY, int64_t nFY, double q, double p, double scale, double* E, double* G) {
    int rc = check_common(ctx, X, V, F, nF, q, p);
    if (rc) return rc;
    if (ctx->quad != 1) return fail(ctx, TPE_ERR_UNSUPPORTED, "the confinement energy uses one point per face");
    if ((rc = check_common(ctx, Y, VY, FY, nFY, q, p))) return rc;
    if (!std::isfinite(scale)) return fail(ctx, TPE_ERR_INVALID_ARG, "scale must be finite");
    const bool grad = G != nullptr;
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    Plan P;
    plan(P, ctx, nF, V, grad, -1, nFY, VY);
    if ((rc = ensure_arena(ctx, P.bytes))) return rc;
    layout(P, ctx->arena, grad);
    hipStream_t st = ctx->stream;
    HIPCHK(launch_init(P.zero_begin, P.zero_end - P.zero_begin, P.bbox, ctx->sync_checks ? ctx->dflags : nullptr, st));
    HIPCHK(launch_bbox(X, V, F, 3, nF, P.bbox, ctx->dflags, st));
    HIPCHK(launch_bbox(Y, VY, FY, 3, nFY, P.bbox, ctx->dflags, st));
    // confining surface: records in Morton order (the sort buffers are reused for the rows below)
    HIPCHK(launch_morton(Y, VY, FY, 3, nFY, 1, P.bbox, P.morton_bits_y, P.keys, P.vals, st));
    HIPCHK(radix_sort(P.keys, P.vals, P.ktmp, P.vtmp, nFY, 3 * P.morton_bits_y, P.hist, P.hoff, st));
    HIPCHK(launch_records(Y, VY, FY, nFY, 1, P.FpY, P.vals, P.bbox, P.orgY, P.colsY, P.colvY, P.c64Y, P.geoY, nullptr,
                          ctx->dflags, st));
    // moving surface: records, corner counts and CSR (no exclusion between different surfaces)
    HIPCHK(launch_morton(X, V, F, 3, nF, 1, P.bbox, P.morton_bits, P.keys, P.vals, st));
    HIPCHK(radix_sort(P.keys, P.vals, P.ktmp, P.vtmp, nF, 3 * P.morton_bits, P.hist, P.hoff, st));
    HIPCHK(launch_records(X, V, F, nF, 1, P.Fp, P.vals, P.bbox, P.org, P.cols, P.colv, P.c64, P.geo, P.cnt, ctx->dflags,
                          st));
    if (grad) HIPCHK(launch_adjacency(P.colv, nF, V, P.cnt, P.voff, P.cursor, P.list, P.scanws, st));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (ctx->kernel_timing) {
        if ((rc = timing_events(ctx, &ev0, &ev1))) return rc;
    }
    if (ctx->kernel_timing == 1) HIPCHK(hipEventRecord(ev0, st));
    HIPCHK(launch_pair_conf(grad, P.cols, P.c64, P.colv, P.colsY, P.colvY, P.orgY, P.sc, P.part, st));
    if (ctx->kernel_timing == 1) HIPCHK(hipEventRecord(ev1, st));
    if (ctx->kernel_timing == 2) HIPCHK(hipEventRecord(ev0, st));
    EnergyOut en = {};  // with the gradient, the energy is summed by the gather's extra work-group
    HIPCHK(launch_finalize(grad, P.part, P.sc, P.Fp, nF, nullptr, P.geo, P.colv, X, P.bbox, q, p, scale, 1.0, 1,
                           P.corner, P.epart, ctx->dflags, E, grad ? &en : nullptr, st));
    if (grad) HIPCHK(launch_gather(P.voff, P.list, V, P.corner, G, en, st));
    if (ctx->kernel_timing == 2) HIPCHK(hipEventRecord(ev1, st));
    if (ctx->sync_checks) return report_flags(ctx);
    return TPE_OK;
}

// Device arrays of a new tree: the permutation (copied from the build's sort) and the per-block
// work record of the far-field walk (zero: the first walk runs in tree order).  Frees the tree on
// failure.
void free_tree(tpe_tree* t) {
    for (uint32_t* p : {t->perm, t->work, t->voff, t->vlist, t->fsum, t->nbl})
        if (p) (void)hipFree(p);
    if (t->xm) (void)hipFree(t->xm);
    delete t;
}

// voff, vlist, fsum (device, nullable: a tree over curved elements keeps none): the gather's vertex
// lists (V + 1 offsets, 3 n slots) and the face-list checksum, copied into the tree; colv: the
// sorted faces' vertex ids, from which the per-block neighbour leaves are listed
int finish_tree(tpe_ctx* ctx, tpe_tree* t, const uint32_t* perm, tpe_tree** out, const uint32_t* voff = nullptr,
                const uint32_t* vlist = nullptr, const uint32_t* fsum = nullptr, const int4* colv = nullptr) {
    hipStream_t st = ctx->stream;
    const int64_t nb = (t->n + 63) / 64;
    auto drop = [&](int code) {
        free_tree(t);
        return code;
    };
    if (hipMalloc(&t->perm, t->n * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&t->work, nb * sizeof(uint32_t)) != hipSuccess ||
        (voff && (hipMalloc(&t->voff, (t->V + 1) * sizeof(uint32_t)) != hipSuccess ||
                  hipMalloc(&t->vlist, 3 * t->n * sizeof(uint32_t)) != hipSuccess ||
                  hipMalloc(&t->fsum, sizeof(uint32_t)) != hipSuccess ||
                  hipMalloc(&t->nbl, block_neighbour_words(t->n) * sizeof(uint32_t)) != hipSuccess ||
                  hipMalloc(&t->xm, block_exclusion_mask_words(t->n) * sizeof(uint2)) != hipSuccess))) {
        (void)hipGetLastError();
        return drop(fail(ctx, TPE_ERR_OOM, "tree allocation failed"));
    }
    hipError_t e = hipMemcpyAsync(t->perm, perm, t->n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && voff)
        e = hipMemcpyAsync(t->voff, voff, (t->V + 1) * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && voff)
        e = hipMemcpyAsync(t->vlist, vlist, 3 * t->n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && voff) e = hipMemcpyAsync(t->fsum, fsum, sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && voff) e = launch_block_neighbours(colv, t->voff, t->vlist, t->n, t->V, t->nbl, t->xm, st);
    if (e == hipSuccess) e = launch_fill(t->work, 0u, nb, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return drop(hip_fail(ctx, e, "tree set-up"));
    int rc;
    if (ctx->sync_checks && (rc = report_flags(ctx))) return drop(rc);
    *out = t;
    return TPE_OK;
}

}  // namespace

extern "C" {

int tpe_version(void) { return 100; }

int tpe_create(tpe_ctx** out, int device, void* hip_stream) {
    if (!out) return TPE_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TPE_ERR_INVALID_ARG;
    tpe_ctx* ctx = new tpe_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    DeviceGuard dg(device);
    if (hipMalloc(&ctx->dflags, 256) != hipSuccess) {
        delete ctx;
        return TPE_ERR_OOM;
    }
    ctx->dstats = reinterpret_cast<unsigned long long*>(ctx->dflags) + 16;  // bytes 128..176 of the same block
    if (hipHostMalloc(&ctx->hflags, sizeof(uint32_t)) != hipSuccess) {
        (void)hipFree(ctx->dflags);
        delete ctx;
        return TPE_ERR_OOM;
    }
    *ctx->hflags = 0;
    noalloc_setup(device);
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu < 1)
            ncu = 1;
        ctx->resident[0] = ncu * pair_blocks_per_cu(false);
        ctx->resident[1] = ncu * pair_blocks_per_cu(true);
        for (int k = 0; k < 4; ++k) {
            ctx->resident_sym[k][0] = ncu * pair_sym_blocks_per_cu(false, 1 << k, false);
            ctx->resident_sym[k][1] = ncu * pair_sym_blocks_per_cu(true, 1 << k, false);
            ctx->resident_symf[k][0] = ncu * pair_sym_blocks_per_cu(false, 1 << k, true);
            ctx->resident_symf[k][1] = ncu * pair_sym_blocks_per_cu(true, 1 << k, true);
        }
    }
    if (launch_fill(ctx->dflags, 0u, 64, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->done) (void)hipEventDestroy(ctx->done);
        if (ctx->join) (void)hipEventDestroy(ctx->join);
        if (ctx->fork) (void)hipEventDestroy(ctx->fork);
        if (ctx->side) (void)hipStreamDestroy(ctx->side);
        (void)hipFree(ctx->dflags);
        (void)hipHostFree(ctx->hflags);
        delete ctx;
        return TPE_ERR_HIP;
    }
    *out = ctx;
    return TPE_OK;
}

int tpe_destroy(tpe_ctx* ctx) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    DeviceGuard dg(ctx->device);
    if (ctx->done_valid) (void)hipEventSynchronize(ctx->done);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamSynchronize(ctx->side);
    if (ctx->arena) (void)hipFree(ctx->arena);
    if (ctx->dflags) (void)hipFree(ctx->dflags);
    if (ctx->hflags) (void)hipHostFree(ctx->hflags);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    (void)hipEventDestroy(ctx->fork);
    (void)hipEventDestroy(ctx->join);
    (void)hipEventDestroy(ctx->done);
    (void)hipStreamDestroy(ctx->side);
    delete ctx;
    return TPE_OK;
}

int tpe_set_stream(tpe_ctx* ctx, void* hip_stream) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return TPE_OK;
}

int tpe_set_option(tpe_ctx* ctx, int option, int64_t value) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    switch (option) {
        case TPE_OPT_SYNC_CHECKS:
            if (value != 0 && value != 1) return fail(ctx, TPE_ERR_INVALID_ARG, "sync checks: 0 or 1");
            ctx->sync_checks = value != 0;
            return TPE_OK;
        case TPE_OPT_TARGET_WAVES:
            if (value < 0 || value > (int64_t)1 << 24) return fail(ctx, TPE_ERR_INVALID_ARG, "target waves");
            ctx->target_waves = value;
            return TPE_OK;
        case TPE_OPT_QUADRATURE:
            if (!quad_rule_ok((int)value) || value != (int)value)
                return fail(ctx, TPE_ERR_INVALID_ARG, "quadrature: 1, 3 or 6 points per face");
            ctx->quad = (int)value;
            return TPE_OK;
        case TPE_OPT_SYMMETRIC:
            if (value != 0 && value != 1) return fail(ctx, TPE_ERR_INVALID_ARG, "symmetric: 0 or 1");
            ctx->symmetric = value != 0;
            return TPE_OK;
        case TPE_OPT_SYM_WAVES:
            if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
                return fail(ctx, TPE_ERR_INVALID_ARG, "symmetric kernel waves: 0, 1, 2, 4 or 8");
            ctx->sym_waves = (int)value;
            return TPE_OK;
        case TPE_OPT_SYM_BARRIERS:
            if (value != 0 && value != 1) return fail(ctx, TPE_ERR_INVALID_ARG, "symmetric barriers: 0 or 1");
            ctx->sym_barriers = value != 0;
            return TPE_OK;
        case TPE_OPT_KERNEL_TIMING:
            if (value < 0 || value > 2) return fail(ctx, TPE_ERR_INVALID_ARG, "kernel timing: 0, 1 or 2");
            ctx->kernel_timing = (int)value;
            return TPE_OK;
        default:
            return fail(ctx, TPE_ERR_INVALID_ARG, "unknown option");
    }
}

const char* tpe_last_error(const tpe_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int tpe_check(tpe_ctx* ctx) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    int rc = report_flags(ctx);
    if (launch_fill(ctx->dflags, 0u, 1, ctx->stream) != hipSuccess) return hip_fail(ctx, hipGetLastError(), "fill");
    return rc;
}

int tpe_energy(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p,
               double scale, double* E_dev) {
    if (ctx && !E_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "null E_dev");
    return run_exact(ctx, X, V, F, nF, q, p, scale, E_dev, nullptr);
}

int tpe_gradient(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF, double q, double p,
                 double scale, double* E_dev, double* G_dev) {
    if (ctx && !G_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "null G_dev");
    if (ctx && (const void*)G_dev == (const void*)X) return fail(ctx, TPE_ERR_INVALID_ARG, "G_dev aliases X");
    return run_exact(ctx, X, V, F, nF, q, p, scale, E_dev, G_dev);
}

int tpe_gradient_noalloc(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF, double q,
                         double p, double scale, double* E_dev, double* G_dev) {
    if (ctx && !G_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "null G_dev");
    if (ctx && (const void*)G_dev == (const void*)X) return fail(ctx, TPE_ERR_INVALID_ARG, "G_dev aliases X");
    return run_exact(ctx, X, V, F, nF, q, p, scale, E_dev, G_dev, false, true);
}

int tpe_sort_pairs(tpe_ctx* ctx, uint32_t* keys, uint32_t* vals, int64_t n, int bits) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (n < 0 || n > ((int64_t)1 << 30) || (n > 0 && (!keys || !vals)))
        return fail(ctx, TPE_ERR_INVALID_ARG, "keys/vals null or n outside [0, 2^30]");
    if (bits < 1 || bits > 32) return fail(ctx, TPE_ERR_INVALID_ARG, "bits must be in [1, 32]");
    if (n <= 1) return TPE_OK;
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    Carve plan_c(nullptr);
    plan_c.take<uint32_t>(n);
    plan_c.take<uint32_t>(n);
    plan_c.take<uint32_t>((size_t)radix_hist_words(n));
    plan_c.take<uint32_t>((size_t)radix_hist_words(n));
    int rc = ensure_arena(ctx, plan_c.off + 256);
    if (rc) return rc;
    Carve c(ctx->arena);
    uint32_t* ktmp = c.take<uint32_t>(n);
    uint32_t* vtmp = c.take<uint32_t>(n);
    uint32_t* hist = c.take<uint32_t>((size_t)radix_hist_words(n));
    uint32_t* hoff = c.take<uint32_t>((size_t)radix_hist_words(n));
    HIPCHK(radix_sort(keys, vals, ktmp, vtmp, n, bits, hist, hoff, ctx->stream));
    if (ctx->sync_checks) HIPCHK(hipStreamSynchronize(ctx->stream));
    return TPE_OK;
}

int tpe_energy_p3(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F10, int64_t nF, double q, double p,
                  double scale, double* E_dev) {
    if (ctx && !E_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "null E_dev");
    return run_exact(ctx, X, V, F10, nF, q, p, scale, E_dev, nullptr, true);
}

int tpe_gradient_p3(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F10, int64_t nF, double q, double p,
                    double scale, double* E_dev, double* G_dev) {
    if (ctx && !G_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "null G_dev");
    if (ctx && (const void*)G_dev == (const void*)X) return fail(ctx, TPE_ERR_INVALID_ARG, "G_dev aliases X");
    return run_exact(ctx, X, V, F10, nF, q, p, scale, E_dev, G_dev, true);
}

int tpe_conf_energy(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF, const double* Y,
                    int64_t VY, const int32_t* FY, int64_t nFY, double q, double p, double scale, double* E_dev) {
    if (ctx && !E_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "null E_dev");
    return run_conf(ctx, X, V, F, nF, Y, VY, FY, nFY, q, p, scale, E_dev, nullptr);
}

int tpe_conf_gradient(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF, const double* Y,
                      int64_t VY, const int32_t* FY, int64_t nFY, double q, double p, double scale, double* E_dev,
                      double* G_dev) {
    if (ctx && !G_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "null G_dev");
    if (ctx && ((const void*)G_dev == (const void*)X || (const void*)G_dev == (const void*)Y))
        return fail(ctx, TPE_ERR_INVALID_ARG, "G_dev aliases an input");
    return run_conf(ctx, X, V, F, nF, Y, VY, FY, nFY, q, p, scale, E_dev, G_dev);
}

int tpe_build_tree(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F, int64_t nF, int32_t leaf_size,
                   tpe_tree** out) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!out) return fail(ctx, TPE_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    int rc = check_common(ctx, X, V, F, nF, 6.0, 12.0);
    if (rc) return rc;
    if (leaf_size < 1 || leaf_size > 4096) return fail(ctx, TPE_ERR_INVALID_ARG, "leaf_size must be in [1, 4096]");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    const int H = tree_height(nF, leaf_size);
    Plan P;
    plan(P, ctx, nF, V, false, H);
    if ((rc = ensure_arena(ctx, P.bytes))) return rc;
    layout(P, ctx->arena, false);
    hipStream_t st = ctx->stream;
    HIPCHK(launch_init(P.zero_begin, P.zero_end - P.zero_begin, P.bbox, ctx->sync_checks ? ctx->dflags : nullptr, st));
    HIPCHK(launch_bbox(X, V, F, 3, nF, P.bbox, ctx->dflags, st));
    HIPCHK(build_kd_order(X, V, F, nF, 0, leaf_size, H, P.cen4, P.nbox, P.vals, P.keys, P.ktmp, P.vtmp, P.hist,
                          P.hoff, st));
    // the gather's vertex lists in tree order, kept with the tree (they depend only on F and the order)
    HIPCHK(launch_records(X, V, F, nF, 1, P.Fp, P.vals, P.bbox, P.org, P.cols, P.colv, P.c64, P.geo, P.cnt,
                          ctx->dflags, st));
    HIPCHK(launch_adjacency(P.colv, nF, V, P.cnt, P.voff, P.cursor, P.list, P.scanws, st));
    tpe_tree* t = new tpe_tree();
    t->device = ctx->device;
    t->nF = nF;
    t->V = V;
    t->leaf = leaf_size;
    t->H = tree_height(nF, leaf_size);
    t->n = nF;
    return finish_tree(ctx, t, P.vals, out, P.voff, P.list, P.bbox + BBOX_FSUM, P.colv);
}

int tpe_build_tree_p3(tpe_ctx* ctx, const double* X, int64_t V, const int32_t* F10, int64_t nF, int32_t leaf_size,
                      tpe_tree** out) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!out) return fail(ctx, TPE_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    int rc = check_common(ctx, X, V, F10, nF, 6.0, 12.0);
    if (rc) return rc;
    if (leaf_size < 1 || leaf_size > 4096) return fail(ctx, TPE_ERR_INVALID_ARG, "leaf_size must be in [1, 4096]");
    const int Q = ctx->quad;
    const int64_t n = nF * Q;
    if (n > (int64_t)1 << 26) return fail(ctx, TPE_ERR_INVALID_ARG, "too many quadrature points (> 2^26)");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    const int H = tree_height(n, leaf_size);
    Plan P;
    plan(P, ctx, nF, V, false, H, 0, 0, Q, false, true);
    if ((rc = ensure_arena(ctx, P.bytes))) return rc;
    layout(P, ctx->arena, false);
    hipStream_t st = ctx->stream;
    HIPCHK(launch_init(P.zero_begin, P.zero_end - P.zero_begin, P.bbox, ctx->sync_checks ? ctx->dflags : nullptr, st));
    HIPCHK(launch_bbox(X, V, F10, P3_NODES, nF, P.bbox, ctx->dflags, st));
    HIPCHK(build_kd_order(X, V, F10, nF, Q, leaf_size, H, P.cen4, P.nbox, P.vals, P.keys, P.ktmp, P.vtmp, P.hist,
                          P.hoff, st));
    tpe_tree* t = new tpe_tree();
    t->device = ctx->device;
    t->nF = nF;
    t->V = V;
    t->leaf = leaf_size;
    t->H = H;
    t->Q = Q;
    t->n = n;
    return finish_tree(ctx, t, P.vals, out);
}

// The far field on curved cubic elements: the tree's items are the quadrature points, so the
// walk, the moments and the near ranges run on point records exactly as on faces, the records'
// vertex ids being the elements' corners; the finalize takes one record per item.
int tpe_farfield_p3(tpe_ctx* ctx, const tpe_tree* tree, const double* X, int64_t V, const int32_t* F10, int64_t nF,
                    double q, double p, double scale, double theta, const tpe_mlp* mlp, double* E_dev,
                    double* G_dev) {
    int rc = check_common(ctx, X, V, F10, nF, q, p);
    if (rc) return rc;
    if (!tree) return fail(ctx, TPE_ERR_INVALID_ARG, "null tree");
    if (tree->Q < 1) return fail(ctx, TPE_ERR_INVALID_ARG, "tree was built over flat faces (tpe_build_tree)");
    if (tree->nF != nF || tree->V != V) return fail(ctx, TPE_ERR_INVALID_ARG, "tree was built for another mesh size");
    if (tree->device != ctx->device) return fail(ctx, TPE_ERR_INVALID_ARG, "tree lives on another device");
    // theta <= 2 keeps every face sharing a vertex with the block out of the far clusters (the radii
    // bound vertices: a shared vertex means |C_T - C_B| - r_T <= r_B); [0, 1] as for the dual tree
    if (!(theta >= 0.0 && theta <= 1.0)) return fail(ctx, TPE_ERR_INVALID_ARG, "theta must be in [0, 1]");
    if (!std::isfinite(scale)) return fail(ctx, TPE_ERR_INVALID_ARG, "scale must be finite");
    if (!E_dev && !G_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "nothing to compute");
    if (G_dev && (const void*)G_dev == (const void*)X) return fail(ctx, TPE_ERR_INVALID_ARG, "G_dev aliases X");
    if (mlp && mlp->device != ctx->device) return fail(ctx, TPE_ERR_INVALID_ARG, "MLP lives on another device");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    const int Q = tree->Q;
    const int64_t n = tree->n;
    Plan P;
    P.ff_leaf = tree->leaf;
    plan(P, ctx, nF, V, true, tree->H, 0, 0, Q, false, true);
    if ((rc = ensure_arena(ctx, P.bytes))) return rc;
    layout(P, ctx->arena, true);
    hipStream_t st = ctx->stream;
    HIPCHK(launch_init(P.zero_begin, P.zero_end - P.zero_begin, P.bbox, ctx->sync_checks ? ctx->dflags : nullptr, st));
    HIPCHK(launch_bbox(X, V, F10, P3_NODES, nF, P.bbox, ctx->dflags, st));
    HIPCHK(launch_p3_records(X, V, F10, nF, Q, P.Fp, tree->perm, P.bbox, P.org, P.cols, P.colv, P.c64, P.geo, P.cnt,
                             ctx->dflags, st));
    HIPCHK(launch_tree_moments(P.c64, P.geo, P.colv, X, P.bbox, n, tree->leaf, tree->H, P.nodes64, P.recs,
                               mlp != nullptr, P.balls, st));
    if (G_dev) {  // the node CSR only serves the gather: built on the side stream during the walk
        HIPCHK(hipEventRecord(ctx->fork, st));
        HIPCHK(hipStreamWaitEvent(ctx->side, ctx->fork, 0));
        HIPCHK(launch_p3_nodes(F10, n, 1, Q, V, tree->perm, P.ncnt, P.noff, P.ncursor, P.nlist, P.scanws,
                               ctx->side));
        HIPCHK(hipEventRecord(ctx->join, ctx->side));
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (ctx->kernel_timing) {
        if ((rc = timing_events(ctx, &ev0, &ev1))) return rc;
    }
    {  // the walk writes all six counts of ctx->dstats; kernel timing 1: events around the evaluation
        uint32_t* const sortbuf[6] = {P.keys, P.vals, P.ktmp, P.vtmp, P.hist, P.hoff};
        const bool t1 = ctx->kernel_timing == 1;
        HIPCHK(launch_farfield(P.cols, P.colv, P.c64, P.org, X, P.bbox, P.recs, tree->H, tree->leaf, n, P.Fp,
                               (float)theta, mlp ? mlp->packed : nullptr, P.balls, P.acc64, ctx->dstats, tree->work,
                               P.ff_ent, P.ff_lst, P.ff_cap, ctx->dflags, sortbuf, nullptr, nullptr,
                               t1 ? ev0 : nullptr, t1 ? ev1 : nullptr, st));
    }
    if (ctx->kernel_timing == 2) HIPCHK(hipEventRecord(ev0, st));
    EnergyOut en = {};  // with the gradient, the energy is summed by the gather's extra work-group
    HIPCHK(launch_p3_finalize(true, nullptr, P.sc, P.Fp, n, 1, Q, P.acc64, tree->perm, F10, V, X, P.bbox, q, p, scale,
                              0.5, P.corner, P.epart, ctx->dflags, E_dev, G_dev ? &en : nullptr, st));
    if (G_dev) {
        HIPCHK(hipStreamWaitEvent(st, ctx->join, 0));
        HIPCHK(launch_gather(P.noff, P.nlist, V, P.corner, G_dev, en, st));
    }
    if (ctx->kernel_timing == 2) HIPCHK(hipEventRecord(ev1, st));
    if (ctx->sync_checks) return report_flags(ctx);
    return TPE_OK;
}

int tpe_tree_order(tpe_ctx* ctx, const tpe_tree* tree, uint32_t* perm_dev, int64_t n) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!tree || !perm_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "null tree or output");
    if (n != tree->n) return fail(ctx, TPE_ERR_INVALID_ARG, "n must be the tree's item count");
    if (tree->device != ctx->device) return fail(ctx, TPE_ERR_INVALID_ARG, "tree lives on another device");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    HIPCHK(hipMemcpyAsync(perm_dev, tree->perm, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx->stream));
    if (ctx->sync_checks) HIPCHK(hipStreamSynchronize(ctx->stream));
    return TPE_OK;
}

int tpe_tree_destroy(tpe_tree* t) {
    if (!t) return TPE_ERR_INVALID_ARG;
    DeviceGuard dg(t->device);
    free_tree(t);
    return TPE_OK;
}

int tpe_farfield(tpe_ctx* ctx, const tpe_tree* tree, const double* X, int64_t V, const int32_t* F, int64_t nF,
                 double q, double p, double scale, double theta, const tpe_mlp* mlp, double* E_dev, double* G_dev) {
    int rc = check_common(ctx, X, V, F, nF, q, p);
    if (rc) return rc;
    if (!tree) return fail(ctx, TPE_ERR_INVALID_ARG, "null tree");
    if (tree->nF != nF || tree->V != V) return fail(ctx, TPE_ERR_INVALID_ARG, "tree was built for another mesh size");
    if (tree->Q != 0) return fail(ctx, TPE_ERR_INVALID_ARG, "tree was built over curved elements");
    if (tree->device != ctx->device) return fail(ctx, TPE_ERR_INVALID_ARG, "tree lives on another device");
    // theta <= 2 keeps every face sharing a vertex with the block out of the far clusters (the radii
    // bound vertices: a shared vertex means |C_T - C_B| - r_T <= r_B); [0, 1] as for the dual tree
    if (!(theta >= 0.0 && theta <= 1.0)) return fail(ctx, TPE_ERR_INVALID_ARG, "theta must be in [0, 1]");
    if (!std::isfinite(scale)) return fail(ctx, TPE_ERR_INVALID_ARG, "scale must be finite");
    if (!E_dev && !G_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "nothing to compute");
    if (G_dev && (const void*)G_dev == (const void*)X) return fail(ctx, TPE_ERR_INVALID_ARG, "G_dev aliases X");
    if (mlp && mlp->device != ctx->device) return fail(ctx, TPE_ERR_INVALID_ARG, "MLP lives on another device");
    if (ctx->quad != 1) return fail(ctx, TPE_ERR_UNSUPPORTED, "the far field uses one point per face");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    Plan P;
    P.ff_leaf = tree->leaf;
    plan(P, ctx, nF, V, true, tree->H);
    if ((rc = ensure_arena(ctx, P.bytes))) return rc;
    layout(P, ctx->arena, true);
    hipStream_t st = ctx->stream;
    HIPCHK(launch_init(P.zero_begin, P.zero_end - P.zero_begin, P.bbox, ctx->sync_checks ? ctx->dflags : nullptr, st));
    // the face list must be the tree's (its gather lists are kept with the tree)
    HIPCHK(launch_bbox(X, V, F, 3, nF, P.bbox, ctx->dflags, st, tree->fsum));
    HIPCHK(launch_records(X, V, F, nF, 1, P.Fp, tree->perm, P.bbox, P.org, P.cols, P.colv, P.c64, P.geo, nullptr,
                          ctx->dflags, st));
    HIPCHK(launch_tree_moments(P.c64, P.geo, P.colv, X, P.bbox, nF, tree->leaf, tree->H, P.nodes64, P.recs,
                               mlp != nullptr, P.balls, st));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (ctx->kernel_timing) {
        if ((rc = timing_events(ctx, &ev0, &ev1))) return rc;
    }
    {  // the walk writes all six counts of ctx->dstats; kernel timing 1: events around the evaluation
        uint32_t* const sortbuf[6] = {P.keys, P.vals, P.ktmp, P.vtmp, P.hist, P.hoff};
        const bool t1 = ctx->kernel_timing == 1;
        HIPCHK(launch_farfield(P.cols, P.colv, P.c64, P.org, X, P.bbox, P.recs, tree->H, tree->leaf, nF, P.Fp,
                               (float)theta, mlp ? mlp->packed : nullptr, P.balls, P.acc64, ctx->dstats, tree->work,
                               P.ff_ent, P.ff_lst, P.ff_cap, ctx->dflags, sortbuf, tree->nbl, tree->xm,
                               t1 ? ev0 : nullptr, t1 ? ev1 : nullptr, st));
    }
    if (ctx->kernel_timing == 2) HIPCHK(hipEventRecord(ev0, st));
    EnergyOut en = {};  // with the gradient, the energy is summed by the gather's extra work-group
    HIPCHK(launch_finalize(true, nullptr, P.sc, P.Fp, nF, P.acc64, P.geo, P.colv, X, P.bbox, q, p, scale, 0.5, 1,
                           P.corner, P.epart, ctx->dflags, E_dev, G_dev ? &en : nullptr, st));
    if (G_dev) HIPCHK(launch_gather(tree->voff, tree->vlist, V, P.corner, G_dev, en, st));
    if (ctx->kernel_timing == 2) HIPCHK(hipEventRecord(ev1, st));
    if (ctx->sync_checks) return report_flags(ctx);
    return TPE_OK;
}

int tpe_farfield_dual(tpe_ctx* ctx, const tpe_tree* tree, const double* X, int64_t V, const int32_t* F, int64_t nF,
                      double q, double p, double scale, double theta, double* E_dev, double* G_dev) {
    int rc = check_common(ctx, X, V, F, nF, q, p);
    if (rc) return rc;
    if (!tree) return fail(ctx, TPE_ERR_INVALID_ARG, "null tree");
    if (tree->nF != nF || tree->V != V) return fail(ctx, TPE_ERR_INVALID_ARG, "tree was built for another mesh size");
    if (tree->Q != 0) return fail(ctx, TPE_ERR_INVALID_ARG, "tree was built over curved elements");
    if (tree->device != ctx->device) return fail(ctx, TPE_ERR_INVALID_ARG, "tree lives on another device");
    if (tree->leaf > 64 || (64 % tree->leaf) != 0)
        return fail(ctx, TPE_ERR_UNSUPPORTED, "the dual-tree far field needs a leaf size dividing 64");
    if (!(theta >= 0.0 && theta <= 1.0)) return fail(ctx, TPE_ERR_INVALID_ARG, "theta must be in [0, 1]");
    if (!std::isfinite(scale)) return fail(ctx, TPE_ERR_INVALID_ARG, "scale must be finite");
    if (!E_dev && !G_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "nothing to compute");
    if (G_dev && (const void*)G_dev == (const void*)X) return fail(ctx, TPE_ERR_INVALID_ARG, "G_dev aliases X");
    if (ctx->quad != 1) return fail(ctx, TPE_ERR_UNSUPPORTED, "the far field uses one point per face");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    Plan P;
    P.dual_leaf = tree->leaf;
    plan(P, ctx, nF, V, true, tree->H);
    if ((rc = ensure_arena(ctx, P.bytes))) return rc;
    layout(P, ctx->arena, true);
    hipStream_t st = ctx->stream;
    HIPCHK(launch_init(P.zero_begin, P.zero_end - P.zero_begin, P.bbox, ctx->sync_checks ? ctx->dflags : nullptr, st));
    // the face list must be the tree's (its gather lists are kept with the tree)
    HIPCHK(launch_bbox(X, V, F, 3, nF, P.bbox, ctx->dflags, st, tree->fsum));
    HIPCHK(launch_records(X, V, F, nF, 1, P.Fp, tree->perm, P.bbox, P.org, P.cols, P.colv, P.c64, P.geo, nullptr,
                          ctx->dflags, st));
    HIPCHK(launch_tree_moments(P.c64, P.geo, P.colv, X, P.bbox, nF, tree->leaf, tree->H, P.nodes64, P.recs, false,
                               nullptr, st));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (ctx->kernel_timing) {
        if ((rc = timing_events(ctx, &ev0, &ev1))) return rc;
    }
    if (ctx->kernel_timing == 1) HIPCHK(hipEventRecord(ev0, st));
    HIPCHK(launch_fill(reinterpret_cast<uint32_t*>(ctx->dstats), 0u, 12, st));
    uint32_t* const sortbuf[6] = {P.keys, P.vals, P.ktmp, P.vtmp, P.hist, P.hoff};
    HIPCHK(launch_dual(tree->H, tree->leaf, (float)theta, P.cols, P.colv, P.c64, P.geo, P.org, P.nodes64, P.recs, nF,
                       P.Fp, q, p, P.doff, P.dnear, P.dfar, P.dcnt, P.drel, P.dent, P.dscan, P.dadj, P.dpart, P.acc64,
                       ctx->dflags, ctx->dstats, sortbuf, st));
    if (ctx->kernel_timing == 1) HIPCHK(hipEventRecord(ev1, st));
    if (ctx->kernel_timing == 2) HIPCHK(hipEventRecord(ev0, st));
    EnergyOut en = {};  // with the gradient, the energy is summed by the gather's extra work-group
    HIPCHK(launch_finalize(true, nullptr, P.sc, P.Fp, nF, P.acc64, P.geo, P.colv, X, P.bbox, q, p, scale, 0.5, 1,
                           P.corner, P.epart, ctx->dflags, E_dev, G_dev ? &en : nullptr, st));
    if (G_dev) HIPCHK(launch_gather(tree->voff, tree->vlist, V, P.corner, G_dev, en, st));
    if (ctx->kernel_timing == 2) HIPCHK(hipEventRecord(ev1, st));
    if (ctx->sync_checks) return report_flags(ctx);
    return TPE_OK;
}

int tpe_farfield_samples(tpe_ctx* ctx, const tpe_tree* tree, const double* X, int64_t V, const int32_t* F, int64_t nF,
                         double theta, uint64_t seed, double select_prob, int32_t quota, int64_t max_cluster_faces,
                         const tpe_mlp* mlp, float* feats, float* targets, float* pred) {
    int rc = check_common(ctx, X, V, F, nF, 6.0, 12.0);
    if (rc) return rc;
    if (!tree || tree->nF != nF || tree->V != V || tree->Q != 0)
        return fail(ctx, TPE_ERR_INVALID_ARG, "tree/mesh mismatch");
    if (!feats || !targets) return fail(ctx, TPE_ERR_INVALID_ARG, "null output");
    if ((mlp == nullptr) != (pred == nullptr)) return fail(ctx, TPE_ERR_INVALID_ARG, "mlp and pred go together");
    if (!(theta > 0.0 && theta <= 1.0) || !(select_prob >= 0.0 && select_prob <= 1.0) || quota < 1 || quota > 1024 ||
        max_cluster_faces < 1)
        return fail(ctx, TPE_ERR_INVALID_ARG, "bad sampling parameters");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    Plan P;
    plan(P, ctx, nF, V, true, tree->H);
    if ((rc = ensure_arena(ctx, P.bytes))) return rc;
    layout(P, ctx->arena, true);
    hipStream_t st = ctx->stream;
    HIPCHK(launch_init(P.zero_begin, P.zero_end - P.zero_begin, P.bbox, ctx->sync_checks ? ctx->dflags : nullptr, st));
    HIPCHK(launch_bbox(X, V, F, 3, nF, P.bbox, ctx->dflags, st, tree->fsum));
    HIPCHK(launch_records(X, V, F, nF, 1, P.Fp, tree->perm, P.bbox, P.org, P.cols, P.colv, P.c64, P.geo, nullptr,
                          ctx->dflags, st));
    HIPCHK(launch_tree_moments(P.c64, P.geo, P.colv, X, P.bbox, nF, tree->leaf, tree->H, P.nodes64, P.recs, true,
                               nullptr, st));
    const uint32_t sel = select_prob >= 1.0 ? 0xffffffffu : (uint32_t)(select_prob * 4294967296.0);
    HIPCHK(launch_farfield_samples(P.cols, P.colv, P.c64, X, P.bbox, P.recs, tree->H, tree->leaf, nF, (float)theta,
                                   (uint32_t)(seed ^ (seed >> 32)), sel, quota, max_cluster_faces, P.balls, feats,
                                   targets, mlp ? mlp->packed : nullptr, pred, st));
    if (ctx->sync_checks) return report_flags(ctx);
    return TPE_OK;
}

int tpe_farfield_stats(tpe_ctx* ctx, int64_t* out_host) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!out_host) return fail(ctx, TPE_ERR_INVALID_ARG, "null output");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    unsigned long long h[6] = {0, 0, 0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(h, ctx->dstats, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < 6; ++i) out_host[i] = (int64_t)h[i];
    return TPE_OK;
}

// ---- learned far-field correction: MLP ------------------------------------------------------------

static int mlp_alloc_parts(tpe_ctx* ctx, tpe_mlp* m, int64_t ntiles) {
    if (ntiles <= m->cap_tiles) return TPE_OK;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (m->gpart) (void)hipFree(m->gpart);
    if (m->lpart) (void)hipFree(m->lpart);
    m->gpart = m->lpart = nullptr;
    m->cap_tiles = 0;
    if (hipMalloc(&m->gpart, (size_t)ntiles * MLP_NPARAM * sizeof(float)) != hipSuccess ||
        hipMalloc(&m->lpart, (size_t)ntiles * 2 * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, TPE_ERR_OOM, "MLP gradient partials");
    }
    m->cap_tiles = ntiles;
    return TPE_OK;
}

int tpe_mlp_create(tpe_ctx* ctx, int32_t d_in, int32_t width, int32_t depth, int32_t d_out, uint64_t seed,
                   tpe_mlp** out) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!out) return fail(ctx, TPE_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    if (d_in != MLP_DIN || width != MLP_W || depth != MLP_DEPTH || d_out != MLP_DOUT)
        return fail(ctx, TPE_ERR_UNSUPPORTED, "only the 32-64-64-64-16 network is implemented");
    DeviceGuard dg(ctx->device);
    tpe_mlp* m = new tpe_mlp();
    m->device = ctx->device;
    const size_t bytes = MLP_NPARAM * sizeof(float);
    if (hipMalloc(&m->P, bytes) != hipSuccess || hipMalloc(&m->M, bytes) != hipSuccess ||
        hipMalloc(&m->V, bytes) != hipSuccess || hipMalloc(&m->packed, mlp_packed_bytes()) != hipSuccess) {
        (void)hipGetLastError();
        tpe_mlp_destroy(m);
        return fail(ctx, TPE_ERR_OOM, "MLP parameters");
    }
    std::vector<float> P;
    mlp_init_params(seed, P);
    std::vector<float> z(MLP_NPARAM, 0.f);
    hipError_t e = hipMemcpy(m->P, P.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->M, z.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->V, z.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = mlp_pack_launch(m->P, m->min_s, m->packed, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        tpe_mlp_destroy(m);
        return hip_fail(ctx, e, "MLP init copy");
    }
    *out = m;
    return TPE_OK;
}

int tpe_mlp_destroy(tpe_mlp* m) {
    if (!m) return TPE_ERR_INVALID_ARG;
    DeviceGuard dg(m->device);
    for (float* p : {m->P, m->M, m->V, m->gpart, m->lpart})
        if (p) (void)hipFree(p);
    if (m->packed) (void)hipFree(m->packed);
    delete m;
    return TPE_OK;
}

int64_t tpe_mlp_num_params(const tpe_mlp* m) { return m ? MLP_NPARAM : -1; }

int tpe_mlp_get_params(tpe_ctx* ctx, const tpe_mlp* m, float* host, int64_t n) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!m || !host || n != MLP_NPARAM) return fail(ctx, TPE_ERR_INVALID_ARG, "bad MLP parameter buffer");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    HIPCHK(hipMemcpyAsync(host, m->P, n * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return TPE_OK;
}

int tpe_mlp_set_params(tpe_ctx* ctx, tpe_mlp* m, const float* host, int64_t n) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!m || !host || n != MLP_NPARAM) return fail(ctx, TPE_ERR_INVALID_ARG, "bad MLP parameter buffer");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    HIPCHK(hipMemcpyAsync(m->P, host, n * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(mlp_pack_launch(m->P, m->min_s, m->packed, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return TPE_OK;
}

int tpe_mlp_set_smoothness(tpe_ctx* ctx, tpe_mlp* m, float lam) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!m || !(lam >= 0.f) || !std::isfinite(lam)) return fail(ctx, TPE_ERR_INVALID_ARG, "bad smoothness weight");
    m->lam = lam;
    return TPE_OK;
}

int tpe_mlp_get_gate(tpe_ctx* ctx, const tpe_mlp* m, float* min_s) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!m || !min_s) return fail(ctx, TPE_ERR_INVALID_ARG, "bad gate arguments");
    *min_s = m->min_s;
    return TPE_OK;
}

int tpe_mlp_set_gate(tpe_ctx* ctx, tpe_mlp* m, float min_s) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!m || !(min_s >= 0.f) || !std::isfinite(min_s)) return fail(ctx, TPE_ERR_INVALID_ARG, "bad gate");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    m->min_s = min_s;
    HIPCHK(mlp_pack_launch(m->P, m->min_s, m->packed, ctx->stream));
    return TPE_OK;
}

int tpe_mlp_forward(tpe_ctx* ctx, const tpe_mlp* m, const float* feats, int64_t n, float* out) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!m || !feats || !out || n < 0) return fail(ctx, TPE_ERR_INVALID_ARG, "bad MLP forward arguments");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    HIPCHK(mlp_infer_launch(m->packed, feats, n, out, ctx->stream));
    return TPE_OK;
}

static int mlp_step(tpe_ctx* ctx, tpe_mlp* m, const float* feats, const float* targets, int64_t n, float lr,
                    float* loss_dev, float* grad_dev) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!m || !feats || !targets || n < 1) return fail(ctx, TPE_ERR_INVALID_ARG, "bad MLP training arguments");
    if (!grad_dev && !(lr > 0.f && std::isfinite(lr))) return fail(ctx, TPE_ERR_INVALID_ARG, "lr must be > 0");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    int rc = mlp_alloc_parts(ctx, m, mlp_tiles(n));
    if (rc) return rc;
    if (!grad_dev) ++m->step;
    HIPCHK(mlp_train_launch(m->P, m->M, m->V, feats, targets, n, lr, m->lam, m->step, m->gpart, m->lpart, loss_dev,
                            grad_dev, ctx->stream));
    if (!grad_dev) HIPCHK(mlp_pack_launch(m->P, m->min_s, m->packed, ctx->stream));
    return TPE_OK;
}

int tpe_mlp_train_step(tpe_ctx* ctx, tpe_mlp* m, const float* feats, const float* targets, int64_t n, float lr,
                       float* loss_dev) {
    return mlp_step(ctx, m, feats, targets, n, lr, loss_dev, nullptr);
}

int tpe_mlp_gradient(tpe_ctx* ctx, tpe_mlp* m, const float* feats, const float* targets, int64_t n,
                     float* grad_dev) {
    if (ctx && !grad_dev) return fail(ctx, TPE_ERR_INVALID_ARG, "null gradient output");
    return mlp_step(ctx, m, feats, targets, n, 0.f, nullptr, grad_dev);
}

static const char MLP_MAGIC[8] = {'T', 'P', 'E', 'M', 'L', 'P', '0', '2'};
static const char MLP_MAGIC_V1[8] = {'T', 'P', 'E', 'M', 'L', 'P', '0', '1'};  // no gate (read as 0)

int tpe_mlp_save(tpe_ctx* ctx, const tpe_mlp* m, const char* path) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!m || !path) return fail(ctx, TPE_ERR_INVALID_ARG, "bad save arguments");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    std::vector<float> buf(3 * (size_t)MLP_NPARAM);
    HIPCHK(hipMemcpyAsync(buf.data(), m->P, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(buf.data() + MLP_NPARAM, m->M, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipMemcpyAsync(buf.data() + 2 * MLP_NPARAM, m->V, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    FILE* f = fopen(path, "wb");
    if (!f) return fail(ctx, TPE_ERR_INVALID_ARG, std::string("cannot open ") + path);
    const int32_t dims[4] = {MLP_DIN, MLP_W, MLP_DEPTH, MLP_DOUT};
    const int64_t step = m->step;
    const float gate[2] = {m->min_s, 0.f};
    bool ok = fwrite(MLP_MAGIC, 1, 8, f) == 8 && fwrite(dims, sizeof(dims), 1, f) == 1 &&
              fwrite(&step, sizeof(step), 1, f) == 1 && fwrite(gate, sizeof(gate), 1, f) == 1 &&
              fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? TPE_OK : fail(ctx, TPE_ERR_INVALID_ARG, std::string("write failed: ") + path);
}

int tpe_mlp_load(tpe_ctx* ctx, const char* path, tpe_mlp** out) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!path || !out) return fail(ctx, TPE_ERR_INVALID_ARG, "bad load arguments");
    *out = nullptr;
    FILE* f = fopen(path, "rb");
    if (!f) return fail(ctx, TPE_ERR_INVALID_ARG, std::string("cannot open ") + path);
    char magic[8];
    int32_t dims[4];
    int64_t step = 0;
    std::vector<float> buf(3 * (size_t)MLP_NPARAM);
    float gate[2] = {0.f, 0.f};
    bool ok = fread(magic, 1, 8, f) == 8;
    const bool v2 = ok && memcmp(magic, MLP_MAGIC, 8) == 0;
    ok = ok && (v2 || memcmp(magic, MLP_MAGIC_V1, 8) == 0) && fread(dims, sizeof(dims), 1, f) == 1 &&
         dims[0] == MLP_DIN && dims[1] == MLP_W && dims[2] == MLP_DEPTH && dims[3] == MLP_DOUT &&
         fread(&step, sizeof(step), 1, f) == 1 && (!v2 || fread(gate, sizeof(gate), 1, f) == 1) &&
         fread(buf.data(), sizeof(float), buf.size(), f) == buf.size() && gate[0] >= 0.f && std::isfinite(gate[0]);
    fclose(f);
    if (!ok) return fail(ctx, TPE_ERR_INVALID_ARG, std::string("not a valid MLP checkpoint: ") + path);
    tpe_mlp* m = nullptr;
    int rc = tpe_mlp_create(ctx, MLP_DIN, MLP_W, MLP_DEPTH, MLP_DOUT, 0, &m);
    if (rc) return rc;
    m->min_s = gate[0];
    DeviceGuard dg(ctx->device);
    hipError_t e = hipMemcpy(m->P, buf.data(), MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(m->M, buf.data() + MLP_NPARAM, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(m->V, buf.data() + 2 * MLP_NPARAM, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = mlp_pack_launch(m->P, m->min_s, m->packed, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        tpe_mlp_destroy(m);
        return hip_fail(ctx, e, "MLP load copy");
    }
    m->step = step;
    *out = m;
    return TPE_OK;
}

int tpe_kernel_time(tpe_ctx* ctx, double* total_ms, int64_t* count) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!total_ms || !count) return fail(ctx, TPE_ERR_INVALID_ARG, "null output");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double tot = 0.0;
    for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev_pool[i], ctx->ev_pool[i + 1]));
        tot += ms;
    }
    *total_ms = tot;
    *count = (int64_t)(ctx->ev_used / 2);
    ctx->ev_used = 0;
    return TPE_OK;
}

int tpe_exact_plan(tpe_ctx* ctx, int64_t nF, int64_t V, int32_t grad, int64_t* out_host) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!out_host || nF < 1 || V < 1 || (grad != 0 && grad != 1))
        return fail(ctx, TPE_ERR_INVALID_ARG, "bad arguments");
    Plan P;
    plan(P, ctx, nF, V, grad != 0, -1, 0, 0, ctx->quad, ctx->symmetric, false);
    out_host[0] = P.sym ? (P.sym_free ? 2 : 1) : 0;
    out_host[1] = P.sym ? P.ssc.nw : 0;
    out_host[2] = P.sym ? sym_colpart_floats(P.ssc, grad != 0) * (int64_t)sizeof(float) : 0;
    out_host[3] = (int64_t)P.bytes;
    return TPE_OK;
}

int tpe_pair_count(tpe_ctx* ctx, const int32_t* F, int64_t nF, int64_t V, int64_t* out_host) {
    if (!ctx) return TPE_ERR_INVALID_ARG;
    if (!F || !out_host || nF < 1 || V < 1) return fail(ctx, TPE_ERR_INVALID_ARG, "bad arguments");
    DeviceGuard dg(ctx->device);
    ORDERED(ctx);
    Plan P;
    plan(P, ctx, nF, V, false);
    int rc = ensure_arena(ctx, P.bytes);
    if (rc) return rc;
    layout(P, ctx->arena, false);
    hipStream_t st = ctx->stream;
    // sorted order is irrelevant for counting: use the identity permutation
    HIPCHK(launch_init(P.zero_begin, P.zero_end - P.zero_begin, P.bbox, ctx->dflags, st));
    HIPCHK(launch_fill(reinterpret_cast<uint32_t*>(P.counter), 0u, 2, st));
    hipLaunchKernelGGL(face_ids, dim3((int)ceil_div(nF, 256)), dim3(256), 0, st, F, nF, V, P.colv, P.cnt, ctx->dflags);
    HIPCHK(hipGetLastError());
    HIPCHK(launch_adjacency(P.colv, nF, V, P.cnt, P.voff, P.cursor, P.list, P.scanws, st));
    hipLaunchKernelGGL(excluded_count, dim3((int)ceil_div(nF, 256)), dim3(256), 0, st, P.colv, nF, V, P.voff, P.list,
                       P.counter);
    HIPCHK(hipGetLastError());
    unsigned long long h = 0;
    HIPCHK(hipMemcpyAsync(&h, P.counter, sizeof(h), hipMemcpyDeviceToHost, st));
    if ((rc = report_flags(ctx))) return rc;
    *out_host = nF * nF - (int64_t)h;
    return TPE_OK;
}

}  // extern "C"
