// Octree build on the GPU (Sec. 4.1 and App. A of Klepitko et al. 2023).
//
// Topology: every node is an ancestor-or-self of a leaf cell.  For each depth d the
// node set is a subset of the dense Morton range [0, 8^d); one u32 occupancy word per
// dense slot (bit0 exists, bit1 leaf, bits 8..15 child mask) is filled bottom-up and a
// single exclusive scan over the concatenated slots of all depths numbers the nodes
// depth-major and in Morton order inside a depth, so the children of a node are
// consecutive.  Content: leaves first (FP64 arithmetic, FP32 storage), then the upward
// pass depth by depth, summing children in Morton order in FP64 so that the stored
// FP32 fields are reproducible bit for bit.
#include <hipcub/hipcub.hpp>

#include "common.hpp"

namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    // bit k of v -> bit 3k
    uint32_t x = v & 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}
__device__ __forceinline__ uint32_t compact3(uint32_t x) {
    x &= 0x09249249u;
    x = (x | (x >> 2)) & 0x030c30c3u;
    x = (x | (x >> 4)) & 0x0300f00fu;
    x = (x | (x >> 8)) & 0x030000ffu;
    x = (x | (x >> 16)) & 0x000003ffu;
    return x;
}
__device__ __forceinline__ uint32_t morton(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

struct DenseLayout {
    int64_t base[TR_MAX_DEPTH + 2]; // first dense slot of each depth
};

__global__ void k_mark_leaves(const int4 *__restrict__ blocks, int64_t n_cells, int D,
                              int max_level, DenseLayout L, uint32_t *__restrict__ occ,
                              int *__restrict__ err) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    int4 b = blocks[c >> 9];
    int lc = (int)(c & 511);
    int dc = D - (max_level - b.x);
    uint32_t m = morton((uint32_t)(b.y * 8 + (lc & 7)), (uint32_t)(b.z * 8 + ((lc >> 3) & 7)),
                        (uint32_t)(b.w * 8 + (lc >> 6)));
    uint32_t old = atomicOr(&occ[L.base[dc] + m], 3u);
    if (old & 2u) atomicOr(err, 1); // two blocks claim the same cell
}

__global__ void k_exist(int d, DenseLayout L, uint32_t *__restrict__ occ, int *__restrict__ err) {
    int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= ((int64_t)1 << (3 * d))) return;
    const uint32_t *ch = occ + L.base[d + 1] + 8 * m;
    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) mask |= (ch[k] != 0u ? 1u : 0u) << k;
    uint32_t v = occ[L.base[d] + m];
    if ((v & 2u) && mask) atomicOr(err, 2); // a leaf cell inside a refined region
    if (mask) v |= 1u | (mask << 8);
    occ[L.base[d] + m] = v;
}

// Optional input check (tr_ctx_set_validation): a density, opacity or dust temperature that
// is not a finite number >= 0 sets bit 8, 9 or 10 of the build's error word.
__global__ void k_validate_cells(int64_t n, const float *__restrict__ rho, const float *__restrict__ kappa,
                                 const float *__restrict__ t_dust, int *__restrict__ err) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    auto bad = [](float v) { return !(v >= 0.0f && v <= 3.402823466e38f); }; // NaN fails both
    int e = bad(rho[c]) ? 256 : 0;
    if (kappa && bad(kappa[c])) e |= 512;
    if (bad(t_dust[c])) e |= 1024;
    if (e) atomicOr(err, e);
}

struct ExistsOp {
    __device__ int operator()(uint32_t v) const { return v != 0u ? 1 : 0; }
};
struct LeafOp {
    __device__ int operator()(uint32_t v) const { return (v & 2u) ? 1 : 0; }
};

__global__ void k_nodes(int D, int64_t root_edge, DenseLayout L, const uint32_t *__restrict__ occ,
                        const int *__restrict__ ids, const int *__restrict__ leaf_rank,
                        int4 *__restrict__ geo, uint32_t *__restrict__ meta,
                        int4 *__restrict__ pcol, int32_t *__restrict__ targets) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= L.base[D + 1]) return;
    uint32_t v = occ[e];
    if (!v) return;
    int d = 0;
    while (e >= L.base[d + 1]) ++d;
    uint32_t m = (uint32_t)(e - L.base[d]);
    int id = ids[e];
    int s = (int)(root_edge >> d);
    int gx = (int)compact3(m) * s + s / 2, gy = (int)compact3(m >> 1) * s + s / 2,
        gz = (int)compact3(m >> 2) * s + s / 2;
    uint32_t mask = (v >> 8) & 255u;
    int first = -1;
    if (mask) first = ids[L.base[d + 1] + 8 * (int64_t)m + __builtin_ctz(mask)];
    geo[id] = make_int4(gx, gy, gz, first);
    meta[id] = (uint32_t)d | (mask << 4) | ((v & 2u) ? (1u << 12) : 0u);
    pcol[id] = make_int4(gx * TR_FX, gy * TR_FX, gz * TR_FX, 0);
    if (v & 2u) targets[leaf_rank[e]] = id;
}

__global__ void k_cells(const int4 *__restrict__ blocks, int64_t n_cells, int D, int max_level,
                        DenseLayout L, const int *__restrict__ ids, int32_t *__restrict__ node_of_cell,
                        int32_t *__restrict__ leaf_cell) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    int4 b = blocks[c >> 9];
    int lc = (int)(c & 511);
    int dc = D - (max_level - b.x);
    uint32_t m = morton((uint32_t)(b.y * 8 + (lc & 7)), (uint32_t)(b.z * 8 + ((lc >> 3) & 7)),
                        (uint32_t)(b.w * 8 + (lc >> 6)));
    int id = ids[L.base[dc] + m];
    node_of_cell[c] = id;
    leaf_cell[id] = (int32_t)c;
}

// Stars in input order, one thread: the per-cell sum then has a fixed order.  A star's host
// cell is the leaf holding its fine cell floor((x - x0) / dx_min) (half-open, clamped to the
// grid), found by descending from the root: at each node the octant of the fine cell's
// centre 2 f + 1 (in u) against the node's centre, then that child among the existing ones.
__global__ void k_stars(const double *__restrict__ stars, int n_star, int64_t n_fine, double x0,
                        double y0, double z0, double dxmin, double u2, const int4 *__restrict__ geo,
                        const uint32_t *__restrict__ meta, const int32_t *__restrict__ leaf_cell,
                        double *__restrict__ src) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int s = 0; s < n_star; ++s) {
        // (x, y, z, L) read as four doubles: a caller's array needs only 8-byte alignment
        const double *st = stars + 4 * (int64_t)s;
        double pos[3] = {st[0] - x0, st[1] - y0, st[2] - z0};
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            double q = floor(pos[a] / dxmin);
            if (q < 0) q = 0;
            if (q > (double)(n_fine - 1)) q = (double)(n_fine - 1);
            c[a] = 2 * (int64_t)q + 1;
        }
        int id = 0;
        for (;;) {
            const uint32_t m = meta[id];
            if (m & (1u << 12)) {
                const int cell = leaf_cell[id];
                src[cell] = src[cell] + st[3] / u2;
                break;
            }
            const int4 g = geo[id];
            const uint32_t k = (c[0] > g.x ? 1u : 0u) | (c[1] > g.y ? 2u : 0u) | (c[2] > g.z ? 4u : 0u);
            const uint32_t mask = (m >> 4) & 255u;
            if (!((mask >> k) & 1u)) break; // no such child: the grid does not cover the star
            id = g.w + __builtin_popcount(mask & ((1u << k) - 1u));
        }
    }
}

__global__ void k_zero_f64(double *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

struct Scratch64 {
    double *Lt, *LVk, *At, *Ak, *Vk, *xi;
};

// b-nodes (Sec. 4.1.1).  Same FP64 operation sequence as the definition the tests hold
// the library to; lattice units (lengths in u, luminosities per u_len^2).
__global__ void k_leaf_fill(int64_t n_cells, const float *__restrict__ rho,
                            const float *__restrict__ kappa, const float *__restrict__ t_dust,
                            const double *__restrict__ src, const int32_t *__restrict__ node_of_cell,
                            uint32_t *__restrict__ meta, int64_t root_edge, double u_len,
                            double sigma, Scratch64 S64, float4 *__restrict__ q,
                            float *__restrict__ vthick, float *__restrict__ cell_tau,
                            float *__restrict__ cell_kappa, float *__restrict__ cell_src) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    int id = node_of_cell[c];
    int d = (int)(meta[id] & 15u);
    double e = (double)(root_edge >> d);
    double tt = (double)t_dust[c];
    double kap = kappa ? (double)kappa[c] : (tt < 150.0 ? 1.0e-3 * (tt * tt) : 22.5);
    double rk = (double)rho[c] * kap;
    double tau = rk * (e * u_len);
    double V = e * e * e;
    double A = (rk * u_len) * V;
    double sT4 = sigma * ((tt * tt) * (tt * tt));
    double lsrc = src[c];
    double Sv = lsrc * exp(-0.5 * tau);
    float4 o;
    if (tau < 1.0) {
        double L = (4.0 * sT4) * A;
        S64.Lt[id] = L + Sv;
        S64.LVk[id] = 0.0;
        S64.At[id] = A;
        S64.Ak[id] = 0.0;
        S64.Vk[id] = 0.0;
        S64.xi[id] = L + Sv;
        o.x = (float)L;
    } else {
        double La = sT4 / kPi;
        S64.Lt[id] = Sv;
        S64.LVk[id] = La * V;
        S64.At[id] = 0.0;
        S64.Ak[id] = A;
        S64.Vk[id] = V;
        S64.xi[id] = La * (e * e) + Sv;
        o.x = copysignf((float)La, -1.0f);
    }
    meta[id] = (meta[id] & ~(1u << 13)) | (tau < 1.0 ? 0u : 1u << 13); // thick content
    o.y = (float)A;
    o.z = (float)Sv;
    o.w = 0.0f;
    q[id] = o;
    vthick[id] = 0.0f;
    cell_tau[c] = (float)tau;
    cell_kappa[c] = (float)kap;
    cell_src[c] = (float)lsrc;
}

// h-nodes of one depth (App. A): thin and thick content summed separately, star light in
// the thin luminosity, centre of luminosity from the sub-nodes' own mapping positions.
__global__ void k_up(int64_t lo, int64_t hi, const int4 *__restrict__ geo,
                     uint32_t *__restrict__ meta, Scratch64 S64, float4 *__restrict__ q,
                     float *__restrict__ vthick, int4 *__restrict__ pcol) {
    int64_t id = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= hi) return;
    uint32_t mt = meta[id];
    if (mt & (1u << 12)) return;
    int4 g = geo[id];
    int64_t g256[3] = {(int64_t)g.x * TR_FX, (int64_t)g.y * TR_FX, (int64_t)g.z * TR_FX};
    double Lt = 0, LVk = 0, At = 0, Ak = 0, Vk = 0, X = 0, n0 = 0, n1 = 0, n2 = 0;
    int c = g.w;
    uint32_t mask = (mt >> 4) & 255u;
    for (int k = 0; k < 8; ++k) {
        if (!((mask >> k) & 1u)) continue;
        Lt = Lt + S64.Lt[c];
        LVk = LVk + S64.LVk[c];
        At = At + S64.At[c];
        Ak = Ak + S64.Ak[c];
        Vk = Vk + S64.Vk[c];
        double xi = S64.xi[c];
        X = X + xi;
        int4 pc = pcol[c];
        n0 = n0 + xi * (double)((int64_t)pc.x - g256[0]);
        n1 = n1 + xi * (double)((int64_t)pc.y - g256[1]);
        n2 = n2 + xi * (double)((int64_t)pc.z - g256[2]);
        ++c;
    }
    S64.Lt[id] = Lt;
    S64.LVk[id] = LVk;
    S64.At[id] = At;
    S64.Ak[id] = Ak;
    S64.Vk[id] = Vk;
    S64.xi[id] = Lt + (Vk > 0.0 ? LVk / cbrt(Vk) : 0.0);
    int4 p = make_int4(g.x * TR_FX, g.y * TR_FX, g.z * TR_FX, 0);
    if (X > 0.0) {
        p.x = (int)(g256[0] + (int64_t)rint(n0 / X));
        p.y = (int)(g256[1] + (int64_t)rint(n1 / X));
        p.z = (int)(g256[2] + (int64_t)rint(n2 / X));
    }
    p.w = __float_as_int((float)Vk); // the walk reads the thick volume with the position
    pcol[id] = p;
    q[id] = make_float4((float)Lt, (float)LVk, (float)At, (float)Ak);
    vthick[id] = (float)Vk;
    meta[id] = (mt & ~(1u << 13)) | (Vk > 0.0 ? 1u << 13 : 0u); // thick content
}

// Walk record of every node, one 16-byte load per visit:
// (gx | depth << 16 | leaf << 20 | thick << 21, gy | child mask << 16, gz, first child)
__global__ void k_pack(int64_t n, const int4 *__restrict__ geo, const uint32_t *__restrict__ meta,
                       int4 *__restrict__ packed) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int4 g = geo[id];
    const uint32_t m = meta[id];
    packed[id] = make_int4(g.x | (int)((m & 15u) << 16) | (int)(((m >> 12) & 3u) << 20),
                           g.y | (int)(((m >> 4) & 255u) << 16), g.z, g.w);
}

template <class T>
int dev_alloc(tr_ctx *ctx, T **p, int64_t n) {
    if (hipMalloc((void **)p, sizeof(T) * (size_t)(n > 0 ? n : 1)) != hipSuccess)
        return tr_fail(ctx, TR_ENOMEM, "device allocation of %lld bytes failed",
                       (long long)(sizeof(T) * n));
    return TR_OK;
}

} // namespace

extern "C" void tr_tree_free(tr_tree *t) {
    if (!t) return;
    hipFree(t->geo); hipFree(t->meta); hipFree(t->q); hipFree(t->vthick); hipFree(t->pcol);
    hipFree(t->packed);
    hipFree(t->leaf_cell); hipFree(t->node_of_cell); hipFree(t->targets);
    hipFree(t->cell_tau); hipFree(t->cell_kappa); hipFree(t->cell_src);
    for (double *p : t->s64) hipFree(p);
    hipFree(t->src);
    delete t;
}

#define TRY(x)                    \
    do {                          \
        int rc_ = (x);            \
        if (rc_) { cleanup(); return rc_; } \
    } while (0)

extern "C" int tr_build_tree(tr_ctx *ctx, const tr_grid *grid, const float *rho,
                             const float *kappa, const float *t_dust, const tr_star *stars,
                             int n_stars, const tr_units *units, tr_tree **out) {
    if (!ctx) return TR_EINVAL;
    if (!grid || !out || !rho || !t_dust || !units || (n_stars > 0 && !stars) || n_stars < 0)
        return tr_fail(ctx, TR_EINVAL, "tr_build_tree: null argument");
    *out = nullptr;
    if (grid->nb <= 0 || grid->max_level < 0 || grid->n_blk <= 0 || !grid->blocks ||
        !(grid->box_len > 0))
        return tr_fail(ctx, TR_EINVAL, "tr_build_tree: bad grid header");
    int64_t n_fine = (int64_t)grid->nb * 8 << grid->max_level;
    int D = 0;
    while (((int64_t)1 << D) < n_fine) ++D;
    if (D > TR_MAX_DEPTH)
        return tr_fail(ctx, TR_EINVAL, "grid too fine: %lld cells per edge (max %d)",
                       (long long)n_fine, 1 << TR_MAX_DEPTH);
    for (int b = 0; b < grid->n_blk; ++b) {
        const int32_t *bl = grid->blocks + 4 * b;
        if (bl[0] < 0 || bl[0] > grid->max_level)
            return tr_fail(ctx, TR_EINVAL, "block %d: level %d out of range", b, bl[0]);
        int64_t nbl = (int64_t)grid->nb << bl[0];
        for (int a = 1; a < 4; ++a)
            if (bl[a] < 0 || bl[a] >= nbl)
                return tr_fail(ctx, TR_EINVAL, "block %d: index out of range", b);
    }
    TR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;

    tr_tree *t = new tr_tree();
    t->ctx = ctx;
    t->nb = grid->nb; t->max_level = grid->max_level; t->n_blk = grid->n_blk; t->D = D;
    t->n_fine = n_fine; t->root_edge = (int64_t)2 << D;
    t->box_len = grid->box_len; t->sigma = units->sigma; t->c_light = units->c;
    for (int a = 0; a < 3; ++a) t->x0[a] = grid->x0[a];
    t->u_len = grid->box_len / (2.0 * (double)n_fine);
    t->n_cells = (int64_t)grid->n_blk * 512;
    {
        int64_t lim = 3 * (2 * n_fine) * (2 * n_fine), i = 1;
        while ((i + 1) * (i + 1) * (i + 1) * (i + 1) < lim) ++i;
        t->n_bins = (int)i;
    }
    DenseLayout L;
    L.base[0] = 0;
    for (int d = 0; d <= D; ++d) L.base[d + 1] = L.base[d] + ((int64_t)1 << (3 * d));
    for (int d = D + 2; d < TR_MAX_DEPTH + 2; ++d) L.base[d] = L.base[D + 1];
    const int64_t T = L.base[D + 1];

    uint32_t *occ = nullptr;
    int *ids = nullptr, *lrank = nullptr, *err = ctx->d_ctl + 17;
    int4 *d_blocks = nullptr;
    double4 *d_stars = nullptr;
    double *src = nullptr;
    void *tmp = nullptr;
    Scratch64 S64 = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    auto cleanup = [&]() {
        hipFree(occ); hipFree(ids); hipFree(lrank); hipFree(d_blocks); hipFree(d_stars);
        hipFree(src); hipFree(tmp);
        hipFree(S64.Lt); hipFree(S64.LVk); hipFree(S64.At); hipFree(S64.Ak); hipFree(S64.Vk);
        hipFree(S64.xi);
        if (t) tr_tree_free(t);
    };
    TRY(dev_alloc(ctx, &occ, T));
    TRY(dev_alloc(ctx, &ids, T));
    TRY(dev_alloc(ctx, &lrank, T));
    TRY(dev_alloc(ctx, &d_blocks, grid->n_blk));
    if (hipMemsetAsync(occ, 0, sizeof(uint32_t) * T, st) != hipSuccess ||
        hipMemsetAsync(err, 0, sizeof(int), st) != hipSuccess ||
        hipMemcpyAsync(d_blocks, grid->blocks, sizeof(int4) * grid->n_blk, hipMemcpyHostToDevice, st) != hipSuccess) {
        cleanup();
        return tr_fail(ctx, TR_EHIP, "tr_build_tree: upload failed");
    }
    const int TPB = 256;
    if (ctx->validate)
        k_validate_cells<<<tr_div_up(t->n_cells, TPB), TPB, 0, st>>>(t->n_cells, rho, kappa, t_dust, err);
    k_mark_leaves<<<tr_div_up(t->n_cells, TPB), TPB, 0, st>>>(d_blocks, t->n_cells, D, t->max_level, L, occ, err);
    for (int d = D - 1; d >= 0; --d)
        k_exist<<<tr_div_up((int64_t)1 << (3 * d), TPB), TPB, 0, st>>>(d, L, occ, err);
    {
        hipcub::TransformInputIterator<int, ExistsOp, const uint32_t *> ex(occ, ExistsOp());
        hipcub::TransformInputIterator<int, LeafOp, const uint32_t *> lf(occ, LeafOp());
        size_t b1 = 0, b2 = 0;
        hipcub::DeviceScan::ExclusiveSum(nullptr, b1, ex, ids, (int)T, st);
        hipcub::DeviceScan::ExclusiveSum(nullptr, b2, lf, lrank, (int)T, st);
        size_t nb = b1 > b2 ? b1 : b2;
        if (hipMalloc(&tmp, nb) != hipSuccess) { cleanup(); return tr_fail(ctx, TR_ENOMEM, "scan scratch"); }
        if (hipcub::DeviceScan::ExclusiveSum(tmp, nb, ex, ids, (int)T, st) != hipSuccess ||
            hipcub::DeviceScan::ExclusiveSum(tmp, nb, lf, lrank, (int)T, st) != hipSuccess) {
            cleanup();
            return tr_fail(ctx, TR_EHIP, "scan failed");
        }
    }
    // node counts per depth and error word back to the host (the one synchronisation)
    std::vector<int> firsts(D + 2, 0);
    uint32_t last_occ = 0;
    int last_id = 0, last_rank = 0, herr = 0;
    for (int d = 0; d <= D; ++d)
        if (hipMemcpyAsync(&firsts[d], ids + L.base[d], sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) {
            cleanup(); return tr_fail(ctx, TR_EHIP, "readback failed");
        }
    if (hipMemcpyAsync(&last_occ, occ + T - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&last_id, ids + T - 1, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&last_rank, lrank + T - 1, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        cleanup(); return tr_fail(ctx, TR_EHIP, "readback failed");
    }
    if (herr & 1792) {
        cleanup();
        return tr_fail(ctx, TR_EINVAL, "tr_build_tree: a cell's %s is negative, infinite or NaN",
                       (herr & 256) ? "density" : ((herr & 512) ? "opacity" : "dust temperature"));
    }
    if (herr) { cleanup(); return tr_fail(ctx, TR_EINVAL, "blocks overlap (code %d)", herr); }
    t->n_node = last_id + (last_occ != 0u ? 1 : 0);
    t->n_leaf = last_rank + ((last_occ & 2u) ? 1 : 0);
    if (t->n_leaf != t->n_cells) {
        cleanup();
        return tr_fail(ctx, TR_EINVAL, "leaf count %lld != cell count %lld", (long long)t->n_leaf,
                       (long long)t->n_cells);
    }
    if (t->n_node >= ((int64_t)1 << 31) - 1) { cleanup(); return tr_fail(ctx, TR_EINVAL, "too many nodes"); }
    for (int d = 0; d <= D; ++d) t->depth_off[d] = firsts[d];
    t->depth_off[D + 1] = t->n_node;

    const int64_t n = t->n_node, nc = t->n_cells;
    TRY(dev_alloc(ctx, &t->geo, n));
    TRY(dev_alloc(ctx, &t->meta, n));
    TRY(dev_alloc(ctx, &t->q, n));
    TRY(dev_alloc(ctx, &t->vthick, n));
    TRY(dev_alloc(ctx, &t->pcol, n));
    TRY(dev_alloc(ctx, &t->packed, n));
    TRY(dev_alloc(ctx, &t->leaf_cell, n));
    TRY(dev_alloc(ctx, &t->node_of_cell, nc));
    TRY(dev_alloc(ctx, &t->targets, nc));
    TRY(dev_alloc(ctx, &t->cell_tau, nc));
    TRY(dev_alloc(ctx, &t->cell_kappa, nc));
    TRY(dev_alloc(ctx, &t->cell_src, nc));
    TRY(dev_alloc(ctx, &src, nc));
    TRY(dev_alloc(ctx, &S64.Lt, n));
    TRY(dev_alloc(ctx, &S64.LVk, n));
    TRY(dev_alloc(ctx, &S64.At, n));
    TRY(dev_alloc(ctx, &S64.Ak, n));
    TRY(dev_alloc(ctx, &S64.Vk, n));
    TRY(dev_alloc(ctx, &S64.xi, n));
    if (hipMemsetAsync(t->leaf_cell, 0xff, sizeof(int32_t) * n, st) != hipSuccess ||
        hipMemsetAsync(src, 0, sizeof(double) * nc, st) != hipSuccess) {
        cleanup(); return tr_fail(ctx, TR_EHIP, "memset failed");
    }
    k_nodes<<<tr_div_up(T, TPB), TPB, 0, st>>>(D, t->root_edge, L, occ, ids, lrank, t->geo, t->meta,
                                               t->pcol, t->targets);
    k_cells<<<tr_div_up(nc, TPB), TPB, 0, st>>>(d_blocks, nc, D, t->max_level, L, ids,
                                                t->node_of_cell, t->leaf_cell);
    if (n_stars > 0) {
        TRY(dev_alloc(ctx, &d_stars, n_stars));
        if (hipMemcpyAsync(d_stars, stars, sizeof(double4) * n_stars, hipMemcpyHostToDevice, st) != hipSuccess) {
            cleanup(); return tr_fail(ctx, TR_EHIP, "star upload failed");
        }
        double dxmin = grid->box_len / (double)n_fine;
        k_stars<<<1, 64, 0, st>>>(reinterpret_cast<const double *>(d_stars), n_stars, n_fine, grid->x0[0], grid->x0[1], grid->x0[2], dxmin,
                                  t->u_len * t->u_len, t->geo, t->meta, t->leaf_cell, src);
    }
    k_leaf_fill<<<tr_div_up(nc, TPB), TPB, 0, st>>>(nc, rho, kappa, t_dust, src, t->node_of_cell, t->meta,
                                                    t->root_edge, t->u_len, units->sigma, S64, t->q,
                                                    t->vthick, t->cell_tau, t->cell_kappa, t->cell_src);
    for (int d = D - 1; d >= 0; --d) {
        int64_t lo = t->depth_off[d], hi = t->depth_off[d + 1];
        if (hi > lo)
            k_up<<<tr_div_up(hi - lo, TPB), TPB, 0, st>>>(lo, hi, t->geo, t->meta, S64, t->q, t->vthick, t->pcol);
    }
    k_pack<<<tr_div_up(n, TPB), TPB, 0, st>>>(n, t->geo, t->meta, t->packed);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        cleanup(); return tr_fail(ctx, TR_EHIP, "tree kernels failed");
    }
    tr_tree *res = t;
    t = nullptr; // keep the tree (with its FP64 sums and star light, for refills), free the rest
    res->s64[0] = S64.Lt; res->s64[1] = S64.LVk; res->s64[2] = S64.At;
    res->s64[3] = S64.Ak; res->s64[4] = S64.Vk; res->s64[5] = S64.xi;
    res->src = src;
    S64 = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    src = nullptr;
    cleanup();
    *out = res;
    return TR_OK;
}

extern "C" int tr_tree_refill(tr_ctx *ctx, tr_tree *t, const float *rho, const float *kappa,
                              const float *t_dust, const tr_star *stars, int n_stars) {
    if (!ctx) return TR_EINVAL;
    if (!t || !rho || !t_dust || n_stars < 0 || (n_stars > 0 && !stars))
        return tr_fail(ctx, TR_EINVAL, "tr_tree_refill: bad argument");
    if (!t->src || !t->s64[0]) return tr_fail(ctx, TR_EINVAL, "tr_tree_refill: tree has no refill buffers");
    TR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int TPB = 256;
    const int64_t n = t->n_node, nc = t->n_cells;
    Scratch64 S64 = {t->s64[0], t->s64[1], t->s64[2], t->s64[3], t->s64[4], t->s64[5]};
    k_zero_f64<<<tr_div_up(nc, TPB), TPB, 0, st>>>(t->src, nc);
    if (n_stars > 0)
        k_stars<<<1, 64, 0, st>>>(reinterpret_cast<const double *>(stars), n_stars, t->n_fine, t->x0[0],
                                  t->x0[1], t->x0[2], t->box_len / (double)t->n_fine, t->u_len * t->u_len,
                                  t->geo, t->meta, t->leaf_cell, t->src);
    k_leaf_fill<<<tr_div_up(nc, TPB), TPB, 0, st>>>(nc, rho, kappa, t_dust, t->src, t->node_of_cell, t->meta,
                                                    t->root_edge, t->u_len, t->sigma, S64, t->q, t->vthick,
                                                    t->cell_tau, t->cell_kappa, t->cell_src);
    for (int d = t->D - 1; d >= 0; --d) {
        int64_t lo = t->depth_off[d], hi = t->depth_off[d + 1];
        if (hi > lo)
            k_up<<<tr_div_up(hi - lo, TPB), TPB, 0, st>>>(lo, hi, t->geo, t->meta, S64, t->q, t->vthick, t->pcol);
    }
    k_pack<<<tr_div_up(n, TPB), TPB, 0, st>>>(n, t->geo, t->meta, t->packed);
    return hipGetLastError() == hipSuccess ? TR_OK : tr_fail(ctx, TR_EHIP, "tr_tree_refill: launch failed");
}

extern "C" int tr_tree_get_info(const tr_tree *t, tr_tree_info *info) {
    if (!t || !info) return TR_EINVAL;
    info->n_node = t->n_node;
    info->n_leaf = t->n_leaf;
    info->n_cells = t->n_cells;
    info->depth = t->D;
    info->root_edge = (int32_t)t->root_edge;
    info->n_bins = t->n_bins;
    info->u_len = t->u_len;
    return TR_OK;
}

extern "C" int tr_tree_export(tr_ctx *ctx, const tr_tree *t, int32_t *geo, uint32_t *meta,
                              float *q, float *vthick, int32_t *pcol, int64_t *leaf_cell) {
    if (!ctx || !t) return TR_EINVAL;
    TR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const size_t n = (size_t)t->n_node;
    if (geo) TR_HIP(ctx, hipMemcpyAsync(geo, t->geo, sizeof(int4) * n, hipMemcpyDeviceToHost, st));
    if (meta) TR_HIP(ctx, hipMemcpyAsync(meta, t->meta, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, st));
    if (q) TR_HIP(ctx, hipMemcpyAsync(q, t->q, sizeof(float4) * n, hipMemcpyDeviceToHost, st));
    if (vthick) TR_HIP(ctx, hipMemcpyAsync(vthick, t->vthick, sizeof(float) * n, hipMemcpyDeviceToHost, st));
    std::vector<int4> pc;
    std::vector<int32_t> lc;
    if (pcol) {
        pc.resize(n);
        TR_HIP(ctx, hipMemcpyAsync(pc.data(), t->pcol, sizeof(int4) * n, hipMemcpyDeviceToHost, st));
    }
    if (leaf_cell) {
        lc.resize(n);
        TR_HIP(ctx, hipMemcpyAsync(lc.data(), t->leaf_cell, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    }
    TR_HIP(ctx, hipStreamSynchronize(st));
    for (size_t i = 0; pcol && i < n; ++i) {
        pcol[3 * i] = pc[i].x;
        pcol[3 * i + 1] = pc[i].y;
        pcol[3 * i + 2] = pc[i].z;
    }
    for (size_t i = 0; leaf_cell && i < n; ++i) leaf_cell[i] = lc[i];
    return TR_OK;
}
