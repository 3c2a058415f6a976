// Backward ray tracing of the diffuse infrared field (Sec. 4.2-4.5 of Klepitko et al.).
//
// One wavefront per target cell, persistent: waves take targets from a global work
// counter.  For every target the optically thin content of the ray segments (HEALPix
// pixel x radial evaluation point: L_thin, A_thin) lives in LDS; the optically thick
// content (L V, A, V and Q of thick material), which only a small minority of nodes
// carries, goes to a per-wave accumulator in global memory with a presence bit per
// segment in LDS.  To keep many waves resident per CU the segments are processed in
// passes of `bins_per_pass` radial points; each pass re-walks the octree, pruning
// subtrees whose material cannot map into the pass, maps the accepted nodes with
// atomics and then integrates the pass outwards with one lane per ray, carrying the
// extinction and an open merged segment to the next pass.
//
// Walk: a stack of child ranges (first child, count) in LDS; each step pops 8 ranges so
// that the 64 lanes test 64 sibling nodes at once (one 16-byte record per node).  The
// opening test, the pruning test and the radial bin search are exact integer
// comparisons; the bin search compares r^2 with the pass's few radial points in 64-bit
// integers (wide passes: a float estimate with a 64-bit fallback near a bin edge).
// Accepted nodes that touch the pass are compacted into one of two LDS queues and mapped
// 64 at a time, so the angular kernel runs with every lane busy on the same code path:
// nodes at least 8 edges away take the tabulated kernel (the walk computes their table
// key, one table load per node), nearer ones the per-node 8-point kernel.  A block holds
// several such waves; with up to 64 rays they share one copy of the direction-cell table
// in LDS, otherwise near nodes read it from global memory.
#include "common.hpp"

namespace {

constexpr float kPiF = 3.14159265358979f;
// accepted nodes waiting to be mapped: the far-node queue (tabulated kernel) grows up from
// 0, the near-node one down from kQueue - 1; each holds < 64 entries before a walk step
// adds at most 64
constexpr int kQueue = 192;
constexpr int kFields = 6;  // L_thin, A_thin, L_thick*V, A_thick, V_thick, Q
constexpr int kThin = 2;    // fields held in LDS: L_thin, A_thin
constexpr int kMaxBp = 16;  // segments per pass: a ray's merge and thick-content flags take
                            // 2 kMaxBp bits (flag_words)

// ranges on a wave's walk stack: each step pops up to 8 ranges and pushes at most 64,
// so at most 56 per level of the tree stay behind
__host__ __device__ inline int stack_size(int depth) { return 56 * depth + 8; }
struct TraceArgs {
    const int4 *nodes;   // packed walk records
    const float4 *q;     // node content
    const int4 *pcol;    // mapping position, .w thick volume
    const int32_t *targets;
    const int32_t *leaf_cell;
    const float *cell_tau;
    const float *cell_src;
    const int16_t *table;
    const unsigned long long *alpha; // tabulated angular kernel [6 M M][classes 6 .. alpha_c1 - 1]
    const float4 *dirs;
    const int4 *near;    // per-node kernel of same-size leaves at offsets up to 7 edges
    int *work;
    int *err;
    float4 *thick;  // per wave: [npix][bp] thick content accumulators (all-zero between uses),
                    // then [npix][2] carry slots of merged segments open across passes
    float *J, *F, *u_rad;
    int32_t *counters;
    int64_t n_cells;
    int n_targets;
    int root_edge;
    int npix;
    int log2m;      // direction cells per face edge = 1 << log2m
    int alpha_c1;   // first distance class served by the pixel table (the cell's own pixel)
    int n_bins;
    int bp;         // bins per pass
    int n_pass;
    int chunk;
    int merge;
    int wide_open;  // opening test needs 64-bit products
    int th_num2, th_den2;
    float omega;
    float j_bg;
    float c_light;
    int kstack;     // ranges per wave stack
    int tab_slot;   // batched launches: which LDS table set the instance uses
    int orient;     // ray-set orientation 0..47, -1 = drawn per target
    int per_node;   // 1: the per-node angular kernel for every node (no table)
    uint32_t orient_seed;
    int per_block;  // waves per block
    int lds_wave;   // bytes of LDS per wave
    int lds_table;  // bytes of the shared tables (0: read the tables from global memory)
};

struct LdsLayout {
    int bins, flg, stk, qnode, qpk, total;
};

// Merge and thick-content flags of a pass, per ray: bit k (merge segment k with the next)
// and bit tsh + k (segment k holds thick content), k relative to the pass.  With at most 8
// segments per pass they take 16 bits and two rays share a word (ray h in half h & 1).
__host__ __device__ inline int flag_words(int npix, int bp) { return bp <= 8 ? (npix + 1) >> 1 : npix; }

__host__ __device__ inline LdsLayout lds_layout(int npix, int bp, int kstack, bool count) {
    LdsLayout L;
    int o = 0;
    L.bins = o;
    o += count ? 0 : npix * bp * kThin * 4;
    L.flg = o;
    o += count ? 0 : flag_words(npix, bp) * 4;
    L.stk = o;
    o += kstack * 4;
    L.qnode = o;
    o += count ? 0 : kQueue * 4;
    L.qpk = o;
    o += count ? 0 : kQueue * 4;
    L.total = (o + 15) & ~15;
    return L;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_s_waitcnt(0xc07f); // lgkmcnt(0): this wave's LDS traffic has landed
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// set bits of a wave-wide mask in the lanes below this one (two mbcnt instructions)
__device__ __forceinline__ int count_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// element i of an array, addressed as the array's (uniform) base plus a 32-bit byte offset,
// which the hardware adds itself (no 64-bit address arithmetic per lane); every array read
// this way is far below 4 GiB
template <typename T>
__device__ __forceinline__ const T &at32(const T *base, int i) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (uint32_t)i * (uint32_t)sizeof(T));
}

// largest i in [0, nb] with R_i + off <= r (lattice units / 256, R_i = 256 i^2), i.e.
// (256 i^2 + off)^2 <= r2 or 256 i^2 + off <= 0.  Float estimate (hardware square root,
// 1 ulp; the sum of squares adds a few more, far inside the 4e-6 r margin), exact
// integer fallback near edges.
__device__ __forceinline__ int bin_below(int dx, int dy, int dz, int off, int nb) {
    const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
    const float r = __builtin_amdgcn_sqrtf(fx * fx + fy * fy + fz * fz);
    const float x = r - (float)off;
    int i = x > 0.0f ? (int)__builtin_amdgcn_sqrtf(x * (1.0f / TR_FX)) : 0;
    i = i > nb ? nb : i;
    const float e0 = (float)(TR_FX * i * i), e1 = (float)(TR_FX * (i + 1) * (i + 1));
    const float tol = 4e-6f * (r + (float)(off < 0 ? -off : off) + 1.0f);
    const bool sure = (i == 0 || x - e0 > tol) && (i == nb || e1 - x > tol);
    if (!sure) {
        const int64_t r2 = (int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz;
        auto ok = [&](int k) {
            const int64_t e = (int64_t)TR_FX * k * k + off;
            return e <= 0 || e * e <= r2;
        };
        i = i < 1 ? 0 : i - 1;
        while (i < nb && ok(i + 1)) ++i;
        while (i > 0 && !ok(i)) --i;
    }
    return i;
}

// exact floor(num / den) for num < 2^31, den < 2^24, quotient < 2^8, from a float reciprocal
__device__ __forceinline__ uint32_t exact_div(uint32_t num, uint32_t den, float rc) {
    uint32_t q = (uint32_t)((float)num * rc);
    q -= (uint32_t)__umul24(q, den) > num ? 1u : 0u;
    q += (uint32_t)__umul24(q + 1u, den) <= num ? 1u : 0u;
    return q;
}

// direction cell of an integer direction (face of the largest component with ties to the
// lower axis, then floor(M (d_a + |d_m|) / (2 |d_m|)) on the other two axes)
__device__ __forceinline__ int cube_cell(int dx, int dy, int dz, int log2m) {
    const int ax = abs(dx), ay = abs(dy), az = abs(dz);
    // the face by selects (no divergent branches): x when it is the largest (ties to the
    // lower axis), else y when it is at least z, else z
    const bool fx = (ax >= ay) & (ax >= az), fy = !fx & (ay >= az);
    const int m = fx ? ax : (fy ? ay : az);
    const int lead = fx ? dx : (fy ? dy : dz);
    const int f = (fx ? 0 : (fy ? 2 : 4)) + (lead < 0 ? 1 : 0);
    const int ua = (fx ? dy : dx) + m, ub = ((fy | fx) ? dz : dy) + m;
    const uint32_t den = 2u * (uint32_t)m;
    const float rc = rcp((float)den);
    const int Mm1 = (1 << log2m) - 1;
    uint32_t i = exact_div((uint32_t)ua << log2m, den, rc);
    uint32_t j = exact_div((uint32_t)ub << log2m, den, rc);
    i = i > (uint32_t)Mm1 ? (uint32_t)Mm1 : i;
    j = j > (uint32_t)Mm1 ? (uint32_t)Mm1 : j;
    return (((f << log2m) + (int)i) << log2m) + (int)j;
}

struct Pass {
    int a, b; // radial points [a, b) held in LDS
};

__device__ __forceinline__ void cswap(int &a, int &b) {
    const int lo = min(a, b), hi = max(a, b);
    a = lo;
    b = hi;
}

// sort 8 pixel ids (19-comparator network), then mark the first of each run of equal ids
__device__ __forceinline__ void sort8_runs(int (&pix)[8], bool valid, uint32_t &starts) {
    cswap(pix[0], pix[2]); cswap(pix[1], pix[3]); cswap(pix[4], pix[6]); cswap(pix[5], pix[7]);
    cswap(pix[0], pix[4]); cswap(pix[1], pix[5]); cswap(pix[2], pix[6]); cswap(pix[3], pix[7]);
    cswap(pix[0], pix[1]); cswap(pix[2], pix[3]); cswap(pix[4], pix[5]); cswap(pix[6], pix[7]);
    cswap(pix[2], pix[4]); cswap(pix[3], pix[5]);
    cswap(pix[1], pix[4]); cswap(pix[3], pix[6]);
    cswap(pix[1], pix[2]); cswap(pix[3], pix[4]); cswap(pix[5], pix[6]);
    starts = valid ? 1u : 0u;
#pragma unroll
    for (int k = 1; k < 8; ++k) starts |= (valid && pix[k] != pix[k - 1] ? 1u : 0u) << k;
}

// Orientation of the ray set (Sec. 7.6 names different HEALPix orientations as the remedy
// for ray artefacts): one of the 48 signed permutations of the axes, which map the lattice
// onto itself.  Index o: axis permutation o / 8 in the order 012 021 102 120 201 210, sign
// flip of axis a for bit a of o % 8; a node offset d enters the angular kernel as
// (s0 d[p0], s1 d[p1], s2 d[p2]).  A per-target draw takes the SplitMix64 generator
// (Steele, Lea and Flood 2014) of seed * 2^32 + cell, modulo 48.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int target_orient(int orient, uint32_t seed, int cell) {
    return orient >= 0 ? orient : (int)(splitmix64(((uint64_t)seed << 32) | (uint32_t)cell) % 48u);
}

__device__ __forceinline__ void orient_axes(int o, int &p0, int &p1, int &p2) {
    const int q = o >> 3;
    p0 = q >> 1;
    p1 = (0x102021 >> (4 * q)) & 3; // 1 2 0 2 0 1
    p2 = 3 - p0 - p1;
}

__device__ __forceinline__ void orient_offset(int o, int &x, int &y, int &z) {
    if (o == 0) return;
    int p0, p1, p2;
    orient_axes(o, p0, p1, p2);
    auto pick = [&](int k) { return k == 0 ? x : (k == 1 ? y : z); };
    const int a = pick(p0), b = pick(p1), c = pick(p2);
    x = (o & 1) ? -a : a;
    y = (o & 2) ? -b : b;
    z = (o & 4) ? -c : c;
}

// a vector from the ray set's frame back to the grid's axes: out[p_a] = s_a f[a]
__device__ __forceinline__ void orient_back(int o, float &fx, float &fy, float &fz) {
    if (o == 0) return;
    int p0, p1, p2;
    orient_axes(o, p0, p1, p2);
    const float f0 = (o & 1) ? -fx : fx, f1 = (o & 2) ? -fy : fy, f2 = (o & 4) ? -fz : fz;
    fx = p0 == 0 ? f0 : (p1 == 0 ? f1 : f2);
    fy = p0 == 1 ? f0 : (p1 == 1 ? f1 : f2);
    fz = p0 == 2 ? f0 : (p1 == 2 ? f1 : f2);
}

// lane-shifted copies within rows of 16 lanes (DPP row_shr / row_shl); lanes whose source
// lies outside the row receive `old`
template <int N>
__device__ __forceinline__ int dpp_shr(int v, int old) {
    return __builtin_amdgcn_update_dpp(old, v, 0x110 | N, 0xf, 0xf, false);
}
template <int N>
__device__ __forceinline__ int dpp_shl(int v, int old) {
    return __builtin_amdgcn_update_dpp(old, v, 0x100 | N, 0xf, 0xf, false);
}
template <int N>
__device__ __forceinline__ float dpp_shr_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 | N, 0xf, 0xf, false));
}

// one step of a segmented inclusive sum over runs of equal run ids inside a row of 16
template <int D>
__device__ __forceinline__ void seg_sum_step(int rl, int rid, float &v0, float &v1) {
    const int r = dpp_shr<D>(rid, -1);
    const float a0 = dpp_shr_f<D>(v0), a1 = dpp_shr_f<D>(v1);
    if (rl >= D && r == rid) {
        v0 += a0;
        v1 += a1;
    }
}

// Tabulated angular kernel (Sec. 4.2): nodes at least 8 edges away (r >= 8 s) take the
// entry of their direction cell and distance class c = floor(log2(r^2 / s^2)), 6 <= c <= 20
// (larger classes count as 20).  Entry: 64 bits, pixels 0..3 (10 bits each from bit 0),
// counts 0..2 out of 64 (7 bits each from bit 40; count 3 = 64 - the others) and bit 61 set
// when the key's sub-points reach more than 4 pixels (the node then takes the per-node
// kernel).  From class alpha_c1 on every entry is the direction cell's own pixel alone, and
// the pixel table serves those keys (a negative key -1 - cell).
constexpr int kAlphaFar = 6;
constexpr int kAlphaMax = 20;

// distance class c = floor(log2(r^2 / s^2)) of an offset (1/256 lattice units, r^2 > 0)
// from a node of edge s = 2^log2s: node edges are powers of two, so s^2 = 2^(16 + 2 log2s)
// and c is exact from the leading bit of r^2.  The node is served by the table when c >= 6,
// i.e. r^2 >= 64 s^2.
__device__ __forceinline__ int dist_class(int dx, int dy, int dz, int log2s) {
    const int64_t r2 = (int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz;
    return (63 - __clzll(r2)) - 2 * (8 + log2s);
}

// table key of a far node (class c >= 6): direction cell of the offset in the ray set's
// frame and the class, or -1 - cell when the class is served by the pixel table
__device__ __forceinline__ int alpha_key(int dx, int dy, int dz, int c, int orient, int log2m, int c1) {
    c = c > kAlphaMax ? kAlphaMax : c; // larger classes count as the last
    orient_offset(orient, dx, dy, dz);
    const int cell = cube_cell(dx, dy, dz, log2m);
    return c >= c1 ? -1 - cell : __mul24(cell, c1 - kAlphaFar) + (c - kAlphaFar);
}

// Segment of an accepted node in the pass [a, b) (Sec. 4.2): i = the largest radial point
// with R_i <= r (R_i = i^2 lattice units, offsets in 1/256 units), content when a <= i < b
// (or i >= a in the last pass).  A node with thick material and merging (ext = s/2 > 0)
// also flags the segments its extent r -+ s/2 spans, k0 .. k1 relative to a.  Without
// thick material r^2 is compared with (256 i^2)^2 exactly in 64 bits, for the points of
// the pass only when it holds a few.
struct SegHit {
    int i, k0, k1;
    bool content;
};
__device__ __forceinline__ SegHit seg_hit(int dx, int dy, int dz, int s, int ext, int a, int b, bool last, int nb) {
    SegHit h{0, 0, 0, false};
    if (ext) {
        const int i = bin_below(dx, dy, dz, 0, nb);
        if (i > 0) {
            h.i = i;
            h.content = i >= a && i < b;
            const int half = TR_FX / 2 * s;
            int lo = bin_below(dx, dy, dz, half, nb);
            lo = lo < 1 ? 1 : lo;
            const int hi = bin_below(dx, dy, dz, -half, nb);
            int k0 = lo > a ? lo : a, k1 = hi < b ? hi : b;
            if (k1 > k0) {
                h.k0 = k0 - a;
                h.k1 = k1 - a;
            }
        }
    } else {
        const int64_t r2 = (int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz;
        auto t = [](int k) {
            const int64_t q = (int64_t)TR_FX * k * k;
            return q * q;
        };
        h.content = r2 >= t(a) && (last || r2 < t(b));
        if (b - a <= 4) {
            int i = a;
            for (int k = a + 1; k < b; ++k) i += r2 >= t(k) ? 1 : 0;
            h.i = i;
        } else {
            h.i = bin_below(dx, dy, dz, 0, nb); // wide passes: float estimate, exact near edges
        }
    }
    return h;
}

// Thresholds of a pass [a, b) of at most four radial points for the segment search, the
// same on every lane: R_k^2 = 2^16 k^4 in 1/256 lattice units, in FP64, for k = a, then
// a + 1 .. a + 3 (each infinite from b on), and b.  An offset below 2^19 per axis has r^2 < 2^40, so r^2, the
// thresholds and their comparisons are exact in FP64, as in 64-bit integers.
struct PassT {
    double ta, t1, t2, t3, tb;
};
__device__ __forceinline__ PassT pass_thresholds(int a, int b) {
    auto t = [](int k) {
        const double q = (double)(k * k);
        return 65536.0 * (q * q);
    };
    const double inf = __builtin_inf();
    return PassT{t(a), a + 1 < b ? t(a + 1) : inf, a + 2 < b ? t(a + 2) : inf, a + 3 < b ? t(a + 3) : inf, t(b)};
}

// radial kernel beta = R_i^2 / r^2 of segment i (offsets in 1/256 lattice units)
__device__ __forceinline__ float beta_of(int dx, int dy, int dz, int i) {
    const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
    const float R2 = (float)(TR_FX * __mul24(i, i));
    return (R2 * R2) * rcp(fx * fx + fy * fy + fz * fz);
}

// Queue record of an accepted node: pk = content segment (i - a + 1, 0 = none) | first
// merge flag << 6 | end of merge flags << 12 (both relative to the pass) | leaf << 18 |
// depth << 19 | thick content << 23 | distance class << 24 (far nodes, at most kAlphaMax).
//
// Map queued nodes (Sec. 4.2.1/4.2.2): one lane per node, one LDS update per distinct pixel.
// FAR: every node of the batch is at least 8 edges away and takes the tabulated kernel,
// keyed by the direction cell and distance class of its offset, which every lane computes
// from the node's mapping position.  Otherwise the per-node kernel: the node cube's 2x2x2
// sub-points, each binned to a direction cell and its pixel, sorted to find the distinct
// pixels.  Merge and thick-content flags go to the rays' flag words (flag_words).
template <bool LDS_TABLE, bool FAR>
__device__ __forceinline__ void map_queue(const TraceArgs &A, int e, bool valid, const int *qnode, const uint32_t *qpk,
                                          int pass_a, int4 c256, int tdepth, int orient, const uint8_t *tab8,
                                          float *bins, uint32_t *flg, float4 *thick) {
    uint32_t starts = 0;
    int pix[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    float Lt = 0, At = 0, LVk = 0, Ak = 0, Vk = 0, beta = 0;
    int seg = -1;
    uint32_t fbits = 0;
    uint32_t counts = 0; // tabulated entries: counts out of 64 of pix[0..3]
    bool tab = false;
    {
        // Every lane reads a queue entry (e is in range on every lane); a lane without one of
        // its own (!valid, only at the end of a pass) repeats another lane's and carries no
        // counts, segment or flags, so the lanes take the same steps without branching.
        const int ev = e;
        const int node = qnode[ev];
        const uint32_t pk = qpk[ev];
        const bool leaf = (pk >> 18) & 1u;
        const int depth = (int)((pk >> 19) & 15u);
        const int s = A.root_edge >> depth;
        seg = valid ? (int)(pk & 63u) - 1 : -1;
        const uint32_t k0 = (pk >> 6) & 63u, k1 = (pk >> 12) & 63u;
        fbits = valid && k1 > k0 ? (k1 >= 32u ? 0xffffffffu : ((1u << k1) - 1u)) & ~((1u << k0) - 1u) : 0u;
        const float4 qv = at32(A.q, node);
        auto lookup = [&](int cell) { return LDS_TABLE ? (int)tab8[cell] : (int)A.table[cell]; };
        unsigned long long en = 1ull << 61; // no entry: the per-node kernel
        int own = -1;                       // key served by the pixel table: the cell's pixel
        float vkh;
        int dx = 0, dy = 0, dz = 0;
        if (FAR) {
            // the node's offset from its mapping position: table key and radial kernel here,
            // with every lane busy
            const int4 p = at32(A.pcol, node);
            vkh = __int_as_float(p.w);
            dx = p.x - c256.x; dy = p.y - c256.y; dz = p.z - c256.z;
            beta = beta_of(dx, dy, dz, (seg > 0 ? seg : 0) + pass_a);
            const int key = alpha_key(dx, dy, dz, (int)(pk >> 24), orient, A.log2m, A.alpha_c1);
            // both reads, the one not needed at a harmless index, instead of a branch
            const unsigned long long ek = at32(A.alpha, key < 0 ? 0 : key);
            const int ok = lookup(key < 0 ? -1 - key : 0);
            en = key < 0 ? 0ull : ek;
            own = key < 0 ? ok : -1;
        } else {
            const int4 p = at32(A.pcol, node);
            vkh = __int_as_float(p.w);
            dx = p.x - c256.x; dy = p.y - c256.y; dz = p.z - c256.z;
            beta = beta_of(dx, dy, dz, (seg > 0 ? seg : 0) + pass_a);
            orient_offset(orient, dx, dy, dz); // the angular kernel works in the ray set's frame
        }
        if (leaf) {
            const bool thick = signbit(qv.x);
            const float V = (float)s * (float)s * (float)s;
            Lt = thick ? qv.z : qv.x + qv.z;
            At = thick ? 0.0f : qv.y;
            LVk = thick ? fabsf(qv.x) * V : 0.0f;
            Ak = thick ? qv.y : 0.0f;
            Vk = thick ? V : 0.0f;
        } else {
            Lt = qv.x; LVk = qv.y; At = qv.z; Ak = qv.w;
            Vk = vkh;
        }
        if (FAR) {
            // the cell's own pixel (all 64 sub-points), or up to 4 tabulated pixels and counts
            const uint32_t lo = (uint32_t)en, hi = (uint32_t)(en >> 32);
            const uint32_t c0 = (hi >> 8) & 127u, c1 = (hi >> 15) & 127u, c2 = (hi >> 22) & 127u;
            tab = own >= 0 || !((en >> 61) & 1ull);
            pix[0] = own >= 0 ? own : (int)(lo & 1023u);
            pix[1] = (int)((lo >> 10) & 1023u);
            pix[2] = (int)((lo >> 20) & 1023u);
            pix[3] = (int)((lo >> 30) | ((hi & 255u) << 2));
            counts = !valid ? 0u : own >= 0 ? 64u : c0 | (c1 << 8) | (c2 << 16) | ((64u - c0 - c1 - c2) << 24);
        }
        if (FAR && !tab) orient_offset(orient, dx, dy, dz); // more than 4 pixels: the per-node kernel
        if (!tab) {
            // A leaf of the target's own size lies a whole number of edges m away, and its
            // sub-points' directions depend on m alone: near ones read their sorted pixels
            // from a table instead of binning and sorting them here
            const int sh = 8 + (31 - __clz(A.root_edge)) - depth;
            const int mx = dx >> sh, my = dy >> sh, mz = dz >> sh;
            const bool tabled = !FAR && ((pk >> 18) & 1u) && depth == tdepth && (uint32_t)(mx + 7) < 15u &&
                                (uint32_t)(my + 7) < 15u && (uint32_t)(mz + 7) < 15u;
            if (tabled) {
                const int4 nt = at32(A.near, __mul24(mx + 7, 225) + __mul24(my + 7, 15) + (mz + 7));
                pix[0] = nt.x & 1023; pix[1] = (nt.x >> 10) & 1023; pix[2] = (nt.x >> 20) & 1023;
                pix[3] = nt.y & 1023; pix[4] = (nt.y >> 10) & 1023; pix[5] = (nt.y >> 20) & 1023;
                pix[6] = nt.z & 1023; pix[7] = (nt.z >> 10) & 1023;
                starts = valid ? (uint32_t)nt.w : 0u;
            } else {
                const int h = (TR_FX / 4) * s;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int cx = dx + ((k & 1) ? h : -h), cy = dy + ((k & 2) ? h : -h), cz = dz + ((k & 4) ? h : -h);
                    pix[k] = lookup(cube_cell(cx, cy, cz, A.log2m));
                }
                sort8_runs(pix, valid, starts);
            }
        }
    }
    // One update per (node, pixel); each loop runs as often as the busiest lane needs.  Thin
    // contributions are first summed over runs of neighbouring lanes that hit the same
    // (pixel, segment) -- siblings of one parent usually do -- so that one LDS atomic per
    // run, not per lane, reaches the bins.
    const int lane = lane_id(), rl = lane & 15;
    // on: the lane has this pixel; thin content goes out through key/v0/v1 (key -1: none),
    // thick content and merge flags (both rare) straight to their accumulators
    auto update = [&](bool on, int px, float al, float ab, int &key, float &v0, float &v1) {
        const bool cs = on && seg >= 0;
        key = cs ? px * A.bp + seg : -1;
        v0 = cs ? ab * Lt : 0.0f;
        v1 = cs ? ab * At : 0.0f;
        uint32_t ft = 0u;
        if (cs && Vk > 0.0f) {
            float *tk = reinterpret_cast<float *>(thick + px * A.bp + seg);
            atomicAdd(tk + 0, al * LVk);
            atomicAdd(tk + 1, al * Ak);
            atomicAdd(tk + 2, al * Vk);
            atomicAdd(tk + 3, ab * Vk);
            ft = 1u << seg;
        }
        const uint32_t fm = on ? fbits : 0u;
        const bool half = A.bp <= 8;
        const uint32_t fl = fm | (ft << (half ? 8 : 16));
        if (fl) atomicOr(flg + (half ? px >> 1 : px), half ? fl << ((px & 1) << 4) : fl);
    };
    auto flush = [&](int key, float v0, float v1) {
        // runs of equal keys within rows of 16 lanes (wave-uniform control flow): run id =
        // number of run heads up to this lane, then a segmented inclusive sum
        const int prev = dpp_shr<1>(key, -2);
        const bool head = rl == 0 || prev != key;
        const uint64_t hb = __ballot(head);
        const int rid = count_below(hb) + (head ? 1 : 0);
        seg_sum_step<1>(rl, rid, v0, v1);
        seg_sum_step<2>(rl, rid, v0, v1);
        seg_sum_step<4>(rl, rid, v0, v1);
        seg_sum_step<8>(rl, rid, v0, v1);
        const int nrid = dpp_shl<1>(rid, 0);
        if (key >= 0 && (rl == 15 || nrid != rid) && (v0 != 0.0f || v1 != 0.0f)) {
            float *bb = bins + key * kThin;
            atomicAdd(bb + 0, v0);
            atomicAdd(bb + 1, v1);
        }
    };
    if (FAR) {
        // tabulated entries: slot t holds the t-th pixel, count 0 = unused (slots are filled
        // from 0), so the slot index is the same on every lane.  Every lane has a slot 0 and
        // most have a slot 1 (far nodes of classes 6-8 reach 1.6-2.1 pixels), and siblings in
        // neighbouring lanes often share those bins: both take the run sums.  Slots 2 and 3
        // are sparse and go to the bins directly.
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint32_t ct = tab ? (counts >> (8 * t)) & 255u : 0u;
            if (!__ballot(ct != 0u)) break;
            int key;
            float v0, v1;
            const float al = (1.0f / 64.0f) * (float)ct;
            update(ct != 0u, pix[t], al, al * beta, key, v0, v1);
            if (t <= 1) {
                flush(key, v0, v1);
            } else if (key >= 0 && (v0 != 0.0f || v1 != 0.0f)) {
                float *bb = bins + key * kThin;
                atomicAdd(bb + 0, v0);
                atomicAdd(bb + 1, v1);
            }
        }
    }
    // per-node kernel: runs of equal pixels among the 8 sorted sub-point pixels
    while (__ballot(starts != 0u)) {
        int key;
        float v0, v1;
        const bool on = starts != 0u;
        const int k = on ? __builtin_ctz(starts) : 0;
        starts &= starts - 1u;
        int px = pix[0];
#pragma unroll
        for (int j = 1; j < 8; ++j) px = k == j ? pix[j] : px;
        const int kn = starts ? __builtin_ctz(starts) : 8;
        const float al = 0.125f * (float)(kn - k);
        update(on, px, al, al * beta, key, v0, v1);
        flush(key, v0, v1);
    }
}

// A ray's state between passes: sum of the thin optical depths of its closed inner segments,
// thick extinction, flux so far and the first point of its open (merged) segment (0 = none;
// that segment's content waits in the wave's carry slots).
struct RayState {
    float tau_thin, eps_thick, Fh;
    int run_i;
};

// The wave's ray states.  Up to 3 rays per lane they stay in registers.  Wide rays (12 per
// lane, 48 registers of states held through the whole walk) keep them in the wave's
// workspace after the thick accumulators and carry slots, one float4 per ray (tau, eps, F,
// run as int bits), written back to zero when the target is done; that frees the registers
// for three waves per SIMD.
__host__ __device__ constexpr int ray_state_floats4(int nslot) { return nslot > 3 ? 64 * nslot : 0; }
template <int NSLOT, bool MEM = (NSLOT > 3)>
struct RayStates {
    RayState r[NSLOT];
    __device__ __forceinline__ void init(float4 *, int) {
#pragma unroll
        for (int k = 0; k < NSLOT; ++k) r[k] = RayState{0.0f, 1.0f, 0.0f, 0};
    }
    __device__ __forceinline__ RayState load(float4 *, int sl) const { return r[sl]; }
    __device__ __forceinline__ void store(float4 *, int sl, const RayState &R) { r[sl] = R; }
    __device__ __forceinline__ RayState take(float4 *, int sl) { return r[sl]; }
};
// (ws: the wave's ray-state area; nothing is held in registers between the calls)
template <int NSLOT>
struct RayStates<NSLOT, true> {
    // only the rays that exist: the others' entries must stay zero
    __device__ __forceinline__ void init(float4 *ws, int npix) {
#pragma unroll
        for (int k = 0; k < NSLOT; ++k)
            if (k * 64 + lane_id() < npix) ws[k * 64 + lane_id()] = make_float4(0.0f, 1.0f, 0.0f, 0.0f);
    }
    __device__ __forceinline__ RayState load(float4 *ws, int sl) const {
        const float4 v = ws[sl * 64 + lane_id()];
        return RayState{v.x, v.y, v.z, __float_as_int(v.w)};
    }
    __device__ __forceinline__ void store(float4 *ws, int sl, const RayState &R) {
        ws[sl * 64 + lane_id()] = make_float4(R.tau_thin, R.eps_thick, R.Fh, __int_as_float(R.run_i));
    }
    // the last read, which leaves the area zero
    __device__ __forceinline__ RayState take(float4 *ws, int sl) {
        const RayState R = load(ws, sl);
        ws[sl * 64 + lane_id()] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return R;
    }
};

// One closed segment at R_i (Sec. 4.3.1, 4.3.2): updates the ray's flux and extinction.
__device__ __forceinline__ void integrate_segment(const float *s, int i, float omega, float &tau_thin,
                                                  float &eps_thick, float &Fh) {
    const float R2 = (float)i * (float)i * (float)i * (float)i;
    const float rR2 = rcp(R2);
    const float tt = s[1] * rcp(omega) * rR2;
    float omt = 0.0f, tk = 0.0f, Fk = 0.0f;
    if (s[4] > 0.0f) {
        const float cb = cbrtf(s[4]);
        const float rv = rcp(s[4]);
        omt = s[5] * rv * (cb * cb) * rR2;
        omt = omt > omega ? omega : omt;
        if (omt > 0.0f) tk = s[3] * rcp(omt) * rR2;
        Fk = omt * s[2] * rv;
    }
    const float f = omt * rcp(omega);
    const float phi = tt > 0.0f ? -expm1f(-tt) * rcp(tt) : 1.0f;
    const float Ft = phi * s[0] * rR2 * (0.25f / kPiF);
    const float den = s[1] + f * s[3];
    const float Fs = den > 0.0f ? (Ft * s[1] + Fk * f * s[3]) * rcp(den) : Ft;
    Fh += __expf(-tau_thin) * eps_thick * Fs;
    tau_thin += tt;
    eps_thick *= (1.0f - f) + f * __expf(-tk);
}

// A trace kernel reads its instance's arguments where it uses them (scalar loads from the
// constant address space), not held in scalar registers across the persistent loop: there
// are more of them than registers, and the spilled copies cost vector instructions to
// restore.  SRC says where they are: ARGS_KERNEL, the kernel's only argument, in the
// kernel-argument segment; ARGS_BATCH, descriptor `inst` of the array whose address is
// the first word of the kernel's argument.  The empty asm hides the segment pointer's value
// from the compiler so that the loads stay where they are.
typedef __attribute__((address_space(4))) const TraceArgs *KernArgs;
enum { ARGS_KERNEL = 1, ARGS_BATCH = 2 };
template <int SRC>
__device__ __forceinline__ const TraceArgs &args_at(int inst) {
    typedef __attribute__((address_space(4))) const KernArgs *KernArgsArray;
    if (SRC == ARGS_KERNEL) {
        KernArgs p = (KernArgs)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(p));
        return *(const TraceArgs *)p;
    }
    KernArgsArray pp = (KernArgsArray)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(pp));
    return *(const TraceArgs *)(*pp + __builtin_amdgcn_readfirstlane(inst));
}

template <int NSLOT, bool COUNT, bool LDS_TABLE, int SRC>
__device__ void trace_target(int inst, int ti, char *lds, const uint8_t *tab8, float4 *thick) {
    const TraceArgs &A = args_at<SRC>(inst);
    const LdsLayout LL = lds_layout(A.npix, A.bp, A.kstack, COUNT);
    float *bins = reinterpret_cast<float *>(lds + LL.bins);
    uint32_t *flg = reinterpret_cast<uint32_t *>(lds + LL.flg);
    uint32_t *stk = reinterpret_cast<uint32_t *>(lds + LL.stk);
    int *qnode = reinterpret_cast<int *>(lds + LL.qnode);
    uint32_t *qpk = reinterpret_cast<uint32_t *>(lds + LL.qpk);
    const int lane = lane_id();
    // the target's values are the same on every lane: held in scalar registers
    const int tid = __builtin_amdgcn_readfirstlane(A.targets[ti]);
    const int4 tr = A.nodes[tid];
    const int tx = __builtin_amdgcn_readfirstlane(tr.x & 0xffff), ty = __builtin_amdgcn_readfirstlane(tr.y & 0xffff),
              tz = __builtin_amdgcn_readfirstlane(tr.z);
    const int4 c256 = make_int4(tx * TR_FX, ty * TR_FX, tz * TR_FX, 0);
    const int tdepth = __builtin_amdgcn_readfirstlane((tr.x >> 16) & 15);
    // copies in vector registers for the walk's per-lane differences and comparisons: as
    // scalars they outnumber the scalar registers and come back from spill lanes every step
    int wtx = tx, wty = ty, wtz = tz, wtid = tid;
    asm volatile("" : "+v"(wtx), "+v"(wty), "+v"(wtz), "+v"(wtid));
    const int orient = __builtin_amdgcn_readfirstlane(target_orient(A.orient, A.orient_seed, A.leaf_cell[tid]));
    // the wave's workspace: [npix][bp] thick accumulators, [npix][2] carry slots, then the
    // ray states of wide rays; all of it is zero whenever no target is being traced
    RayStates<NSLOT> RS;
    if (!COUNT) RS.init(thick + A.npix * (A.bp + 2), A.npix);
    int n_b = 0, n_h = 0, n_open = 0;
    const int n_pass = COUNT ? 1 : A.n_pass;
    for (int ps = 0; ps < n_pass; ++ps) {
        const TraceArgs &A = args_at<SRC>(inst);
        Pass P;
        P.a = 1 + ps * A.bp;
        P.b = P.a + A.bp;
        if (P.b > A.n_bins + 1) P.b = A.n_bins + 1;
        const int lo_cut = P.a * P.a, hi_cut = P.b * P.b;
        const int a4 = lo_cut * lo_cut, b4 = hi_cut * hi_cut; // R_a^2, R_b^2 in lattice units
        const bool last = P.b > A.n_bins;
        const bool narrow = P.b - P.a <= 4;
        const PassT PT = pass_thresholds(P.a, P.b);
        // vector copies of the pass's radial bounds for the walk's per-lane test: as scalars
        // they would come back from spill lanes every step
        int wa4 = a4, wb4 = b4;
        asm volatile("" : "+v"(wa4), "+v"(wb4));
        if (!COUNT) {
            const int nf = A.npix * A.bp * kThin;
            for (int k = lane; k < nf; k += 64) bins[k] = 0.0f;
            for (int k = lane; k < flag_words(A.npix, A.bp); k += 64) flg[k] = 0u;
        }
        if (lane == 0) stk[0] = 0u; // the root: first node 0, one node
        int sp = 1, qf = 0, qs = 0; // stack depth, far and near queue lengths
        bool ovf = false;
        wave_sync();
        for (;;) {
            // The three counts are the same on every lane (they change only by ballot
            // counts and kernel arguments); read from the first lane they are scalar values
            // to the compiler too, so the walk's control flow is scalar branches rather than
            // execution-mask updates.  Every lane is active here (top level of the loop).
            sp = __builtin_amdgcn_readfirstlane(sp);
            qf = __builtin_amdgcn_readfirstlane(qf);
            qs = __builtin_amdgcn_readfirstlane(qs);
            if ((sp | qf | qs) == 0) break; // all three are >= 0
            if (sp > 0) {
                const int npop = sp < 8 ? sp : 8;
                const int r = lane >> 3, k = lane & 7;
                const uint32_t rg = r < npop ? stk[sp - 1 - r] : 0u;
                sp -= npop;
                wave_sync();
                const int node = (r < npop && k <= (int)(rg & 7u)) ? (int)(rg >> 3) + k : -1;
                bool open, enq = false, far1 = false;
                uint32_t push, pk = 0;
                {
                    // Every lane takes the same steps and selects by its node's kind instead
                    // of branching (a lane without a node reads the root and keeps nothing).
                    const bool valid = node >= 0;
                    const int nid = valid ? node : 0;
                    const int4 nd = at32(A.nodes, nid);
                    // mapping position, needed by accepted h-nodes: fetched beside the walk
                    // record rather than after the tests that depend on it
                    const int4 pfc = at32(A.pcol, nid);
                    const int depth = (nd.x >> 16) & 15;
                    const bool leaf = (nd.x >> 20) & 1;
                    const bool thick = (nd.x >> 21) & 1;
                    const int s = A.root_edge >> depth;
                    const int vx = (nd.x & 0xffff) - wtx, vy = (nd.y & 0xffff) - wty, vz = nd.z - wtz;
                    // |v| < 2^12, s < 2^12: d2 and s^2 fit 24 bits
                    const int d2 = __mul24(vx, vx) + __mul24(vy, vy) + __mul24(vz, vz);
                    const int s2 = __mul24(s, s);
                    const bool accept = A.wide_open ? (int64_t)s2 * A.th_den2 < (int64_t)A.th_num2 * d2
                                                    : __umul24(s2, A.th_den2) < __umul24(A.th_num2, d2);
                    // (bitwise rather than short-circuit operators: no branches)
                    const bool acc = valid & (leaf ? nid != wtid : accept); // leaves always, but the target
                    const bool opn = valid & !leaf & !accept;
                    n_b += (valid & leaf & (nid != wtid)) ? 1 : 0;
                    n_h += (valid & !leaf & accept) ? 1 : 0;
                    n_open += opn ? 1 : 0;
                    const int ext = (acc & thick & (A.merge != 0)) ? (s >> 1) : 0;
                    // One box test serves both kinds of node (a lane is opened or accepted, not
                    // both), in lattice units with R_i = i^2:
                    //  - an opened h-node keeps its subtree when r_max + s/4 >= R_a and
                    //    r_min - s/4 < R_b, with r over the node cube (half edge s/2) and the
                    //    s/4 only when the subtree holds thick content to be merged;
                    //  - an accepted node can reach the pass when r_max >= R_a and r_min < R_b:
                    //    its mapping position lies in its cube (a leaf's is its centre, half
                    //    edge 0), and thick material reaches a further s/2 for the merge flags.
                    //    For a leaf with no extent the test is exact.
                    const int he = opn ? (s >> 1) : (leaf ? 0 : (s >> 1)) + ext;
                    const int ax = abs(vx), ay = abs(vy), az = abs(vz);
                    const int nx = max(ax - he, 0), ny = max(ay - he, 0), nz = max(az - he, 0);
                    const int fx = ax + he, fy = ay + he, fz = az + he;
                    const int rmin2 = __mul24(nx, nx) + __mul24(ny, ny) + __mul24(nz, nz);
                    const int rmax2 = __mul24(fx, fx) + __mul24(fy, fy) + __mul24(fz, fz);
                    bool keep = true;
                    if (!COUNT) {
                        // the s/4 margin covers the merge extents of thick descendants; a
                        // subtree without thick content keeps exactly its cube's range
                        const int q4 = (thick & (A.merge != 0)) ? s >> 2 : 0;
                        const int lo = lo_cut - q4, hi = hi_cut + q4;
                        keep = !((lo > 0) & (rmax2 < __mul24(lo, lo))) & (last | (rmin2 < __mul24(hi, hi)));
                    }
                    open = opn & keep;
                    push = ((uint32_t)nd.w << 3) | (uint32_t)(__builtin_popcount((nd.y >> 16) & 255) - 1);
                    if (!COUNT) {
                        const bool maybe = acc & (rmax2 >= wa4) & (last | (rmin2 < wb4));
                        const int dx = leaf ? vx * TR_FX : pfc.x - c256.x;
                        const int dy = leaf ? vy * TR_FX : pfc.y - c256.y;
                        const int dz = leaf ? vz * TR_FX : pfc.z - c256.z;
                        const int log2s = (31 - __clz(A.root_edge)) - depth;
                        SegHit h;
                        int c;
                        if (ext == 0 && narrow) {
                            // r^2 exact in FP64 (a leaf's is 2^16 d2); the class is its binary
                            // exponent
                            const double r2 = (double)dx * dx + (double)dy * dy + (double)dz * dz;
                            h.content = (r2 >= PT.ta) & (last | (r2 < PT.tb));
                            h.k0 = h.k1 = 0;
                            h.i = P.a + (r2 >= PT.t1 ? 1 : 0) + (r2 >= PT.t2 ? 1 : 0) + (r2 >= PT.t3 ? 1 : 0);
                            c = (__builtin_amdgcn_frexp_exp(r2) - 1) - 2 * (8 + log2s);
                        } else {
                            h = seg_hit(dx, dy, dz, s, ext, P.a, P.b, last, A.n_bins);
                            c = dist_class(dx, dy, dz, log2s);
                        }
                        enq = maybe & (h.content | (h.k1 > h.k0));
                        far1 = enq & (A.per_node == 0) & (c >= kAlphaFar);
                        pk = (h.content ? (uint32_t)(h.i - P.a + 1) : 0u) | ((uint32_t)h.k0 << 6) |
                             ((uint32_t)h.k1 << 12) | ((leaf ? 1u : 0u) << 18) | ((uint32_t)depth << 19) |
                             ((thick ? 1u : 0u) << 23) |
                             (far1 ? (uint32_t)(c < kAlphaMax ? c : kAlphaMax) << 24 : 0u);
                    }
                }
                const uint64_t bal = __ballot(open);
                const int pos = count_below(bal);
                const int npush = __builtin_popcountll(bal);
                if (open && sp + pos < A.kstack) stk[sp + pos] = push;
                // an overflow drops the pushes past the stack and is reported once per pass
                ovf |= sp + npush > A.kstack;
                sp = min(sp + npush, A.kstack);
                if (!COUNT) {
                    const uint64_t fb = __ballot(enq && far1), gb = __ballot(enq && !far1);
                    if (enq) {
                        const int qp = far1 ? qf + count_below(fb) : kQueue - 1 - qs - count_below(gb);
                        qnode[qp] = node;
                        qpk[qp] = pk;
                    }
                    qf += __builtin_popcountll(fb);
                    qs += __builtin_popcountll(gb);
                }
                wave_sync();
            }
            if (COUNT) continue;
            // map full batches, or whatever is left once the walk of the pass is done
            if (qf >= 64 || (sp == 0 && qf > 0)) {
                const int nq = qf >= 64 ? 64 : qf;
                const int e = qf - nq + (lane < nq ? lane : 0);
                map_queue<LDS_TABLE, true>(A, e, lane < nq, qnode, qpk, P.a, c256, tdepth, orient, tab8, bins, flg, thick);
                qf -= nq;
                wave_sync();
            }
            if (qs >= 64 || (sp == 0 && qs > 0)) {
                const int nq = qs >= 64 ? 64 : qs;
                const int e = kQueue - qs + (lane < nq ? lane : 0);
                map_queue<LDS_TABLE, false>(A, e, lane < nq, qnode, qpk, P.a, c256, tdepth, orient, tab8, bins, flg, thick);
                qs -= nq;
                wave_sync();
            }
        }
        if (ovf && lane == 0) atomicOr(A.err, 4);
        if (COUNT) break;
        // the thick accumulators' atomics of every lane have been performed at the device
        // cache before any lane reads them back
        __threadfence_block();
        // integrate the pass's segments outwards, one lane per ray
#pragma unroll
        for (int sl = 0; sl < NSLOT; ++sl) {
            const int h = lane + 64 * sl;
            if (h >= A.npix) continue;
            RayState R = RS.load(thick + A.npix * (A.bp + 2), sl);
            const bool half = A.bp <= 8;
            const uint32_t fl = half ? (flg[h >> 1] >> ((h & 1) << 4)) & 0xffffu : flg[h];
            const int tsh = half ? 8 : 16;
            float4 *carry = thick + A.npix * A.bp + 2 * h;
            float acc[kFields] = {0, 0, 0, 0, 0, 0};
            if (R.run_i != 0) {
                // take the carried content and clear the slots: the accumulator memory is
                // all-zero whenever no target is being traced
                const float4 c0 = carry[0], c1 = carry[1];
                acc[0] = c0.x; acc[1] = c0.y; acc[2] = c0.z; acc[3] = c0.w; acc[4] = c1.x; acc[5] = c1.y;
                carry[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                carry[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
            for (int i = P.a; i < P.b; ++i) {
                const float *th = bins + (h * A.bp + (i - P.a)) * kThin;
                float v[kFields] = {th[0], th[1], 0.0f, 0.0f, 0.0f, 0.0f};
                if ((fl >> (tsh + i - P.a)) & 1u) {
                    // read and clear the segment's thick content
                    float *tk = reinterpret_cast<float *>(thick + h * A.bp + (i - P.a));
#pragma unroll
                    for (int f = 0; f < 4; ++f) v[2 + f] = atomicExch(tk + f, 0.0f);
                }
                if (R.run_i == 0) {
                    R.run_i = i;
#pragma unroll
                    for (int f = 0; f < kFields; ++f) acc[f] = v[f];
                } else {
                    // inverse-square content moves to the merged segment's R_i
                    const float T = (float)R.run_i * rcp((float)i);
                    const float T4 = (T * T) * (T * T);
                    acc[0] += T4 * v[0];
                    acc[1] += T4 * v[1];
                    acc[2] += v[2];
                    acc[3] += v[3];
                    acc[4] += v[4];
                    acc[5] += T4 * v[5];
                }
                const bool link = ((fl >> (i - P.a)) & 1u) && i < A.n_bins;
                if (!link) {
                    integrate_segment(acc, R.run_i, A.omega, R.tau_thin, R.eps_thick, R.Fh);
                    R.run_i = 0;
                }
            }
            if (R.run_i != 0) {
                // a merged segment still open at the pass end continues in the next pass
                carry[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
                carry[1] = make_float4(acc[4], acc[5], 0.0f, 0.0f);
            }
            RS.store(thick + A.npix * (A.bp + 2), sl, R);
        }
        wave_sync();
    }
    const int cell = A.leaf_cell[tid];
    if (COUNT) {
        for (int o = 32; o > 0; o >>= 1) {
            n_b += __shfl_xor(n_b, o);
            n_h += __shfl_xor(n_h, o);
            n_open += __shfl_xor(n_open, o);
        }
        if (lane == 0) {
            A.counters[3 * (int64_t)cell] = n_b;
            A.counters[3 * (int64_t)cell + 1] = n_h;
            A.counters[3 * (int64_t)cell + 2] = n_open;
        }
        return;
    }
    // finalisation (Sec. 4.4): F = -sum F^h n^h, J = sum F^h / 4 pi + J_src
    float js = 0.0f, fx = 0.0f, fy = 0.0f, fz = 0.0f;
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) {
        const int h = lane + 64 * sl;
        if (h >= A.npix) continue;
        const RayState R = RS.take(thick + A.npix * (A.bp + 2), sl);
        const float Fh = R.Fh + __expf(-R.tau_thin) * R.eps_thick * A.omega * A.j_bg;
        const float4 n = A.dirs[h];
        js += Fh;
        fx -= Fh * n.x;
        fy -= Fh * n.y;
        fz -= Fh * n.z;
    }
    for (int o = 32; o > 0; o >>= 1) {
        js += __shfl_xor(js, o);
        fx += __shfl_xor(fx, o);
        fy += __shfl_xor(fy, o);
        fz += __shfl_xor(fz, o);
    }
    if (lane == 0) {
        const float src = A.cell_src[cell];
        float Jv = js * (0.25f / kPiF);
        if (src > 0.0f) {
            const float e = (float)(A.root_edge >> ((tr.x >> 16) & 15));
            Jv += -expm1f(-0.5f * A.cell_tau[cell]) * src / (4.0f * kPiF * (e * e));
        }
        orient_back(orient, fx, fy, fz); // the flux back to the grid's axes
        A.J[cell] = Jv;
        A.F[cell] = fx;
        A.F[A.n_cells + cell] = fy;
        A.F[2 * A.n_cells + cell] = fz;
        if (A.u_rad) A.u_rad[cell] = 4.0f * kPiF * Jv / A.c_light;
    }
}

// wide rays (12 per lane): three waves per SIMD, which their ray states' leaving the
// registers allows (168 VGPRs)
template <int NSLOT, bool COUNT, bool LDS_TABLE>
__global__ __launch_bounds__(NSLOT > 3 ? 256 : 1024) __attribute__((amdgpu_waves_per_eu(NSLOT > 3 ? 3 : 1)))
void k_trace(TraceArgs A) {
    extern __shared__ __align__(16) char smem[];
    const uint8_t *tab8 = reinterpret_cast<const uint8_t *>(smem);
    const int ncell = 6 << (2 * A.log2m);

    if (LDS_TABLE) {
        uint8_t *t = reinterpret_cast<uint8_t *>(smem);
        for (int k = threadIdx.x; k < ncell; k += blockDim.x) t[k] = (uint8_t)A.table[k];

        __syncthreads();
    }
    char *lds = smem + A.lds_table + (threadIdx.x >> 6) * A.lds_wave;
    float4 *thick = COUNT ? nullptr
                          : A.thick + (int64_t)(blockIdx.x * A.per_block + (threadIdx.x >> 6)) *
                                          (A.npix * (A.bp + 2) + ray_state_floats4(NSLOT));
    // XCD-aware work distribution: blocks are dispatched round-robin over the 8 XCDs, so
    // block b runs on XCD b % 8; each XCD takes targets from its own contiguous range of
    // the (Morton-ordered) target list and keeps that region of the tree in its L2.  A
    // wave whose range is exhausted helps the next XCD's range.
    const int home = blockIdx.x & 7;
    const int per = (A.n_targets + 7) >> 3;
    for (int x = 0; x < 8; ++x) {
        const int r = (home + x) & 7;
        const int lo = r * per;
        const int hi = min(lo + per, A.n_targets);
        for (;;) {
            int t0 = 0;
            if (lane_id() == 0) t0 = atomicAdd(A.work + r, A.chunk);
            t0 = __builtin_amdgcn_readfirstlane(t0) + lo;
            if (t0 >= hi) break;
            const int t1 = t0 + A.chunk < hi ? t0 + A.chunk : hi;
            for (int ti = t0; ti < t1; ++ti) trace_target<NSLOT, COUNT, LDS_TABLE, ARGS_KERNEL>(0, ti, lds, tab8, thick);
        }
    }
}

// Batched launch: many trees (instances) in one persistent grid.  The targets of all
// instances form one index space (prefix sums `start`, optionally every `stride`-th
// target); waves take chunks of it exactly as in k_trace and trace each target with its
// instance's arguments.  The LDS holds one copy of every distinct direction-cell table of
// the batch.
constexpr int kMaxTabs = 4;

struct BatchArgs {
    const TraceArgs *__restrict__ inst; // [n_inst]; the first member (read through the kernel
                                        // argument segment's first word by the trace)
    const int *start;      // [n_inst + 1]
    int n_inst;
    int n_total;
    int stride;
    int *work;
    int chunk;
    int per_block;
    int lds_wave;
    int lds_table;
    int n_tab;
    const int16_t *tab[kMaxTabs];
    int tab_off[kMaxTabs];
    int tab_ncell[kMaxTabs];
    float4 *thick;
    int thick_wave; // float4 per wave
};

template <int NSLOT, bool LDS_TABLE>
__global__ __launch_bounds__(NSLOT > 3 ? 256 : 1024) __attribute__((amdgpu_waves_per_eu(NSLOT > 3 ? 3 : 1)))
void k_trace_batch(BatchArgs B) {
    extern __shared__ __align__(16) char smem[];
    if (LDS_TABLE) {
        for (int s = 0; s < B.n_tab; ++s) {
            uint8_t *t = reinterpret_cast<uint8_t *>(smem) + B.tab_off[s];
            const int nc = B.tab_ncell[s];
            for (int k = threadIdx.x; k < nc; k += blockDim.x) t[k] = (uint8_t)B.tab[s][k];
        }
        __syncthreads();
    }
    char *lds = smem + B.lds_table + (threadIdx.x >> 6) * B.lds_wave;
    float4 *thick = B.thick + (int64_t)(blockIdx.x * B.per_block + (threadIdx.x >> 6)) * B.thick_wave;
    const int home = blockIdx.x & 7;
    const int per = (B.n_total + 7) >> 3;
    for (int x = 0; x < 8; ++x) {
        const int r = (home + x) & 7;
        const int lo = r * per;
        const int hi = min(lo + per, B.n_total);
        for (;;) {
            int t0 = 0;
            if (lane_id() == 0) t0 = atomicAdd(B.work + r, B.chunk);
            t0 = __builtin_amdgcn_readfirstlane(t0) + lo;
            if (t0 >= hi) break;
            const int t1 = t0 + B.chunk < hi ? t0 + B.chunk : hi;
            for (int ti = t0; ti < t1; ++ti) {
                // the instance holding global target ti: start[k] <= ti < start[k + 1]
                int a = 0, b = B.n_inst;
                while (b - a > 1) {
                    const int m = (a + b) >> 1;
                    if (B.start[m] <= ti) a = m; else b = m;
                }
                const int k = __builtin_amdgcn_readfirstlane(a);
                const TraceArgs &A = B.inst[k];
                const uint8_t *tab8 = reinterpret_cast<const uint8_t *>(smem) + B.tab_off[A.tab_slot];
                trace_target<NSLOT, false, LDS_TABLE, ARGS_BATCH>(k, (ti - B.start[k]) * B.stride, lds, tab8, thick);
            }
        }
    }
}

__global__ void k_zero_int(int *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_zero_f32(float *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// Radiation pressure (Sec. 4.5)
__global__ void k_rad_force(int64_t n, const float *__restrict__ F, const float *__restrict__ kap,
                            const float *__restrict__ tau, const float *__restrict__ src,
                            const int32_t *__restrict__ node_of_cell, const uint32_t *__restrict__ meta,
                            int root_edge, float c_light, float *__restrict__ a, float *__restrict__ p_src) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const float t = tau[c];
    const float fac = t < 1e-4f ? 1.0f : -expm1f(-t) / t;
    const float k = kap[c] * fac / c_light;
    a[c] = k * F[c];
    a[n + c] = k * F[n + c];
    a[2 * n + c] = k * F[2 * n + c];
    if (p_src) {
        const float s = src[c];
        float ps = 0.0f;
        if (s > 0.0f) {
            const float e = (float)(root_edge >> (meta[node_of_cell[c]] & 15u));
            ps = -expm1f(-0.5f * t) * s / (c_light * (e * e));
        }
        p_src[c] = ps;
    }
}

// Validated set-up of one traced tree: the knob-independent kernel arguments.
struct Inst {
    TraceArgs A;
    RayTable *rt = nullptr;
    int M = 0, npix = 0;
};

constexpr int kLdsCu = 160 * 1024;

int table_bytes(int M) { return (6 * M * M + 15) & ~15; }
int max_waves_for(int npix) { return npix > 192 ? 4 : 16; } // the kernel's launch bound
// waves a CU should hold at once; passes are sized so that this many waves share the CU's
// LDS.  Wide rays (168 VGPRs, three waves per SIMD): 12, one segment per pass on the 128^3
// core (8.8 s, against 10.6 s for 2 segments and 8 waves, which the registers allowed
// before the ray states left them).  Otherwise 16, four per SIMD, the most the registers
// allow.  Each pass re-walks the tree, so the LDS left beside the bins decides the walk's
// cost: with two rays per flag word and no far-node offsets in the queue, the 128^3 core
// and the AMR 256^3-equivalent tree take 4 segments per pass at 16 waves (1.39 s and
// 1.91 s, against 1.42 s and 2.00 s with 3).
int waves_cu_for(int npix) { return npix > 192 ? 12 : 16; }
int nslot_for(int npix) { return npix <= 64 ? 1 : (npix <= 192 ? 3 : 12); }
// the one-wave kernels keep the pixel table in LDS for up to 64 rays (N_side <= 2, at most
// 6 KB); beyond that only near nodes read it, from global memory, and the LDS holds more
// segments per pass instead
bool table_in_lds(int npix) { return npix <= 64; }

int setup_instance(tr_ctx *ctx, const tr_tree *t, const tr_trace_params *p, float *J, float *F, float *u_rad,
                   int32_t *counters, bool count, Inst &I) {
    if (!t || !p) return tr_fail(ctx, TR_EINVAL, "trace: null argument");
    if (!count && (!J || !F)) return tr_fail(ctx, TR_EINVAL, "trace: null output");
    const int ns = p->n_side;
    if (ns != 1 && ns != 2 && ns != 4 && ns != 8)
        return tr_fail(ctx, TR_EINVAL, "n_side must be 1, 2, 4 or 8 (got %d)", ns);
    int64_t num = p->theta_num, den = p->theta_den;
    if (num == 0 && den == 0) { num = 1; den = 2 * ns; }
    if (num < 0 || den <= 0 || num > 1024 || den > 1024)
        return tr_fail(ctx, TR_EINVAL, "bad opening angle %lld/%lld", (long long)num, (long long)den);
    const int M = p->cube_m ? p->cube_m : 16 * ns;
    if (M < 2 || M > 256 || (M & (M - 1)))
        return tr_fail(ctx, TR_EINVAL, "cube_m must be a power of two in [2, 256]");
    int log2m = 0;
    while ((1 << log2m) < M) ++log2m;
    if (t->n_bins > 63) return tr_fail(ctx, TR_EINVAL, "too many ray segments (%d)", t->n_bins);
    if (t->n_node >= ((int64_t)1 << 29)) return tr_fail(ctx, TR_EINVAL, "too many nodes for the walk stack");
    if (t->root_edge > 2048) return tr_fail(ctx, TR_EINVAL, "grid too fine for the walk's integer ranges");
    if (t->n_node >= ((int64_t)1 << 28))
        return tr_fail(ctx, TR_EINVAL, "tree of %lld nodes: the trace addresses node records with 32-bit offsets "
                       "(at most 2^28 nodes)", (long long)t->n_node);
    if (t->n_cells >= ((int64_t)1 << 31)) return tr_fail(ctx, TR_EINVAL, "too many cells");
    if (t->ctx != ctx && t->ctx && t->ctx->device != ctx->device)
        return tr_fail(ctx, TR_EINVAL, "tree lives on another device");
    int rc = tr_get_table(ctx, ns, M, &I.rt);
    if (rc) return rc;
    I.M = M;
    I.npix = 12 * ns * ns;
    TraceArgs &A = I.A;
    A = TraceArgs{};
    A.nodes = t->packed; A.q = t->q; A.pcol = t->pcol;
    A.targets = t->targets; A.leaf_cell = t->leaf_cell; A.cell_tau = t->cell_tau; A.cell_src = t->cell_src;
    A.table = I.rt->table; A.alpha = I.rt->alpha; A.alpha_c1 = I.rt->alpha_c1; A.dirs = I.rt->dirs;
    A.near = I.rt->near;
    A.per_node = p->per_node_kernel ? 1 : 0;
    A.work = ctx->d_ctl; A.err = ctx->d_ctl + 16;
    A.J = J; A.F = F; A.u_rad = u_rad; A.counters = counters;
    A.n_cells = t->n_cells; A.n_targets = (int)t->n_cells; A.root_edge = (int)t->root_edge;
    A.npix = I.npix; A.log2m = log2m; A.n_bins = t->n_bins;
    A.merge = p->merge ? 1 : 0;
    A.th_num2 = (int)(num * num); A.th_den2 = (int)(den * den);
    // 32-bit products are exact when num^2 d^2 and den^2 s^2 stay below 2^31, and take the
    // 24-bit multiplier when every factor is below 2^24 (d^2 < 3 * 2048^2 always is)
    const int64_t max_d2 = 3 * t->root_edge * t->root_edge, max_s2 = t->root_edge * t->root_edge;
    A.wide_open = (num * num * max_d2 >= ((int64_t)1 << 31) || den * den * max_s2 >= ((int64_t)1 << 31) ||
                   num * num >= ((int64_t)1 << 24) || den * den >= ((int64_t)1 << 24)) ? 1 : 0;
    A.omega = (float)(4.0 * 3.14159265358979323846 / I.npix);
    A.j_bg = p->j_bg;
    A.c_light = (float)t->c_light;
    if (p->stack_limit < 0) return tr_fail(ctx, TR_EINVAL, "stack_limit must be >= 0");
    A.kstack = stack_size(t->D);
    if (p->stack_limit > 0 && p->stack_limit < A.kstack) A.kstack = p->stack_limit < 9 ? 9 : p->stack_limit;
    A.tab_slot = 0;
    if (p->orientation < -1 || p->orientation > 47)
        return tr_fail(ctx, TR_EINVAL, "orientation must be -1 (per target) or 0..47");
    A.orient = p->orientation;
    A.orient_seed = p->orient_seed;
    return TR_OK;
}

// segments per pass of one instance under a requested value (0 = automatic: the longest
// pass that lets waves_cu waves share the CU's LDS next to `lds_table` bytes of tables)
int choose_bp(const Inst &I, int want, int lds_table, int waves_cu, bool count) {
    int bp = want;
    if (bp <= 0) {
        bp = I.A.n_bins < kMaxBp ? I.A.n_bins : kMaxBp;
        while (bp > 1 && lds_table + waves_cu * lds_layout(I.npix, bp, I.A.kstack, count).total > kLdsCu) --bp;
    }
    if (bp > I.A.n_bins) bp = I.A.n_bins;
    if (bp > kMaxBp) bp = kMaxBp;
    if (bp < 1) bp = 1;
    return bp;
}

void set_bp(Inst &I, int bp, bool count) {
    I.A.bp = bp;
    I.A.n_pass = (int)tr_div_up(I.A.n_bins, bp);
    I.A.lds_wave = lds_layout(I.npix, bp, I.A.kstack, count).total;
}

// grow-only per-wave thick-content accumulators, kept all-zero between uses
int ensure_thick(tr_ctx *ctx, int64_t need) {
    if (ctx->ws_thick_n >= need) return TR_OK;
    hipFree(ctx->ws_thick);
    ctx->ws_thick = nullptr;
    ctx->ws_thick_n = 0;
    if (hipMalloc(&ctx->ws_thick, sizeof(float4) * need) != hipSuccess)
        return tr_fail(ctx, TR_ENOMEM, "thick-content accumulators (%lld bytes)", (long long)(sizeof(float4) * need));
    k_zero_f32<<<(int)tr_div_up(4 * need, 256 * 64), 256, 0, ctx->stream>>>(reinterpret_cast<float *>(ctx->ws_thick),
                                                                           4 * need);
    ctx->ws_thick_n = need;
    return TR_OK;
}

int launch_trace(tr_ctx *ctx, const tr_tree *t, const tr_trace_params *p, float *J, float *F,
                 float *u_rad, int32_t *counters, bool count) {
    if (!ctx) return TR_EINVAL;
    TR_HIP(ctx, hipSetDevice(ctx->device));
    Inst I;
    int rc = setup_instance(ctx, t, p, J, F, u_rad, counters, count, I);
    if (rc) return rc;
    if (p->kernel == 2)
        return tr_fail(ctx, TR_EINVAL, "kernel 2 (one block of waves per target) is withdrawn: the one-wave kernel "
                       "(0 or 1) was faster on every workload measured");
    if (p->kernel < 0 || p->kernel > 1) return tr_fail(ctx, TR_EINVAL, "kernel must be 0 or 1");
    const int npix = I.npix;
    const bool tab_lds = !count && table_in_lds(npix);
    const int lds_table = tab_lds ? table_bytes(I.M) : 0;
    const int max_waves = max_waves_for(npix);
    set_bp(I, choose_bp(I, p->bins_per_pass, lds_table, waves_cu_for(npix), count), count);
    TraceArgs &A = I.A;
    A.chunk = p->chunk > 0 ? p->chunk : 1; // one target per grab: a short tail (128^3 core: 1.59 s, 1.61 s with 4)
    A.lds_table = lds_table;
    // waves per block: as many as fit in the CU's LDS together with the shared tables
    int per_block = p->waves_per_block > 0 ? p->waves_per_block : (kLdsCu - lds_table) / A.lds_wave;
    if (per_block > max_waves) per_block = max_waves;
    if (per_block < 1) per_block = 1;
    A.per_block = per_block;
    const size_t lds = (size_t)lds_table + (size_t)per_block * A.lds_wave;
    if (lds > (size_t)kLdsCu) return tr_fail(ctx, TR_EINVAL, "LDS per block too large (%zu bytes)", lds);
    // one block per CU when the tables sit in LDS; otherwise as many blocks as fit
    int blocks_cu = tab_lds ? 1 : (int)(kLdsCu / lds);
    if (blocks_cu > 8) blocks_cu = 8;
    const int grid = ctx->n_cu * blocks_cu;
    A.thick = nullptr;
    if (!count) {
        rc = ensure_thick(ctx, (int64_t)grid * per_block * (npix * (A.bp + 2) + ray_state_floats4(nslot_for(npix))));
        if (rc) return rc;
        A.thick = ctx->ws_thick;
    }
    k_zero_int<<<1, 64, 0, ctx->stream>>>(ctx->d_ctl, 8);
    const dim3 blk(64 * per_block);
#define LAUNCH(NS_, C_, T_) hipLaunchKernelGGL((k_trace<NS_, C_, T_>), dim3(grid), blk, lds, ctx->stream, A)
    if (count) {
        LAUNCH(1, true, false);
    } else if (nslot_for(npix) == 1) {
        LAUNCH(1, false, true);
    } else if (nslot_for(npix) == 3) {
        LAUNCH(3, false, false);
    } else {
        LAUNCH(12, false, false);
    }
#undef LAUNCH
    if (hipGetLastError() != hipSuccess) return tr_fail(ctx, TR_EHIP, "trace kernel launch failed");
    return TR_OK;
}

// ---------------------------------------------------------------------------------------
// Batched launches
// ---------------------------------------------------------------------------------------
struct Knobs {
    int bp = 0, waves = 0, chunk = 0;
};

// Per-node angular kernel of the leaves of a target's own size within 7 edges of it
// (RayTable::near), built with the mapping's own direction cells.  Offsets are in units of
// one edge (s = 1): the direction cells of the sub-points d +- s/4 do not change when d and
// s scale together, since the cell index is an exact quotient of two of their components.
__global__ void k_near_table(int log2m, const int16_t *__restrict__ table, int4 *__restrict__ near) {
    const int key = blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= 15 * 15 * 15) return;
    const int mx = key / 225 - 7, my = (key / 15) % 15 - 7, mz = key % 15 - 7;
    const int h = TR_FX / 4;
    int pix[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int cx = TR_FX * mx + ((k & 1) ? h : -h), cy = TR_FX * my + ((k & 2) ? h : -h),
                  cz = TR_FX * mz + ((k & 4) ? h : -h);
        pix[k] = table[cube_cell(cx, cy, cz, log2m)];
    }
    uint32_t starts = 0;
    sort8_runs(pix, true, starts);
    near[key] = make_int4(pix[0] | (pix[1] << 10) | (pix[2] << 20), pix[3] | (pix[4] << 10) | (pix[5] << 20),
                          pix[6] | (pix[7] << 10), (int)starts);
}

} // namespace

int tr_build_near_table(tr_ctx *ctx, RayTable &rt, int log2m) {
    const int n = 15 * 15 * 15;
    if (hipMalloc(&rt.near, sizeof(int4) * n) != hipSuccess) {
        rt.near = nullptr;
        return tr_fail(ctx, TR_ENOMEM, "near-leaf pixel table");
    }
    k_near_table<<<tr_div_up(n, 256), 256, 0, ctx->stream>>>(log2m, rt.table, rt.near);
    TR_HIP(ctx, hipGetLastError());
    return TR_OK;
}

struct tr_batch {
    tr_ctx *ctx = nullptr;
    std::vector<Inst> inst;
    std::vector<int> start;   // prefix of target counts
    TraceArgs *d_inst = nullptr;
    int *d_start = nullptr;   // [2][n + 1]: all targets, then the tuner's sample
    int sample_stride = 0;
    std::vector<std::pair<int, int>> tabs; // (n_side, M) of each LDS table slot
    int nslot = 1;
    bool tab_lds = true;
    int lds_table = 0;
    Knobs knobs;
    BatchArgs B{};
    int grid = 0;
    size_t lds = 0;
    float4 *thick = nullptr;
    int64_t thick_n = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float tuned_ms = 0.0f;
};

namespace {

int batch_configure(tr_batch *b, Knobs k) {
    tr_ctx *ctx = b->ctx;
    int max_npix = 0;
    for (auto &I : b->inst) max_npix = I.npix > max_npix ? I.npix : max_npix;
    const int max_waves = max_waves_for(max_npix);
    int lds_wave = 16, thick_wave = 0;
    for (auto &I : b->inst) {
        set_bp(I, choose_bp(I, k.bp, b->lds_table, waves_cu_for(max_npix), false), false);
        lds_wave = I.A.lds_wave > lds_wave ? I.A.lds_wave : lds_wave;
        thick_wave = I.npix * (I.A.bp + 2) > thick_wave ? I.npix * (I.A.bp + 2) : thick_wave;
    }
    thick_wave += ray_state_floats4(b->nslot); // the ray states of wide rays
    int per_block = k.waves > 0 ? k.waves : (kLdsCu - b->lds_table) / lds_wave;
    if (per_block > max_waves) per_block = max_waves;
    if (per_block < 1) return tr_fail(ctx, TR_EINVAL, "batch: LDS too small for one wave (%d + %d bytes)",
                                      b->lds_table, lds_wave);
    const size_t lds = (size_t)b->lds_table + (size_t)per_block * lds_wave;
    if (lds > (size_t)kLdsCu) return tr_fail(ctx, TR_EINVAL, "batch: LDS per block too large (%zu bytes)", lds);
    int blocks_cu = b->tab_lds ? 1 : (int)(kLdsCu / lds);
    if (blocks_cu > 8) blocks_cu = 8;
    const int grid = ctx->n_cu * blocks_cu;
    const int64_t need = (int64_t)grid * per_block * thick_wave;
    if (b->thick_n < need) {
        TR_HIP(ctx, hipStreamSynchronize(ctx->stream));
        hipFree(b->thick);
        b->thick = nullptr;
        b->thick_n = 0;
        if (hipMalloc(&b->thick, sizeof(float4) * need) != hipSuccess)
            return tr_fail(ctx, TR_ENOMEM, "batch thick-content accumulators");
        k_zero_f32<<<(int)tr_div_up(4 * need, 256 * 64), 256, 0, ctx->stream>>>(reinterpret_cast<float *>(b->thick),
                                                                               4 * need);
        b->thick_n = need;
    }
    std::vector<TraceArgs> h(b->inst.size());
    for (size_t i = 0; i < b->inst.size(); ++i) {
        h[i] = b->inst[i].A;
        h[i].per_block = per_block;
        h[i].thick = b->thick;
        h[i].lds_table = b->lds_table;
    }
    TR_HIP(ctx, hipMemcpyAsync(b->d_inst, h.data(), sizeof(TraceArgs) * h.size(), hipMemcpyHostToDevice, ctx->stream));
    TR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    BatchArgs &B = b->B;
    B.inst = b->d_inst;
    B.n_inst = (int)b->inst.size();
    B.work = ctx->d_ctl;
    B.chunk = k.chunk > 0 ? k.chunk : 1;
    B.per_block = per_block;
    B.lds_wave = lds_wave;
    B.lds_table = b->lds_table;
    B.thick = b->thick;
    B.thick_wave = thick_wave;
    b->knobs = k;
    b->grid = grid;
    b->lds = lds;
    return TR_OK;
}

// one persistent launch on stream st over all targets (stride 1) or the tuner's sample
int batch_enqueue(tr_batch *b, hipStream_t st, bool sample) {
    BatchArgs B = b->B;
    const int n = (int)b->inst.size();
    B.start = b->d_start + (sample ? n + 1 : 0);
    B.stride = sample ? b->sample_stride : 1;
    if (sample) {
        int tot = 0;
        for (auto &I : b->inst) tot += (int)tr_div_up(I.A.n_targets, b->sample_stride);
        B.n_total = tot;
    } else {
        B.n_total = b->start.back();
    }
    k_zero_int<<<1, 64, 0, st>>>(b->ctx->d_ctl, 8);
    const dim3 blk(64 * B.per_block);
#define LAUNCHB(NS_, T_) hipLaunchKernelGGL((k_trace_batch<NS_, T_>), dim3(b->grid), blk, b->lds, st, B)
    if (b->nslot == 1) {
        LAUNCHB(1, true);
    } else if (b->nslot == 3) {
        LAUNCHB(3, false);
    } else {
        LAUNCHB(12, false);
    }
#undef LAUNCHB
    if (hipGetLastError() != hipSuccess) return tr_fail(b->ctx, TR_EHIP, "batched trace launch failed");
    return TR_OK;
}

// the batch's current setting as tr_batch_tuning: the knobs as set (0 = automatic) and the
// widest pass any instance takes under them
void batch_report(const tr_batch *b, float ms, tr_batch_tuning *out) {
    int bp = 1;
    for (auto &I : b->inst) bp = I.A.bp > bp ? I.A.bp : bp;
    out->bins_per_pass = b->knobs.bp;
    out->waves_per_block = b->knobs.waves;
    out->chunk = b->knobs.chunk;
    out->sample_ms = ms;
    out->widest_pass = bp;
    out->waves_used = b->B.per_block;
}

void batch_drop_graph(tr_batch *b) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

int batch_capture(tr_batch *b) {
    tr_ctx *ctx = b->ctx;
    batch_drop_graph(b);
    if (!b->cap) TR_HIP(ctx, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    TR_HIP(ctx, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const int rc = batch_enqueue(b, b->cap, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc) {
        if (g) hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) return tr_fail(ctx, TR_EHIP, "batch graph capture failed");
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        batch_drop_graph(b);
        return tr_fail(ctx, TR_EHIP, "batch graph instantiation failed");
    }
    return TR_OK;
}

void batch_release(tr_batch *b) {
    if (!b) return;
    if (b->ctx) {
        hipSetDevice(b->ctx->device);
        hipStreamSynchronize(b->ctx->stream);
    }
    batch_drop_graph(b);
    if (b->cap) hipStreamDestroy(b->cap);
    hipFree(b->d_inst);
    hipFree(b->d_start);
    hipFree(b->thick);
    delete b;
}

int batch_build(tr_ctx *ctx, int n, const tr_tree *const *trees, const tr_trace_params *p, float *const *J,
                float *const *F, float *const *u_rad, tr_batch **out) {
    if (!ctx) return TR_EINVAL;
    if (!out || n < 1 || !trees || !p || !J || !F) return tr_fail(ctx, TR_EINVAL, "batch: bad argument");
    *out = nullptr;
    TR_HIP(ctx, hipSetDevice(ctx->device));
    tr_batch *b = new tr_batch;
    b->ctx = ctx;
    b->inst.resize(n);
    b->start.assign(n + 1, 0);
    int64_t tot = 0;
    int max_npix = 0;
    for (int i = 0; i < n; ++i) {
        int rc = setup_instance(ctx, trees[i], p + i, J[i], F[i], u_rad ? u_rad[i] : nullptr, nullptr, false,
                                b->inst[i]);
        if (rc) {
            batch_release(b);
            return rc;
        }
        Inst &I = b->inst[i];
        tot += I.A.n_targets;
        if (tot >= ((int64_t)1 << 31)) {
            batch_release(b);
            return tr_fail(ctx, TR_EINVAL, "batch: more than 2^31 targets");
        }
        b->start[i + 1] = (int)tot;
        max_npix = I.npix > max_npix ? I.npix : max_npix;
        const std::pair<int, int> key(I.npix, I.M);
        int slot = -1;
        for (size_t s = 0; s < b->tabs.size(); ++s)
            if (b->tabs[s] == key) slot = (int)s;
        if (slot < 0) {
            if ((int)b->tabs.size() == kMaxTabs) {
                batch_release(b);
                return tr_fail(ctx, TR_EINVAL, "batch: more than %d distinct (N_side, cube_m)", kMaxTabs);
            }
            slot = (int)b->tabs.size();
            b->tabs.push_back(key);
            b->B.tab[slot] = I.rt->table;
            b->B.tab_ncell[slot] = 6 * I.M * I.M;
        }
        I.A.tab_slot = slot;
    }
    b->nslot = nslot_for(max_npix);
    b->tab_lds = table_in_lds(max_npix);
    b->B.n_tab = (int)b->tabs.size();
    int off = 0;
    for (int s = 0; s < b->B.n_tab; ++s) {
        b->B.tab_off[s] = off;
        if (b->tab_lds) off += table_bytes(b->tabs[s].second);
    }
    b->lds_table = off;
    if (hipMalloc(&b->d_inst, sizeof(TraceArgs) * n) != hipSuccess ||
        hipMalloc(&b->d_start, sizeof(int) * 2 * (n + 1)) != hipSuccess) {
        batch_release(b);
        return tr_fail(ctx, TR_ENOMEM, "batch descriptors");
    }
    if (hipMemcpy(b->d_start, b->start.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice) != hipSuccess) {
        batch_release(b);
        return tr_fail(ctx, TR_EHIP, "batch descriptor upload");
    }
    Knobs k;
    k.bp = p[0].bins_per_pass;
    k.waves = p[0].waves_per_block;
    k.chunk = p[0].chunk;
    int rc = batch_configure(b, k);
    if (rc) {
        batch_release(b);
        return rc;
    }
    *out = b;
    return TR_OK;
}

int batch_set_sample(tr_batch *b, int stride) {
    if (stride < 1) stride = 1;
    if (b->sample_stride == stride) return TR_OK;
    const int n = (int)b->inst.size();
    std::vector<int> st(n + 1, 0);
    for (int i = 0; i < n; ++i) st[i + 1] = st[i] + (int)tr_div_up(b->inst[i].A.n_targets, stride);
    TR_HIP(b->ctx, hipMemcpy(b->d_start + n + 1, st.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
    b->sample_stride = stride;
    return TR_OK;
}

// time one configuration on the tuner's sample: best of `reps` launches, in ms
int batch_time(tr_batch *b, Knobs k, int reps, float *ms) {
    tr_ctx *ctx = b->ctx;
    int rc = batch_configure(b, k);
    if (rc) return rc;
    hipEvent_t e0, e1;
    TR_HIP(ctx, hipEventCreate(&e0));
    TR_HIP(ctx, hipEventCreate(&e1));
    float best = 1e30f;
    rc = batch_enqueue(b, ctx->stream, true); // warm-up
    for (int r = 0; r < reps && rc == TR_OK; ++r) {
        hipEventRecord(e0, ctx->stream);
        rc = batch_enqueue(b, ctx->stream, true);
        hipEventRecord(e1, ctx->stream);
        if (hipEventSynchronize(e1) != hipSuccess) rc = tr_fail(ctx, TR_EHIP, "batch tuning: event wait failed");
        float t = 0.0f;
        hipEventElapsedTime(&t, e0, e1);
        best = t < best ? t : best;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc == TR_OK && ctx->d_ctl) {
        rc = tr_sync(ctx);
    }
    *ms = best;
    return rc;
}

} // namespace

extern "C" int tr_batch_create(tr_ctx *ctx, int n, const tr_tree *const *trees, const tr_trace_params *p,
                               float *const *J, float *const *F, float *const *u_rad, tr_batch **out) {
    int rc = batch_build(ctx, n, trees, p, J, F, u_rad, out);
    if (rc) return rc;
    rc = batch_capture(*out);
    if (rc) {
        batch_release(*out);
        *out = nullptr;
    }
    return rc;
}

extern "C" int tr_batch_launch(tr_batch *b) {
    if (!b) return TR_EINVAL;
    TR_HIP(b->ctx, hipSetDevice(b->ctx->device));
    if (!b->exec) return tr_fail(b->ctx, TR_EINVAL, "batch has no graph");
    TR_HIP(b->ctx, hipGraphLaunch(b->exec, b->ctx->stream));
    return TR_OK;
}

extern "C" int tr_batch_launch_eager(tr_batch *b) {
    if (!b) return TR_EINVAL;
    TR_HIP(b->ctx, hipSetDevice(b->ctx->device));
    return batch_enqueue(b, b->ctx->stream, false);
}

extern "C" int tr_batch_tune(tr_batch *b, int sample_stride, tr_batch_tuning *best) {
    if (!b) return TR_EINVAL;
    tr_ctx *ctx = b->ctx;
    TR_HIP(ctx, hipSetDevice(ctx->device));
    int rc = batch_set_sample(b, sample_stride);
    if (rc) return rc;
    int max_bins = 1;
    for (auto &I : b->inst) max_bins = I.A.n_bins > max_bins ? I.A.n_bins : max_bins;
    // coordinate descent: segments per pass, then waves per block, then the queue chunk
    Knobs cur;
    cur.chunk = 4;
    float cur_ms = 0.0f;
    rc = batch_time(b, cur, 2, &cur_ms);
    if (rc) return rc;
    const int bps[] = {1, 2, 3, 4, 6, 8, 12, 16};
    for (int v : bps) {
        if (v > max_bins) break;
        Knobs k = cur;
        k.bp = v;
        float ms = 0.0f;
        if (batch_time(b, k, 2, &ms) != TR_OK) continue; // does not fit: skip
        if (ms < cur_ms) { cur = k; cur_ms = ms; }
    }
    const int waves[] = {4, 8, 12};
    for (int v : waves) {
        Knobs k = cur;
        k.waves = v;
        float ms = 0.0f;
        if (batch_time(b, k, 2, &ms) != TR_OK) continue;
        if (ms < cur_ms) { cur = k; cur_ms = ms; }
    }
    const int chunks[] = {1, 2, 8, 16, 32};
    for (int v : chunks) {
        Knobs k = cur;
        k.chunk = v;
        float ms = 0.0f;
        if (batch_time(b, k, 2, &ms) != TR_OK) continue;
        if (ms < cur_ms) { cur = k; cur_ms = ms; }
    }
    ctx->err.clear();
    rc = batch_configure(b, cur);
    if (rc) return rc;
    b->tuned_ms = cur_ms;
    rc = batch_capture(b);
    if (rc) return rc;
    if (best) batch_report(b, cur_ms, best);
    return TR_OK;
}

extern "C" int tr_batch_set_tuning(tr_batch *b, const tr_batch_tuning *t) {
    if (!b) return TR_EINVAL;
    tr_ctx *ctx = b->ctx;
    if (!t || t->bins_per_pass < 0 || t->waves_per_block < 0 || t->chunk < 0)
        return tr_fail(ctx, TR_EINVAL, "tr_batch_set_tuning: negative setting");
    TR_HIP(ctx, hipSetDevice(ctx->device));
    Knobs k;
    k.bp = t->bins_per_pass;
    k.waves = t->waves_per_block;
    k.chunk = t->chunk;
    const Knobs old = b->knobs;
    int rc = batch_configure(b, k);
    if (rc) {
        const std::string why = ctx->err;
        if (batch_configure(b, old) == TR_OK) ctx->err = why; // the batch keeps its setting
        return rc;
    }
    b->tuned_ms = 0.0f;
    return batch_capture(b);
}

extern "C" int tr_batch_get_tuning(const tr_batch *b, tr_batch_tuning *out) {
    if (!b || !out) return TR_EINVAL;
    batch_report(b, b->tuned_ms, out);
    return TR_OK;
}

extern "C" void tr_batch_free(tr_batch *b) { batch_release(b); }

extern "C" int tr_trace_rays_batched(tr_ctx *ctx, int n, const tr_tree *const *trees, const tr_trace_params *p,
                                     float *const *J, float *const *F, float *const *u_rad) {
    tr_batch *b = nullptr;
    int rc = batch_build(ctx, n, trees, p, J, F, u_rad, &b);
    if (rc) return rc;
    rc = batch_enqueue(b, ctx->stream, false);
    batch_release(b); // waits for the launch before the descriptors go
    return rc;
}

extern "C" int tr_trace_rays(tr_ctx *ctx, const tr_tree *t, const tr_trace_params *p, float *J,
                             float *F, float *u_rad) {
    return launch_trace(ctx, t, p, J, F, u_rad, nullptr, false);
}

extern "C" int tr_walk_counts(tr_ctx *ctx, const tr_tree *t, const tr_trace_params *p,
                              int32_t *counters) {
    if (!ctx) return TR_EINVAL;
    if (!counters) return tr_fail(ctx, TR_EINVAL, "tr_walk_counts: null output");
    return launch_trace(ctx, t, p, nullptr, nullptr, nullptr, counters, true);
}

extern "C" int tr_rad_force(tr_ctx *ctx, const tr_tree *t, const float *F, float *a_rp, float *p_src) {
    if (!ctx) return TR_EINVAL;
    if (!t || !F || !a_rp) return tr_fail(ctx, TR_EINVAL, "tr_rad_force: null argument");
    TR_HIP(ctx, hipSetDevice(ctx->device));
    k_rad_force<<<tr_div_up(t->n_cells, 256), 256, 0, ctx->stream>>>(
        t->n_cells, F, t->cell_kappa, t->cell_tau, t->cell_src, t->node_of_cell, t->meta, (int)t->root_edge,
        (float)t->c_light, a_rp, p_src);
    if (hipGetLastError() != hipSuccess) return tr_fail(ctx, TR_EHIP, "rad_force launch failed");
    return TR_OK;
}
