// Backward ray tracing of the diffuse infrared field (Sec. 4.2-4.5 of Klepitko et al.).
//
// One wavefront per target cell, persistent: waves take targets from a global work
// counter.  For every target the ray segments (HEALPix pixel x radial evaluation point)
// live in LDS.  To keep several waves resident per CU the segments are processed in
// passes of `bins_per_pass` radial points; each pass re-walks the octree, pruning
// subtrees whose material cannot map into the pass, maps the accepted nodes with LDS
// atomics and then integrates the pass outwards with one lane per ray, carrying the
// extinction and an open merged segment to the next pass.
//
// Walk: a stack of child ranges (first child, count) in LDS; each step pops 8 ranges so
// that the 64 lanes test 64 sibling nodes at once; the opening test and the radial
// bin search are exact integer comparisons.
#include "common.hpp"

namespace {

constexpr float kPiF = 3.14159265358979f;
constexpr int kStack = 640;      // ranges per wave; the walk needs at most 56 * depth + 8
constexpr int kFields = 6;       // L_thin, A_thin, L_thick*V, A_thick, V_thick, Q

struct TraceArgs {
    const int4 *geo;
    const uint32_t *meta;
    const float4 *q;
    const float *vthick;
    const int4 *pcol;
    const int32_t *targets;
    const int32_t *leaf_cell;
    const float *cell_tau;
    const float *cell_src;
    const int16_t *table;
    const float4 *dirs;
    int *work;
    int *err;
    float *J, *F, *u_rad;
    int32_t *counters;
    int64_t n_cells;
    int n_targets;
    int root_edge;
    int npix;
    int cube_m;
    int n_bins;
    int bp;      // bins per pass
    int n_pass;
    int chunk;
    int merge;
    int64_t th_num2, th_den2; // opening test s^2 den^2 < num^2 d^2
    float omega;
    float j_bg;
    float c_light;
    int lds_wave; // bytes of LDS per wave
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_s_waitcnt(0xc07f); // lgkmcnt(0): this wave's LDS traffic has landed
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// largest i in [0, nb] with R_i + off <= r, i.e. (FX i^2 + off)^2 <= r2 (or FX i^2 + off <= 0)
__device__ __forceinline__ int bin_below(int64_t r2, int off, int nb) {
    float rr = sqrtf((float)r2) - (float)off;
    int i = rr > 0.0f ? (int)sqrtf(rr * (1.0f / TR_FX)) : 0;
    i = i < 0 ? 0 : (i > nb ? nb : i);
    auto ok = [&](int k) {
        int64_t e = (int64_t)TR_FX * k * k + off;
        return e <= 0 || e * e <= r2;
    };
    while (i < nb && ok(i + 1)) ++i;
    while (i > 0 && !ok(i)) --i;
    return i;
}

// direction cell of an integer direction (same binning as the table: face of the largest
// component with ties to the lower axis, then floor(M (d_a + |d_m|) / (2 |d_m|)))
__device__ __forceinline__ int cube_cell(int dx, int dy, int dz, int M) {
    int ax = abs(dx), ay = abs(dy), az = abs(dz);
    int f, m, ua, ub;
    if (ax >= ay && ax >= az) {
        m = ax; f = dx < 0 ? 1 : 0; ua = dy + m; ub = dz + m;
    } else if (ay >= az) {
        m = ay; f = dy < 0 ? 3 : 2; ua = dx + m; ub = dz + m;
    } else {
        m = az; f = dz < 0 ? 5 : 4; ua = dx + m; ub = dy + m;
    }
    uint32_t den = 2u * (uint32_t)m;
    uint32_t i = ((uint32_t)M * (uint32_t)ua) / den;
    uint32_t j = ((uint32_t)M * (uint32_t)ub) / den;
    i = i > (uint32_t)(M - 1) ? (uint32_t)(M - 1) : i;
    j = j > (uint32_t)(M - 1) ? (uint32_t)(M - 1) : j;
    return (f * M + (int)i) * M + (int)j;
}

struct Pass {
    int a, b; // radial points [a, b) held in LDS
};

// Map one accepted node (Sec. 4.2.1/4.2.2) into the pass's LDS segments.
__device__ __forceinline__ void map_node(const TraceArgs &A, int node, bool leaf, int s, int4 c256,
                                         Pass P, float *bins, uint32_t *flg) {
    int4 p = A.pcol[node];
    int dx = p.x - c256.x, dy = p.y - c256.y, dz = p.z - c256.z;
    int64_t r2 = (int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz;
    int i = bin_below(r2, 0, A.n_bins);
    if (i == 0) return;
    float4 qv = A.q[node];
    float Lt, At, LVk, Ak, Vk;
    if (leaf) {
        bool thick = signbit(qv.x);
        float V = (float)s * (float)s * (float)s;
        Lt = thick ? qv.z : qv.x + qv.z;
        At = thick ? 0.0f : qv.y;
        LVk = thick ? fabsf(qv.x) * V : 0.0f;
        Ak = thick ? qv.y : 0.0f;
        Vk = thick ? V : 0.0f;
    } else {
        Lt = qv.x; LVk = qv.y; At = qv.z; Ak = qv.w;
        Vk = A.vthick[node];
    }
    const bool content = i >= P.a && i < P.b;
    uint32_t fbits = 0;
    if (Vk > 0.0f && A.merge) {
        int half = TR_FX / 2 * s;
        int lo = bin_below(r2, half, A.n_bins);
        lo = lo < 1 ? 1 : lo;
        int hi = bin_below(r2, -half, A.n_bins);
        int k0 = lo > P.a ? lo : P.a, k1 = hi < P.b ? hi : P.b;
        for (int k = k0; k < k1; ++k) fbits |= 1u << (k - P.a);
    }
    if (!content && !fbits) return;
    // radial kernel beta = R_i^2 / r^2 and the 8-point angular kernel
    float beta = (float)((int64_t)TR_FX * TR_FX * i * i * i * i) / (float)r2;
    int h = 64 * s;
    int pix[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int cx = dx + ((k & 1) ? h : -h), cy = dy + ((k & 2) ? h : -h), cz = dz + ((k & 4) ? h : -h);
        pix[k] = A.table[cube_cell(cx, cy, cz, A.cube_m)];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        bool first = true;
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            bool eq = pix[j] == pix[k];
            cnt += eq ? 1 : 0;
            if (j < k && eq) first = false;
        }
        if (!first) continue;
        float al = 0.125f * (float)cnt;
        if (content) {
            float *bb = bins + ((size_t)pix[k] * A.bp + (i - P.a)) * kFields;
            float ab = al * beta;
            if (Lt != 0.0f) atomicAdd(bb + 0, ab * Lt);
            if (At != 0.0f) atomicAdd(bb + 1, ab * At);
            if (Vk > 0.0f) {
                atomicAdd(bb + 2, al * LVk);
                atomicAdd(bb + 3, al * Ak);
                atomicAdd(bb + 4, al * Vk);
                atomicAdd(bb + 5, ab * Vk);
            }
        }
        if (fbits) atomicOr(flg + pix[k], fbits);
    }
}

template <int NSLOT>
struct RayState {
    float tau_thin[NSLOT]; // sum of thin optical depths of closed inner segments
    float eps_thick[NSLOT];
    float Fh[NSLOT];
    int run_i[NSLOT];      // first point of the open (merged) segment, 0 = none
    float acc[NSLOT][kFields];
};

// One closed segment at R_i (Sec. 4.3.1, 4.3.2): returns nothing, updates the ray.
__device__ __forceinline__ void integrate_segment(const float *s, int i, float omega, float &tau_thin,
                                                  float &eps_thick, float &Fh) {
    float R2 = (float)i * (float)i * (float)i * (float)i;
    float tt = s[1] / (omega * R2);
    float omt = 0.0f, tk = 0.0f, Fk = 0.0f;
    if (s[4] > 0.0f) {
        float cb = cbrtf(s[4]);
        omt = (s[5] / s[4]) * (cb * cb) / R2;
        omt = omt > omega ? omega : omt;
        if (omt > 0.0f) tk = s[3] / (omt * R2);
        Fk = omt * s[2] / s[4];
    }
    float f = omt / omega;
    float phi = tt > 0.0f ? -expm1f(-tt) / tt : 1.0f;
    float Ft = phi * s[0] / (4.0f * kPiF * R2);
    float den = s[1] + f * s[3];
    float Fs = den > 0.0f ? (Ft * s[1] + Fk * f * s[3]) / den : Ft;
    Fh += __expf(-tau_thin) * eps_thick * Fs;
    tau_thin += tt;
    eps_thick *= (1.0f - f) + f * __expf(-tk);
}

template <int NSLOT, bool COUNT>
__device__ void trace_target(const TraceArgs &A, int ti, float *bins, uint32_t *flg, int2 *stk) {
    const int lane = lane_id();
    const int tid = A.targets[ti];
    const int4 tg = A.geo[tid];
    const int4 c256 = make_int4(tg.x * TR_FX, tg.y * TR_FX, tg.z * TR_FX, 0);
    RayState<NSLOT> R;
#pragma unroll
    for (int k = 0; k < NSLOT; ++k) {
        R.tau_thin[k] = 0.0f;
        R.eps_thick[k] = 1.0f;
        R.Fh[k] = 0.0f;
        R.run_i[k] = 0;
#pragma unroll
        for (int f = 0; f < kFields; ++f) R.acc[k][f] = 0.0f;
    }
    int n_b = 0, n_h = 0, n_open = 0;
    const int n_pass = COUNT ? 1 : A.n_pass;
    for (int ps = 0; ps < n_pass; ++ps) {
        Pass P;
        P.a = 1 + ps * A.bp;
        P.b = P.a + A.bp;
        if (P.b > A.n_bins + 1) P.b = A.n_bins + 1;
        if (!COUNT) {
            const int nf = A.npix * A.bp * kFields;
            for (int k = lane; k < nf; k += 64) bins[k] = 0.0f;
            for (int k = lane; k < A.npix; k += 64) flg[k] = 0u;
        }
        // squared pruning radii (lattice units): keep a subtree when
        // r_max + s/4 >= R_a and r_min - s/4 < R_b
        if (lane == 0) stk[0] = make_int2(0, 1);
        int sp = 1;
        wave_sync();
        while (sp > 0) {
            const int npop = sp < 8 ? sp : 8;
            const int r = lane >> 3, k = lane & 7;
            int2 rg = r < npop ? stk[sp - 1 - r] : make_int2(0, 0);
            sp -= npop;
            wave_sync();
            int node = (r < npop && k < rg.y) ? rg.x + k : -1;
            bool open = false;
            int2 push = make_int2(0, 0);
            if (node >= 0) {
                const int4 g = A.geo[node];
                const uint32_t mt = A.meta[node];
                const int s = A.root_edge >> (mt & 15u);
                const bool leaf = (mt >> 12) & 1u;
                if (leaf) {
                    if (node != tid) {
                        ++n_b;
                        if (!COUNT) map_node(A, node, true, s, c256, P, bins, flg);
                    }
                } else {
                    const int64_t ddx = g.x - tg.x, ddy = g.y - tg.y, ddz = g.z - tg.z;
                    const int64_t d2 = ddx * ddx + ddy * ddy + ddz * ddz;
                    if ((int64_t)s * s * A.th_den2 < A.th_num2 * d2) {
                        ++n_h;
                        if (!COUNT) map_node(A, node, false, s, c256, P, bins, flg);
                    } else {
                        ++n_open;
                        bool keep = true;
                        if (!COUNT) {
                            const int hs = s / 2, q4 = s / 4;
                            const int ax = abs((int)ddx), ay = abs((int)ddy), az = abs((int)ddz);
                            const int64_t nx = ax > hs ? ax - hs : 0, ny = ay > hs ? ay - hs : 0,
                                          nz = az > hs ? az - hs : 0;
                            const int64_t fx = ax + hs, fy = ay + hs, fz = az + hs;
                            const int64_t rmin2 = nx * nx + ny * ny + nz * nz;
                            const int64_t rmax2 = fx * fx + fy * fy + fz * fz;
                            const int64_t lo = (int64_t)P.a * P.a - q4;
                            const int64_t hi = (int64_t)P.b * P.b + q4;
                            if (lo > 0 && rmax2 < lo * lo) keep = false;
                            if (P.b <= A.n_bins && rmin2 >= hi * hi) keep = false;
                        }
                        if (keep) {
                            open = true;
                            push = make_int2(g.w, __builtin_popcount((mt >> 4) & 255u));
                        }
                    }
                }
            }
            const uint64_t bal = __ballot(open);
            const int pos = __builtin_popcountll(bal & ((1ull << lane) - 1ull));
            const int npush = __builtin_popcountll(bal);
            if (open && sp + pos < kStack) stk[sp + pos] = push;
            if (sp + npush > kStack) {
                if (lane == 0) atomicOr(A.err, 4);
                sp = kStack;
            } else {
                sp += npush;
            }
            wave_sync();
        }
        if (COUNT) break;
        // integrate the pass's segments outwards, one lane per ray
#pragma unroll
        for (int sl = 0; sl < NSLOT; ++sl) {
            const int h = lane + 64 * sl;
            if (h >= A.npix) continue;
            const uint32_t fl = flg[h];
            for (int i = P.a; i < P.b; ++i) {
                const float *v = bins + ((size_t)h * A.bp + (i - P.a)) * kFields;
                if (R.run_i[sl] == 0) {
                    R.run_i[sl] = i;
#pragma unroll
                    for (int f = 0; f < kFields; ++f) R.acc[sl][f] = v[f];
                } else {
                    // inverse-square content moves to the merged segment's R_i
                    const float T = (float)R.run_i[sl] / (float)i;
                    const float T4 = (T * T) * (T * T);
                    R.acc[sl][0] += T4 * v[0];
                    R.acc[sl][1] += T4 * v[1];
                    R.acc[sl][2] += v[2];
                    R.acc[sl][3] += v[3];
                    R.acc[sl][4] += v[4];
                    R.acc[sl][5] += T4 * v[5];
                }
                const bool link = ((fl >> (i - P.a)) & 1u) && i < A.n_bins;
                if (!link) {
                    integrate_segment(R.acc[sl], R.run_i[sl], A.omega, R.tau_thin[sl], R.eps_thick[sl],
                                      R.Fh[sl]);
                    R.run_i[sl] = 0;
                }
            }
        }
        wave_sync();
    }
    const int cell = A.leaf_cell[tid];
    if (COUNT) {
        // reduce the per-lane counters
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
        const float Fh = R.Fh[sl] + __expf(-R.tau_thin[sl]) * R.eps_thick[sl] * A.omega * A.j_bg;
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
        float Jv = js / (4.0f * kPiF);
        if (src > 0.0f) {
            const float e = (float)(A.root_edge >> (A.meta[tid] & 15u));
            Jv += -expm1f(-0.5f * A.cell_tau[cell]) * src / (4.0f * kPiF * (e * e));
        }
        A.J[cell] = Jv;
        A.F[cell] = fx;
        A.F[A.n_cells + cell] = fy;
        A.F[2 * A.n_cells + cell] = fz;
        if (A.u_rad) A.u_rad[cell] = 4.0f * kPiF * Jv / A.c_light;
    }
}

template <int NSLOT, bool COUNT>
__global__ __launch_bounds__(64) void k_trace(TraceArgs A) {
    extern __shared__ __align__(16) char smem[];
    float *bins = reinterpret_cast<float *>(smem);
    uint32_t *flg = reinterpret_cast<uint32_t *>(bins + (COUNT ? 0 : A.npix * A.bp * kFields));
    int2 *stk = reinterpret_cast<int2 *>(smem + (COUNT ? 0 : A.lds_wave - kStack * sizeof(int2)));
    for (;;) {
        int t0 = 0;
        if (lane_id() == 0) t0 = atomicAdd(A.work, A.chunk);
        t0 = __shfl(t0, 0);
        if (t0 >= A.n_targets) break;
        const int t1 = t0 + A.chunk < A.n_targets ? t0 + A.chunk : A.n_targets;
        for (int ti = t0; ti < t1; ++ti) trace_target<NSLOT, COUNT>(A, ti, bins, flg, stk);
    }
}

__global__ void k_zero_int(int *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
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

int launch_trace(tr_ctx *ctx, const tr_tree *t, const tr_trace_params *p, float *J, float *F,
                 float *u_rad, int32_t *counters, bool count) {
    if (!ctx) return TR_EINVAL;
    if (!t || !p) return tr_fail(ctx, TR_EINVAL, "tr_trace_rays: null argument");
    if (!count && (!J || !F)) return tr_fail(ctx, TR_EINVAL, "tr_trace_rays: null output");
    const int ns = p->n_side;
    if (ns != 1 && ns != 2 && ns != 4 && ns != 8)
        return tr_fail(ctx, TR_EINVAL, "n_side must be 1, 2, 4 or 8 (got %d)", ns);
    int64_t num = p->theta_num, den = p->theta_den;
    if (num == 0 && den == 0) { num = 1; den = 2 * ns; }
    if (num < 0 || den <= 0) return tr_fail(ctx, TR_EINVAL, "bad opening angle %lld/%lld", (long long)num, (long long)den);
    const int M = p->cube_m ? p->cube_m : 16 * ns;
    if (M < 1 || M > 256) return tr_fail(ctx, TR_EINVAL, "cube_m must be in [1, 256]");
    TR_HIP(ctx, hipSetDevice(ctx->device));
    RayTable *rt = nullptr;
    int rc = tr_get_table(ctx, ns, M, &rt);
    if (rc) return rc;
    const int npix = 12 * ns * ns;
    int bp = p->bins_per_pass;
    if (bp <= 0) {
        // largest pass that keeps at least 4 waves per CU within 160 KB of LDS
        bp = t->n_bins;
        while (bp > 1 && (size_t)npix * bp * kFields * 4 + npix * 4 + kStack * 8 > 40 * 1024) --bp;
    }
    if (bp > t->n_bins) bp = t->n_bins;
    if (bp > 32) bp = 32;
    if (bp < 1) bp = 1;
    TraceArgs A;
    A.geo = t->geo; A.meta = t->meta; A.q = t->q; A.vthick = t->vthick; A.pcol = t->pcol;
    A.targets = t->targets; A.leaf_cell = t->leaf_cell; A.cell_tau = t->cell_tau; A.cell_src = t->cell_src;
    A.table = rt->table; A.dirs = rt->dirs;
    A.work = ctx->d_ctl; A.err = ctx->d_ctl + 16;
    A.J = J; A.F = F; A.u_rad = u_rad; A.counters = counters;
    A.n_cells = t->n_cells; A.n_targets = (int)t->n_cells; A.root_edge = (int)t->root_edge;
    A.npix = npix; A.cube_m = M; A.n_bins = t->n_bins; A.bp = bp;
    A.n_pass = (int)tr_div_up(t->n_bins, bp);
    A.chunk = p->chunk > 0 ? p->chunk : 4;
    A.merge = p->merge ? 1 : 0;
    A.th_num2 = num * num; A.th_den2 = den * den;
    A.omega = (float)(4.0 * 3.14159265358979323846 / npix);
    A.j_bg = p->j_bg;
    A.c_light = (float)t->c_light;
    A.lds_wave = count ? (int)(kStack * sizeof(int2))
                       : (int)((size_t)npix * bp * kFields * 4 + (size_t)npix * 4 + kStack * sizeof(int2));
    A.lds_wave = (A.lds_wave + 15) & ~15;
    int per_cu = p->blocks_per_cu > 0 ? p->blocks_per_cu : (int)((160 * 1024) / A.lds_wave);
    if (per_cu > 16) per_cu = 16;
    if (per_cu < 1) per_cu = 1;
    const int grid = ctx->n_cu * per_cu;
    k_zero_int<<<1, 64, 0, ctx->stream>>>(ctx->d_ctl, 1);
    const size_t lds = (size_t)A.lds_wave;
#define LAUNCH(NS_, C_)                                                                     \
    hipLaunchKernelGGL((k_trace<NS_, C_>), dim3(grid), dim3(64), lds, ctx->stream, A)
    if (count) {
        LAUNCH(1, true);
    } else if (npix <= 64) {
        LAUNCH(1, false);
    } else if (npix <= 192) {
        LAUNCH(3, false);
    } else {
        LAUNCH(12, false);
    }
#undef LAUNCH
    if (hipGetLastError() != hipSuccess) return tr_fail(ctx, TR_EHIP, "trace kernel launch failed");
    return TR_OK;
}

} // namespace

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
