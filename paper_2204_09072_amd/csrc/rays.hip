// Ray set and angular-kernel table (Sec. 4.2 of Klepitko et al. 2023).
//
// Rays are the HEALPix pixels (Gorski et al. 2005, NESTED numbering).  The angular
// kernel maps a direction to its pixel through a table over discrete directions: the
// six faces of a cube split into M x M cells, each cell holding the pixel of its centre
// direction.  Both tables are built once per (N_side, M) on the device in FP64; the
// tabulated angular kernel of distant nodes follows from the pixel table on the host.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ int hp_interleave(int x, int y) {
    int r = 0;
    for (int b = 0; b < 10; ++b) r |= ((x >> b) & 1) << (2 * b) | ((y >> b) & 1) << (2 * b + 1);
    return r;
}

// pixel of direction (x, y, z)
__device__ int hp_vec2pix(int ns, double x, double y, double z0) {
    double r = sqrt(x * x + y * y + z0 * z0);
    double z = z0 / r;
    double phi = atan2(y, x);
    if (phi < 0) phi += 2.0 * kPi;
    double tt = phi / (kPi / 2.0);
    if (tt >= 4.0) tt -= 4.0;
    int face, fx, fy;
    if (fabs(z) > 2.0 / 3.0) {
        // polar cap: the cap is cut along the four meridians tt = 0, 1, 2, 3
        int q = tt >= 3.0 ? 3 : (int)tt;
        double tp = tt - q;
        double w = ns * sqrt(3.0 * (1.0 - fabs(z)));
        int a = (int)floor(tp * w), b = (int)floor((1.0 - tp) * w);
        a = a < ns - 1 ? a : ns - 1;
        b = b < ns - 1 ? b : ns - 1;
        if (z > 0) {
            face = q;
            fx = ns - 1 - b;
            fy = ns - 1 - a;
        } else {
            face = q + 8;
            fx = a;
            fy = b;
        }
    } else {
        // equatorial belt: two families of straight pixel edges in (tt, z)
        double up = ns * (0.5 + tt - 0.75 * z), dn = ns * (0.5 + tt + 0.75 * z);
        int ju = (int)floor(up), jd = (int)floor(dn);
        int fu = ju / ns, fd = jd / ns;
        face = fu == fd ? (fu & 3) + 4 : (fu < fd ? fu : fd + 8);
        fx = jd % ns;
        fy = ns - 1 - ju % ns;
    }
    return face * ns * ns + hp_interleave(fx, fy);
}

// centre of a pixel
__device__ void hp_pix2vec(int ns, int pix, double *v) {
    const int row[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
    const int col[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};
    int face = pix / (ns * ns), w = pix % (ns * ns), x = 0, y = 0;
    for (int b = 0; b < 10; ++b) {
        x |= ((w >> (2 * b)) & 1) << b;
        y |= ((w >> (2 * b + 1)) & 1) << b;
    }
    int ring = row[face] * ns - x - y - 1;
    int nr = ns, shift = 0;
    double z;
    if (ring < ns) {
        nr = ring;
        z = 1.0 - (double)(nr * nr) / (3.0 * ns * ns);
    } else if (ring > 3 * ns) {
        nr = 4 * ns - ring;
        z = -1.0 + (double)(nr * nr) / (3.0 * ns * ns);
    } else {
        shift = (ring - ns) & 1;
        z = (double)(2 * ns - ring) * 2.0 / (3.0 * ns);
    }
    int jp = (col[face] * nr + x - y + 1 + shift) / 2;
    if (jp > 4 * nr) jp -= 4 * nr;
    if (jp < 1) jp += 4 * nr;
    double phi = ((double)jp - 0.5 * (double)(shift + 1)) * (kPi / 2.0) / (double)nr;
    double st = sqrt((1.0 - z) * (1.0 + z));
    v[0] = st * cos(phi);
    v[1] = st * sin(phi);
    v[2] = z;
}

__global__ void k_cube_table(int ns, int M, int16_t *__restrict__ tab) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 6 * (int64_t)M * M) return;
    int f = (int)(e / ((int64_t)M * M));
    int i = (int)((e / M) % M), j = (int)(e % M);
    int ax = f >> 1;
    double v[3];
    v[ax] = (f & 1) ? -1.0 : 1.0;
    v[ax == 0 ? 1 : 0] = (2.0 * i + 1.0) / M - 1.0;
    v[ax == 2 ? 1 : 2] = (2.0 * j + 1.0) / M - 1.0;
    tab[e] = (int16_t)hp_vec2pix(ns, v[0], v[1], v[2]);
}

__global__ void k_dirs(int ns, float4 *__restrict__ dirs) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= 12 * ns * ns) return;
    double v[3];
    hp_pix2vec(ns, p, v);
    dirs[p] = make_float4((float)v[0], (float)v[1], (float)v[2], 0.0f);
}

} // namespace

int tr_get_table(tr_ctx *ctx, int n_side, int cube_m, RayTable **out) {
    auto key = std::make_pair(n_side, cube_m);
    auto it = ctx->tables.find(key);
    if (it != ctx->tables.end()) {
        *out = &it->second;
        return TR_OK;
    }
    if (n_side < 1 || n_side > 8 || (n_side & (n_side - 1)) || cube_m < 1 || cube_m > 1024)
        return tr_fail(ctx, TR_EINVAL, "bad ray table request (n_side %d, cube_m %d)", n_side, cube_m);
    RayTable rt;
    rt.n_side = n_side;
    rt.cube_m = cube_m;
    const int64_t ne = 6 * (int64_t)cube_m * cube_m;
    const int npix = 12 * n_side * n_side;
    if (hipMalloc(&rt.table, sizeof(int16_t) * ne) != hipSuccess) return tr_fail(ctx, TR_ENOMEM, "table");
    if (hipMalloc(&rt.dirs, sizeof(float4) * npix) != hipSuccess) {
        hipFree(rt.table);
        return tr_fail(ctx, TR_ENOMEM, "dirs");
    }
    k_cube_table<<<tr_div_up(ne, 256), 256, 0, ctx->stream>>>(n_side, cube_m, rt.table);
    k_dirs<<<tr_div_up(npix, 256), 256, 0, ctx->stream>>>(n_side, rt.dirs);
    if (hipGetLastError() != hipSuccess) {
        hipFree(rt.table);
        hipFree(rt.dirs);
        return tr_fail(ctx, TR_EHIP, "table kernels failed to launch");
    }
    // Tabulated angular kernel (Sec. 4.2.1), built on the host from the pixel table in exact
    // integers: for direction cell (f, i, j) with centre d = K (2i + 1 - M, 2j + 1 - M, +-M)
    // on its face (K = 2^16) and distance class c = 6 .. 20, the 4^3 stratified sub-points
    // of a cube of edge s_c = |d| 2^(-(c + 1/2)/2) (rounded to a multiple of 8) centred on
    // d, each binned to its direction cell and that cell's pixel.
    std::vector<int16_t> pix(ne);
    if (hipMemcpyAsync(pix.data(), rt.table, sizeof(int16_t) * ne, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        hipFree(rt.table);
        hipFree(rt.dirs);
        return tr_fail(ctx, TR_EHIP, "direction-cell table readback failed");
    }
    const int M = cube_m;
    const int64_t K = (int64_t)1 << 16;
    auto cell_of = [&](const int64_t *d) {
        const int64_t a0 = d[0] < 0 ? -d[0] : d[0], a1 = d[1] < 0 ? -d[1] : d[1], a2 = d[2] < 0 ? -d[2] : d[2];
        const int ax = (a0 >= a1 && a0 >= a2) ? 0 : (a1 >= a2 ? 1 : 2);
        const int oa = ax == 0 ? 1 : 0, ob = ax == 2 ? 1 : 2;
        const int64_t m = ax == 0 ? a0 : (ax == 1 ? a1 : a2);
        const int f = 2 * ax + (d[ax] < 0 ? 1 : 0);
        int64_t i = ((int64_t)M * (d[oa] + m)) / (2 * m), j = ((int64_t)M * (d[ob] + m)) / (2 * m);
        i = i > M - 1 ? M - 1 : i;
        j = j > M - 1 ? M - 1 : j;
        return (int64_t)(f * M + i) * M + j;
    };
    constexpr int nclass = 15;
    struct Entry {
        int np, px[4], cnt[4];
    };
    std::vector<Entry> full(ne * nclass);
    for (int f = 0; f < 6; ++f) {
        const int ax = f / 2, oa = ax == 0 ? 1 : 0, ob = ax == 2 ? 1 : 2;
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                int64_t d[3];
                d[ax] = (f & 1) ? -(int64_t)M * K : (int64_t)M * K;
                d[oa] = K * (2 * i + 1 - M);
                d[ob] = K * (2 * j + 1 - M);
                const double len = std::sqrt((double)d[0] * d[0] + (double)d[1] * d[1] + (double)d[2] * d[2]);
                for (int c = 6; c <= 20; ++c) {
                    const double x = len * 0.8408964152537145 * ((c & 1) ? 0.7071067811865476 : 1.0) *
                                     std::ldexp(1.0, -(c / 2));
                    const int64_t S = 8 * std::llround(x / 8.0);
                    int px[64], cnt[64], np = 0;
                    for (int q = 0; q < 64; ++q) {
                        const int64_t e[3] = {d[0] + (2 * (q % 4) - 3) * S / 8, d[1] + (2 * ((q / 4) % 4) - 3) * S / 8,
                                              d[2] + (2 * (q / 16) - 3) * S / 8};
                        const int p = pix[cell_of(e)];
                        int k = 0;
                        while (k < np && px[k] != p) ++k;
                        if (k == np) { px[np] = p; cnt[np] = 0; ++np; }
                        cnt[k]++;
                    }
                    for (int u = 1; u < np; ++u)
                        for (int v = u; v > 0 && px[v - 1] > px[v]; --v) {
                            std::swap(px[v], px[v - 1]);
                            std::swap(cnt[v], cnt[v - 1]);
                        }
                    Entry &en = full[(((int64_t)f * M + i) * M + j) * nclass + (c - 6)];
                    en.np = np;
                    for (int k = 0; k < 4; ++k) {
                        en.px[k] = k < np && np <= 4 ? px[k] : 0;
                        en.cnt[k] = k < np && np <= 4 ? cnt[k] : 0;
                    }
                }
            }
    }
    // the first class from which every entry is the direction cell's own pixel alone
    int c1 = 21;
    for (; c1 > 6; --c1) {
        bool own = true;
        for (int64_t cell = 0; own && cell < ne; ++cell) {
            const Entry &en = full[cell * nclass + (c1 - 1 - 6)];
            own = en.np == 1 && en.px[0] == pix[cell];
        }
        if (!own) break;
    }
    const int ncls = c1 - 6;
    std::vector<unsigned long long> packed(ne * (ncls > 0 ? ncls : 1), 0ull);
    for (int64_t cell = 0; cell < ne; ++cell)
        for (int c = 6; c < c1; ++c) {
            const Entry &en = full[cell * nclass + (c - 6)];
            unsigned long long w = 0;
            if (en.np > 4) {
                w = 1ull << 61;
            } else {
                for (int k = 0; k < 4; ++k) w |= (unsigned long long)en.px[k] << (10 * k);
                for (int k = 0; k < 3; ++k) w |= (unsigned long long)en.cnt[k] << (40 + 7 * k);
            }
            packed[cell * ncls + (c - 6)] = w;
        }
    rt.alpha_c1 = c1;
    if (hipMalloc(&rt.alpha, sizeof(unsigned long long) * packed.size()) != hipSuccess ||
        hipMemcpy(rt.alpha, packed.data(), sizeof(unsigned long long) * packed.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
        hipFree(rt.table);
        hipFree(rt.dirs);
        hipFree(rt.alpha);
        return tr_fail(ctx, TR_ENOMEM, "tabulated angular kernel");
    }
    ctx->tables[key] = rt;
    *out = &ctx->tables[key];
    return TR_OK;
}

extern "C" int tr_ray_tables(tr_ctx *ctx, int n_side, int cube_m, int32_t *table, float *dirs) {
    if (!ctx) return TR_EINVAL;
    TR_HIP(ctx, hipSetDevice(ctx->device));
    if (cube_m == 0) cube_m = 16 * n_side;
    RayTable *rt = nullptr;
    int rc = tr_get_table(ctx, n_side, cube_m, &rt);
    if (rc) return rc;
    const int64_t ne = 6 * (int64_t)cube_m * cube_m;
    const int npix = 12 * n_side * n_side;
    std::vector<int16_t> t16(ne);
    std::vector<float4> d4(npix);
    TR_HIP(ctx, hipMemcpyAsync(t16.data(), rt->table, sizeof(int16_t) * ne, hipMemcpyDeviceToHost, ctx->stream));
    TR_HIP(ctx, hipMemcpyAsync(d4.data(), rt->dirs, sizeof(float4) * npix, hipMemcpyDeviceToHost, ctx->stream));
    TR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t e = 0; table && e < ne; ++e) table[e] = t16[e];
    for (int p = 0; dirs && p < npix; ++p) {
        dirs[3 * p] = d4[p].x;
        dirs[3 * p + 1] = d4[p].y;
        dirs[3 * p + 2] = d4[p].z;
    }
    return TR_OK;
}

extern "C" int tr_alpha_table(tr_ctx *ctx, int n_side, int cube_m, int32_t *out) {
    if (!ctx) return TR_EINVAL;
    if (!out) return tr_fail(ctx, TR_EINVAL, "tr_alpha_table: null output");
    TR_HIP(ctx, hipSetDevice(ctx->device));
    if (cube_m == 0) cube_m = 16 * n_side;
    RayTable *rt = nullptr;
    int rc = tr_get_table(ctx, n_side, cube_m, &rt);
    if (rc) return rc;
    const int64_t ne = 6 * (int64_t)cube_m * cube_m;
    const int c1 = rt->alpha_c1, ncls = c1 - 6;
    std::vector<unsigned long long> a(ne * (ncls > 0 ? ncls : 1));
    std::vector<int16_t> pix(ne);
    TR_HIP(ctx, hipMemcpyAsync(a.data(), rt->alpha, sizeof(unsigned long long) * a.size(), hipMemcpyDeviceToHost,
                               ctx->stream));
    TR_HIP(ctx, hipMemcpyAsync(pix.data(), rt->table, sizeof(int16_t) * ne, hipMemcpyDeviceToHost, ctx->stream));
    TR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t cell = 0; cell < ne; ++cell)
        for (int c = 6; c <= 20; ++c) {
            int32_t *o = out + 9 * (cell * 15 + (c - 6));
            for (int k = 0; k < 9; ++k) o[k] = 0;
            if (c >= c1) {
                o[0] = pix[cell];
                o[4] = 64;
                continue;
            }
            const unsigned long long w = a[cell * ncls + (c - 6)];
            if ((w >> 61) & 1ull) {
                o[8] = 1;
                continue;
            }
            for (int k = 0; k < 4; ++k) o[k] = (int32_t)((w >> (10 * k)) & 1023ull);
            int sum = 0;
            for (int k = 0; k < 3; ++k) {
                o[4 + k] = (int32_t)((w >> (40 + 7 * k)) & 127ull);
                sum += o[4 + k];
            }
            o[7] = 64 - sum;
        }
    return TR_OK;
}
