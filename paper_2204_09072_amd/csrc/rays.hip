// Ray set and angular-kernel tables (Sec. 4.2 of Klepitko et al. 2023).
//
// Rays are the HEALPix pixels (Gorski et al. 2005, NESTED numbering).  The library locates
// pixels on the plane of the HEALPix map projection (Calabretta & Roukema 2007, the
// projection with H = 4 facets around the equator and K = 3): there the twelve base pixels
// are squares rotated by 45 degrees on a regular lattice, so a direction's pixel is a pair
// of floors in rotated plane coordinates and a pixel's centre is the inverse projection of
// its square's centre.
//
// The angular kernel takes directions through a cube map: the six faces of a cube split
// into M x M direction cells (M a power of two), each cell holding the pixel of its centre
// direction.  For distant nodes the kernel is tabulated over (direction cell, distance
// class): the share per pixel of the 4^3 stratified sub-points of a cube seen under the
// class's middle edge-to-distance ratio.  Everything is built once per (N_side, M) by
// device kernels: the cell table and ray directions in FP64, the tabulated kernel in exact
// integers with one wavefront per table key (a lane per sub-point, distinct pixels found
// by repeated wave minima).
#include <cmath>

#include "common.hpp"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kClassFirst = 6; // first tabulated distance class (r^2 >= 64 s^2)
constexpr int kClassLast = 20; // last class, which also takes every farther node
constexpr int kClasses = kClassLast - kClassFirst + 1;

// bits of v (< 2^16) spread to the even bit positions
__host__ __device__ inline uint32_t spread_bits(uint32_t v) {
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// the even bit positions of v gathered into the low half
__host__ __device__ inline uint32_t gather_bits(uint32_t v) {
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0f0f0f0fu;
    v = (v | (v >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0x0000ffffu;
    return v;
}

// Pixel of the direction (x, y, z), not necessarily normalised.  Projection plane in units
// of pi/4: the equatorial zone |z| <= 2/3 maps linearly, X = 4 phi / pi, Y = 3 z / 2; a
// polar zone compresses each quarter of longitude towards its central meridian X_m by
// sigma = sqrt(3 (1 - |z|)), X = X_m + (4 phi / pi - X_m) sigma, Y = +-(2 - sigma).  In the
// rotated coordinates P = X + Y, Q = X - Y the base pixels are the unit cells of a lattice
// of spacing 2 centred on even (P, Q); a base pixel's row is (P_c - Q_c) / 2 (north 1,
// equator 0, south -1) and its column (P_c + Q_c) / 2 (mod 8).  Inside it the NESTED
// coordinates run along P (x, towards north-east) and against Q (y, towards north-west).
__host__ __device__ int pixel_of_direction(int ns, double x, double y, double z) {
    const double zn = z / sqrt(x * x + y * y + z * z);
    double lon = atan2(y, x);
    lon = lon < 0.0 ? lon + 2.0 * kPi : lon;
    double q4 = lon * (2.0 / kPi); // longitude in quarter turns, [0, 4)
    q4 = q4 >= 4.0 ? q4 - 4.0 : q4;
    const double az = fabs(zn);
    double X, Y;
    if (az > 2.0 / 3.0) {
        const double sg = sqrt(3.0 * (1.0 - az));
        const double quarter = fmin(floor(q4), 3.0);
        const double xm = 2.0 * quarter + 1.0;
        X = xm + (2.0 * q4 - xm) * sg;
        Y = zn > 0.0 ? 2.0 - sg : sg - 2.0;
    } else {
        X = 2.0 * q4;
        Y = 1.5 * zn;
    }
    const double P = X + Y, Q = X - Y;
    const double pa = floor(0.5 * (P + 1.0)), qa = floor(0.5 * (Q + 1.0));
    const int row = (int)(pa - qa);                  // 1, 0, -1
    const int col = ((int)(pa + qa) % 8 + 8) % 8;    // 0 .. 7
    const int face = row > 0 ? (col - 1) / 2 : (row < 0 ? 8 + (col - 1) / 2 : 4 + col / 2);
    int ix = (int)floor(0.5 * ns * (P - 2.0 * pa + 1.0));
    int iy = (int)floor(0.5 * ns * (2.0 * qa - Q + 1.0));
    ix = ix < 0 ? 0 : (ix > ns - 1 ? ns - 1 : ix);
    iy = iy < 0 ? 0 : (iy > ns - 1 ? ns - 1 : iy);
    return face * ns * ns + (int)(spread_bits((uint32_t)ix) | (spread_bits((uint32_t)iy) << 1));
}

// Centre of a pixel: the centre of its cell on the projection plane, projected back.
__host__ __device__ void pixel_centre(int ns, int pix, double *v) {
    const int face = pix / (ns * ns), w = pix % (ns * ns);
    const int ix = (int)gather_bits((uint32_t)w), iy = (int)gather_bits((uint32_t)w >> 1);
    const int row = 1 - face / 4;                        // north 1, equator 0, south -1
    const int col = 2 * (face % 4) + (row == 0 ? 0 : 1); // the base pixel's centre X
    const double u = (ix + 0.5) / ns, t = (iy + 0.5) / ns;
    double X = col + (u - t), Y = row + (u + t - 1.0);
    X = X < 0.0 ? X + 8.0 : X;
    double zc, lon;
    if (fabs(Y) <= 1.0) {
        zc = Y / 1.5;
        lon = X * (kPi / 4.0);
    } else {
        const double sg = 2.0 - fabs(Y);
        zc = Y > 0.0 ? 1.0 - sg * sg / 3.0 : sg * sg / 3.0 - 1.0;
        const double xm = 2.0 * floor(0.5 * X) + 1.0;
        lon = (xm + (X - xm) / sg) * (kPi / 4.0);
    }
    const double st = sqrt((1.0 - zc) * (1.0 + zc));
    v[0] = st * cos(lon);
    v[1] = st * sin(lon);
    v[2] = zc;
}

// Direction cell of an integer direction: the face of the component of largest magnitude
// (ties to the lower axis; face 2 axis + 1 when it is negative), then on the two other axes,
// in increasing order, the cell floor(M (e_a + |e_m|) / (2 |e_m|)), at most M - 1.
__host__ __device__ int cell_of_direction(int64_t e0, int64_t e1, int64_t e2, int log2m) {
    const int64_t a0 = e0 < 0 ? -e0 : e0, a1 = e1 < 0 ? -e1 : e1, a2 = e2 < 0 ? -e2 : e2;
    const int axis = (a0 >= a1 && a0 >= a2) ? 0 : (a1 >= a2 ? 1 : 2);
    const int64_t m = axis == 0 ? a0 : (axis == 1 ? a1 : a2);
    const int64_t neg = (axis == 0 ? e0 : (axis == 1 ? e1 : e2)) < 0 ? 1 : 0;
    const int64_t u = axis == 0 ? e1 : e0, t = axis == 2 ? e1 : e2;
    const int64_t top = ((int64_t)1 << log2m) - 1;
    int64_t i = ((u + m) << log2m) / (2 * m), j = ((t + m) << log2m) / (2 * m);
    i = i > top ? top : i;
    j = j > top ? top : j;
    return (int)((((2 * axis + neg) << log2m) + i) << log2m) + (int)j;
}

// integer direction of the centre of cell (face, i, j), scaled by 2^16 per unit of the
// cube's half edge M
__host__ __device__ void cell_centre(int cell, int log2m, int64_t *d) {
    const int M = 1 << log2m;
    const int face = cell >> (2 * log2m), i = (cell >> log2m) & (M - 1), j = cell & (M - 1);
    const int axis = face >> 1;
    const int64_t K = (int64_t)1 << 16;
    const int64_t along = (face & 1) ? -(int64_t)M * K : (int64_t)M * K;
    const int64_t u = K * (2 * i + 1 - M), t = K * (2 * j + 1 - M);
    d[0] = axis == 0 ? along : u;
    d[1] = axis == 1 ? along : (axis == 0 ? u : t);
    d[2] = axis == 2 ? along : t;
}

__global__ void k_cell_pixels(int ns, int log2m, int16_t *__restrict__ tab) {
    const int n = 6 << (2 * log2m);
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= n) return;
    int64_t d[3];
    cell_centre(cell, log2m, d);
    tab[cell] = (int16_t)pixel_of_direction(ns, (double)d[0], (double)d[1], (double)d[2]);
}

__global__ void k_ray_dirs(int ns, float4 *__restrict__ dirs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= 12 * ns * ns) return;
    double v[3];
    pixel_centre(ns, p, v);
    dirs[p] = make_float4((float)v[0], (float)v[1], (float)v[2], 0.0f);
}

// Edge of the sub-sampled cube of distance class c around a direction of squared length
// len2: the class's middle ratio s / r = 2^(-(c + 1/2) / 2) times |d|, rounded to the
// nearest multiple of 8 so that the sub-point offsets are integers.  With k = edge / 8,
// round-to-nearest means (2k - 1)^4 <= 16 (|d| 2^(-(2c + 1) / 4) / 8)^4 < (2k + 1)^4,
// i.e. (2k - 1)^4 2^(2c + 9) <= len2^2 < (2k + 1)^4 2^(2c + 9): decided exactly in 128-bit
// integers around a floating-point estimate.
__host__ __device__ int64_t class_edge(int64_t len2, int c) {
    const double est = sqrt(sqrt((double)len2 * (double)len2 * ldexp(1.0, -(2 * c + 13))));
    int64_t k = (int64_t)rint(est);
    const unsigned __int128 L = (unsigned __int128)len2 * (unsigned __int128)len2;
    auto bound = [&](int64_t odd) { // odd^4 2^(2c + 9)
        const unsigned __int128 o2 = (unsigned __int128)(odd * odd);
        return (o2 * o2) << (2 * c + 9);
    };
    while (k > 0 && bound(2 * k - 1) > L) --k;
    while (bound(2 * k + 1) <= L) ++k;
    return 8 * k;
}

// Tabulated angular kernel: one wavefront per key (direction cell, class), lane q holding
// sub-point q = (qx, qy, qz) in [0, 4)^3 at offset (2 q_a - 3) edge / 8 from the cell's
// centre direction.  Distinct pixels are taken in ascending order as repeated wave minima,
// each with the number of lanes that hold it.  Entry (64 bits): pixels 0..3 (10 bits each
// from bit 0), counts 0..2 out of 64 (7 bits each from bit 40; count 3 is the rest), or
// bit 61 alone when more than 4 pixels are reached.
__global__ __launch_bounds__(256) void k_alpha_keys(int log2m, const int16_t *__restrict__ pixtab,
                                                     unsigned long long *__restrict__ out) {
    const int64_t n_keys = (int64_t)(6 << (2 * log2m)) * kClasses;
    const int64_t key = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (key >= n_keys) return; // whole waves leave together
    const int lane = threadIdx.x & 63;
    const int cell = (int)(key / kClasses), c = kClassFirst + (int)(key % kClasses);
    int64_t d[3];
    cell_centre(cell, log2m, d);
    const int64_t h = class_edge(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], c) / 8;
    const int64_t e0 = d[0] + (2 * (lane & 3) - 3) * h;
    const int64_t e1 = d[1] + (2 * ((lane >> 2) & 3) - 3) * h;
    const int64_t e2 = d[2] + (2 * (lane >> 4) - 3) * h;
    const int pix = pixtab[cell_of_direction(e0, e1, e2, log2m)];
    bool left = true;
    int found = 0;
    unsigned long long w = 0ull;
    for (;;) {
        int m = left ? pix : 0x7fffffff;
        for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o));
        if (m == 0x7fffffff) break; // uniform: every lane holds the same minimum
        const int cnt = __popcll(__ballot(left && pix == m));
        if (found < 4) {
            w |= (unsigned long long)m << (10 * found);
            if (found < 3) w |= (unsigned long long)cnt << (40 + 7 * found);
        }
        ++found;
        left = left && pix != m;
    }
    if (lane == 0) out[key] = found > 4 ? (1ull << 61) : w;
}

// first class from which every key holds its cell's own pixel alone: one more than the
// largest class of a key that does not
__global__ void k_alpha_first_own(int log2m, const int16_t *__restrict__ pixtab,
                                  const unsigned long long *__restrict__ full, int *__restrict__ c_own) {
    const int64_t n_keys = (int64_t)(6 << (2 * log2m)) * kClasses;
    const int64_t key = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= n_keys) return;
    const int cell = (int)(key / kClasses), c = kClassFirst + (int)(key % kClasses);
    const unsigned long long own = (unsigned long long)(uint16_t)pixtab[cell] | (64ull << 40);
    if (full[key] != own) atomicMax(c_own, c + 1);
}

// keep the classes below the first own-pixel class: [cell][ncls]
__global__ void k_alpha_compact(int64_t n_cells, int ncls, const unsigned long long *__restrict__ full,
                                unsigned long long *__restrict__ alpha) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_cells * ncls) return;
    alpha[e] = full[(e / ncls) * kClasses + e % ncls];
}

} // namespace

int tr_get_table(tr_ctx *ctx, int n_side, int cube_m, RayTable **out) {
    const auto key = std::make_pair(n_side, cube_m);
    auto it = ctx->tables.find(key);
    if (it != ctx->tables.end()) {
        *out = &it->second;
        return TR_OK;
    }
    if (n_side < 1 || n_side > 8 || (n_side & (n_side - 1)) || cube_m < 2 || cube_m > 256 || (cube_m & (cube_m - 1)))
        return tr_fail(ctx, TR_EINVAL, "bad ray table request (n_side %d, cube_m %d; powers of two, n_side <= 8, "
                       "2 <= cube_m <= 256)", n_side, cube_m);
    int log2m = 0;
    while ((1 << log2m) < cube_m) ++log2m;
    const int64_t n_cells = 6 * (int64_t)cube_m * cube_m;
    const int64_t n_keys = n_cells * kClasses;
    const int npix = 12 * n_side * n_side;
    RayTable rt;
    rt.n_side = n_side;
    rt.cube_m = cube_m;
    unsigned long long *full = nullptr;
    int *c_own = nullptr;
    auto cleanup = [&]() {
        hipFree(rt.table);
        hipFree(rt.dirs);
        hipFree(rt.alpha);
        hipFree(rt.near);
        hipFree(full);
        hipFree(c_own);
    };
    if (hipMalloc(&rt.table, sizeof(int16_t) * n_cells) != hipSuccess ||
        hipMalloc(&rt.dirs, sizeof(float4) * npix) != hipSuccess ||
        hipMalloc(&full, sizeof(unsigned long long) * n_keys) != hipSuccess ||
        hipMalloc(&c_own, sizeof(int)) != hipSuccess) {
        cleanup();
        return tr_fail(ctx, TR_ENOMEM, "ray tables");
    }
    const int c_init = kClassFirst;
    int c1 = kClassFirst;
    bool ok = hipMemcpyAsync(c_own, &c_init, sizeof(int), hipMemcpyHostToDevice, ctx->stream) == hipSuccess;
    k_cell_pixels<<<tr_div_up(n_cells, 256), 256, 0, ctx->stream>>>(n_side, log2m, rt.table);
    k_ray_dirs<<<tr_div_up(npix, 256), 256, 0, ctx->stream>>>(n_side, rt.dirs);
    k_alpha_keys<<<tr_div_up(n_keys, 4), 256, 0, ctx->stream>>>(log2m, rt.table, full);
    k_alpha_first_own<<<tr_div_up(n_keys, 256), 256, 0, ctx->stream>>>(log2m, rt.table, full, c_own);
    ok = ok && hipGetLastError() == hipSuccess;
    ok = ok && hipMemcpyAsync(&c1, c_own, sizeof(int), hipMemcpyDeviceToHost, ctx->stream) == hipSuccess;
    ok = ok && hipStreamSynchronize(ctx->stream) == hipSuccess;
    if (!ok) {
        cleanup();
        return tr_fail(ctx, TR_EHIP, "ray table kernels failed");
    }
    const int ncls = c1 - kClassFirst;
    const int64_t n_alpha = n_cells * (ncls > 0 ? ncls : 1);
    if (hipMalloc(&rt.alpha, sizeof(unsigned long long) * n_alpha) != hipSuccess) {
        cleanup();
        return tr_fail(ctx, TR_ENOMEM, "tabulated angular kernel");
    }
    if (ncls > 0)
        k_alpha_compact<<<tr_div_up(n_cells * ncls, 256), 256, 0, ctx->stream>>>(n_cells, ncls, full, rt.alpha);
    else
        ok = hipMemsetAsync(rt.alpha, 0, sizeof(unsigned long long), ctx->stream) == hipSuccess;
    ok = ok && hipGetLastError() == hipSuccess && hipStreamSynchronize(ctx->stream) == hipSuccess;
    hipFree(full);
    hipFree(c_own);
    full = nullptr;
    c_own = nullptr;
    if (!ok) {
        cleanup();
        return tr_fail(ctx, TR_EHIP, "tabulated angular kernel compaction failed");
    }
    rt.alpha_c1 = c1;
    if (int rc = tr_build_near_table(ctx, rt, log2m)) {
        cleanup();
        return rc;
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
    const int rc = tr_get_table(ctx, n_side, cube_m, &rt);
    if (rc) return rc;
    const int64_t n_cells = 6 * (int64_t)cube_m * cube_m;
    const int npix = 12 * n_side * n_side;
    std::vector<int16_t> t16(n_cells);
    std::vector<float4> d4(npix);
    TR_HIP(ctx, hipMemcpyAsync(t16.data(), rt->table, sizeof(int16_t) * n_cells, hipMemcpyDeviceToHost, ctx->stream));
    TR_HIP(ctx, hipMemcpyAsync(d4.data(), rt->dirs, sizeof(float4) * npix, hipMemcpyDeviceToHost, ctx->stream));
    TR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t e = 0; table && e < n_cells; ++e) table[e] = t16[e];
    for (int p = 0; dirs && p < npix; ++p) {
        dirs[3 * p] = d4[p].x;
        dirs[3 * p + 1] = d4[p].y;
        dirs[3 * p + 2] = d4[p].z;
    }
    return TR_OK;
}

// unpack the device table to [cell][class 6 .. 20][pixel 0..3, count 0..3, overflow flag]
extern "C" int tr_alpha_table(tr_ctx *ctx, int n_side, int cube_m, int32_t *out) {
    if (!ctx) return TR_EINVAL;
    if (!out) return tr_fail(ctx, TR_EINVAL, "tr_alpha_table: null output");
    TR_HIP(ctx, hipSetDevice(ctx->device));
    if (cube_m == 0) cube_m = 16 * n_side;
    RayTable *rt = nullptr;
    const int rc = tr_get_table(ctx, n_side, cube_m, &rt);
    if (rc) return rc;
    const int64_t n_cells = 6 * (int64_t)cube_m * cube_m;
    const int c1 = rt->alpha_c1, ncls = c1 - kClassFirst;
    std::vector<unsigned long long> a(n_cells * (ncls > 0 ? ncls : 1));
    std::vector<int16_t> pix(n_cells);
    TR_HIP(ctx, hipMemcpyAsync(a.data(), rt->alpha, sizeof(unsigned long long) * a.size(), hipMemcpyDeviceToHost,
                               ctx->stream));
    TR_HIP(ctx, hipMemcpyAsync(pix.data(), rt->table, sizeof(int16_t) * n_cells, hipMemcpyDeviceToHost, ctx->stream));
    TR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t cell = 0; cell < n_cells; ++cell)
        for (int c = kClassFirst; c <= kClassLast; ++c) {
            int32_t *o = out + 9 * (cell * kClasses + (c - kClassFirst));
            for (int k = 0; k < 9; ++k) o[k] = 0;
            if (c >= c1) { // the cell's own pixel, all 64 sub-points
                o[0] = pix[cell];
                o[4] = 64;
                continue;
            }
            const unsigned long long w = a[cell * ncls + (c - kClassFirst)];
            if ((w >> 61) & 1ull) {
                o[8] = 1;
                continue;
            }
            int rest = 64;
            for (int k = 0; k < 4; ++k) o[k] = (int32_t)((w >> (10 * k)) & 1023ull);
            for (int k = 0; k < 3; ++k) {
                o[4 + k] = (int32_t)((w >> (40 + 7 * k)) & 127ull);
                rest -= o[4 + k];
            }
            o[7] = rest;
        }
    return TR_OK;
}
