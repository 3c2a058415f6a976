// Self-consistent dust temperature (Sec. 2 and 4.6 of Klepitko et al. 2023): the dust
// temperature sets the Planck-mean opacity and the thermal emission of every cell (the
// b-node content of Sec. 4.1), the traced radiation field sets the dust temperature
// through the equilibrium of Sec. 4.6.  Inside FLASH the two meet over time steps; here
// the loop build -> trace -> equilibrium is repeated to a fixed point.
#include <cstring>

#include "common.hpp"

namespace {

// largest |T_new - T_old| / T_new, as the bit pattern of a positive float (ordered like
// the float) combined with an integer atomic maximum
__global__ __launch_bounds__(256) void k_max_rel_change(int64_t n, const float *__restrict__ t_old,
                                                        const float *__restrict__ t_new, int *__restrict__ out) {
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float a = t_old[i], b = t_new[i];
        const float r = fabsf(b - a) / fmaxf(b, 1e-30f);
        m = r > m ? r : m;
        m = r != r ? 3.0e38f : m; // NaN counts as no convergence
    }
    for (int o = 32; o > 0; o >>= 1) {
        const float v = __shfl_xor(m, o);
        m = v > m ? v : m;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_int(m));
}

__global__ void k_copy(int64_t n, const float *__restrict__ a, float *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

__global__ void k_zero1(int *p) { *p = 0; }

} // namespace

extern "C" int tr_dust_fixed_point(tr_ctx *ctx, const tr_grid *grid, const float *rho, const float *t_gas,
                                   const tr_star *stars, int n_stars, const tr_units *units,
                                   const tr_trace_params *tp, const tr_dust_params *dp, const tr_mlp *mlp,
                                   int max_iter, float tol, float *t_dust, float *J, float *F, float *u_rad,
                                   int32_t *iterations, float *max_rel_change) {
    if (!ctx) return TR_EINVAL;
    if (!grid || !rho || !t_gas || !units || !tp || !dp || !t_dust || !J || !F || !u_rad || max_iter < 1)
        return tr_fail(ctx, TR_EINVAL, "tr_dust_fixed_point: bad argument");
    TR_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t n = (int64_t)grid->n_blk * 512;
    float *t_new = nullptr;
    int *d_max = ctx->d_ctl + 24;
    if (hipMalloc(&t_new, sizeof(float) * n) != hipSuccess) return tr_fail(ctx, TR_ENOMEM, "fixed point workspace");
    int rc = TR_OK, it = 0;
    float change = 0.0f;
    const int blocks = (int)(tr_div_up(n, 256) < 4096 ? tr_div_up(n, 256) : 4096);
    // the tree is built once; each later sweep refills its content for the new dust
    // temperature (kappa = kappa_P(T_dust)) on the same blocks, without allocating
    tr_tree *tree = nullptr;
    tr_star *d_stars = nullptr;
    if (n_stars > 0 && (hipMalloc(&d_stars, sizeof(tr_star) * n_stars) != hipSuccess ||
                        hipMemcpyAsync(d_stars, stars, sizeof(tr_star) * n_stars, hipMemcpyHostToDevice,
                                       ctx->stream) != hipSuccess)) {
        hipFree(d_stars);
        hipFree(t_new);
        return tr_fail(ctx, TR_ENOMEM, "fixed point star buffer");
    }
    for (it = 1; it <= max_iter; ++it) {
        rc = it == 1 ? tr_build_tree(ctx, grid, rho, nullptr, t_dust, stars, n_stars, units, &tree)
                     : tr_tree_refill(ctx, tree, rho, nullptr, t_dust, d_stars, n_stars);
        if (rc) break;
        rc = tr_trace_rays(ctx, tree, tp, J, F, u_rad);
        if (rc == TR_OK) rc = tr_dust_equilibrium(ctx, n, rho, u_rad, t_gas, dp, mlp, t_new, nullptr);
        if (rc == TR_OK) {
            k_zero1<<<1, 1, 0, ctx->stream>>>(d_max);
            k_max_rel_change<<<blocks, 256, 0, ctx->stream>>>(n, t_dust, t_new, d_max);
            k_copy<<<blocks, 256, 0, ctx->stream>>>(n, t_new, t_dust);
            int bits = 0;
            if (hipMemcpyAsync(ctx->h_err, d_max, sizeof(int), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
                hipStreamSynchronize(ctx->stream) != hipSuccess)
                rc = tr_fail(ctx, TR_EHIP, "fixed point: readback failed");
            else
                bits = *ctx->h_err;
            memcpy(&change, &bits, sizeof(float));
        }
        if (rc == TR_OK) rc = tr_sync(ctx); // device-side failures of the trace
        if (rc || change <= tol) break;
    }
    hipStreamSynchronize(ctx->stream);
    tr_tree_free(tree);
    hipFree(d_stars);
    hipFree(t_new);
    if (iterations) *iterations = it > max_iter ? max_iter : it;
    if (max_rel_change) *max_rel_change = change;
    return rc;
}
