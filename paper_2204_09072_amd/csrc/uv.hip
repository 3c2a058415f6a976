// Ionising side of the stellar sources (Sec. 7.2) and the UV radiation pressure on dust and
// gas (App. C of Klepitko et al. 2023).  The ionising photon flux itself comes from the
// ionising-radiation solver and is an input here.
#include <cmath>

#include "common.hpp"

namespace {

constexpr double kPi = 3.14159265358979323846;

// gamma(T) = fraction of a black body's power above the Lyman limit.  The Planck integral
// int_x0^inf x^3 / (e^x - 1) dx with x0 = t_lyc / T is summed as the series of its
// geometric expansion, sum_k e^{-k x0} (x0^3/k + 3 x0^2/k^2 + 6 x0/k^3 + 6/k^4), until the
// terms fall below 1e-17 of the sum; the missing tail of the 6/k^4 terms (~ 2/K^3) is added
// in closed form when x0 is small.
__device__ double lyman_fraction(double T, double t_lyc) {
    if (!(T > 0.0)) return 0.0;
    const double x0 = t_lyc / T;
    const double I0 = kPi * kPi * kPi * kPi / 15.0;
    double s = 0.0;
    int k = 1;
    for (; k <= 20000; ++k) {
        const double dk = (double)k;
        const double e = exp(-dk * x0);
        const double term = e * (x0 * x0 * x0 / dk + 3.0 * x0 * x0 / (dk * dk) + 6.0 * x0 / (dk * dk * dk) +
                                 6.0 / (dk * dk * dk * dk));
        s += term;
        if (term < 1e-17 * s) break;
    }
    if (k > 20000) {
        // remaining sum_{k > K} 6 e^{-k x0} / k^4 ~ 2 / K^3 (x0 K << 1), with K = 20000
        const double K = 20000.0;
        s += 2.0 / (K * K * K) * exp(-K * x0);
    }
    const double g = s / I0;
    return g > 1.0 ? 1.0 : g;
}

__global__ void k_star_split(int n, const double *__restrict__ L_int, const double *__restrict__ L_acc,
                             const double *__restrict__ r_star, double f_fill, double sigma, double t_lyc,
                             double *__restrict__ L_uv, double *__restrict__ L_ir) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double area = 4.0 * kPi * r_star[s] * r_star[s];
    const double T_int = pow(L_int[s] / (sigma * area), 0.25);
    const double T_acc = pow(L_acc[s] / (f_fill * sigma * area), 0.25);
    const double uv = lyman_fraction(T_int, t_lyc) * L_int[s] + lyman_fraction(T_acc, t_lyc) * L_acc[s];
    L_uv[s] = uv;
    L_ir[s] = L_int[s] + L_acc[s] - uv;
}

// Written per unit mass so that single precision stays in range: with q = e_ph / (c mu m_H),
// a_dust + a_H = q n_ph (sigma_d + sigma_h (1 - x)) and a_H+ = q x^2 (rho / mu m_H) alpha_b;
// the rates per volume are rho times these.
__global__ __launch_bounds__(256) void k_uv_rp(int64_t n, const float *__restrict__ rho, const float *__restrict__ x_ion,
                                               const float *__restrict__ nph, const float *__restrict__ uph,
                                               float q, float sigma_d, float sigma_h, float alpha_b,
                                               float inv_mu_mh, float *__restrict__ a, float *__restrict__ parts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float r = rho[i], x = x_ion[i], N = nph[i];
    const float qN = q * N;
    const float ad = qN * sigma_d;
    const float ah = qN * (sigma_h * (1.0f - x));
    const float ai = q * (x * x) * (r * inv_mu_mh) * alpha_b;
    const float f = ad + ah + ai;
    a[i] = f * uph[i];
    a[n + i] = f * uph[n + i];
    a[2 * n + i] = f * uph[2 * n + i];
    if (parts) {
        parts[i] = r * ad;
        parts[n + i] = r * ah;
        parts[2 * n + i] = r * ai;
    }
}

} // namespace

extern "C" int tr_star_luminosity_split(tr_ctx *ctx, int n, const double *L_int, const double *L_acc,
                                        const double *r_star, double f_fill, double sigma, double t_lyc,
                                        double *L_uv, double *L_ir) {
    if (!ctx) return TR_EINVAL;
    if (n < 0 || (n > 0 && (!L_int || !L_acc || !r_star || !L_uv || !L_ir)) || !(f_fill > 0) || !(sigma > 0) ||
        !(t_lyc > 0))
        return tr_fail(ctx, TR_EINVAL, "tr_star_luminosity_split: bad argument");
    if (n == 0) return TR_OK;
    TR_HIP(ctx, hipSetDevice(ctx->device));
    k_star_split<<<(n + 63) / 64, 64, 0, ctx->stream>>>(n, L_int, L_acc, r_star, f_fill, sigma, t_lyc, L_uv, L_ir);
    return hipGetLastError() == hipSuccess ? TR_OK : tr_fail(ctx, TR_EHIP, "star split launch failed");
}

extern "C" int tr_uv_rad_pressure(tr_ctx *ctx, int64_t n, const float *rho, const float *x_ion, const float *n_ph,
                                  const float *u_ph, const tr_uv_params *p, float *a_uv, float *parts) {
    if (!ctx) return TR_EINVAL;
    if (n < 0 || !p || (n > 0 && (!rho || !x_ion || !n_ph || !u_ph || !a_uv)) || !(p->c > 0) || !(p->mu_mh > 0))
        return tr_fail(ctx, TR_EINVAL, "tr_uv_rad_pressure: bad argument");
    if (n == 0) return TR_OK;
    TR_HIP(ctx, hipSetDevice(ctx->device));
    k_uv_rp<<<(int)tr_div_up(n, 256), 256, 0, ctx->stream>>>(
        n, rho, x_ion, n_ph, u_ph, (float)(p->e_ph / (p->c * p->mu_mh)), (float)p->sigma_d, (float)p->sigma_h,
        (float)p->alpha_b, (float)(1.0 / p->mu_mh), a_uv, parts);
    return hipGetLastError() == hipSuccess ? TR_OK : tr_fail(ctx, TR_EHIP, "uv radiation pressure launch failed");
}
