// Guess network for the dust-equilibrium solve: training and inference on the matrix
// cores (bfloat16 operands, FP32 accumulation).
//
// One wavefront handles 32 samples at a time.  The hidden layer products that are real
// matrix products run on v_mfma_f32_32x32x8bf16_1k:
//   forward   a2[s][n]  = sum_i h1[s][i] W2[n][i]          (32 x 64 x 64)
//   backward  dh1[s][i] = sum_n da2[s][n] W2[n][i]         (32 x 64 x 64)
//             gW2[n][i] += sum_s da2[s][n] h1[s][i]        (64 x 64 x 32, kept in registers)
// The 3-wide input layer and the 1-wide output layer are per-lane dot products.
// 32x32x8 operand layout: lane l holds A[l%32][4(l/32)+0..3] and B[4(l/32)+0..3][l%32];
// the 16 accumulators of lane l are C[8(v/4) + 4(l/32) + v%4][l%32], v = 0..15.
#include <cmath>

#include "mlp.hpp"

typedef short sh4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

namespace {

constexpr int H = MLP_H;
constexpr int S = 32;          // samples per wave step
constexpr int LD = H + 4;      // padded row of a bfloat16 tile

__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

enum Mode { TRAIN = 0, FORWARD = 1, GUESS = 2 };

struct MlpArgs {
    int64_t n;
    const float *x;      // TRAIN/FORWARD: [n][3] normalised inputs
    const float *y;      // TRAIN: targets
    const float *rho, *u_rad, *t_gas; // GUESS: raw fields
    float *out;          // FORWARD: y; GUESS: temperature guess
    float *grad, *loss;  // TRAIN
    const float *p;      // FP32 parameters
    float shift[3], scale[3], out_shift, out_scale;
    float inv_n;
};

struct WaveLds {
    uint16_t h1[S * LD];
    uint16_t da2[S * LD];
    float xs[S][3];
    float t[S];
    float dy[S];
};

template <int MODE>
__global__ __launch_bounds__(256) void k_mlp(MlpArgs A) {
    __shared__ uint16_t w2[H * LD];   // W2[n][i]
    __shared__ uint16_t w2t[H * LD];  // W2[n][i] stored as [i][n]
    __shared__ float w1[3 * H], b1[H], b2[H], w3[H];
    __shared__ float gacc[MLP_NPARAM];
    __shared__ WaveLds wl[4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int k = tid; k < H * H; k += 256) {
        const int n = k / H, i = k % H;
        const uint16_t b = bf16_bits(A.p[MLP_OFF_W2 + k]);
        w2[n * LD + i] = b;
        w2t[i * LD + n] = b;
    }
    for (int k = tid; k < 3 * H; k += 256) w1[k] = bf16_val(bf16_bits(A.p[k]));
    for (int k = tid; k < H; k += 256) {
        b1[k] = bf16_val(bf16_bits(A.p[MLP_OFF_B1 + k]));
        b2[k] = bf16_val(bf16_bits(A.p[MLP_OFF_B2 + k]));
        w3[k] = bf16_val(bf16_bits(A.p[MLP_OFF_W3 + k]));
    }
    if (MODE == TRAIN)
        for (int k = tid; k < MLP_NPARAM; k += 256) gacc[k] = 0.0f;
    __syncthreads();
    const float b3 = bf16_val(bf16_bits(A.p[MLP_OFF_B3]));
    WaveLds &L = wl[wv];
    const int col = lane & 31, half = lane >> 5;

    f16v gw2[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) gw2[a][b][v] = 0.0f;
    float gw1[2][3] = {{0, 0, 0}, {0, 0, 0}}, gb1[2] = {0, 0}, gb2[2] = {0, 0}, gw3[2] = {0, 0};
    float gb3 = 0.0f, lsum = 0.0f;

    const int64_t nchunk = (A.n + S - 1) / S;
    for (int64_t ch = (int64_t)blockIdx.x * 4 + wv; ch < nchunk; ch += (int64_t)gridDim.x * 4) {
        const int64_t s0 = ch * S;
        const int cnt = A.n - s0 < S ? (int)(A.n - s0) : S;
        // inputs, rounded to bfloat16
        if (lane < S) {
            float x0 = 0, x1 = 0, x2 = 0, t = 0;
            if (lane < cnt) {
                const int64_t s = s0 + lane;
                if (MODE == GUESS) {
                    x0 = (log10f(fmaxf(A.rho[s], 1e-37f)) - A.shift[0]) * A.scale[0];
                    x1 = (log10f(fmaxf(A.u_rad[s], 1e-37f)) - A.shift[1]) * A.scale[1];
                    x2 = (log10f(fmaxf(A.t_gas[s], 1e-37f)) - A.shift[2]) * A.scale[2];
                } else {
                    x0 = A.x[3 * s];
                    x1 = A.x[3 * s + 1];
                    x2 = A.x[3 * s + 2];
                }
                if (MODE == TRAIN) t = A.y[s];
            }
            L.xs[lane][0] = bf16_val(bf16_bits(x0));
            L.xs[lane][1] = bf16_val(bf16_bits(x1));
            L.xs[lane][2] = bf16_val(bf16_bits(x2));
            L.t[lane] = t;
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        // first layer: lane = hidden unit
        {
            const int j = lane;
            const float wa = w1[3 * j], wb = w1[3 * j + 1], wc = w1[3 * j + 2], bj = b1[j];
            for (int s = 0; s < S; ++s) {
                const float a = bj + wa * L.xs[s][0] + wb * L.xs[s][1] + wc * L.xs[s][2];
                L.h1[s * LD + j] = bf16_bits(tanh_fast(a));
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        // second layer on the matrix cores: a2 = h1 W2^T
        f16v acc[2];
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) {
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[tn][v] = 0.0f;
#pragma unroll
            for (int kk = 0; kk < H / 8; ++kk) {
                const int k = 8 * kk + 4 * half;
                sh4 a = *reinterpret_cast<const sh4 *>(&L.h1[col * LD + k]);
                sh4 b = *reinterpret_cast<const sh4 *>(&w2[(32 * tn + col) * LD + k]);
                acc[tn] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc[tn], 0, 0, 0);
            }
        }
        // hidden activations (unrounded kept for the derivative) and the output layer
        float h2[2][16];
        float yp[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) yp[v] = 0.0f;
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) {
            const int n = 32 * tn + col;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                h2[tn][v] = tanh_fast(acc[tn][v] + b2[n]);
                yp[v] += w3[n] * bf16_val(bf16_bits(h2[tn][v]));
            }
        }
        // rows held by this lane: s = 8 (v/4) + 4 half + v%4
        if (MODE != TRAIN) {
            // sum over the 32 lanes of a half-wave by halving exchanges: after the steps
            // over lane bits 4, 3, 2, 1 (8 + 4 + 2 + 1 shuffles) and a last one over bit
            // 0, lane l holds the full sum of row v = 8 b4 + 4 b3 + 2 b2 + b1, b_k being
            // bit k of the lane
            float r8[8], r4[4], r2[2], r1;
            const bool k4 = col & 16, k3 = col & 8, k2 = col & 4, k1 = col & 2;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float keep = k4 ? yp[j + 8] : yp[j], send = k4 ? yp[j] : yp[j + 8];
                r8[j] = keep + __shfl_xor(send, 16);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float keep = k3 ? r8[j + 4] : r8[j], send = k3 ? r8[j] : r8[j + 4];
                r4[j] = keep + __shfl_xor(send, 8);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const float keep = k2 ? r4[j + 2] : r4[j], send = k2 ? r4[j] : r4[j + 2];
                r2[j] = keep + __shfl_xor(send, 4);
            }
            {
                const float keep = k1 ? r2[1] : r2[0], send = k1 ? r2[0] : r2[1];
                r1 = keep + __shfl_xor(send, 2);
            }
            r1 += __shfl_xor(r1, 1);
            const int v = (k4 ? 8 : 0) + (k3 ? 4 : 0) + (k2 ? 2 : 0) + (k1 ? 1 : 0);
            const int s = 8 * (v >> 2) + 4 * half + (v & 3);
            if ((col & 1) == 0 && s < cnt) {
                const float yv = r1 + b3;
                A.out[s0 + s] = MODE == GUESS ? exp10f(yv / A.out_scale + A.out_shift) : yv;
            }
            continue;
        }
#pragma unroll
        for (int v = 0; v < 16; ++v)
            for (int o = 1; o < 32; o <<= 1) yp[v] += __shfl_xor(yp[v], o);
        float dy[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int s = 8 * (v >> 2) + 4 * half + (v & 3);
            const float r = s < cnt ? yp[v] + b3 - L.t[s] : 0.0f;
            dy[v] = 2.0f * r * A.inv_n;
            if (col == 0) {
                lsum += r * r;
                gb3 += dy[v];
            }
        }
        // backward through the output layer and the second tanh
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) {
            const int n = 32 * tn + col;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int s = 8 * (v >> 2) + 4 * half + (v & 3);
                const float da = dy[v] * w3[n] * (1.0f - h2[tn][v] * h2[tn][v]);
                gw3[tn] += dy[v] * bf16_val(bf16_bits(h2[tn][v]));
                gb2[tn] += da;
                L.da2[s * LD + n] = bf16_bits(da);
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        // gW2 += da2^T h1 (K = the 32 samples)
#pragma unroll
        for (int tn = 0; tn < 2; ++tn)
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int kk = 0; kk < S / 8; ++kk) {
                    const int s = 8 * kk + 4 * half;
                    sh4 a, b;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        a[r] = (short)L.da2[(s + r) * LD + 32 * tn + col];
                        b[r] = (short)L.h1[(s + r) * LD + 32 * ti + col];
                    }
                    gw2[tn][ti] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, gw2[tn][ti], 0, 0, 0);
                }
        // dh1 = da2 W2, then through the first tanh to the input layer's gradients
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) {
            f16v d;
#pragma unroll
            for (int v = 0; v < 16; ++v) d[v] = 0.0f;
#pragma unroll
            for (int kk = 0; kk < H / 8; ++kk) {
                const int k = 8 * kk + 4 * half;
                sh4 a = *reinterpret_cast<const sh4 *>(&L.da2[col * LD + k]);
                sh4 b = *reinterpret_cast<const sh4 *>(&w2t[(32 * ti + col) * LD + k]);
                d = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, d, 0, 0, 0);
            }
            const int i = 32 * ti + col;
            const float wa = w1[3 * i], wb = w1[3 * i + 1], wc = w1[3 * i + 2], bi = b1[i];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int s = 8 * (v >> 2) + 4 * half + (v & 3);
                const float h = tanh_fast(bi + wa * L.xs[s][0] + wb * L.xs[s][1] + wc * L.xs[s][2]);
                const float da1 = d[v] * (1.0f - h * h);
                gb1[ti] += da1;
                gw1[ti][0] += da1 * L.xs[s][0];
                gw1[ti][1] += da1 * L.xs[s][1];
                gw1[ti][2] += da1 * L.xs[s][2];
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
    }
    if (MODE != TRAIN) return;
    // block reduction of the gradients in LDS, then one global add per parameter
#pragma unroll
    for (int tn = 0; tn < 2; ++tn)
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int n = 32 * tn + 8 * (v >> 2) + 4 * half + (v & 3);
                const int i = 32 * ti + col;
                atomicAdd(&gacc[MLP_OFF_W2 + H * n + i], gw2[tn][ti][v]);
            }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int j = 32 * t + col;
        atomicAdd(&gacc[MLP_OFF_B1 + j], gb1[t]);
        atomicAdd(&gacc[3 * j], gw1[t][0]);
        atomicAdd(&gacc[3 * j + 1], gw1[t][1]);
        atomicAdd(&gacc[3 * j + 2], gw1[t][2]);
        atomicAdd(&gacc[MLP_OFF_B2 + j], gb2[t]);
        atomicAdd(&gacc[MLP_OFF_W3 + j], gw3[t]);
    }
    if (col == 0) atomicAdd(&gacc[MLP_OFF_B3], gb3);
    __syncthreads();
    for (int k = tid; k < MLP_NPARAM; k += 256) atomicAdd(&A.grad[k], gacc[k]);
    if (col == 0) atomicAdd(A.loss, lsum * A.inv_n);
}

__global__ void k_fill(float *p, int n, float v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_adam(float *p, float *m, float *v, const float *g, float *wq, int n, float lr, float c1,
                       float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
    p[i] = pi;
    wq[i] = bf16_round(pi);
}

__global__ void k_round(const float *p, float *wq, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wq[i] = bf16_round(p[i]);
}

int grid_for(tr_ctx *ctx, int64_t n) {
    const int64_t waves = (n + S - 1) / S;
    int64_t blocks = (waves + 3) / 4;
    const int64_t cap = (int64_t)ctx->n_cu * 4;
    if (blocks > cap) blocks = cap;
    return (int)(blocks < 1 ? 1 : blocks);
}

MlpArgs base_args(const tr_mlp *m, int64_t n) {
    MlpArgs A = {};
    A.n = n;
    A.p = m->p;
    for (int k = 0; k < 3; ++k) {
        A.shift[k] = m->norm[k];
        A.scale[k] = m->norm[3 + k];
    }
    A.out_shift = m->norm[6];
    A.out_scale = m->norm[7];
    A.inv_n = n > 0 ? 1.0f / (float)n : 0.0f;
    return A;
}

} // namespace

int mlp_guess(tr_ctx *ctx, const tr_mlp *m, int64_t n, const float *rho, const float *u_rad,
              const float *t_gas, float *guess) {
    MlpArgs A = base_args(m, n);
    A.rho = rho; A.u_rad = u_rad; A.t_gas = t_gas; A.out = guess;
    k_mlp<GUESS><<<grid_for(ctx, n), 256, 0, ctx->stream>>>(A);
    return hipGetLastError() == hipSuccess ? TR_OK : tr_fail(ctx, TR_EHIP, "mlp guess launch failed");
}

extern "C" int tr_mlp_n_params(void) { return MLP_NPARAM; }

extern "C" int tr_mlp_create(tr_ctx *ctx, const float *params, const float *norm, tr_mlp **out) {
    if (!ctx) return TR_EINVAL;
    if (!params || !out) return tr_fail(ctx, TR_EINVAL, "tr_mlp_create: null argument");
    TR_HIP(ctx, hipSetDevice(ctx->device));
    tr_mlp *m = new tr_mlp();
    m->ctx = ctx;
    if (norm)
        for (int k = 0; k < 8; ++k) m->norm[k] = norm[k];
    const size_t b = sizeof(float) * MLP_NPARAM;
    if (hipMalloc(&m->p, b) != hipSuccess || hipMalloc(&m->wq, b) != hipSuccess ||
        hipMalloc(&m->m, b) != hipSuccess || hipMalloc(&m->v, b) != hipSuccess ||
        hipMalloc(&m->grad, b) != hipSuccess || hipMalloc(&m->loss, sizeof(float)) != hipSuccess) {
        tr_mlp_free(m);
        return tr_fail(ctx, TR_ENOMEM, "tr_mlp_create: allocation failed");
    }
    if (hipMemcpyAsync(m->p, params, b, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        hipMemsetAsync(m->m, 0, b, ctx->stream) != hipSuccess ||
        hipMemsetAsync(m->v, 0, b, ctx->stream) != hipSuccess) {
        tr_mlp_free(m);
        return tr_fail(ctx, TR_EHIP, "tr_mlp_create: upload failed");
    }
    k_round<<<tr_div_up(MLP_NPARAM, 256), 256, 0, ctx->stream>>>(m->p, m->wq, MLP_NPARAM);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
        tr_mlp_free(m);
        return tr_fail(ctx, TR_EHIP, "tr_mlp_create: sync failed");
    }
    *out = m;
    return TR_OK;
}

extern "C" void tr_mlp_free(tr_mlp *m) {
    if (!m) return;
    hipFree(m->p); hipFree(m->wq); hipFree(m->m); hipFree(m->v); hipFree(m->grad); hipFree(m->loss);
    delete m;
}

extern "C" int tr_mlp_get_params(tr_ctx *ctx, const tr_mlp *m, float *params) {
    if (!ctx || !m || !params) return TR_EINVAL;
    TR_HIP(ctx, hipMemcpyAsync(params, m->p, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, ctx->stream));
    TR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return TR_OK;
}

extern "C" int tr_mlp_forward(tr_ctx *ctx, const tr_mlp *m, int64_t n, const float *x, float *y) {
    if (!ctx) return TR_EINVAL;
    if (!m || !x || !y || n < 0) return tr_fail(ctx, TR_EINVAL, "tr_mlp_forward: bad argument");
    if (n == 0) return TR_OK;
    MlpArgs A = base_args(m, n);
    A.x = x; A.out = y;
    k_mlp<FORWARD><<<grid_for(ctx, n), 256, 0, ctx->stream>>>(A);
    return hipGetLastError() == hipSuccess ? TR_OK : tr_fail(ctx, TR_EHIP, "mlp forward launch failed");
}

extern "C" int tr_mlp_grad(tr_ctx *ctx, const tr_mlp *m, int64_t n, const float *x, const float *y,
                           float *grad, float *loss) {
    if (!ctx) return TR_EINVAL;
    if (!m || !x || !y || !grad || !loss || n <= 0) return tr_fail(ctx, TR_EINVAL, "tr_mlp_grad: bad argument");
    k_fill<<<tr_div_up(MLP_NPARAM, 256), 256, 0, ctx->stream>>>(grad, MLP_NPARAM, 0.0f);
    k_fill<<<1, 64, 0, ctx->stream>>>(loss, 1, 0.0f);
    MlpArgs A = base_args(m, n);
    A.x = x; A.y = y; A.grad = grad; A.loss = loss;
    k_mlp<TRAIN><<<grid_for(ctx, n), 256, 0, ctx->stream>>>(A);
    return hipGetLastError() == hipSuccess ? TR_OK : tr_fail(ctx, TR_EHIP, "mlp grad launch failed");
}

extern "C" int tr_mlp_train_step(tr_ctx *ctx, tr_mlp *m, int64_t n, const float *x, const float *y,
                                 float lr, float *loss) {
    if (!ctx) return TR_EINVAL;
    int rc = tr_mlp_grad(ctx, m, n, x, y, m->grad, loss ? loss : m->loss);
    if (rc) return rc;
    m->step += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, m->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, m->step)));
    k_adam<<<tr_div_up(MLP_NPARAM, 256), 256, 0, ctx->stream>>>(m->p, m->m, m->v, m->grad, m->wq, MLP_NPARAM,
                                                                 lr, c1, c2);
    return hipGetLastError() == hipSuccess ? TR_OK : tr_fail(ctx, TR_EHIP, "adam launch failed");
}
