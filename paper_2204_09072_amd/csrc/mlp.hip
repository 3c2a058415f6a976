// Guess network for the dust-equilibrium solve (3 -> 64 -> 64 -> 1, ReLU hidden layers):
// training and inference on the matrix cores (bfloat16 operands, FP32 accumulation).
//
// One wavefront handles 32 samples at a time, on v_mfma_f32_32x32x8bf16_1k.
// 32x32x8 operand layout: lane l holds A[l%32][4(l/32)+0..3] and B[4(l/32)+0..3][l%32];
// the 16 accumulators of lane l are C[8(v/4) + 4(l/32) + v%4][l%32], v = 0..15.
//
// Training (k_mlp_train), with the hidden activations staged in LDS:
//   forward   a2[s][n]  = sum_i h1[s][i] W2[n][i]          (32 x 64 x 64)
//   backward  dh1[s][i] = sum_n da2[s][n] W2[n][i]         (32 x 64 x 64)
//             gW2[n][i] += sum_s da2[s][n] h1[s][i]        (64 x 64 x 32, kept in registers)
// and the 3-wide input and 1-wide output layers as per-lane dot products.
//
// Inference (k_mlp_infer) keeps everything in registers by working on transposed
// products, hidden units as rows and samples as columns:
//   a1[n][s] = sum_k [W1 | b1][n][k] [x; 1][k][s]          (K = 3 inputs + bias, padded to 8)
//   a2[n][s] = sum_k W2[n][k] h1[k][s] + b2[n]             (bias as one more K step)
// The accumulators of the first product are, lane for lane, the B operands of the second
// (rows 8 kk + 4(l/32) + j of column l%32), so h1 never leaves the registers; the output
// y[s] = w3 . h2[:, s] + b3 is a per-lane sum over the lane's 32 rows plus one exchange
// between the two half-waves.
#include <cmath>

#include "mlp.hpp"

using trnet::f16v;
using trnet::sh4;

namespace {

constexpr int H = MLP_H;
constexpr int S = 32;          // samples per wave step
constexpr int64_t kMaxInfer = (int64_t)1 << 28; // inference: byte offsets of [n][3] inputs fit 32 bits
constexpr int LD = H + 4;      // padded row of a bfloat16 tile

__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

enum Mode { FORWARD = 1, GUESS = 2 };

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

__global__ __launch_bounds__(256) void k_mlp_train(MlpArgs A) {
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
                x0 = A.x[3 * s];
                x1 = A.x[3 * s + 1];
                x2 = A.x[3 * s + 2];
                t = A.y[s];
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
                L.h1[s * LD + j] = bf16_bits(a > 0.0f ? a : 0.0f);
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
                const float a2 = acc[tn][v] + b2[n];
                h2[tn][v] = a2 > 0.0f ? a2 : 0.0f;
                yp[v] += w3[n] * bf16_val(bf16_bits(h2[tn][v]));
            }
        }
        // rows held by this lane: s = 8 (v/4) + 4 half + v%4
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
        // backward through the output layer and the second ReLU
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) {
            const int n = 32 * tn + col;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int s = 8 * (v >> 2) + 4 * half + (v & 3);
                const float da = h2[tn][v] > 0.0f ? dy[v] * w3[n] : 0.0f;
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
        // dh1 = da2 W2, then through the first ReLU to the input layer's gradients
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
                const float a1 = bi + wa * L.xs[s][0] + wb * L.xs[s][1] + wc * L.xs[s][2];
                const float da1 = a1 > 0.0f ? d[v] : 0.0f;
                gb1[ti] += da1;
                gw1[ti][0] += da1 * L.xs[s][0];
                gw1[ti][1] += da1 * L.xs[s][1];
                gw1[ti][2] += da1 * L.xs[s][2];
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
    }
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

// Inference, 32 samples per wave step, all operands in registers (layouts in the header).
// The second product runs on v_mfma_f32_32x32x16_bf16 (K = 16 per instruction): lane l
// contributes 8 K-slots, A and B slot for slot, and a contraction may visit K in any
// order, so K-block kk takes accumulators v = 8 (kk % 2) + j of first-layer tile kk / 2 as
// its B slots and the matching columns of W2 as its A slots.  Its bias enters as the
// accumulators' starting value (accumulator v of lane l is hidden unit 32 t + 8 (v / 4) +
// 4 half + v % 4).  The next step's inputs are loaded while the current step computes.
// The output layer is a third product, y[s] = sum_k w3[k] h2[k][s], with w3 as row 0 of
// its A operand and h2 packed exactly as h1 was; row 0 of the result is accumulator 0 of
// lanes 0..31.  Logarithm and exponential are the hardware's base-2 instructions (about
// 1 ulp, far finer than the bfloat16 rounding of the inputs and the solve's tolerance).
template <int MODE>
__global__ __launch_bounds__(256) void k_mlp_infer(MlpArgs A) {
    const int lane = threadIdx.x & 63, col = lane & 31, half = lane >> 5;
    const int wave = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    const int nwave = (int)((gridDim.x * (int64_t)blockDim.x) >> 6);
    trnet::Net net;
    net.load(A.p, col, half);
    const float inv_out = 1.0f / A.out_scale;
    const int64_t nchunk = (A.n + S - 1) / S;
    // Inputs and outputs go through buffer descriptors, whose range check returns 0 for a
    // load and drops a store at an offset beyond the array: every lane issues every load
    // and store (lanes without a sample at an out-of-range offset), so no memory operation
    // sits under a lane mask and a step waits only for the loads it reads.
    constexpr uint32_t kOut = 0xfffffff0u; // beyond any array (n < 2^28)
    const uint32_t nb = (uint32_t)A.n * 4u;
    const __amdgpu_buffer_rsrc_t rin0 = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(MODE == GUESS ? A.rho : A.x), (short)0, (int)(MODE == GUESS ? nb : 3u * nb), 0x00020000);
    const __amdgpu_buffer_rsrc_t rin1 =
        __builtin_amdgcn_make_buffer_rsrc((void *)(MODE == GUESS ? A.u_rad : A.x), (short)0, (int)(MODE == GUESS ? nb : 3u * nb), 0x00020000);
    const __amdgpu_buffer_rsrc_t rin2 =
        __builtin_amdgcn_make_buffer_rsrc((void *)(MODE == GUESS ? A.t_gas : A.x), (short)0, (int)(MODE == GUESS ? nb : 3u * nb), 0x00020000);
    const __amdgpu_buffer_rsrc_t rout = __builtin_amdgcn_make_buffer_rsrc((void *)A.out, (short)0, (int)nb, 0x00020000);
    // raw inputs of sample ch * 32 + col (half-wave 0 only; 0 elsewhere)
    auto load = [&](int64_t ch, float &x0, float &x1, float &x2) {
        const int64_t s = ch * S + col;
        const bool own = half == 0 && s < A.n;
        const uint32_t o = own ? (uint32_t)s * (MODE == GUESS ? 4u : 12u) : kOut;
        x0 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rin0, o, 0, 0));
        x1 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rin1, MODE == GUESS ? o : o + 4u, 0, 0));
        x2 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rin2, MODE == GUESS ? o : o + 8u, 0, 0));
    };
    // one 32-sample step on inputs already in registers
    auto step = [&](int64_t ch, float x0, float x1, float x2) {
        const int64_t s = ch * S + col;
        const bool live = half == 0 && s < A.n;
        if (MODE == GUESS) {
            x0 = trnet::feature(x0, A.shift[0], A.scale[0]);
            x1 = trnet::feature(x1, A.shift[1], A.scale[1]);
            x2 = trnet::feature(x2, A.shift[2], A.scale[2]);
        }
        // B operand of the first product: column s = (x0, x1, x2, 1) in half-wave 0
        const trnet::sh4 bx = live ? trnet::input_operand(x0, x1, x2) : trnet::sh4_of(0u, 0u);
        const float yv = net.eval(bx);
        const float yo = MODE == GUESS ? trnet::temperature(yv, inv_out, A.out_shift) : yv;
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(yo), rout, live ? (uint32_t)s * 4u : kOut, 0, 0);
    };
    // a wave takes steps wave, wave + nwave, ...; the inputs of the next three are in flight
    // while one computes (three register sets, so no step waits on a load issued just before)
    float a0, a1, a2, b0, b1, b2, c0, c1, c2;
    load(wave, a0, a1, a2);
    load(wave + nwave, b0, b1, b2);
    load(wave + 2 * (int64_t)nwave, c0, c1, c2);
    for (int64_t ch = wave; ch < nchunk; ch += 3 * (int64_t)nwave) {
        step(ch, a0, a1, a2);
        load(ch + 3 * (int64_t)nwave, a0, a1, a2);
        if (ch + nwave >= nchunk) break; // uniform over the wave
        step(ch + nwave, b0, b1, b2);
        load(ch + 4 * (int64_t)nwave, b0, b1, b2);
        if (ch + 2 * (int64_t)nwave >= nchunk) break;
        step(ch + 2 * (int64_t)nwave, c0, c1, c2);
        load(ch + 5 * (int64_t)nwave, c0, c1, c2);
    }
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

// blocks of 4 waves for n samples, at most per_cu blocks per compute unit (the kernels
// loop over 32-sample steps)
int grid_for(tr_ctx *ctx, int64_t n, int per_cu = 4) {
    const int64_t waves = (n + S - 1) / S;
    int64_t blocks = (waves + 3) / 4;
    const int64_t cap = (int64_t)ctx->n_cu * per_cu;
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
    if (n >= kMaxInfer) return tr_fail(ctx, TR_EINVAL, "guess network: %lld states, fewer than 2^28 required", (long long)n);
    MlpArgs A = base_args(m, n);
    A.rho = rho; A.u_rad = u_rad; A.t_gas = t_gas; A.out = guess;
    k_mlp_infer<GUESS><<<grid_for(ctx, n, 3), 256, 0, ctx->stream>>>(A); // 3 waves/SIMD fit
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

extern "C" int tr_mlp_get_state(tr_ctx *ctx, const tr_mlp *m, float *params, float *adam_m, float *adam_v,
                                int64_t *steps, float *norm) {
    if (!ctx) return TR_EINVAL;
    if (!m) return tr_fail(ctx, TR_EINVAL, "tr_mlp_get_state: null network");
    TR_HIP(ctx, hipSetDevice(ctx->device));
    const size_t b = sizeof(float) * MLP_NPARAM;
    if (params) TR_HIP(ctx, hipMemcpyAsync(params, m->p, b, hipMemcpyDeviceToHost, ctx->stream));
    if (adam_m) TR_HIP(ctx, hipMemcpyAsync(adam_m, m->m, b, hipMemcpyDeviceToHost, ctx->stream));
    if (adam_v) TR_HIP(ctx, hipMemcpyAsync(adam_v, m->v, b, hipMemcpyDeviceToHost, ctx->stream));
    TR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (steps) *steps = m->step;
    if (norm)
        for (int k = 0; k < 8; ++k) norm[k] = m->norm[k];
    return TR_OK;
}

extern "C" int tr_mlp_set_state(tr_ctx *ctx, tr_mlp *m, const float *params, const float *adam_m,
                                const float *adam_v, int64_t steps) {
    if (!ctx) return TR_EINVAL;
    if (!m || !params || steps < 0) return tr_fail(ctx, TR_EINVAL, "tr_mlp_set_state: bad argument");
    TR_HIP(ctx, hipSetDevice(ctx->device));
    const size_t b = sizeof(float) * MLP_NPARAM;
    TR_HIP(ctx, hipMemcpyAsync(m->p, params, b, hipMemcpyHostToDevice, ctx->stream));
    if (adam_m) TR_HIP(ctx, hipMemcpyAsync(m->m, adam_m, b, hipMemcpyHostToDevice, ctx->stream));
    else k_fill<<<tr_div_up(MLP_NPARAM, 256), 256, 0, ctx->stream>>>(m->m, MLP_NPARAM, 0.0f);
    if (adam_v) TR_HIP(ctx, hipMemcpyAsync(m->v, adam_v, b, hipMemcpyHostToDevice, ctx->stream));
    else k_fill<<<tr_div_up(MLP_NPARAM, 256), 256, 0, ctx->stream>>>(m->v, MLP_NPARAM, 0.0f);
    k_round<<<tr_div_up(MLP_NPARAM, 256), 256, 0, ctx->stream>>>(m->p, m->wq, MLP_NPARAM);
    TR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    m->step = steps;
    return TR_OK;
}

extern "C" int tr_mlp_forward(tr_ctx *ctx, const tr_mlp *m, int64_t n, const float *x, float *y) {
    if (!ctx) return TR_EINVAL;
    if (!m || n < 0) return tr_fail(ctx, TR_EINVAL, "tr_mlp_forward: bad argument");
    if (n == 0) return TR_OK;
    if (!x || !y) return tr_fail(ctx, TR_EINVAL, "tr_mlp_forward: null buffer");
    if (n >= kMaxInfer) return tr_fail(ctx, TR_EINVAL, "tr_mlp_forward: %lld samples, fewer than 2^28 required", (long long)n);
    MlpArgs A = base_args(m, n);
    A.x = x; A.out = y;
    k_mlp_infer<FORWARD><<<grid_for(ctx, n, 3), 256, 0, ctx->stream>>>(A);
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
    k_mlp_train<<<grid_for(ctx, n), 256, 0, ctx->stream>>>(A);
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
