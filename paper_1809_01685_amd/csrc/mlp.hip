// Early-stopping surrogate: a 19 -> 256 -> 256 -> 2 perceptron with ReLU,
// BF16-rounded weights and FP32 sums, its Gaussian-NLL gradient and Adam.
//
// All products go through one tiled FP32 kernel C = op(A * B) with optional
// BF16 rounding of the weight operand, bias, ReLU and ReLU-mask epilogues;
// every sum runs over its reduction index in ascending order.
#include <math.h>

#include "tnslq_internal.h"

namespace tnslq {
namespace {

constexpr int NIN = TNSLQ_MLP_NIN, NH = TNSLQ_MLP_NHID, NOUT = TNSLQ_MLP_NOUT;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NOUT * NH, NPAR = OFF_B3 + NOUT;
static_assert(NPAR == TNSLQ_MLP_NPARAMS, "parameter layout");

__device__ inline float bf16_round_f(float x) { return bf16_to_f32(f32_to_bf16_rne(x)); }

// C[i][j] = sum_l A[i*sai + l*sal] * Bq[l*sbl + j*sbj]  (+ bias[j]) (relu) (* mask)
// where Bq = bf16(B) if qb.  Optional row gather on A: row i reads gather[i].
struct MM {
    const float *A;
    int64_t sai, sal;
    const int *gather;
    const float *B;
    int64_t sbl, sbj;
    int qb;
    float *C;
    int64_t ldc;
    int M, N, Kr;
    const float *bias;
    int relu;
    const float *mask;   // same layout as C; keep where mask > 0
};

__global__ void __launch_bounds__(256) k_mm(MM p) {
    __shared__ float As[16][17], Bs[16][17];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
    float acc = 0.0f;
    for (int l0 = 0; l0 < p.Kr; l0 += 16) {
        {
            const int ii = blockIdx.y * 16 + ty, ll = l0 + tx;
            float v = 0.0f;
            if (ii < p.M && ll < p.Kr) {
                const int64_t row = p.gather ? p.gather[ii] : ii;
                v = p.A[row * p.sai + (int64_t)ll * p.sal];
            }
            As[ty][tx] = v;
            const int lb = l0 + ty, jb = blockIdx.x * 16 + tx;
            float u = 0.0f;
            if (lb < p.Kr && jb < p.N) {
                u = p.B[(int64_t)lb * p.sbl + (int64_t)jb * p.sbj];
                if (p.qb) u = bf16_round_f(u);
            }
            Bs[ty][tx] = u;
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < 16; ++l) acc = fmaf(As[ty][l], Bs[l][tx], acc);
        __syncthreads();
    }
    if (i < p.M && j < p.N) {
        if (p.bias) acc += p.bias[j];
        if (p.relu) acc = fmaxf(acc, 0.0f);
        if (p.mask && !(p.mask[(int64_t)i * p.ldc + j] > 0.0f)) acc = 0.0f;
        p.C[(int64_t)i * p.ldc + j] = acc;
    }
}

// xhat = (t(x[gather]) - mean) / scale, t = asinh on the 16 Lanczos-coefficient
// features (which span many decades) and the identity on the three log2 sizes.
constexpr int N_COEF = 16;
__global__ void k_standardise(const float *__restrict__ x, const int *__restrict__ gather,
                              const float *__restrict__ norm, int B, float *__restrict__ xh) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * NIN) return;
    const int b = t / NIN, f = t % NIN;
    const int64_t row = gather ? gather[b] : b;
    float v = x[row * NIN + f];
    if (f < N_COEF) v = asinhf(v);
    xh[t] = (v - norm[f]) / norm[NIN + f];
}

// Loss and dL/du for L = (1/B) sum 0.5 (u1 + (r - u0)^2 exp(-u1)).
__global__ void __launch_bounds__(256) k_nll(const float *__restrict__ u, const float *__restrict__ r,
                                             const int *__restrict__ gather, int B, float *__restrict__ du,
                                             float *__restrict__ loss) {
    __shared__ float sh[256];
    float s = 0.0f;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const float rb = r[gather ? gather[b] : b];
        const float u0 = u[2 * b], u1 = u[2 * b + 1];
        const float d = rb - u0, ex = expf(-u1);
        du[2 * b] = -d * ex / B;
        du[2 * b + 1] = 0.5f * (1.0f - d * d * ex) / B;
        s += 0.5f * (u1 + d * d * ex);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = sh[0] / B;
}

// db[j] = sum_b dY[b][j]
__global__ void k_colsum(const float *__restrict__ dy, int B, int N, float *__restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += dy[(int64_t)b * N + j];
    db[j] = s;
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    p[i] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

inline void run_mm(const MM &p, hipStream_t st) {
    dim3 grid((p.N + 15) / 16, (p.M + 15) / 16), block(256);
    hipLaunchKernelGGL(k_mm, grid, block, 0, st, p);
}

struct Ws {
    float *xh, *z1, *z2, *u, *du, *d2, *d1;
};
inline Ws carve(void *ws, int B) {
    float *f = (float *)ws;
    Ws w;
    auto take = [&](int64_t n) {
        float *p = f;
        f += (n + 63) / 64 * 64;
        return p;
    };
    w.xh = take((int64_t)B * NIN);
    w.z1 = take((int64_t)B * NH);
    w.z2 = take((int64_t)B * NH);
    w.u = take((int64_t)B * NOUT);
    w.du = take((int64_t)B * NOUT);
    w.d2 = take((int64_t)B * NH);
    w.d1 = take((int64_t)B * NH);
    return w;
}

// Forward pass into the workspace: z1, z2 hold post-ReLU activations h1, h2
// (the ReLU masks of the backward pass are h > 0, identical to z > 0).
void forward_ws(const float *params, const float *norm, const float *x, const int *gather, int B, Ws &w,
                float *out, hipStream_t st) {
    hipLaunchKernelGGL(k_standardise, dim3((B * NIN + 255) / 256), dim3(256), 0, st, x, gather, norm, B, w.xh);
    MM p{};
    // h1 = relu(xh W1^T + b1): A = xh [B x 19], B(l=i, j=o) = W1[o][i]
    p = MM{w.xh, NIN, 1, nullptr, params + OFF_W1, 1, NIN, 1, w.z1, NH, B, NH, NIN, params + OFF_B1, 1, nullptr};
    run_mm(p, st);
    p = MM{w.z1, NH, 1, nullptr, params + OFF_W2, 1, NH, 1, w.z2, NH, B, NH, NH, params + OFF_B2, 1, nullptr};
    run_mm(p, st);
    p = MM{w.z2, NH, 1, nullptr, params + OFF_W3, 1, NH, 1, out, NOUT, B, NOUT, NH, params + OFF_B3, 0, nullptr};
    run_mm(p, st);
}

}  // namespace

size_t mlp_ws_bytes(int B) {
    auto r = [](int64_t n) { return (n + 63) / 64 * 64; };
    return sizeof(float) * (size_t)(r((int64_t)B * NIN) + 4 * r((int64_t)B * NH) + 2 * r((int64_t)B * NOUT));
}

hipError_t mlp_forward(const float *params, const float *norm, const float *x, int B, float *out, void *ws,
                       hipStream_t st) {
    Ws w = carve(ws, B);
    forward_ws(params, norm, x, nullptr, B, w, out, st);
    return hipGetLastError();
}

hipError_t mlp_loss_grad(const float *params, const float *norm, const float *x, const float *r, const int *idx,
                         int B, float *loss, float *grad, void *ws, hipStream_t st) {
    Ws w = carve(ws, B);
    forward_ws(params, norm, x, idx, B, w, w.u, st);
    hipLaunchKernelGGL(k_nll, dim3(1), dim3(256), 0, st, (const float *)w.u, r, idx, B, w.du, loss);
    MM p{};
    // dW3[o][i] = sum_b du[b][o] h2[b][i]; A(i=o, l=b) = du[b*2 + o], B(l=b, j=i) = h2[b*NH + i]
    p = MM{w.du, 1, NOUT, nullptr, w.z2, NH, 1, 0, grad + OFF_W3, NH, NOUT, NH, B, nullptr, 0, nullptr};
    run_mm(p, st);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(64), 0, st, (const float *)w.du, B, NOUT, grad + OFF_B3);
    // dz2[b][i] = (sum_o du[b][o] bf(W3[o][i])) * (h2 > 0)
    p = MM{w.du, NOUT, 1, nullptr, params + OFF_W3, NH, 1, 1, w.d2, NH, B, NH, NOUT, nullptr, 0, w.z2};
    run_mm(p, st);
    // dW2[o][i] = sum_b dz2[b][o] h1[b][i]
    p = MM{w.d2, 1, NH, nullptr, w.z1, NH, 1, 0, grad + OFF_W2, NH, NH, NH, B, nullptr, 0, nullptr};
    run_mm(p, st);
    hipLaunchKernelGGL(k_colsum, dim3((NH + 63) / 64), dim3(64), 0, st, (const float *)w.d2, B, NH, grad + OFF_B2);
    // dz1[b][i] = (sum_o dz2[b][o] bf(W2[o][i])) * (h1 > 0)
    p = MM{w.d2, NH, 1, nullptr, params + OFF_W2, NH, 1, 1, w.d1, NH, B, NH, NH, nullptr, 0, w.z1};
    run_mm(p, st);
    // dW1[o][i] = sum_b dz1[b][o] xh[b][i]
    p = MM{w.d1, 1, NH, nullptr, w.xh, NIN, 1, 0, grad + OFF_W1, NIN, NH, NIN, B, nullptr, 0, nullptr};
    run_mm(p, st);
    hipLaunchKernelGGL(k_colsum, dim3((NH + 63) / 64), dim3(64), 0, st, (const float *)w.d1, B, NH, grad + OFF_B1);
    return hipGetLastError();
}

hipError_t mlp_adam(float *params, float *m, float *v, const float *grad, int n, int t, float lr,
                    hipStream_t st) {
    const float bc1 = 1.0f - powf(0.9f, (float)t), bc2 = 1.0f - powf(0.999f, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, params, m, v, grad, n, lr, bc1, bc2);
    return hipGetLastError();
}

}  // namespace tnslq
