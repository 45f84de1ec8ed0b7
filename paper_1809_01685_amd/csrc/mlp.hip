// Early-stopping surrogate: a 19 -> 256 -> 256 -> 2 perceptron with ReLU,
// BF16-rounded weights and FP32 sums, its Gaussian-NLL gradient and Adam.
//
// All products go through one kernel C = A op(B) on the BF16 matrix
// instructions (v_mfma_f32_16x16x32_bf16, one wave per 16 x 16 output tile)
// with bias, ReLU and ReLU-mask epilogues.  The FP32 activations enter as
// three BF16 pieces whose sum is the FP32 value exactly; a weight operand is
// rounded to BF16 (one piece, the network's weights), an activation operand
// is split too.  Every product of pieces is exact in FP32 and the matrix
// instruction sums in FP32, so the products are those of FP32 arithmetic on
// the BF16 weights (the pairs of pieces below 2^-24 of a term are left out
// when both operands are split).
#include <math.h>

#include "tnslq_internal.h"

namespace tnslq {
namespace {

constexpr int NIN = TNSLQ_MLP_NIN, NH = TNSLQ_MLP_NHID, NOUT = TNSLQ_MLP_NOUT;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NOUT * NH, NPAR = OFF_B3 + NOUT;
static_assert(NPAR == TNSLQ_MLP_NPARAMS, "parameter layout");

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

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ inline bf16x8 pack8(const uint16_t (&h)[8]) {
    uint4 v;
    v.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
    v.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
    v.z = (uint32_t)h[4] | ((uint32_t)h[5] << 16);
    v.w = (uint32_t)h[6] | ((uint32_t)h[7] << 16);
    return __builtin_bit_cast(bf16x8, v);
}

// the 16 Lanczos-coefficient features (which span many decades) are mapped
// by asinh before standardisation; the three log2 sizes are not
constexpr int N_COEF = 16;

// xhat of feature f of one raw input row x
__device__ inline float standardise(const float *__restrict__ xr, int f, const float *__restrict__ norm) {
    float v = xr[f];
    if (f < N_COEF) v = asinhf(v);
    return (v - norm[f]) / norm[NIN + f];
}

// 8 consecutive reduction terms l .. l + 7 of a row (stride `step` between
// terms), zero past K; one 32-byte vector load when the row is contiguous and
// aligned.
__device__ inline void load8(const float *__restrict__ row, int64_t step, int l, int K, bool vec, float (&v)[8]) {
    if (vec && l + 8 <= K) {
        const float4 u0 = *(const float4 *)(row + l), u1 = *(const float4 *)(row + l + 4);
        v[0] = u0.x, v[1] = u0.y, v[2] = u0.z, v[3] = u0.w, v[4] = u1.x, v[5] = u1.y, v[6] = u1.z, v[7] = u1.w;
        return;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = l + t < K ? row[(int64_t)(l + t) * step] : 0.0f;
}

// One 16 x 16 tile of C per workgroup of four waves, which take the steps of
// 32 reduction terms in turn and add their partial tiles in a fixed order.
// Per step, lane l loads A[row l % 16][k = 8 (l / 16) .. +7] and B[k][column
// l % 16] for the same k; accumulator register r holds C[4 (l / 16) + r]
// [l % 16].  BSPLIT: B is an activation (three pieces), else a weight (bf16
// of it).  STD: A is the raw network input, standardised as it is loaded
// (the tile row's xhat is also written to xh when given, by the first
// column of tiles).
template <bool BSPLIT, bool STD>
__global__ void __launch_bounds__(256) k_mm_mfma(MM p, const float *__restrict__ norm, float *__restrict__ xh) {
    __shared__ f32x4 red[4][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, fr = lane & 15, fk = lane >> 4;
    const int i = blockIdx.y * 16 + fr, j = blockIdx.x * 16 + fr;
    const int64_t arow = i < p.M ? (p.gather ? (int64_t)p.gather[i] : (int64_t)i) : -1;
    const float *Ar = arow >= 0 ? p.A + arow * p.sai : nullptr;
    const float *Bc = j < p.N ? p.B + (int64_t)j * p.sbj : nullptr;
    const bool va = !STD && p.sal == 1 && p.sai % 4 == 0 && ((uintptr_t)p.A & 15) == 0;
    const bool vb = p.sbl == 1 && p.sbj % 4 == 0 && ((uintptr_t)p.B & 15) == 0;
    if (STD && xh && blockIdx.x == 0)
        for (int e = tid; e < 16 * NIN; e += 256) {
            const int r = blockIdx.y * 16 + e / NIN, f = e % NIN;
            if (r < p.M) xh[(int64_t)r * NIN + f] = standardise(p.A + (p.gather ? p.gather[r] : r) * p.sai, f, norm);
        }
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int l0 = 32 * w; l0 < p.Kr; l0 += 128) {
        const int l = l0 + 8 * fk;
        float av[8], bv[8];
        if (Ar) {
            if constexpr (STD) {
#pragma unroll
                for (int t = 0; t < 8; ++t) av[t] = l + t < p.Kr ? standardise(Ar, l + t, norm) : 0.0f;
            } else {
                load8(Ar, p.sal, l, p.Kr, va, av);
            }
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) av[t] = 0.0f;
        }
        if (Bc) {
            load8(Bc, p.sbl, l, p.Kr, vb, bv);
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) bv[t] = 0.0f;
        }
        uint16_t a[3][8], b[3][8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            uint16_t pa[3];
            split_bf16<3>(av[t], pa);
            a[0][t] = pa[0];
            a[1][t] = pa[1];
            a[2][t] = pa[2];
            if constexpr (BSPLIT) {
                uint16_t pb[3];
                split_bf16<3>(bv[t], pb);
                b[0][t] = pb[0];
                b[1][t] = pb[1];
                b[2][t] = pb[2];
            } else {
                b[0][t] = f32_to_bf16_rne(bv[t]);
            }
        }
        const bf16x8 a0 = pack8(a[0]), a1 = pack8(a[1]), a2 = pack8(a[2]), b0 = pack8(b[0]);
        // smaller terms first
        if constexpr (BSPLIT) {
            const bf16x8 b1 = pack8(b[1]), b2 = pack8(b[2]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b2, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc, 0, 0, 0);
        } else {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc, 0, 0, 0);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc, 0, 0, 0);
    }
    red[w][lane] = acc;
    __syncthreads();
    if (w != 0) return;
    const f32x4 s = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    const int jj = blockIdx.x * 16 + fr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ii = blockIdx.y * 16 + 4 * fk + r;
        if (ii < p.M && jj < p.N) {
            float v = s[r];
            if (p.bias) v += p.bias[jj];
            if (p.relu) v = fmaxf(v, 0.0f);
            if (p.mask && !(p.mask[(int64_t)ii * p.ldc + jj] > 0.0f)) v = 0.0f;
            p.C[(int64_t)ii * p.ldc + jj] = v;
        }
    }
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

inline void run_mm(const MM &p, hipStream_t st, const float *norm = nullptr, float *xh = nullptr) {
    dim3 grid((p.N + 15) / 16, (p.M + 15) / 16), block(256);
    if (norm)
        hipLaunchKernelGGL((k_mm_mfma<false, true>), grid, block, 0, st, p, norm, xh);
    else if (p.qb)
        hipLaunchKernelGGL((k_mm_mfma<false, false>), grid, block, 0, st, p, norm, xh);
    else
        hipLaunchKernelGGL((k_mm_mfma<true, false>), grid, block, 0, st, p, norm, xh);
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

// Forward pass into the workspace: xh the standardised input, z1, z2 the
// post-ReLU activations h1, h2 (the ReLU masks of the backward pass are
// h > 0, identical to z > 0).  Three launches; the first standardises the
// raw input as it loads it.
void forward_ws(const float *params, const float *norm, const float *x, const int *gather, int B, Ws &w,
                float *out, hipStream_t st) {
    MM p{};
    // h1 = relu(xh W1^T + b1): A = x [B x 19] (standardised on load), B(l=i, j=o) = W1[o][i]
    p = MM{x, NIN, 1, gather, params + OFF_W1, 1, NIN, 1, w.z1, NH, B, NH, NIN, params + OFF_B1, 1, nullptr};
    run_mm(p, st, norm, w.xh);
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
