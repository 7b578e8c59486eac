// Warm-start MLP: d_in -> hidden -> hidden -> d_out with ReLU, on the
// bfloat16 matrix cores of gfx950 (v_mfma_f32_16x16x32_bf16, float32
// accumulation).  A project form around the paper's method: the network maps
// a system descriptor to initial ansatz angles; plain random initialisation
// stays the reference.
//
// Every GEMM operand is rounded to bfloat16 (round to nearest, ties to even)
// as it is loaded; products are exact in float32 and accumulated in float32;
// bias, ReLU and the ReLU mask of the backward pass are applied in float32.
// One generic kernel covers all eight GEMMs of a training step: operands are
// addressed through (row, column) strides, so transposed operands need no
// copies.  Each wavefront computes one 16 x 16 output tile.
#include "mlp_common.h"

namespace dvq {

struct GemmArgs {
    int M, N, K;
    const float* A;  // A(m, k) = A[m * sam + k * sak]
    int64_t sam, sak;
    const float* B;  // B(k, n) = B[k * sbk + n * sbn]
    int64_t sbk, sbn;
    float* C;  // C[m * ldc + n]
    int64_t ldc;
    const float* bias;  // [N] or null
    const float* mask;  // C(m, n) = 0 unless mask[m * ldm + n] > 0 (or null)
    int64_t ldm;
    int relu;
};

__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tiles_n = (g.N + 15) / 16;
    const int tm = wave / tiles_n, tn = wave - tm * tiles_n;
    if (tm * 16 >= g.M) return;  // no barriers below: a wave may leave early
    const int r = lane & 15, kb = (lane >> 4) * 8;
    const int m = tm * 16 + r, n = tn * 16 + r;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    // operands of k-step k0 (zero outside the matrices)
    auto load = [&](int k0, bf16x8& a, bf16x8& b) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k0 + kb + j;
            const float av = (m < g.M && k < g.K) ? g.A[m * g.sam + k * g.sak] : 0.f;
            const float bv = (n < g.N && k < g.K) ? g.B[k * g.sbk + n * g.sbn] : 0.f;
            a[j] = to_bf16(av);
            b[j] = to_bf16(bv);
        }
    };
    // the loads of step k0 + 32 are issued before the product of step k0
    bf16x8 a, b;
    load(0, a, b);
    for (int k0 = 0; k0 < g.K; k0 += 32) {
        bf16x8 an = a, bn = b;
        if (k0 + 32 < g.K) load(k0 + 32, an, bn);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        a = an;
        b = bn;
    }
    const int nn = tn * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int mm = tm * 16 + 4 * (lane >> 4) + i;
        if (mm < g.M && nn < g.N) {
            float v = acc[i];
            if (g.bias) v += g.bias[nn];
            if (g.relu) v = fmaxf(v, 0.f);
            if (g.mask && !(g.mask[mm * g.ldm + nn] > 0.f)) v = 0.f;
            g.C[mm * g.ldc + nn] = v;
        }
    }
}

static dvq_status gemm(const GemmArgs& g, hipStream_t s) {
    const int tiles = ((g.M + 15) / 16) * ((g.N + 15) / 16);
    hipLaunchKernelGGL(k_gemm_bf16, dim3((tiles + 3) / 4), dim3(256), 0, s, g);
    DVQ_CHECK_LAUNCH("k_gemm_bf16");
    return DVQ_OK;
}

// out[n] = sum_m X[m * ld + n] (float32, fixed order).  A workgroup covers
// 64 columns with 16 row groups: wave g sums rows g, g + 16, ... (lanes read
// 64 consecutive columns of a row), then lane c of wave 0 adds the 16
// partials of its column in group order.  One thread per column would chain
// M dependent loads; this chains M / 16.
constexpr int kColsumGroups = 16;

__global__ void __launch_bounds__(64 * kColsumGroups)
k_colsum(const float* __restrict__ X, int M, int N, int64_t ld, float* __restrict__ out) {
    __shared__ float part[kColsumGroups][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    float s = 0.f;
    if (n < N)
        for (int m = g; m < M; m += kColsumGroups) s += X[(int64_t)m * ld + n];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && n < N) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < kColsumGroups; ++k) t += part[k][c];
        out[n] = t;
    }
}

static dvq_status colsum(const float* X, int M, int N, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3((N + 63) / 64), dim3(64 * kColsumGroups), 0, s, X, M, N, (int64_t)N, out);
    DVQ_CHECK_LAUNCH("k_colsum");
    return DVQ_OK;
}

// dY = sin(Y - T) / count; loss = mean(1 - cos(Y - T)) in float64.
__global__ void __launch_bounds__(1024)
k_loss_grad(const float* __restrict__ Y, const float* __restrict__ T, int64_t count,
            float* __restrict__ dY, double* __restrict__ loss) {
    __shared__ double red[16];
    double acc = 0.0;
    const float inv = 1.0f / (float)count;
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
        const float d = Y[i] - T[i];
        dY[i] = sinf(d) * inv;
        acc += 1.0 - cos((double)d);
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0 && loss) *loss = acc / (double)count;
}

__global__ void k_adamw(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, int64_t count, float lr, float b1, float b2, float eps,
                        float wd, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float mh = mi / c1, vh = vi / c2;
        p[i] -= lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
    }
}

static GemmArgs ga(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B,
                   int64_t sbk, int64_t sbn, float* C, int64_t ldc) {
    GemmArgs g{};
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.sbk = sbk;
    g.sbn = sbn;
    g.C = C;
    g.ldc = ldc;
    return g;
}

}  // namespace dvq

using namespace dvq;

extern "C" {

int64_t dvq_mlp_param_count(const dvq_mlp_shape* s) {
    if (!s) return 0;
    return offsets(*s).total;
}

size_t dvq_mlp_workspace_bytes(const dvq_mlp_shape* s, int32_t batch) {
    if (!s || batch < 1) return 0;
    return 2 * (size_t)batch * s->hidden * sizeof(float);
}

dvq_status dvq_mlp_forward(const dvq_mlp_shape* shape, const float* params, const float* X,
                           int32_t batch, float* H1, float* H2, float* Y, dvq_stream stream) {
    dvq_status st = check_shape(shape, batch);
    if (st != DVQ_OK) return st;
    DVQ_REQUIRE(params && X && H1 && H2 && Y, "null device pointer");
    const dvq_mlp_shape s = *shape;
    const MlpOffsets o = offsets(s);
    hipStream_t hs = stream_of(stream);
    const int H = s.hidden;
    GemmArgs g = ga(batch, H, s.d_in, X, s.d_in, 1, params + o.W1, 1, s.d_in, H1, H);
    g.bias = params + o.b1;
    g.relu = 1;
    if ((st = gemm(g, hs)) != DVQ_OK) return st;
    g = ga(batch, H, H, H1, H, 1, params + o.W2, 1, H, H2, H);
    g.bias = params + o.b2;
    g.relu = 1;
    if ((st = gemm(g, hs)) != DVQ_OK) return st;
    g = ga(batch, s.d_out, H, H2, H, 1, params + o.W3, 1, H, Y, s.d_out);
    g.bias = params + o.b3;
    return gemm(g, hs);
}

dvq_status dvq_mlp_loss_grad(const float* Y, const float* T, int64_t count, float* dY, double* loss,
                             dvq_stream stream) {
    DVQ_REQUIRE(Y && T && dY, "null device pointer");
    DVQ_REQUIRE(count >= 1, "count < 1");
    hipLaunchKernelGGL(k_loss_grad, dim3(1), dim3(1024), 0, stream_of(stream), Y, T, count, dY, loss);
    DVQ_CHECK_LAUNCH("k_loss_grad");
    return DVQ_OK;
}

dvq_status dvq_mlp_backward(const dvq_mlp_shape* shape, const float* params, const float* X,
                            const float* H1, const float* H2, const float* dY, int32_t batch,
                            float* dparams, void* workspace, size_t workspace_bytes,
                            dvq_stream stream) {
    dvq_status st = check_shape(shape, batch);
    if (st != DVQ_OK) return st;
    DVQ_REQUIRE(params && X && H1 && H2 && dY && dparams, "null device pointer");
    const size_t need = dvq_mlp_workspace_bytes(shape, batch);
    if (!workspace || workspace_bytes < need)
        return fail(DVQ_ECAPACITY, "mlp workspace %zu B < %zu B", workspace_bytes, need);
    const dvq_mlp_shape s = *shape;
    const MlpOffsets o = offsets(s);
    const int H = s.hidden, D = s.d_out, B = batch;
    float* dZ2 = static_cast<float*>(workspace);
    float* dZ1 = dZ2 + (size_t)B * H;
    hipStream_t hs = stream_of(stream);
    // dW3 = dY^T H2 ; db3 = colsum(dY)
    if ((st = gemm(ga(D, H, B, dY, 1, D, H2, H, 1, dparams + o.W3, H), hs)) != DVQ_OK) return st;
    if ((st = colsum(dY, B, D, dparams + o.b3, hs)) != DVQ_OK) return st;
    // dZ2 = (dY W3) * [H2 > 0]
    GemmArgs g = ga(B, H, D, dY, D, 1, params + o.W3, H, 1, dZ2, H);
    g.mask = H2;
    g.ldm = H;
    if ((st = gemm(g, hs)) != DVQ_OK) return st;
    // dW2 = dZ2^T H1 ; db2 = colsum(dZ2)
    if ((st = gemm(ga(H, H, B, dZ2, 1, H, H1, H, 1, dparams + o.W2, H), hs)) != DVQ_OK) return st;
    if ((st = colsum(dZ2, B, H, dparams + o.b2, hs)) != DVQ_OK) return st;
    // dZ1 = (dZ2 W2) * [H1 > 0]
    g = ga(B, H, H, dZ2, H, 1, params + o.W2, H, 1, dZ1, H);
    g.mask = H1;
    g.ldm = H;
    if ((st = gemm(g, hs)) != DVQ_OK) return st;
    // dW1 = dZ1^T X ; db1 = colsum(dZ1)
    if ((st = gemm(ga(H, s.d_in, B, dZ1, 1, H, X, s.d_in, 1, dparams + o.W1, s.d_in), hs)) != DVQ_OK)
        return st;
    return colsum(dZ1, B, H, dparams + o.b1, hs);
}

dvq_status dvq_adamw_step(float* params, const float* grads, float* m, float* v, int64_t count,
                          int32_t t, float lr, float beta1, float beta2, float eps,
                          float weight_decay, dvq_stream stream) {
    DVQ_REQUIRE(params && grads && m && v, "null device pointer");
    DVQ_REQUIRE(count >= 1 && t >= 1, "count >= 1 and t >= 1 required");
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    const int64_t blocks = (count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024;
    hipLaunchKernelGGL(k_adamw, dim3((unsigned)blocks), dim3(256), 0, stream_of(stream), params, grads, m,
                       v, count, lr, beta1, beta2, eps, weight_decay, c1, c2);
    DVQ_CHECK_LAUNCH("k_adamw");
    return DVQ_OK;
}

}  // extern "C"
