// Fused warm-start MLP: one training step (input standardisation, forward,
// loss, backward, AdamW) in three launches, and a one-launch forward pass.
//
// Same arithmetic as the GEMM-per-layer path of mlp.hip: every GEMM operand
// rounded to bfloat16, float32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16), bias, ReLU, ReLU masks and the bias gradients
// in float32 on the unrounded values; the loss term and its output gradient
// come from one float sincos of half the difference (the same quantities to
// float rounding).
//
// Layout.  A workgroup (16 wavefronts) owns a chunk of 32 batch rows and
// keeps that chunk's activations in LDS as bfloat16, row-major where they
// are the A operand of a product and transposed where the batch index is
// the contraction index (the weight-gradient products), so every operand
// fragment is one 16-byte LDS read.  The inference pass reads the weights
// from the float32 master copy (L2-resident, 77 K parameters) and rounds them
// as they are loaded; the training step first makes a bfloat16 copy laid out
// so that every weight fragment of the step is one 16-byte load (W2 and W3
// also transposed for the backward products), and each wavefront of a chunk
// loads the fragments of its output columns one phase ahead of their use.
// Everything a chunk contributes to
// the gradient is a sum over its own rows, so the backward pass needs no
// other chunk: each workgroup writes its partial gradient; the last launch
// sums the partials in chunk order (bit-reproducible) and applies AdamW.
#include "mlp_common.h"

namespace dvq {

constexpr int kFR = 32;          // batch rows per workgroup
constexpr int kFRS = kFR + 8;    // row stride (elements) of the transposed [*][rows] arrays
constexpr int kFKin = 32;        // first-layer contraction (d_in padded)
constexpr int kFDmax = 128;      // largest d_out of the fused kernels
constexpr int kFDS = kFDmax + 8; // row stride of dY
constexpr int kFWaves = 16;     // wavefronts per workgroup: the output tiles of a product spread over them
constexpr int kFThreads = 64 * kFWaves;

template <int H>
struct FusedLds {
    static constexpr int HS = H + 8;  // row stride of the [rows][H] arrays
    __bf16 xs[kFR * (kFKin + 8)];     // standardised X, [r][k]
    __bf16 xT[kFKin * kFRS];          // the same, [k][r]
    __bf16 h1[kFR * HS];              // relu(layer 1), [r][h]
    __bf16 h1T[H * kFRS];             // [h][r]
    __bf16 h2[kFR * HS];              // relu(layer 2), [r][h]; dZ2 after the mask
    __bf16 h2T[H * kFRS];             // [h][r]; dZ1^T after dW3
    __bf16 dy[kFR * kFDS];            // dY, [r][d]
    __bf16 dyT[kFDmax * kFRS];        // [d][r]
    __bf16 dz2T[H * kFRS];            // [h][r]
    float colsum[2][H > kFDmax ? H : kFDmax];  // column sums for b3, then b1
    float cs2[2][H];                           // column sums for b2
    double loss[kFThreads / 64];
};

// MFMA 16x16x32 fragments: lane l holds row (or column) l & 15 and the
// contraction indices 8 (l >> 4) .. 8 (l >> 4) + 7.
__device__ __forceinline__ bf16x8 frag_lds(const __bf16* base, int ld, int row0, int k0, int lane) {
    return *reinterpret_cast<const bf16x8*>(base + (row0 + (lane & 15)) * ld + k0 + 8 * (lane >> 4));
}

// B[k][n] = W[n][k] from a row-major float32 W[nmax][ldw] (contiguous in k):
// two 16-byte loads when the fragment is inside W and aligned.
__device__ __forceinline__ bf16x8 frag_w(const float* __restrict__ W, int ldw, int nmax, int kmax, int n0, int k0,
                                         int lane) {
    const int n = n0 + (lane & 15), kb = k0 + 8 * (lane >> 4);
    bf16x8 v;
    if (n < nmax && kb + 8 <= kmax && (ldw & 3) == 0) {
        const float4* p = reinterpret_cast<const float4*>(W + (int64_t)n * ldw + kb);
        const float4 a = p[0], b = p[1];
        v[0] = to_bf16(a.x), v[1] = to_bf16(a.y), v[2] = to_bf16(a.z), v[3] = to_bf16(a.w);
        v[4] = to_bf16(b.x), v[5] = to_bf16(b.y), v[6] = to_bf16(b.z), v[7] = to_bf16(b.w);
        return v;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (n < nmax && kb + j < kmax) ? to_bf16(W[(int64_t)n * ldw + kb + j]) : to_bf16(0.f);
    return v;
}

// A fragment of a bfloat16 matrix in device memory (row stride ld elements,
// multiple of 8): one 16-byte load per lane.
__device__ __forceinline__ bf16x8 frag_g(const __bf16* __restrict__ W, int ld, int row0, int k0, int lane) {
    return *reinterpret_cast<const bf16x8*>(W + (int64_t)(row0 + (lane & 15)) * ld + k0 + 8 * (lane >> 4));
}

// The weights of one training step, rounded to bfloat16 once and laid out so
// that every B fragment of the step is contiguous (zero padding past d_in and
// d_out): w1 [H][32] = W1; w2 [H][H] = W2; w2t [H][H] = W2^T; w3 [128][H] =
// W3; w3t [H][128] = W3^T.
struct W16 {
    __bf16 *w1, *w2, *w2t, *w3, *w3t;
};

__host__ __device__ inline size_t w16_elems(int H) {
    return (size_t)H * kFKin + 2 * (size_t)H * H + 2 * (size_t)kFDmax * H;
}

__host__ __device__ inline W16 w16_layout(void* base, int H) {
    W16 w;
    w.w1 = static_cast<__bf16*>(base);
    w.w2 = w.w1 + (size_t)H * kFKin;
    w.w2t = w.w2 + (size_t)H * H;
    w.w3 = w.w2t + (size_t)H * H;
    w.w3t = w.w3 + (size_t)kFDmax * H;
    return w;
}

// H a compile-time constant: the index splits are shifts (the layouts hold
// at most 2^18 elements, 32-bit indices).
template <int H>
__global__ void __launch_bounds__(256)
k_mlp_weights_bf16(const float* __restrict__ params, int d_in, int d_out, W16 w) {
    const dvq_mlp_shape sh{d_in, H, d_out};
    const MlpOffsets o = offsets(sh);
    constexpr int n1 = H * kFKin, n2 = H * H, n3 = kFDmax * H;
    constexpr int total = n1 + 2 * n2 + 2 * n3;
    const float* W1 = params + o.W1;
    const float* W2 = params + o.W2;
    const float* W3 = params + o.W3;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        if (e < n1) {
            const int h = e / kFKin, i = e % kFKin;
            w.w1[e] = to_bf16(i < d_in ? W1[h * d_in + i] : 0.f);
        } else if (e < n1 + n2) {
            const int x = e - n1;
            w.w2[x] = to_bf16(W2[x]);
        } else if (e < n1 + 2 * n2) {
            const int x = e - n1 - n2;
            const int r = x / H, c = x % H;
            w.w2t[x] = to_bf16(W2[c * H + r]);
        } else if (e < n1 + 2 * n2 + n3) {
            const int x = e - n1 - 2 * n2;
            const int d = x / H, k = x % H;
            w.w3[x] = to_bf16(d < d_out ? W3[d * H + k] : 0.f);
        } else {
            const int x = e - n1 - 2 * n2 - n3;
            const int h = x / kFDmax, d = x % kFDmax;
            w.w3t[x] = to_bf16(d < d_out ? W3[d * H + h] : 0.f);
        }
    }
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Sum over the 16 rows of an output tile of one column (lanes l, l + 16,
// l + 32, l + 48 hold rows 4q .. 4q + 3 of column l & 15); lanes 0..15 get it.
__device__ __forceinline__ float tile_colsum(f32x4 v) {
    float s = (v[0] + v[1]) + (v[2] + v[3]);
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    return s;
}

// Inference forward pass of one chunk up to layer 2: xs/xT, h1/h1T, h2/h2T
// in LDS, weights rounded from the float32 master copy as they are loaded.
template <int H>
__device__ __forceinline__ void fused_forward_hidden(FusedLds<H>& S, const float* __restrict__ params,
                                                     const MlpOffsets& o, int d_in,
                                                     const float* __restrict__ X,
                                                     int x_rows, const int32_t* __restrict__ rows, int row0,
                                                     int nrows, const float* __restrict__ mu,
                                                     const float* __restrict__ isd) {
    constexpr int HS = FusedLds<H>::HS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // standardised inputs (zeros past the batch and past d_in)
    for (int e = tid; e < kFR * kFKin; e += kFThreads) {
        const int r = e / kFKin, k = e - r * kFKin;
        float v = 0.f;
        if (r < nrows && k < d_in) {
            const int64_t src = rows ? (int64_t)rows[row0 + r] : (int64_t)(row0 + r);
            if (src >= 0 && src < x_rows) {
                v = X[src * d_in + k];
                if (mu) v = (v - mu[k]) * isd[k];
            }
        }
        const __bf16 q = to_bf16(v);
        S.xs[r * (kFKin + 8) + k] = q;
        S.xT[k * kFRS + r] = q;
    }
    __syncthreads();
    // layer 1: [32 x 32] x W1^T, one contraction step per tile
    for (int t = wave; t < 2 * (H / 16); t += kFWaves) {
        const int tm = t & 1, tn = t >> 1;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const bf16x8 b = frag_w(params + o.W1, d_in, H, d_in, 16 * tn, 0, lane);
        acc = mfma(frag_lds(S.xs, kFKin + 8, 16 * tm, 0, lane), b, acc);
        const int n = 16 * tn + (lane & 15);
        const float bias = params[o.b1 + n];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * tm + 4 * (lane >> 4) + i;
            const __bf16 q = to_bf16(fmaxf(acc[i] + bias, 0.f));
            S.h1[r * HS + n] = q;
            S.h1T[n * kFRS + r] = q;
        }
    }
    __syncthreads();
    // layer 2: [32 x H] x W2^T
    for (int t = wave; t < 2 * (H / 16); t += kFWaves) {
        const int tm = t & 1, tn = t >> 1;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < H; k0 += 32)
            acc = mfma(frag_lds(S.h1, HS, 16 * tm, k0, lane),
                       frag_w(params + o.W2, H, H, H, 16 * tn, k0, lane), acc);
        const int n = 16 * tn + (lane & 15);
        const float bias = params[o.b2 + n];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * tm + 4 * (lane >> 4) + i;
            const __bf16 q = to_bf16(fmaxf(acc[i] + bias, 0.f));
            S.h2[r * HS + n] = q;
            S.h2T[n * kFRS + r] = q;
        }
    }
    __syncthreads();
}

// Layer 3 of tile t: returns the float32 outputs (bias added).
template <int H>
__device__ __forceinline__ f32x4 fused_layer3(const FusedLds<H>& S, const float* __restrict__ params,
                                              const MlpOffsets& o, int d_out, int tm, int tn, int lane) {
    constexpr int HS = FusedLds<H>::HS;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < H; k0 += 32)
        acc = mfma(frag_lds(S.h2, HS, 16 * tm, k0, lane),
                   frag_w(params + o.W3, H, d_out, H, 16 * tn, k0, lane), acc);
    const int n = 16 * tn + (lane & 15);
    const float bias = n < d_out ? params[o.b3 + n] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += bias;
    return acc;
}

template <int H>
__global__ void __launch_bounds__(kFThreads)
k_mlp_predict(const float* __restrict__ params, int d_in, int d_out, const float* __restrict__ X, int batch,
              const float* __restrict__ mu, const float* __restrict__ isd, float* __restrict__ Y) {
    extern __shared__ __align__(16) unsigned char smem[];
    FusedLds<H>& S = *reinterpret_cast<FusedLds<H>*>(smem);
    const dvq_mlp_shape sh{d_in, H, d_out};
    const MlpOffsets o = offsets(sh);
    const int row0 = blockIdx.x * kFR, nrows = batch - row0 < kFR ? batch - row0 : kFR;
    fused_forward_hidden<H>(S, params, o, d_in, X, batch, nullptr, row0, nrows, mu, isd);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ntn = (d_out + 15) / 16;
    for (int t = wave; t < 2 * ntn; t += kFWaves) {
        const int tm = t & 1, tn = t >> 1;
        const f32x4 y = fused_layer3<H>(S, params, o, d_out, tm, tn, lane);
        const int n = 16 * tn + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * tm + 4 * (lane >> 4) + i;
            if (r < nrows && n < d_out) Y[(int64_t)(row0 + r) * d_out + n] = y[i];
        }
    }
}

// One chunk's forward pass, loss and partial gradient (same packing as the
// parameters) into pg[blockIdx.x][*]; its loss sum into lossp[blockIdx.x].
// Wavefront w owns column tile w of every product whose output is H wide
// (both 16-row halves of the chunk, so each weight fragment is loaded once)
// and output tile (w mod 2, w / 2) when w < 2 ceil(d_out / 16).  The
// weights of the step live in device memory and each phase ends at a
// barrier (which waits for LDS traffic only), so each wavefront issues its
// global loads one phase ahead of their use: the input and target rows and
// the layer-1/2 fragments at the start, the layer-3 and W3^T fragments during
// layer 2, the W2^T fragments during layer 3.  Loads complete in issue
// order, hence the order of use; they are not all issued at the start
// because the compute unit's memory pipeline serves them in turn, and the
// bulk of the weights would then delay the input rows the first product
// waits for.
template <int H>
__global__ void __launch_bounds__(kFThreads)
k_mlp_train_chunk(const float* __restrict__ params, int d_in, int d_out, const float* __restrict__ X,
                  const float* __restrict__ T, int x_rows, const int32_t* __restrict__ rows, int batch,
                  const float* __restrict__ mu, const float* __restrict__ isd, W16 w, float* __restrict__ pg,
                  double* __restrict__ lossp) {
    constexpr int HS = FusedLds<H>::HS;
    constexpr int HT = H / 16, KH = H / 32, KDM = kFDmax / 32;
    static_assert(HT <= kFWaves, "one hidden column tile per wavefront");
    static_assert(2 * (kFDmax / 16) <= kFWaves, "one output tile per wavefront");
    extern __shared__ __align__(16) unsigned char smem[];
    FusedLds<H>& S = *reinterpret_cast<FusedLds<H>*>(smem);
    const dvq_mlp_shape sh{d_in, H, d_out};
    const MlpOffsets o = offsets(sh);
    const int row0 = blockIdx.x * kFR, nrows = batch - row0 < kFR ? batch - row0 : kFR;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    float* g = pg + (int64_t)blockIdx.x * o.total;
    const int ntn = (d_out + 15) / 16, nkd = (d_out + 31) / 32;
    const bool hcol = wave < HT, ytile = wave < 2 * ntn;
    const int cn = 16 * wave + (lane & 15);  // the lane's column in its tiles
    const int rq = 4 * (lane >> 4);          // its first row in a 16-row tile
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero8 = {};

    // Source rows: the thread's input row and, in the wavefronts of the
    // output layer, the lane's four target rows (-1: none).  Every global
    // load of the chunk depends on these or on nothing, so two round trips
    // to device memory precede the first product.
    static_assert(kFR * kFKin == kFThreads, "one input element per thread");
    const int xr = tid / kFKin, xk = tid - xr * kFKin;
    const int ytm = wave & 1, yn = 16 * (wave >> 1) + (lane & 15);  // output tile (ytm, wave / 2)
    // (rows r >= nrows load row nrows - 1 and are then dropped, so the five
    // loads are unconditional and in flight together)
    int rr[5];
    rr[0] = xr;
#pragma unroll
    for (int i = 0; i < 4; ++i) rr[1 + i] = 16 * ytm + rq + i;
    int64_t rv[5];
    if (rows) {
#pragma unroll
        for (int j = 0; j < 5; ++j) rv[j] = rows[row0 + (rr[j] < nrows ? rr[j] : nrows - 1)];
    } else {
#pragma unroll
        for (int j = 0; j < 5; ++j) rv[j] = row0 + rr[j];
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) rv[j] = rr[j] < nrows && rv[j] >= 0 && rv[j] < x_rows ? rv[j] : -1;
    const int64_t xsrc = rv[0];
    // the standardised input element (zero past the batch and past d_in)
    // and the targets (every lane loads, an in-bounds element where there is
    // no target, so the loads are in flight together)
    const bool xin = xsrc >= 0 && xk < d_in;
    const int xkc = xk < d_in ? xk : 0;
    const float xraw = X[(xin ? xsrc : 0) * d_in + xkc];
    const float xmu = mu ? mu[xkc] : 0.f, xisd = mu ? isd[xkc] : 1.f;
    float tv[4] = {0.f, 0.f, 0.f, 0.f};
    int valid = 0;  // bit i: row 16 ytm + rq + i has a target in column yn
    if (ytile) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool ok = rv[1 + i] >= 0 && yn < d_out;
            tv[i] = T[(ok ? rv[1 + i] : 0) * d_out + (yn < d_out ? yn : 0)];
            valid |= (int)ok << i;
        }
    }
    // weights of layers 1 and 2 (hidden column tile), in the order of use
    // (loads complete in order)
    bf16x8 f1 = zero8, fa[KH], fb[KH], fc[KDM];
    float bias1 = 0.f, bias2 = 0.f, bias3 = 0.f;
#pragma unroll
    for (int k = 0; k < KH; ++k) fa[k] = fb[k] = zero8;
#pragma unroll
    for (int k = 0; k < KDM; ++k) fc[k] = zero8;
    if (hcol) {
        bias1 = params[o.b1 + cn];
        f1 = frag_g(w.w1, kFKin, 16 * wave, 0, lane);
        bias2 = params[o.b2 + cn];
#pragma unroll
        for (int k = 0; k < KH; ++k) fa[k] = frag_g(w.w2, H, 16 * wave, 32 * k, lane);
    }
    {
        const float xv = xin ? (mu ? (xraw - xmu) * xisd : xraw) : 0.f;
        const __bf16 q = to_bf16(xv);
        S.xs[xr * (kFKin + 8) + xk] = q;
        S.xT[xk * kFRS + xr] = q;
    }
    // dY cleared (columns past d_out stay zero)
    for (int e = tid; e < kFR * kFDS; e += kFThreads) S.dy[e] = to_bf16(0.f);
    for (int e = tid; e < kFDmax * kFRS; e += kFThreads) S.dyT[e] = to_bf16(0.f);
    __syncthreads();

    // layer 1: [32 x 32] x W1^T, one contraction step per tile
    if (hcol) {
#pragma unroll
        for (int tm = 0; tm < 2; ++tm) {
            const f32x4 acc = mfma(frag_lds(S.xs, kFKin + 8, 16 * tm, 0, lane), f1, zero4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * tm + rq + i;
                const __bf16 q = to_bf16(fmaxf(acc[i] + bias1, 0.f));
                S.h1[r * HS + cn] = q;
                S.h1T[cn * kFRS + r] = q;
            }
        }
    }
    __syncthreads();

    // layer 2: [32 x H] x W2^T
    if (hcol) {
#pragma unroll
        for (int tm = 0; tm < 2; ++tm) {
            f32x4 acc = zero4;
#pragma unroll
            for (int k = 0; k < KH; ++k) acc = mfma(frag_lds(S.h1, HS, 16 * tm, 32 * k, lane), fa[k], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * tm + rq + i;
                const __bf16 q = to_bf16(fmaxf(acc[i] + bias2, 0.f));
                S.h2[r * HS + cn] = q;
                S.h2T[cn * kFRS + r] = q;
            }
        }
    }
    // loads for layer 3 (output tile) and for dZ2 = dY W3 (W3^T)
    if (ytile) {
        bias3 = yn < d_out ? params[o.b3 + yn] : 0.f;
#pragma unroll
        for (int k = 0; k < KH; ++k) fb[k] = frag_g(w.w3, H, 16 * (wave >> 1), 32 * k, lane);
    }
    if (hcol) {
#pragma unroll
        for (int k = 0; k < KDM; ++k)
            if (k < nkd) fc[k] = frag_g(w.w3t, kFDmax, 16 * wave, 32 * k, lane);
    }
    __syncthreads();

    // layer 3, loss and dY = sin(Y - T) / (batch * d_out); zeros past the batch
    const float inv = 1.0f / ((float)batch * (float)d_out);
    double lsum = 0.0;
    if (ytile) {
        f32x4 acc = zero4;
#pragma unroll
        for (int k = 0; k < KH; ++k) acc = mfma(frag_lds(S.h2, HS, 16 * ytm, 32 * k, lane), fb[k], acc);
        f32x4 d = zero4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * ytm + rq + i;
            if (valid & (1 << i)) {
                // sin(x) = 2 sin(x/2) cos(x/2) and 1 - cos(x) = 2 sin(x/2)^2
                // from one float sincos (the loss term without the
                // cancellation of 1 - cos near x = 0)
                const float diff = (acc[i] + bias3) - tv[i];
                float sh, ch;
                sincosf(0.5f * diff, &sh, &ch);
                d[i] = 2.f * sh * ch * inv;
                lsum += 2.0 * (double)sh * (double)sh;
            }
            const __bf16 q = to_bf16(d[i]);
            S.dy[r * kFDS + yn] = q;
            S.dyT[yn * kFRS + r] = q;
        }
        const float cs = tile_colsum(d);
        if (lane < 16) S.colsum[ytm][yn] = cs;
    }
    // loads for dZ1 = dZ2 W2 (W2^T fragments, over the layer-2 ones)
    if (hcol) {
#pragma unroll
        for (int k = 0; k < KH; ++k) fa[k] = frag_g(w.w2t, H, 16 * wave, 32 * k, lane);
    }
    lsum = wave_sum(lsum);
    if (lane == 0) S.loss[wave] = lsum;
    __syncthreads();
    if (tid == 0) {
        double ls = 0.0;
        for (int v = 0; v < kFWaves; ++v) ls += S.loss[v];
        lossp[blockIdx.x] = ls;
    }
    for (int n = tid; n < d_out; n += kFThreads) g[o.b3 + n] = S.colsum[0][n] + S.colsum[1][n];

    // dZ2 = (dY W3) * [h2 > 0] (written over h2, each element read and
    // written by the lane that owns it, and as dz2T; column sums for b2 into
    // cs2), beside dW3 = dY^T h2 (contraction over the chunk's rows: one step)
    if (hcol) {
#pragma unroll
        for (int tm = 0; tm < 2; ++tm) {
            f32x4 acc = zero4;
#pragma unroll
            for (int k = 0; k < KDM; ++k)
                if (k < nkd) acc = mfma(frag_lds(S.dy, kFDS, 16 * tm, 32 * k, lane), fc[k], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * tm + rq + i;
                const bool on = (float)S.h2[r * HS + cn] > 0.f;
                acc[i] = on ? acc[i] : 0.f;
                const __bf16 q = to_bf16(acc[i]);
                S.h2[r * HS + cn] = q;
                S.dz2T[cn * kFRS + r] = q;
            }
            const float cs = tile_colsum(acc);
            if (lane < 16) S.cs2[tm][cn] = cs;
        }
    }
    for (int u = wave; u < ntn * HT; u += kFWaves) {
        const int tm = u % ntn, tn = u / ntn;  // tm over d_out, tn over H
        const f32x4 acc = mfma(frag_lds(S.dyT, kFRS, 16 * tm, 0, lane), frag_lds(S.h2T, kFRS, 16 * tn, 0, lane), zero4);
        const int n = 16 * tn + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int d = 16 * tm + rq + i;
            if (d < d_out) g[o.W3 + (int64_t)d * H + n] = acc[i];
        }
    }
    __syncthreads();
    for (int n = tid; n < H; n += kFThreads) g[o.b2 + n] = S.cs2[0][n] + S.cs2[1][n];

    // dZ1 = (dZ2 W2) * [h1 > 0] as dZ1^T over h2T (h2T was last read by dW3;
    // column sums for b1 into colsum), beside dW2 = dZ2^T h1
    if (hcol) {
#pragma unroll
        for (int tm = 0; tm < 2; ++tm) {
            f32x4 acc = zero4;
#pragma unroll
            for (int k = 0; k < KH; ++k) acc = mfma(frag_lds(S.h2, HS, 16 * tm, 32 * k, lane), fa[k], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * tm + rq + i;
                const bool on = (float)S.h1[r * HS + cn] > 0.f;
                acc[i] = on ? acc[i] : 0.f;
                S.h2T[cn * kFRS + r] = to_bf16(acc[i]);
            }
            const float cs = tile_colsum(acc);
            if (lane < 16) S.colsum[tm][cn] = cs;
        }
    }
    for (int u = wave; u < HT * HT; u += kFWaves) {
        const int tm = u % HT, tn = u / HT;
        const f32x4 acc = mfma(frag_lds(S.dz2T, kFRS, 16 * tm, 0, lane), frag_lds(S.h1T, kFRS, 16 * tn, 0, lane), zero4);
        const int n = 16 * tn + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) g[o.W2 + (int64_t)(16 * tm + rq + i) * H + n] = acc[i];
    }
    __syncthreads();
    for (int n = tid; n < H; n += kFThreads) g[o.b1 + n] = S.colsum[0][n] + S.colsum[1][n];

    // dW1 = dZ1^T X
    const int nti = (d_in + 15) / 16;
    for (int t = wave; t < HT * nti; t += kFWaves) {
        const int tm = t % HT, tn = t / HT;
        const f32x4 acc = mfma(frag_lds(S.h2T, kFRS, 16 * tm, 0, lane), frag_lds(S.xT, kFRS, 16 * tn, 0, lane), zero4);
        const int n = 16 * tn + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (n < d_in) g[o.W1 + (int64_t)(16 * tm + rq + i) * d_in + n] = acc[i];
    }
}

// Sum of the chunks' partial gradients (chunk order), then AdamW; the loss
// sum over chunks into loss[0] (mean over batch x d_out).
__global__ void __launch_bounds__(256)
k_mlp_reduce_adamw(const float* __restrict__ pg, int chunks, int64_t count, float* __restrict__ p,
                   float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2, float eps, float wd,
                   float c1, float c2, float* __restrict__ grads, const double* __restrict__ lossp, double inv_count,
                   double* __restrict__ loss) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        float gi = 0.f;
        for (int c = 0; c < chunks; ++c) gi += pg[(int64_t)c * count + i];
        if (grads) grads[i] = gi;
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * p[i]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
        double s = 0.0;
        for (int c = 0; c < chunks; ++c) s += lossp[c];
        *loss = s * inv_count;
    }
}

// Column mean and 1 / standard deviation (n - 1 denominator, at least
// 1e-12) of X [rows][d], float64 sums in row order.
__global__ void __launch_bounds__(64) k_feature_stats(const float* __restrict__ X, int rows, int d,
                                                     float* __restrict__ mean, float* __restrict__ inv_std) {
    const int k = blockIdx.x;
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += 64) s += X[(int64_t)r * d + k];
    s = wave_sum(s);
    const double mu = s / rows;
    double q = 0.0;
    for (int r = threadIdx.x; r < rows; r += 64) {
        const double e = X[(int64_t)r * d + k] - mu;
        q += e * e;
    }
    q = wave_sum(q);
    if (threadIdx.x == 0) {
        const double sd = rows > 1 ? sqrt(q / (rows - 1)) : 0.0;
        mean[k] = (float)mu;
        inv_std[k] = (float)(1.0 / (sd > 1e-12 ? sd : 1e-12));
    }
}

static bool fused_shape(const dvq_mlp_shape& s) {
    return s.d_in <= kFKin && s.d_out <= kFDmax && (s.hidden == 64 || s.hidden == 128 || s.hidden == 256);
}

template <int H>
static dvq_status launch_train_chunks(const dvq_mlp_shape& s, const float* params, const float* X, const float* T,
                                      int x_rows, const int32_t* rows, int batch, const float* mu, const float* isd,
                                      const W16& w, float* pg, double* lossp, hipStream_t hs) {
    const size_t lds = sizeof(FusedLds<H>);
    DVQ_TRY_HIP(allow_lds((const void*)k_mlp_train_chunk<H>, lds));
    hipLaunchKernelGGL(k_mlp_train_chunk<H>, dim3((batch + kFR - 1) / kFR), dim3(kFThreads), lds, hs, params, s.d_in,
                       s.d_out, X, T, x_rows, rows, batch, mu, isd, w, pg, lossp);
    DVQ_CHECK_LAUNCH("k_mlp_train_chunk");
    return DVQ_OK;
}

template <int H>
static dvq_status launch_predict(const dvq_mlp_shape& s, const float* params, const float* X, int batch,
                                 const float* mu, const float* isd, float* Y, hipStream_t hs) {
    const size_t lds = sizeof(FusedLds<H>);
    DVQ_TRY_HIP(allow_lds((const void*)k_mlp_predict<H>, lds));
    hipLaunchKernelGGL(k_mlp_predict<H>, dim3((batch + kFR - 1) / kFR), dim3(kFThreads), lds, hs, params, s.d_in,
                       s.d_out, X, batch, mu, isd, Y);
    DVQ_CHECK_LAUNCH("k_mlp_predict");
    return DVQ_OK;
}

}  // namespace dvq

using namespace dvq;

extern "C" {

size_t dvq_mlp_train_workspace_bytes(const dvq_mlp_shape* s, int32_t batch) {
    if (!s || batch < 1) return 0;
    const int64_t chunks = (batch + kFR - 1) / kFR;
    const size_t part = ((size_t)chunks * (size_t)offsets(*s).total * sizeof(float) + (size_t)chunks * sizeof(double) +
                         255) / 256 * 256;
    return part + w16_elems(s->hidden) * sizeof(__bf16);
}

dvq_status dvq_mlp_train_step(const dvq_mlp_shape* shape, float* params, float* m, float* v, int32_t t, float lr,
                              float beta1, float beta2, float eps, float weight_decay, const float* X,
                              const float* T, int32_t x_rows, const int32_t* rows, int32_t batch, const float* feat_mean,
                              const float* feat_inv_std, float* grads, double* loss, void* workspace,
                              size_t workspace_bytes, dvq_stream stream) {
    dvq_status st = check_shape(shape, batch);
    if (st != DVQ_OK) return st;
    DVQ_REQUIRE(params && m && v && X && T, "null device pointer");
    DVQ_REQUIRE((feat_mean == nullptr) == (feat_inv_std == nullptr), "feat_mean and feat_inv_std go together");
    DVQ_REQUIRE(t >= 1, "t=%d < 1", t);
    DVQ_REQUIRE(x_rows >= 1 && (rows != nullptr || batch <= x_rows), "x_rows=%d, batch=%d", x_rows, batch);
    if (!fused_shape(*shape))
        return fail(DVQ_EUNSUPPORTED, "fused MLP needs d_in <= %d, d_out <= %d, hidden 64/128/256", kFKin, kFDmax);
    const size_t need = dvq_mlp_train_workspace_bytes(shape, batch);
    if (!workspace || workspace_bytes < need)
        return fail(DVQ_ECAPACITY, "mlp train workspace %zu B < %zu B", workspace_bytes, need);
    const dvq_mlp_shape s = *shape;
    const int64_t count = offsets(s).total;
    const int chunks = (batch + kFR - 1) / kFR;
    float* pg = static_cast<float*>(workspace);
    double* lossp = reinterpret_cast<double*>(static_cast<char*>(workspace) + (size_t)chunks * count * sizeof(float));
    const size_t part = ((size_t)chunks * count * sizeof(float) + (size_t)chunks * sizeof(double) + 255) / 256 * 256;
    const W16 w = w16_layout(static_cast<char*>(workspace) + part, s.hidden);
    hipStream_t hs = stream_of(stream);
    const int64_t welems = (int64_t)w16_elems(s.hidden);
    const dim3 wgrid((unsigned)((welems + 255) / 256 < 1024 ? (welems + 255) / 256 : 1024));
    if (s.hidden == 64)
        hipLaunchKernelGGL(k_mlp_weights_bf16<64>, wgrid, dim3(256), 0, hs, params, s.d_in, s.d_out, w);
    else if (s.hidden == 128)
        hipLaunchKernelGGL(k_mlp_weights_bf16<128>, wgrid, dim3(256), 0, hs, params, s.d_in, s.d_out, w);
    else
        hipLaunchKernelGGL(k_mlp_weights_bf16<256>, wgrid, dim3(256), 0, hs, params, s.d_in, s.d_out, w);
    DVQ_CHECK_LAUNCH("k_mlp_weights_bf16");
    if (s.hidden == 64)
        st = launch_train_chunks<64>(s, params, X, T, x_rows, rows, batch, feat_mean, feat_inv_std, w, pg, lossp, hs);
    else if (s.hidden == 128)
        st = launch_train_chunks<128>(s, params, X, T, x_rows, rows, batch, feat_mean, feat_inv_std, w, pg, lossp, hs);
    else
        st = launch_train_chunks<256>(s, params, X, T, x_rows, rows, batch, feat_mean, feat_inv_std, w, pg, lossp, hs);
    if (st != DVQ_OK) return st;
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    const int64_t blocks = (count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024;
    hipLaunchKernelGGL(k_mlp_reduce_adamw, dim3((unsigned)blocks), dim3(256), 0, hs, pg, chunks, count, params, m, v,
                       lr, beta1, beta2, eps, weight_decay, c1, c2, grads, lossp, 1.0 / ((double)batch * s.d_out),
                       loss);
    DVQ_CHECK_LAUNCH("k_mlp_reduce_adamw");
    return DVQ_OK;
}

dvq_status dvq_mlp_predict(const dvq_mlp_shape* shape, const float* params, const float* X, int32_t batch,
                           const float* feat_mean, const float* feat_inv_std, float* Y, dvq_stream stream) {
    dvq_status st = check_shape(shape, batch);
    if (st != DVQ_OK) return st;
    DVQ_REQUIRE(params && X && Y, "null device pointer");
    DVQ_REQUIRE((feat_mean == nullptr) == (feat_inv_std == nullptr), "feat_mean and feat_inv_std go together");
    if (!fused_shape(*shape))
        return fail(DVQ_EUNSUPPORTED, "fused MLP needs d_in <= %d, d_out <= %d, hidden 64/128/256", kFKin, kFDmax);
    const dvq_mlp_shape s = *shape;
    hipStream_t hs = stream_of(stream);
    if (s.hidden == 64) return launch_predict<64>(s, params, X, batch, feat_mean, feat_inv_std, Y, hs);
    if (s.hidden == 128) return launch_predict<128>(s, params, X, batch, feat_mean, feat_inv_std, Y, hs);
    return launch_predict<256>(s, params, X, batch, feat_mean, feat_inv_std, Y, hs);
}

dvq_status dvq_feature_stats(const float* X, int32_t rows, int32_t d, float* mean, float* inv_std,
                             dvq_stream stream) {
    DVQ_REQUIRE(X && mean && inv_std, "null device pointer");
    DVQ_REQUIRE(rows >= 1 && d >= 1 && d <= 65536, "rows=%d, d=%d out of range", rows, d);
    hipLaunchKernelGGL(k_feature_stats, dim3(d), dim3(64), 0, stream_of(stream), X, rows, d, mean, inv_std);
    DVQ_CHECK_LAUNCH("k_feature_stats");
    return DVQ_OK;
}

}  // extern "C"
