// FWHT-based Pauli decomposition of a real matrix and magnitude pruning
// (Section II-B, Eq. (5); Algorithm 1 Steps 1-2).
//
// For each x-mask, c[x][z] = (-i)^{|x&z|} / N * sum_k (-1)^{|z&k|} A[k^x][k].
// The transform over k is split into its low nl = min(n, 6) and high
// nh = n - nl bits (a Walsh-Hadamard transform is the tensor product of its
// per-bit butterflies):
//   pass 1, one workgroup per (xh, kh): the 2^nl x 2^nl tile of A at row
//     block kh^xh and column block kh is read once, coalesced; for every xl
//     the xor-diagonal v[kl] = tile[kl^xl][kl] is transformed across the 64
//     lanes of a wavefront; result T[xh][kh][xl][zl];
//   pass 2, one workgroup per x = (xh, xl): T[xh][*][xl][*] is loaded,
//     transformed over kh across lanes, and c[x][*] written contiguously.
// A is real, so every coefficient is a real number times a power of -i; the
// selection path stores that real value r = w / N once (8 bytes) and
// applies the phase only to the kept terms.
//
// Selection ranks by the 96-bit key (bits of |r|, ~flat index): magnitude
// descending, index ascending.  Threshold mode keeps |r| > tau; top-L mode
// finds the L-th key with most-significant-digit-first radix selection
// (8-bit digits, histogram per pass), then compacts the kept set and ranks
// it exactly (each kept term counts the terms that precede it).
#include "common.h"

namespace dvq {

constexpr int kDecThreads = 256;
constexpr int kSortMax = 65536;
constexpr int kPartials = 1024;

__host__ __device__ constexpr int dec_nl(int n) { return n < 6 ? n : 6; }

// WHT across the first `len` lanes of a wavefront (len a power of two <= 64).
__device__ __forceinline__ double wave_wht(double v, int len) {
    const int lane = threadIdx.x & 63;
    for (int s = 1; s < len; s <<= 1) {
        const double p = __shfl_xor(v, s, 64);
        v = (lane & s) ? (p - v) : (v + p);
    }
    return v;
}

__device__ __forceinline__ dvq_c128 phase_mul(double w, uint32_t x, uint32_t z) {
    switch (__popc(x & z) & 3) {  // (-i)^p * w
        case 0: return {w, 0.0};
        case 1: return {0.0, -w};
        case 2: return {-w, 0.0};
        default: return {0.0, w};
    }
}

// Pass 1.  If nh == 0 it is the only pass and writes the result itself.
__global__ void __launch_bounds__(kDecThreads)
k_fwht_pass1(const double* __restrict__ A, int n, double* __restrict__ Tout,
             dvq_c128* __restrict__ dense, double* __restrict__ values) {
    __shared__ double tile[64 * 65];
    const int nl = dec_nl(n), nh = n - nl, Nl = 1 << nl, Nh = 1 << nh;
    const int64_t N = int64_t(1) << n;
    const int xh = blockIdx.x / Nh, kh = blockIdx.x % Nh;
    const int rowb = (kh ^ xh) * Nl, colb = kh * Nl;
    for (int e = threadIdx.x; e < Nl * Nl; e += blockDim.x) {
        const int r = e / Nl, c = e % Nl;
        tile[r * 65 + c] = A[(int64_t)(rowb + r) * N + colb + c];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const double invN = 1.0 / (double)N;
    for (int xl = wid; xl < Nl; xl += kDecThreads / 64) {
        double v = lane < Nl ? tile[(lane ^ xl) * 65 + lane] : 0.0;
        v = wave_wht(v, Nl);
        if (lane < Nl) {
            if (nh > 0) {
                Tout[((int64_t)(xh * Nh + kh) * Nl + xl) * Nl + lane] = v;
            } else {
                const uint32_t x = (uint32_t)xl, z = (uint32_t)lane;
                if (dense) dense[(int64_t)x * N + z] = phase_mul(v * invN, x, z);
                if (values) values[(int64_t)x * N + z] = v * invN;
            }
        }
    }
}

// Pass 2 (nh > 0): one workgroup per x-mask.
__global__ void __launch_bounds__(kDecThreads)
k_fwht_pass2(const double* __restrict__ Tin, int n, dvq_c128* __restrict__ dense,
             double* __restrict__ values) {
    __shared__ double tile[64 * 65];
    const int nl = dec_nl(n), nh = n - nl, Nl = 1 << nl, Nh = 1 << nh;
    const int64_t N = int64_t(1) << n;
    const int x = blockIdx.x;
    const int xh = x >> nl, xl = x & (Nl - 1);
    for (int e = threadIdx.x; e < Nh * Nl; e += blockDim.x) {
        const int kh = e / Nl, zl = e % Nl;
        tile[kh * 65 + zl] = Tin[((int64_t)(xh * Nh + kh) * Nl + xl) * Nl + zl];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int zl = wid; zl < Nl; zl += kDecThreads / 64) {
        double v = lane < Nh ? tile[lane * 65 + zl] : 0.0;
        v = wave_wht(v, Nh);
        if (lane < Nh) tile[lane * 65 + zl] = v;
    }
    __syncthreads();
    const double invN = 1.0 / (double)N;
    for (int z = threadIdx.x; z < N; z += blockDim.x) {
        const double w = tile[(z >> nl) * 65 + (z & (Nl - 1))] * invN;
        if (dense) dense[(int64_t)x * N + z] = phase_mul(w, (uint32_t)x, (uint32_t)z);
        if (values) values[(int64_t)x * N + z] = w;
    }
}

static dvq_status run_fwht(const double* A, int n, double* T, dvq_c128* dense, double* values,
                           hipStream_t s) {
    const int nl = dec_nl(n), nh = n - nl;
    const int tiles = 1 << (2 * nh);
    hipLaunchKernelGGL(k_fwht_pass1, dim3(tiles), dim3(kDecThreads), 0, s, A, n, T, dense, values);
    DVQ_CHECK_LAUNCH("k_fwht_pass1");
    if (nh > 0) {
        hipLaunchKernelGGL(k_fwht_pass2, dim3(1 << n), dim3(kDecThreads), 0, s, T, n, dense, values);
        DVQ_CHECK_LAUNCH("k_fwht_pass2");
    }
    return DVQ_OK;
}

// ------------------------------------------------------------------ selection

struct Key96 {
    uint64_t hi;  // bits of |r|
    uint32_t lo;  // ~flat index
};

__device__ __forceinline__ uint64_t mag_bits(double r) { return (uint64_t)__double_as_longlong(fabs(r)); }

// Digit d (0 = most significant) of the 96-bit key; digits 0..7 come from
// the magnitude, 8..11 from ~index.
__device__ __forceinline__ uint32_t key_digit(uint64_t hi, uint32_t lo, int d) {
    return d < 8 ? (uint32_t)(hi >> (56 - 8 * d)) & 0xFF : (lo >> (24 - 8 * (d - 8))) & 0xFF;
}

// True when the first d digits of the key equal those of the prefix.
__device__ __forceinline__ bool key_prefix_match(uint64_t hi, uint32_t lo, int d, uint64_t phi,
                                                 uint32_t plo) {
    if (d == 0) return true;
    if (d <= 8) {
        const int sh = 64 - 8 * d;
        return (hi >> sh) == (phi >> sh);
    }
    if (hi != phi) return false;
    const int sh = 32 - 8 * (d - 8);
    return sh >= 32 ? true : (lo >> sh) == (plo >> sh);
}

__global__ void k_fill_u32(uint32_t* p, int count, uint32_t v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = v;
}

__global__ void __launch_bounds__(kDecThreads)
k_digit_hist(const double* __restrict__ values, int64_t total, int d, uint64_t phi, uint32_t plo,
             uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t hi = mag_bits(values[i]);
        const uint32_t lo = ~(uint32_t)i;
        if (key_prefix_match(hi, lo, d, phi, plo)) atomicAdd(&h[key_digit(hi, lo, d)], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Compact the kept terms (flat indices) into cand[0..count).
//   mode 0: |r| > tau.   mode 1: key >= (thi, tlo).
__global__ void __launch_bounds__(kDecThreads)
k_compact(const double* __restrict__ values, int64_t total, int mode, double tau, uint64_t thi,
          uint32_t tlo, uint32_t* __restrict__ counter, uint32_t* __restrict__ cand, int cap) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double r = values[i];
        bool keep;
        if (mode == 0) {
            keep = fabs(r) > tau;
        } else {
            const uint64_t hi = mag_bits(r);
            const uint32_t lo = ~(uint32_t)i;
            keep = hi > thi || (hi == thi && lo >= tlo);
        }
        if (keep) {
            const uint32_t slot = atomicAdd(counter, 1u);
            if ((int)slot < cap) cand[slot] = (uint32_t)i;
        }
    }
}

// Count |r| > tau (mode 0) per block into partial counts.
__global__ void __launch_bounds__(kDecThreads)
k_count_tau(const double* __restrict__ values, int64_t total, double tau, uint32_t* __restrict__ counter) {
    uint32_t c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        c += fabs(values[i]) > tau ? 1u : 0u;
    __shared__ uint32_t red[kDecThreads / 64];
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kDecThreads / 64; ++w) s += red[w];
        if (s) atomicAdd(counter, s);
    }
}

// Exact rank of each kept term; writes the outputs in ranking order.
__global__ void __launch_bounds__(kDecThreads)
k_rank_write(const double* __restrict__ values, const uint32_t* __restrict__ cand, int count, int n,
             dvq_c128* __restrict__ coeffs, dvq_pauli* __restrict__ strings) {
    __shared__ uint64_t th[kDecThreads];
    __shared__ uint32_t ti[kDecThreads];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t mh = 0;
    uint32_t mi = 0;
    if (i < count) {
        mi = cand[i];
        mh = mag_bits(values[mi]);
    }
    int rank = 0;
    for (int base = 0; base < count; base += kDecThreads) {
        const int j = base + threadIdx.x;
        if (j < count) {
            ti[threadIdx.x] = cand[j];
            th[threadIdx.x] = mag_bits(values[cand[j]]);
        }
        __syncthreads();
        const int lim = count - base < kDecThreads ? count - base : kDecThreads;
        if (i < count)
            for (int t = 0; t < lim; ++t) rank += (th[t] > mh) || (th[t] == mh && ti[t] < mi);
        __syncthreads();
    }
    if (i < count) {
        const uint32_t x = mi >> n, z = mi & ((1u << n) - 1);
        coeffs[rank] = phase_mul(values[mi], x, z);
        strings[rank] = {x, z};
    }
}

// Per-block partial sums (fixed grid, fixed order) of r^2 over the dropped
// terms (mode 0: |r| <= tau; mode 1: key < threshold) and of A^2.
__global__ void __launch_bounds__(kDecThreads)
k_partial_sq(const double* __restrict__ v, int64_t total, int mode, double tau, uint64_t thi,
             uint32_t tlo, double* __restrict__ partials) {
    __shared__ double red[kDecThreads / 64];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double r = v[i];
        bool use;
        if (mode == 0) use = fabs(r) <= tau;
        else if (mode == 1) {
            const uint64_t hi = mag_bits(r);
            const uint32_t lo = ~(uint32_t)i;
            use = hi < thi || (hi == thi && lo < tlo);
        } else use = true;  // mode 2: all (||A||^2)
        if (use) acc += r * r;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// Fixed-order sum of the partials (thread-strided, then the block tree).
__global__ void __launch_bounds__(kDecThreads)
k_sum_partials(const double* __restrict__ partials, int count, double* __restrict__ out) {
    __shared__ double red[kDecThreads / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) s += partials[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *out = s;
}

// A_tilde[r][c] = sum_l c_l P_l[r][c], P[r][c] = i^{|x&z|} (-1)^{|z&c|} [r == c^x]
// (Eq. (3) with the kept terms).  One thread per matrix entry.
__global__ void __launch_bounds__(256)
k_pauli_sum_dense(const dvq_c128* __restrict__ coeffs, const dvq_pauli* __restrict__ strings, int L,
                  int n, dvq_c128* __restrict__ out) {
    const int64_t N = int64_t(1) << n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N * N;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t r = (uint32_t)(e >> n), c = (uint32_t)(e & (N - 1));
        double ar = 0.0, ai = 0.0;
        for (int l = 0; l < L; ++l) {
            const dvq_pauli p = strings[l];
            if ((c ^ p.x) != r) continue;
            const int ph = (int)__popc(p.x & p.z) + 2 * parity(p.z & c);
            const dvq_c128 w = coeffs[l];
            switch (ph & 3) {  // w * i^ph
                case 0: ar += w.re; ai += w.im; break;
                case 1: ar -= w.im; ai += w.re; break;
                case 2: ar -= w.re; ai -= w.im; break;
                default: ar += w.im; ai -= w.re; break;
            }
        }
        out[e] = {ar, ai};
    }
}

struct DecWs {
    double* T;
    double* values;
    uint32_t* hist;     // 256
    uint32_t* counter;  // 1
    uint32_t* cand;     // kSortMax
    double* partials;   // kPartials
    double* sums;       // 2
};

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

static size_t dec_ws_layout(int n, DecWs* ws, void* base) {
    const size_t total = size_t(1) << (2 * n);
    const bool two_pass = n > 6;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? static_cast<char*>(base) + off : nullptr;
        off += align256(bytes);
        return p;
    };
    DecWs w;
    w.T = reinterpret_cast<double*>(take(two_pass ? total * sizeof(double) : 0));
    w.values = reinterpret_cast<double*>(take(total * sizeof(double)));
    w.hist = reinterpret_cast<uint32_t*>(take(256 * sizeof(uint32_t)));
    w.counter = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t)));
    w.cand = reinterpret_cast<uint32_t*>(take(kSortMax * sizeof(uint32_t)));
    w.partials = reinterpret_cast<double*>(take(kPartials * sizeof(double)));
    w.sums = reinterpret_cast<double*>(take(2 * sizeof(double)));
    if (ws) *ws = w;
    return off;
}

static dvq_status fill_u32(uint32_t* p, int count, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3((count + 255) / 256), dim3(256), 0, s, p, count, v);
    DVQ_CHECK_LAUNCH("k_fill_u32");
    return DVQ_OK;
}

static int stream_blocks(int64_t total) {
    const int64_t b = (total + kDecThreads - 1) / kDecThreads;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

}  // namespace dvq

using namespace dvq;

extern "C" {

dvq_status dvq_pauli_sum_dense(const dvq_c128* coeffs, const dvq_pauli* strings, int32_t L, int32_t n,
                               dvq_c128* out, dvq_stream stream) {
    DVQ_REQUIRE(n >= 1 && n <= 14, "n=%d outside 1..14", n);
    DVQ_REQUIRE(L >= 0, "L < 0");
    DVQ_REQUIRE(out && (L == 0 || (coeffs && strings)), "null device pointer");
    const int64_t total = int64_t(1) << (2 * n);
    const int64_t blocks = (total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536;
    hipLaunchKernelGGL(k_pauli_sum_dense, dim3((unsigned)blocks), dim3(256), 0, stream_of(stream), coeffs,
                       strings, L, n, out);
    DVQ_CHECK_LAUNCH("k_pauli_sum_dense");
    return DVQ_OK;
}

size_t dvq_decompose_workspace_bytes(int32_t n) {
    if (n < 1 || n > 12) return 0;
    return dec_ws_layout(n, nullptr, nullptr);
}

dvq_status dvq_pauli_decompose_dense(const double* A, int32_t n, dvq_c128* coeffs_all,
                                     void* workspace, size_t workspace_bytes, dvq_stream stream) {
    DVQ_REQUIRE(n >= 1 && n <= 12, "n=%d outside 1..12", n);
    DVQ_REQUIRE(A && coeffs_all, "null device pointer");
    const size_t need = dvq_decompose_workspace_bytes(n);
    if (workspace_bytes < need || (need && !workspace))
        return fail(DVQ_ECAPACITY, "decompose workspace %zu B < %zu B", workspace_bytes, need);
    DecWs w;
    dec_ws_layout(n, &w, workspace);
    return run_fwht(A, n, w.T, coeffs_all, nullptr, stream_of(stream));
}

dvq_status dvq_pauli_decompose(const double* A, int32_t n, double tau, int64_t top_L,
                               dvq_c128* coeffs, dvq_pauli* strings, int64_t capacity,
                               int64_t* L_out_host, double* frob_err_host, void* workspace,
                               size_t workspace_bytes, dvq_stream stream) {
    DVQ_REQUIRE(n >= 1 && n <= 12, "n=%d outside 1..12", n);
    DVQ_REQUIRE(A && coeffs && strings && L_out_host, "null pointer");
    DVQ_REQUIRE(capacity >= 0, "capacity < 0");
    if (top_L <= 0) DVQ_REQUIRE(tau >= 0.0 && tau < INFINITY, "tau must be finite and >= 0");
    const size_t need = dvq_decompose_workspace_bytes(n);
    if (workspace == nullptr || workspace_bytes < need)
        return fail(DVQ_ECAPACITY, "decompose workspace %zu B < %zu B", workspace_bytes, need);
    const int64_t total = int64_t(1) << (2 * n);
    if (top_L > total) top_L = total;
    hipStream_t s = stream_of(stream);
    DecWs w;
    dec_ws_layout(n, &w, workspace);
    dvq_status st = run_fwht(A, n, w.T, nullptr, w.values, s);
    if (st != DVQ_OK) return st;
    const int blocks = stream_blocks(total);

    int mode;
    uint64_t thi = 0;
    uint32_t tlo = 0;
    int64_t kept;
    if (top_L <= 0) {
        mode = 0;
        if ((st = fill_u32(w.counter, 1, 0u, s)) != DVQ_OK) return st;
        hipLaunchKernelGGL(k_count_tau, dim3(blocks), dim3(kDecThreads), 0, s, w.values, total, tau,
                           w.counter);
        DVQ_CHECK_LAUNCH("k_count_tau");
        uint32_t cnt = 0;
        DVQ_TRY_HIP(hipMemcpyAsync(&cnt, w.counter, sizeof(cnt), hipMemcpyDeviceToHost, s));
        DVQ_TRY_HIP(hipStreamSynchronize(s));
        kept = cnt;
    } else {
        // most-significant-digit-first radix selection of the top_L-th key
        mode = 1;
        uint64_t phi = 0;
        uint32_t plo = 0;
        int64_t need_sel = top_L;
        for (int d = 0; d < 12; ++d) {
            if ((st = fill_u32(w.hist, 256, 0u, s)) != DVQ_OK) return st;
            hipLaunchKernelGGL(k_digit_hist, dim3(blocks), dim3(kDecThreads), 0, s, w.values, total, d,
                               phi, plo, w.hist);
            DVQ_CHECK_LAUNCH("k_digit_hist");
            uint32_t h[256];
            DVQ_TRY_HIP(hipMemcpyAsync(h, w.hist, sizeof(h), hipMemcpyDeviceToHost, s));
            DVQ_TRY_HIP(hipStreamSynchronize(s));
            int64_t above = 0;
            int dig = -1;
            for (int b = 255; b >= 0; --b) {
                if (above + h[b] >= need_sel) {
                    dig = b;
                    break;
                }
                above += h[b];
            }
            if (dig < 0) return fail(DVQ_EDEVICE, "radix selection lost elements at digit %d", d);
            need_sel -= above;
            if (d < 8)
                phi |= (uint64_t)dig << (56 - 8 * d);
            else
                plo |= (uint32_t)dig << (24 - 8 * (d - 8));
            if (h[dig] == need_sel) break;  // every key in this bin is kept
        }
        thi = phi;
        tlo = plo;
        kept = top_L;
    }
    *L_out_host = kept;
    if (kept > capacity)
        return fail(DVQ_ECAPACITY, "%lld kept terms > capacity %lld", (long long)kept, (long long)capacity);
    if (kept > kSortMax)
        return fail(DVQ_ECAPACITY, "%lld kept terms > %d (sort limit)", (long long)kept, kSortMax);
    if ((st = fill_u32(w.counter, 1, 0u, s)) != DVQ_OK) return st;
    hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(kDecThreads), 0, s, w.values, total, mode, tau, thi,
                       tlo, w.counter, w.cand, kSortMax);
    DVQ_CHECK_LAUNCH("k_compact");
    // The ranking kernel reads cand[0 .. kept): confirm every slot was written.
    uint32_t compacted = 0;
    DVQ_TRY_HIP(hipMemcpyAsync(&compacted, w.counter, sizeof(compacted), hipMemcpyDeviceToHost, s));
    DVQ_TRY_HIP(hipStreamSynchronize(s));
    if ((int64_t)compacted != kept)
        return fail(DVQ_EDEVICE, "compaction kept %u terms, expected %lld", compacted, (long long)kept);
    if (kept > 0) {
        hipLaunchKernelGGL(k_rank_write, dim3((unsigned)((kept + kDecThreads - 1) / kDecThreads)),
                           dim3(kDecThreads), 0, s, w.values, w.cand, (int)kept, n, coeffs, strings);
        DVQ_CHECK_LAUNCH("k_rank_write");
    }
    if (frob_err_host) {
        const int pb = kPartials;
        hipLaunchKernelGGL(k_partial_sq, dim3(pb), dim3(kDecThreads), 0, s, w.values, total, mode, tau, thi,
                           tlo, w.partials);
        DVQ_CHECK_LAUNCH("k_partial_sq");
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kDecThreads), 0, s, w.partials, pb, w.sums);
        DVQ_CHECK_LAUNCH("k_sum_partials");
        hipLaunchKernelGGL(k_partial_sq, dim3(pb), dim3(kDecThreads), 0, s, A, total, 2, 0.0, 0ull, 0u,
                           w.partials);
        DVQ_CHECK_LAUNCH("k_partial_sq");
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kDecThreads), 0, s, w.partials, pb, w.sums + 1);
        DVQ_CHECK_LAUNCH("k_sum_partials");
        double sums[2];
        DVQ_TRY_HIP(hipMemcpyAsync(sums, w.sums, sizeof(sums), hipMemcpyDeviceToHost, s));
        DVQ_TRY_HIP(hipStreamSynchronize(s));
        const double N = (double)(int64_t(1) << n);
        *frob_err_host = sums[1] > 0.0 ? sqrt(N * sums[0]) / sqrt(sums[1]) : 0.0;
    } else {
        DVQ_TRY_HIP(hipStreamSynchronize(s));
    }
    return DVQ_OK;
}

}  // extern "C"
