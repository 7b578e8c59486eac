// FWHT-based Pauli decomposition of a real matrix and magnitude pruning
// (Section II-B, Eq. (5); Algorithm 1 Steps 1-2).
//
// For each x-mask, c[x][z] = (-i)^{|x&z|} / N * sum_k (-1)^{|z&k|} A[k^x][k].
// The transform over k is split into its low nl = min(n, 6) and high
// nh = n - nl bits (a Walsh-Hadamard transform is the tensor product of its
// per-bit butterflies).  For n = 10..12 one fused pass does both parts
// (k_fwht_fused, below); for n <= 9 two passes run:
//   pass 1, one workgroup per (xh, kh): the 2^nl x 2^nl tile of A at row
//     block kh^xh and column block kh is read once, coalesced; for every xl
//     the xor-diagonal v[kl] = tile[kl^xl][kl] is transformed in LDS;
//     result T[xh][kh][xl][zl];
//   pass 2, one workgroup per x = (xh, xl): T[xh][*][xl][*] is loaded,
//     transformed over kh in LDS, and c[x][*] written contiguously.
// Both forms are bound by HBM traffic: A read once and c written once, plus
// the intermediate T written and read once in the two-pass form.
// A is real, so every coefficient is a real number times a power of -i; the
// selection path stores that real value r = w / N once (8 bytes) and
// applies the phase only to the kept terms.
//
// Selection ranks by the 96-bit key (bits of |r|, ~flat index): magnitude
// descending, index ascending.  Threshold mode keeps |r| > tau; top-L mode
// finds the L-th key with most-significant-digit-first radix selection
// (8-bit digits, histogram per pass, the digit chosen on the device), then
// compacts the kept set and ranks it exactly (each kept term counts the
// terms that precede it).  The whole selection is enqueued without a host
// round trip; one copy at the end returns the count and the error sums.
#include "common.h"

namespace dvq {

constexpr int kDecThreads = 256;
constexpr int kSortMax = 65536;
constexpr int kPartials = 1024;

__host__ __device__ constexpr int dec_nl(int n) { return n < 6 ? n : 6; }

__device__ __forceinline__ dvq_c128 phase_mul(double w, uint32_t x, uint32_t z) {
    switch (__popc(x & z) & 3) {  // (-i)^p * w
        case 0: return {w, 0.0};
        case 1: return {0.0, -w};
        case 2: return {-w, 0.0};
        default: return {0.0, w};
    }
}

// In-place Walsh-Hadamard transform of length 2^M of `rows` vectors in LDS,
// element j of vector r at addr(r, j).  Bits are taken in ascending order,
// up to three per stage: each task holds the (at most) 8 elements that
// differ in the stage's bits in registers, so a stage is one LDS read and
// one LDS write per element and one barrier.
template <int M, int S, class Addr>
__device__ __forceinline__ void lds_wht(double* buf, int rows, const Addr& addr) {
    if constexpr (S < M) {
        constexpr int B = (M - S) < 3 ? (M - S) : 3;
        constexpr int R = 1 << B, REST = M - B;
        const int tasks = rows << REST;
        for (int t = threadIdx.x; t < tasks; t += blockDim.x) {
            const int row = t >> REST, rest = t & ((1 << REST) - 1);
            const int base = (rest & ((1 << S) - 1)) | ((rest >> S) << (S + B));
            double v[R];
#pragma unroll
            for (int u = 0; u < R; ++u) v[u] = buf[addr(row, base | (u << S))];
#pragma unroll
            for (int h = 1; h < R; h <<= 1)
#pragma unroll
                for (int u = 0; u < R; ++u)
                    if (!(u & h)) {
                        const double a = v[u], b = v[u | h];
                        v[u] = a + b;
                        v[u | h] = a - b;
                    }
#pragma unroll
            for (int u = 0; u < R; ++u) buf[addr(row, base | (u << S))] = v[u];
        }
        __syncthreads();
        lds_wht<M, S + B>(buf, rows, addr);
    }
}

// Pass 1, one workgroup per (xh, kh): the 2^NL x 2^NL tile of A at row
// block rb = kh^xh and column block kh, all of its loads issued before the first
// use; the NL-bit transform of every xor-diagonal v_xl[kl] = tile[kl^xl][kl]
// runs in place.  With nh = n - NL > 0 the result goes to
// T[xh][kh][xl][zl]; otherwise (n = NL) it is the decomposition itself.
template <int NL>
__global__ void __launch_bounds__(kDecThreads)
k_fwht_pass1(const double* __restrict__ A, int n, double* __restrict__ Tout,
             dvq_c128* __restrict__ dense, double* __restrict__ values) {
    constexpr int M = 1 << NL, LD = M + 1, E = M * M;
    constexpr int EPT = (E + kDecThreads - 1) / kDecThreads;
    __shared__ double tile[M * LD];
    const int nh = n - NL;
    const int64_t N = int64_t(1) << n;
    // consecutive workgroups take consecutive column blocks of one row
    // block, so the rows of A are streamed in order
    const int rb = blockIdx.x >> nh, kh = blockIdx.x & ((1 << nh) - 1), xh = rb ^ kh;
    const int64_t rowb = (int64_t)rb * M, colb = (int64_t)kh * M;
    const int64_t tbase = ((int64_t)xh * (1 << nh) + kh) * E;
    double v[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = i * kDecThreads + threadIdx.x;
        if (E % kDecThreads == 0 || e < E) v[i] = A[(rowb + e / M) * N + colb + e % M];
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = i * kDecThreads + threadIdx.x;
        if (E % kDecThreads == 0 || e < E) tile[(e / M) * LD + e % M] = v[i];
    }
    __syncthreads();
    lds_wht<NL, 0>(tile, M, [](int xl, int kl) { return (kl ^ xl) * LD + kl; });
    const double invN = 1.0 / (double)N;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = i * kDecThreads + threadIdx.x;
        if (E % kDecThreads == 0 || e < E) {
            const int xl = e >> NL, zl = e & (M - 1);
            const double w = tile[(zl ^ xl) * LD + zl];
            if (nh > 0) {
                Tout[tbase + e] = w;
            } else {
                if (dense) dense[(int64_t)xl * N + zl] = phase_mul(w * invN, (uint32_t)xl, (uint32_t)zl);
                if (values) values[(int64_t)xl * N + zl] = w * invN;
            }
        }
    }
}

// Pass 2 (n = 6 + NH), one workgroup per x-mask x = (xh, xl): the 2^NH
// segments T[xh][*][xl][*] are loaded, transformed over kh in place, and
// c[x][*] is written contiguously (z = zh * 64 + zl).
template <int NH>
__global__ void __launch_bounds__(kDecThreads)
k_fwht_pass2(const double* __restrict__ Tin, int n, dvq_c128* __restrict__ dense,
             double* __restrict__ values) {
    constexpr int M = 64, LD = M + 1, MH = 1 << NH, E = MH * M;
    constexpr int EPT = (E + kDecThreads - 1) / kDecThreads;
    __shared__ double tile[MH * LD];
    const int64_t N = int64_t(1) << n;
    const int x = blockIdx.x;
    const int xh = x >> 6, xl = x & 63;
    double v[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = i * kDecThreads + threadIdx.x;
        if (E % kDecThreads == 0 || e < E)
            v[i] = Tin[((int64_t)(xh * MH + (e >> 6)) * M + xl) * M + (e & 63)];
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = i * kDecThreads + threadIdx.x;
        if (E % kDecThreads == 0 || e < E) tile[(e >> 6) * LD + (e & 63)] = v[i];
    }
    __syncthreads();
    lds_wht<NH, 0>(tile, M, [](int zl, int kh) { return kh * LD + zl; });
    const double invN = 1.0 / (double)N;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int z = i * kDecThreads + threadIdx.x;
        if (E % kDecThreads == 0 || z < E) {
            const double w = tile[(z >> 6) * LD + (z & 63)] * invN;
            if (dense) dense[(int64_t)x * N + z] = phase_mul(w, (uint32_t)x, (uint32_t)z);
            if (values) values[(int64_t)x * N + z] = w;
        }
    }
}

// Single pass for n = 6 + NH, NH = 4..6 (n = 10..12): the intermediate T
// never leaves the chip.  One workgroup of 128 XB threads per (xh, a), where
// a selects the XB consecutive x-masks xl = XB a + b (b < XB).  In tile
// (kh^xh, kh) the elements of these XB xor-diagonals are, in every row r,
// the XB contiguous columns XB ((r / XB) ^ a) + 0..XB-1, so the workgroups
// of one xh read the 2^NH tiles exactly once between them.  Tiles are taken
// in batches of eight (kh = 8 kh1 + kh0), the next batch's loads in flight
// while one is transformed: each batch's 8 XB diagonals (kh0, b) are
// transformed over kl in LDS; each thread (b, half, zl) then takes the
// eight values T[kh0][b][zl], transforms them over kh0 in registers, and
// accumulates them with the sign
// (-1)^{|zh1 & kh1|} into its 2^(NH-1) outputs zh = 8 zh1 + zh0 (zh1 in its
// half of the range).  The transform over kh is therefore the same
// Walsh-Hadamard sum, split into an 8-point fast part and a direct part.
// The outputs are written with non-temporal stores (nothing here reads them
// again), which leaves L2 to the shared input lines.  XB = 2 (256 threads,
// eight workgroups per 128-byte line, 4 workgroups per CU) measured fastest
// of XB = 1, 2, 4, 8 on MI355X.
template <int NH, int XB>
__global__ void __launch_bounds__(128 * XB, 4)
k_fwht_fused(const double* __restrict__ A, int n, dvq_c128* __restrict__ dense,
             double* __restrict__ values) {
    constexpr int THREADS = 128 * XB, MH = 1 << NH, NB = MH / 8, ZH1 = NB / 2, ACC = 8 * ZH1, LD = 65;
    constexpr int EPT = 8 * 64 * XB / THREADS;  // batch elements per thread (4)
    constexpr int SHARE = 16 / XB;              // workgroups reading one 128-byte line
    __shared__ double d[8 * XB * LD];           // row kh0 * XB + b, column kl
    const int64_t N = int64_t(1) << n;
    // The SHARE workgroups that read the parts of the same 128-byte lines
    // are placed 8 apart: workgroups go to the 8 XCDs round robin (blockIdx
    // mod 8), so they run on one XCD, one after another, and all but the
    // first read of each line is served by that XCD's L2.
    const int c = blockIdx.x & 7, sq = blockIdx.x >> 3;
    const int grp = (sq / SHARE) * 8 + c;
    const int xh = grp >> 2, a = SHARE * (grp & 3) + sq % SHARE;
    const int t = threadIdx.x, zl = t & 63, b = t >> 7, half = (t >> 6) & 1;

    auto load = [&](double* v, int kh1) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = i * THREADS + t;
            const int kh = kh1 * 8 + e / (64 * XB), r = (e / XB) & 63, cl = e & (XB - 1);
            v[i] = A[((int64_t)(kh ^ xh) * 64 + r) * N + (int64_t)kh * 64 + XB * ((r / XB) ^ a) + cl];
        }
    };
    double v[EPT];
    double acc[ACC];
#pragma unroll
    for (int i = 0; i < ACC; ++i) acc[i] = 0.0;
    load(v, 0);
#pragma unroll 1
    for (int kh1 = 0; kh1 < NB; ++kh1) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = i * THREADS + t;
            const int kh0 = e / (64 * XB), r = (e / XB) & 63, cl = e & (XB - 1);
            const int kl = XB * ((r / XB) ^ a) + cl, bb = (r & (XB - 1)) ^ cl;
            d[(kh0 * XB + bb) * LD + kl] = v[i];
        }
        if (kh1 + 1 < NB) load(v, kh1 + 1);
        __syncthreads();
        lds_wht<6, 0>(d, 8 * XB, [](int row, int kl) { return row * LD + kl; });  // ends with a barrier
        double u[8];
#pragma unroll
        for (int k0 = 0; k0 < 8; ++k0) u[k0] = d[(k0 * XB + b) * LD + zl];
#pragma unroll
        for (int h = 1; h < 8; h <<= 1)
#pragma unroll
            for (int k0 = 0; k0 < 8; ++k0)
                if (!(k0 & h)) {
                    const double p = u[k0], q = u[k0 | h];
                    u[k0] = p + q;
                    u[k0 | h] = p - q;
                }
#pragma unroll
        for (int j = 0; j < ZH1; ++j) {
            const bool neg = __popc((unsigned)((half * ZH1 + j) & kh1)) & 1;
#pragma unroll
            for (int z0 = 0; z0 < 8; ++z0) acc[j * 8 + z0] += neg ? -u[z0] : u[z0];
        }
        __syncthreads();
    }
    const double invN = 1.0 / (double)N;
    const uint32_t x = (uint32_t)(xh * 64 + a * XB + b);
#pragma unroll
    for (int j = 0; j < ZH1; ++j)
#pragma unroll
        for (int z0 = 0; z0 < 8; ++z0) {
            const uint32_t z = (uint32_t)(((half * ZH1 + j) * 8 + z0) * 64 + zl);
            const double w = acc[j * 8 + z0] * invN;
            if (dense) {
                typedef double d2 __attribute__((ext_vector_type(2)));
                const dvq_c128 cz = phase_mul(w, x, z);
                __builtin_nontemporal_store(d2{cz.re, cz.im}, reinterpret_cast<d2*>(dense + (int64_t)x * N + z));
            }
            if (values) __builtin_nontemporal_store(w, values + (int64_t)x * N + z);
        }
}

template <int NH, int XB = 2>
static void launch_fused(const double* A, int n, dvq_c128* dense, double* values, hipStream_t s) {
    hipLaunchKernelGGL((k_fwht_fused<NH, XB>), dim3((64 / XB) << NH), dim3(128 * XB), 0, s, A, n, dense, values);
}

// n for which the decomposition runs as the single fused pass.
__host__ __device__ constexpr bool fwht_fused(int n) { return n >= 10 && n <= 12; }

template <int NL>
static void launch_pass1(const double* A, int n, double* T, dvq_c128* dense, double* values, hipStream_t s) {
    hipLaunchKernelGGL(k_fwht_pass1<NL>, dim3(1u << (2 * (n - NL))), dim3(kDecThreads), 0, s, A, n, T, dense,
                       values);
}

template <int NH>
static void launch_pass2(const double* T, int n, dvq_c128* dense, double* values, hipStream_t s) {
    hipLaunchKernelGGL(k_fwht_pass2<NH>, dim3(1u << n), dim3(kDecThreads), 0, s, T, n, dense, values);
}

static dvq_status run_fwht(const double* A, int n, double* T, dvq_c128* dense, double* values,
                           hipStream_t s) {
    if (fwht_fused(n)) {
        if (n == 10) launch_fused<4>(A, n, dense, values, s);
        else if (n == 11) launch_fused<5>(A, n, dense, values, s);
        else launch_fused<6>(A, n, dense, values, s);
        DVQ_CHECK_LAUNCH("k_fwht_fused");
        return DVQ_OK;
    }
    switch (dec_nl(n)) {
        case 1: launch_pass1<1>(A, n, T, dense, values, s); break;
        case 2: launch_pass1<2>(A, n, T, dense, values, s); break;
        case 3: launch_pass1<3>(A, n, T, dense, values, s); break;
        case 4: launch_pass1<4>(A, n, T, dense, values, s); break;
        case 5: launch_pass1<5>(A, n, T, dense, values, s); break;
        default: launch_pass1<6>(A, n, T, dense, values, s); break;
    }
    DVQ_CHECK_LAUNCH("k_fwht_pass1");
    switch (n - dec_nl(n)) {
        case 0: return DVQ_OK;
        case 1: launch_pass2<1>(T, n, dense, values, s); break;
        case 2: launch_pass2<2>(T, n, dense, values, s); break;
        case 3: launch_pass2<3>(T, n, dense, values, s); break;
        case 4: launch_pass2<4>(T, n, dense, values, s); break;
        case 5: launch_pass2<5>(T, n, dense, values, s); break;
        default: launch_pass2<6>(T, n, dense, values, s); break;
    }
    DVQ_CHECK_LAUNCH("k_fwht_pass2");
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

// State of the top-L radix selection, kept in device memory so that the
// digit passes run without a host round trip: the key prefix chosen so far,
// how many keys of the current bin are still needed, and flags.
struct SelState {
    uint64_t phi;   // magnitude bits of the prefix
    int64_t need;   // keys still to take from the current prefix's bin
    uint32_t plo;   // ~index bits of the prefix
    uint32_t done;  // every key of the chosen bin is kept: later passes do nothing
    uint32_t error; // a pass found fewer keys than needed
    uint32_t pad;
};

__global__ void k_sel_init(SelState* __restrict__ st, uint32_t* __restrict__ hist, int64_t need) {
    hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) *st = SelState{0ull, need, 0u, 0u, 0u, 0u};  // prefix 0, nothing done
}

// Choose digit d: the bin, scanned from the largest digit down, in which the
// need-th key falls; then clear the histogram for the next pass.
__global__ void __launch_bounds__(256) k_pick_digit(uint32_t* __restrict__ hist, int d, SelState* __restrict__ st) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = hist[threadIdx.x];
    hist[threadIdx.x] = 0;
    __syncthreads();
    if (threadIdx.x != 0 || st->done) return;
    int64_t above = 0;
    int dig = -1;
    for (int b = 255; b >= 0; --b) {
        if (above + h[b] >= st->need) {
            dig = b;
            break;
        }
        above += h[b];
    }
    if (dig < 0) {
        st->error = 1;
        st->done = 1;
        return;
    }
    st->need -= above;
    if (d < 8)
        st->phi |= (uint64_t)dig << (56 - 8 * d);
    else
        st->plo |= (uint32_t)dig << (24 - 8 * (d - 8));
    if ((int64_t)h[dig] == st->need || d == 11) st->done = 1;
}

__global__ void __launch_bounds__(kDecThreads)
k_digit_hist(const double* __restrict__ values, int64_t total, int d, const SelState* __restrict__ st,
             uint32_t* __restrict__ hist) {
    if (st->done) return;
    const uint64_t phi = st->phi;
    const uint32_t plo = st->plo;
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
k_compact(const double* __restrict__ values, int64_t total, int mode, double tau, const SelState* __restrict__ st,
          uint32_t* __restrict__ counter, uint32_t* __restrict__ cand, int cap) {
    const uint64_t thi = mode == 1 ? st->phi : 0ull;
    const uint32_t tlo = mode == 1 ? st->plo : 0u;
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

// Exact rank of each kept term; writes the outputs in ranking order.  The
// count is the device-side compaction count (at most `limit` candidates were
// stored); ranks at or beyond `cap` (the caller's capacity) are not written,
// the host reports that case after the final synchronisation.
__global__ void __launch_bounds__(kDecThreads)
k_rank_write(const double* __restrict__ values, const uint32_t* __restrict__ cand,
             const uint32_t* __restrict__ counter, int limit, int64_t cap, int n, dvq_c128* __restrict__ coeffs,
             dvq_pauli* __restrict__ strings) {
    __shared__ uint64_t th[kDecThreads];
    __shared__ uint32_t ti[kDecThreads];
    const int count = (int)(*counter < (uint32_t)limit ? *counter : (uint32_t)limit);
    if ((int)(blockIdx.x * blockDim.x) >= count) return;  // whole block idle
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
    if (i < count && rank < cap) {
        const uint32_t x = mi >> n, z = mi & ((1u << n) - 1);
        coeffs[rank] = phase_mul(values[mi], x, z);
        strings[rank] = {x, z};
    }
}

// Per-block partial sums (fixed grid, fixed order) of r^2 over the dropped
// terms (mode 0: |r| <= tau; mode 1: key < threshold) and of A^2.
__global__ void __launch_bounds__(kDecThreads)
k_partial_sq(const double* __restrict__ v, int64_t total, int mode, double tau, const SelState* __restrict__ st,
             double* __restrict__ partials) {
    __shared__ double red[kDecThreads / 64];
    const uint64_t thi = mode == 1 ? st->phi : 0ull;
    const uint32_t tlo = mode == 1 ? st->plo : 0u;
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
    SelState* sel;      // 1
};

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

static size_t dec_ws_layout(int n, DecWs* ws, void* base) {
    const size_t total = size_t(1) << (2 * n);
    const bool two_pass = n > 6 && !fwht_fused(n);
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
    w.sel = reinterpret_cast<SelState*>(take(sizeof(SelState)));
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

}  // extern "C"

namespace dvq {

// Enqueue the whole decomposition + selection of one matrix on `s` (no host
// round trip); the results that the host checks go to sel, counter, sums.
static dvq_status enqueue_decompose(const double* A, int n, double tau, int64_t top_L, dvq_c128* coeffs,
                                    dvq_pauli* strings, int64_t capacity, bool frob, const DecWs& w,
                                    SelState* sel, uint32_t* counter, double* sums, hipStream_t s) {
    const int64_t total = int64_t(1) << (2 * n);
    const int blocks = stream_blocks(total);
    dvq_status st = run_fwht(A, n, w.T, nullptr, w.values, s);
    if (st != DVQ_OK) return st;
    const int mode = top_L <= 0 ? 0 : 1;
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, sel, w.hist, mode ? top_L : 0);
    DVQ_CHECK_LAUNCH("k_sel_init");
    if (mode == 1) {
        // most-significant-digit-first radix selection of the top_L-th key
        for (int d = 0; d < 12; ++d) {
            hipLaunchKernelGGL(k_digit_hist, dim3(blocks), dim3(kDecThreads), 0, s, w.values, total, d, sel,
                               w.hist);
            DVQ_CHECK_LAUNCH("k_digit_hist");
            hipLaunchKernelGGL(k_pick_digit, dim3(1), dim3(256), 0, s, w.hist, d, sel);
            DVQ_CHECK_LAUNCH("k_pick_digit");
        }
    }
    if ((st = fill_u32(counter, 1, 0u, s)) != DVQ_OK) return st;
    hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(kDecThreads), 0, s, w.values, total, mode, tau, sel, counter,
                       w.cand, kSortMax);
    DVQ_CHECK_LAUNCH("k_compact");
    hipLaunchKernelGGL(k_rank_write, dim3(kSortMax / kDecThreads), dim3(kDecThreads), 0, s, w.values, w.cand,
                       counter, kSortMax, capacity, n, coeffs, strings);
    DVQ_CHECK_LAUNCH("k_rank_write");
    if (frob) {
        const int pb = kPartials;
        hipLaunchKernelGGL(k_partial_sq, dim3(pb), dim3(kDecThreads), 0, s, w.values, total, mode, tau, sel,
                           w.partials);
        DVQ_CHECK_LAUNCH("k_partial_sq");
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kDecThreads), 0, s, w.partials, pb, sums);
        DVQ_CHECK_LAUNCH("k_sum_partials");
        hipLaunchKernelGGL(k_partial_sq, dim3(pb), dim3(kDecThreads), 0, s, A, total, 2, 0.0, sel, w.partials);
        DVQ_CHECK_LAUNCH("k_partial_sq");
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kDecThreads), 0, s, w.partials, pb, sums + 1);
        DVQ_CHECK_LAUNCH("k_sum_partials");
    }
    return DVQ_OK;
}

// The host checks of one decomposition after the final synchronisation.
static dvq_status check_decompose(int n, int64_t top_L, int64_t capacity, const SelState& sel, uint32_t counter,
                                  const double* sums, int64_t* L_out, double* frob_err, int index) {
    if (sel.error) return fail(DVQ_EDEVICE, "matrix %d: radix selection lost elements", index);
    const int64_t kept = top_L > 0 ? top_L : (int64_t)counter;
    if (L_out) *L_out = kept;
    if (kept > capacity)
        return fail(DVQ_ECAPACITY, "%lld kept terms > capacity %lld", (long long)kept, (long long)capacity);
    if (kept > kSortMax)
        return fail(DVQ_ECAPACITY, "%lld kept terms > %d (sort limit)", (long long)kept, kSortMax);
    if ((int64_t)counter != kept)
        return fail(DVQ_EDEVICE, "matrix %d: compaction kept %u terms, expected %lld", index, counter,
                    (long long)kept);
    if (frob_err) {
        const double N = (double)(int64_t(1) << n);
        *frob_err = sums[1] > 0.0 ? sqrt(N * sums[0]) / sqrt(sums[1]) : 0.0;
    }
    return DVQ_OK;
}

// Per-matrix result slot of the batched form, after the shared workspace.
struct DecSlot {
    SelState sel;
    uint32_t counter;
    uint32_t pad;
    double sums[2];
};

}  // namespace dvq

extern "C" {

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
    dvq_status st = enqueue_decompose(A, n, tau, top_L, coeffs, strings, capacity, frob_err_host != nullptr, w,
                                      w.sel, w.counter, w.sums, s);
    if (st != DVQ_OK) return st;
    uint32_t counter = 0;
    SelState sel;
    double sums[2] = {0.0, 0.0};
    DVQ_TRY_HIP(hipMemcpyAsync(&counter, w.counter, sizeof(counter), hipMemcpyDeviceToHost, s));
    DVQ_TRY_HIP(hipMemcpyAsync(&sel, w.sel, sizeof(sel), hipMemcpyDeviceToHost, s));
    if (frob_err_host) DVQ_TRY_HIP(hipMemcpyAsync(sums, w.sums, sizeof(sums), hipMemcpyDeviceToHost, s));
    DVQ_TRY_HIP(hipStreamSynchronize(s));
    return check_decompose(n, top_L, capacity, sel, counter, sums, L_out_host, frob_err_host, 0);
}

size_t dvq_decompose_batch_workspace_bytes(int32_t n, int32_t B) {
    if (n < 1 || n > 12 || B < 1) return 0;
    return dec_ws_layout(n, nullptr, nullptr) + (size_t)B * sizeof(DecSlot);
}

dvq_status dvq_pauli_decompose_batch(const double* A, int32_t n, int32_t B, int64_t top_L, dvq_c128* coeffs,
                                     dvq_pauli* strings, double* frob_err_host, void* workspace,
                                     size_t workspace_bytes, dvq_stream stream) {
    DVQ_REQUIRE(n >= 1 && n <= 12, "n=%d outside 1..12", n);
    DVQ_REQUIRE(B >= 1, "B=%d < 1", B);
    DVQ_REQUIRE(A && coeffs && strings && frob_err_host, "null pointer");
    const int64_t total = int64_t(1) << (2 * n);
    DVQ_REQUIRE(top_L >= 1 && top_L <= total && top_L <= kSortMax, "top_L=%lld outside 1..min(4^n, %d)",
                (long long)top_L, kSortMax);
    const size_t need = dvq_decompose_batch_workspace_bytes(n, B);
    if (workspace == nullptr || workspace_bytes < need)
        return fail(DVQ_ECAPACITY, "decompose workspace %zu B < %zu B", workspace_bytes, need);
    hipStream_t s = stream_of(stream);
    DecWs w;
    const size_t shared = dec_ws_layout(n, &w, workspace);
    DecSlot* slots = reinterpret_cast<DecSlot*>(static_cast<char*>(workspace) + shared);
    const int64_t N2 = total;
    for (int b = 0; b < B; ++b) {
        dvq_status st = enqueue_decompose(A + (int64_t)b * N2, n, 0.0, top_L, coeffs + (int64_t)b * top_L,
                                          strings + (int64_t)b * top_L, top_L, true, w, &slots[b].sel,
                                          &slots[b].counter, slots[b].sums, s);
        if (st != DVQ_OK) return st;
    }
    DecSlot* host = static_cast<DecSlot*>(malloc(sizeof(DecSlot) * (size_t)B));
    if (!host) return fail(DVQ_EDEVICE, "host allocation of %d result slots failed", B);
    hipError_t e = hipMemcpyAsync(host, slots, sizeof(DecSlot) * (size_t)B, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dvq_status st = DVQ_OK;
    if (e != hipSuccess) st = fail(DVQ_EDEVICE, "batched decomposition: %s", hipGetErrorString(e));
    for (int b = 0; b < B && st == DVQ_OK; ++b)
        st = check_decompose(n, top_L, top_L, host[b].sel, host[b].counter, host[b].sums, nullptr,
                             &frob_err_host[b], b);
    free(host);
    return st;
}

}  // extern "C"
