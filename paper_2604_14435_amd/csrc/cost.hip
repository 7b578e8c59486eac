// Cost assembly from the Hadamard-test terms (Section II-C stages ii-iii,
// Eq. (1)), the parameter-shift gradient of the plain path, the
// gradient-descent step and the solution fidelity (Section III-A).
#include "circuits.h"
#include "gates_lds.h"

#include <mutex>

namespace dvq {

constexpr int kCostThreads = 1024;

// One workgroup per theta row sums the weighted terms (Section II-C stage ii,
// weights w_lm = conj(c_l) c_m) and applies stage iii:
//   Psi = sum_lm w_lm beta_lm;
//   local:  E = sum_j sum_lm w_lm delta^j_lm, C = 1/2 - Re[E / (n Psi)] / 2;
//   global: g = sum_l c_l gamma_l, G = |g|^2, C = 1 - G / Psi  (Eq. (1)).
// The terms are rows of length L (beta rows, then the n delta rows of each
// l); wavefront w takes the rows in blocks of kCostRows (block w, w + 16,
// ...), the row index, and with it l and c_l, uniform over the wavefront,
// and lane i the columns m = i, i + 64, ..., so c_m stays in registers.  A
// block's loads are all issued before the first is used (the terms come
// from HBM, and one workgroup needs many loads in flight).  Thread partial
// sums in a fixed order, then the fixed-order block reduction: the result
// is bit-reproducible.
constexpr int kCostWaves = kCostThreads / 64;
constexpr int kCostRows = 8;

__global__ void __launch_bounds__(kCostThreads)
k_cost(const dvq_c128* __restrict__ coeffs, int L, int n, int kind,
       const dvq_c128* __restrict__ beta, const dvq_c128* __restrict__ other,
       double* __restrict__ C, dvq_c128* __restrict__ parts) {
    __shared__ double red[kCostThreads / 64];
    const int64_t row = blockIdx.x;
    const int64_t L2 = (int64_t)L * L;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // rows 0..L-1: beta; rows L..(n+1)L-1: delta (local only)
    const int rows = kind == DVQ_COST_LOCAL ? (n + 1) * L : L;
    const dvq_c128* bt = beta + row * L2;
    const dvq_c128* dt = other + row * (int64_t)n * L2;
    double pr = 0.0, pi = 0.0, nr = 0.0, ni = 0.0;
    for (int m0 = 0; m0 < L; m0 += 64) {
        const int m = m0 + lane;
        const bool on = m < L;
        const dvq_c128 cm = on ? coeffs[m] : dvq_c128{0.0, 0.0};
        for (int r0 = wave * kCostRows; r0 < rows; r0 += kCostWaves * kCostRows) {
            dvq_c128 t[kCostRows];
#pragma unroll
            for (int u = 0; u < kCostRows; ++u) {
                const int r = r0 + u;
                const dvq_c128* src = r < L ? bt + (int64_t)r * L : dt + (int64_t)(r - L) * L;
                t[u] = (on && r < rows) ? src[m] : dvq_c128{0.0, 0.0};
            }
#pragma unroll
            for (int u = 0; u < kCostRows; ++u) {
                const int r = r0 + u;  // rows past the end loaded zeros
                const dvq_c128 cl = coeffs[r % L];
                const double wr = cl.re * cm.re + cl.im * cm.im, wi = cl.re * cm.im - cl.im * cm.re;
                const double ar = wr * t[u].re - wi * t[u].im, ai = wr * t[u].im + wi * t[u].re;
                if (r < L) {
                    pr += ar;
                    pi += ai;
                } else {
                    nr += ar;
                    ni += ai;
                }
            }
        }
    }
    pr = block_sum(pr, red);
    pi = block_sum(pi, red);
    double cost;
    if (kind == DVQ_COST_LOCAL) {
        nr = block_sum(nr, red);
        ni = block_sum(ni, red);
        cost = 0.5 - 0.5 * (nr * pr + ni * pi) / (n * (pr * pr + pi * pi));  // Re[E / (n Psi)]
    } else {
        const dvq_c128* gt = other + row * (int64_t)L;
        double gr = 0.0, gi = 0.0;
        for (int l = threadIdx.x; l < L; l += kCostThreads) {
            const dvq_c128 cl = coeffs[l], t = gt[l];
            gr += cl.re * t.re - cl.im * t.im;
            gi += cl.re * t.im + cl.im * t.re;
        }
        gr = block_sum(gr, red);
        gi = block_sum(gi, red);
        nr = gr * gr + gi * gi;
        ni = 0.0;
        cost = 1.0 - nr * pr / (pr * pr + pi * pi);  // 1 - Re[G / Psi]
    }
    if (threadIdx.x == 0) {
        C[row] = cost;
        if (parts) {
            parts[2 * row] = {nr, ni};
            parts[2 * row + 1] = {pr, pi};
        }
    }
}

dvq_status launch_cost(const dvq_c128* coeffs, int L, int n, int kind, const dvq_c128* beta,
                       const dvq_c128* other, int B, double* C, dvq_c128* parts, hipStream_t s) {
    hipLaunchKernelGGL(k_cost, dim3(B), dim3(kCostThreads), 0, s, coeffs, L, n, kind, beta, other, C,
                       parts);
    DVQ_CHECK_LAUNCH("k_cost");
    return DVQ_OK;
}

// Rows of the shift rule: row 0 = theta, row 1+2k = theta + pi/2 e_k,
// row 2+2k = theta - pi/2 e_k.
__global__ void k_shift_rows(const double* __restrict__ theta, int P, double* __restrict__ rows) {
    const int r = blockIdx.x;
    const int k = (r - 1) >> 1;
    const double d = (r == 0) ? 0.0 : ((r & 1) ? 1.5707963267948966 : -1.5707963267948966);
    for (int i = threadIdx.x; i < P; i += blockDim.x) rows[(int64_t)r * P + i] = theta[i] + (i == k ? d : 0.0);
}

// Shift rule on the expectation values N (E or G) and Psi, then the quotient
// rule: local C = 1/2 - N/(2 n Psi), global C = 1 - N/Psi.
__global__ void k_shift_combine(const dvq_c128* __restrict__ parts, int P, int n, int kind,
                                const double* __restrict__ Crows, double* __restrict__ C,
                                double* __restrict__ grad) {
    const double N0 = parts[0].re, Psi0 = parts[1].re;
    for (int k = threadIdx.x; k < P; k += blockDim.x) {
        const int rp = 1 + 2 * k, rm = 2 + 2 * k;
        const double dN = 0.5 * (parts[2 * rp].re - parts[2 * rm].re);
        const double dPsi = 0.5 * (parts[2 * rp + 1].re - parts[2 * rm + 1].re);
        const double q = (dN * Psi0 - N0 * dPsi) / (Psi0 * Psi0);
        grad[k] = kind == DVQ_COST_LOCAL ? -0.5 / n * q : -q;
    }
    if (threadIdx.x == 0) C[0] = Crows[0];
}

__global__ void k_gd_step(double* __restrict__ theta, const double* __restrict__ grad, int64_t count,
                          double lr) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        theta[i] -= lr * grad[i];
}

// F = |<target|V(theta)|0>|^2, float64 state in LDS, one workgroup per row.
__global__ void __launch_bounds__(256)
k_fidelity(const double* __restrict__ theta, int n, int layers, int ent,
           const dvq_c128* __restrict__ target, double* __restrict__ F) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = 1 << n, P = n * layers;
    cplx<double>* a = reinterpret_cast<cplx<double>*>(smem);
    double* trig = reinterpret_cast<double*>(a + N);
    double* red = trig + 2 * P;
    const int64_t row = blockIdx.x;
    lds_trig<double>(trig, theta + row * P, P);
    for (int i = threadIdx.x; i < N; i += blockDim.x) a[i] = {i == 0 ? 1.0 : 0.0, 0.0};
    __syncthreads();
    lds_ansatz<double>(a, n, n, layers, ent, trig, -1);
    double ore = 0.0, oim = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const dvq_c128 t = target[i];
        ore += t.re * a[i].re + t.im * a[i].im;  // conj(t) * a
        oim += t.re * a[i].im - t.im * a[i].re;
    }
    ore = block_sum(ore, red);
    oim = block_sum(oim, red);
    if (threadIdx.x == 0) F[row] = ore * ore + oim * oim;
}

// ---------------------------------------------------------- shift rule

// Memory of one shift-rule gradient: the 2P + 1 angle rows, their (N, Psi)
// parts and costs (all rows), then the terms of `chunk` rows at a time.
static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

static size_t shift_fixed_bytes(int64_t P) {
    const int64_t R = 2 * P + 1;
    return align256((size_t)(R * P) * sizeof(double)) + align256((size_t)R * 2 * sizeof(dvq_c128)) +
           align256((size_t)R * sizeof(double));
}

static size_t shift_row_bytes(int n, int L, int cost_kind) {
    const int64_t L2 = (int64_t)L * L;
    const int64_t other = cost_kind == DVQ_COST_LOCAL ? (int64_t)n * L2 : L;
    return (size_t)(L2 + other) * sizeof(dvq_c128);
}

// Enqueue the plain gradient: the shifted rows, then, `chunk` rows at a
// time, every circuit of those rows and their cost, then the shift rule.
// `mem` holds shift_fixed_bytes(P) + chunk * shift_row_bytes(n, L, kind).
// Every argument is checked before the first launch.
static dvq_status enqueue_shift(const dvq_ansatz* an, const double* theta, int precision,
                                const dvq_c128* coeffs, const dvq_pauli* strings, int L, int b_kind,
                                const double* b, int cost_kind, double* C, double* grad, char* mem,
                                int chunk, hipStream_t s) {
    const int P = an->n * an->layers, R = 2 * P + 1;
    double* rows = reinterpret_cast<double*>(mem);
    mem += align256((size_t)R * P * sizeof(double));
    dvq_c128* parts = reinterpret_cast<dvq_c128*>(mem);
    mem += align256((size_t)R * 2 * sizeof(dvq_c128));
    double* crow = reinterpret_cast<double*>(mem);
    mem += align256((size_t)R * sizeof(double));
    dvq_c128* beta = reinterpret_cast<dvq_c128*>(mem);
    dvq_c128* other = beta + (int64_t)chunk * L * L;
    TermsArgs g;
    dvq_status st = make_terms_args(g, an, rows, chunk, precision, strings, L, b_kind, b, cost_kind, beta,
                                    other);
    if (st != DVQ_OK) return st;
    DVQ_REQUIRE(theta != nullptr, "theta is NULL");
    hipLaunchKernelGGL(k_shift_rows, dim3(R), dim3(64), 0, s, theta, P, rows);
    DVQ_CHECK_LAUNCH("k_shift_rows");
    for (int r0 = 0; r0 < R; r0 += chunk) {
        const int cnt = R - r0 < chunk ? R - r0 : chunk;
        TermsArgs gc = g;
        gc.theta = rows + (int64_t)r0 * P;
        gc.B = cnt;
        gc.total = gc.per_row * cnt;
        if ((st = launch_terms(gc, precision, DVQ_EXEC_LITERAL, s)) != DVQ_OK) return st;
        if ((st = launch_cost(coeffs, L, an->n, cost_kind, beta, other, cnt, crow + r0, parts + 2 * r0, s)) !=
            DVQ_OK)
            return st;
    }
    hipLaunchKernelGGL(k_shift_combine, dim3(1), dim3(256), 0, s, parts, P, an->n, cost_kind, crow, C, grad);
    DVQ_CHECK_LAUNCH("k_shift_combine");
    return DVQ_OK;
}

// Device scratch of dvq_vqls_grad_shift_noalloc: a file-scope array, one copy
// per GPU, held until the process ends.  Host code never passes the array's
// name to a kernel: its device address is looked up once per device with
// hipGetSymbolAddress (that device current) and kept in scratch_addr.
constexpr size_t kShiftScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kShiftScratchBytes];
static std::mutex scratch_mu;
static char* scratch_addr[kMaxDevices];

// The scratch address on the device `s` belongs to.
static dvq_status shift_scratch(hipStream_t s, char** out) {
    int cur = 0, dev = 0;
    DVQ_TRY_HIP(hipGetDevice(&cur));
    dev = cur;
    if (s != nullptr) DVQ_TRY_HIP(hipStreamGetDevice(s, &dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DVQ_EUNSUPPORTED, "device %d >= %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_addr[dev] == nullptr) {
        if (dev != cur) DVQ_TRY_HIP(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) DVQ_TRY_HIP(hipSetDevice(cur));
        if (e != hipSuccess) return fail(DVQ_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        if (p == nullptr) return fail(DVQ_EDEVICE, "hipGetSymbolAddress(scratch) gave NULL");
        scratch_addr[dev] = static_cast<char*>(p);
    }
    *out = scratch_addr[dev];
    return DVQ_OK;
}

}  // namespace dvq

using namespace dvq;

extern "C" {

dvq_status dvq_vqls_cost(const dvq_c128* coeffs, int32_t L, int32_t n, int32_t cost_kind,
                         const dvq_c128* beta, const dvq_c128* other, int32_t B, double* C,
                         dvq_c128* parts, dvq_stream stream) {
    DVQ_REQUIRE(coeffs && beta && other && C, "null device pointer");
    DVQ_REQUIRE(L >= 1 && L <= 65536, "L=%d outside 1..65536", L);
    DVQ_REQUIRE(n >= 1 && n <= 13, "n=%d outside 1..13", n);
    DVQ_REQUIRE(B >= 1, "B=%d < 1", B);
    DVQ_REQUIRE(cost_kind == DVQ_COST_GLOBAL || cost_kind == DVQ_COST_LOCAL, "unknown cost kind %d",
                cost_kind);
    return launch_cost(coeffs, L, n, cost_kind, beta, other, B, C, parts, stream_of(stream));
}

size_t dvq_grad_shift_workspace_bytes(const dvq_ansatz* an, int32_t L, int32_t cost_kind) {
    if (!an || an->n < 1 || an->n > 13 || an->layers < 1 || an->layers > 64 || L < 1 || L > 65536) return 0;
    const int64_t P = (int64_t)an->n * an->layers, R = 2 * P + 1;
    return shift_fixed_bytes(P) + (size_t)R * shift_row_bytes(an->n, L, cost_kind);
}

dvq_status dvq_vqls_grad_shift(const dvq_ansatz* ansatz, const double* theta, int32_t precision,
                               const dvq_c128* coeffs, const dvq_pauli* strings, int32_t L,
                               int32_t b_kind, const double* b, int32_t cost_kind, double* C,
                               double* grad, void* workspace, size_t workspace_bytes,
                               dvq_stream stream) {
    DVQ_REQUIRE(coeffs && C && grad, "null device pointer");
    const size_t need = dvq_grad_shift_workspace_bytes(ansatz, L, cost_kind);
    DVQ_REQUIRE(ansatz != nullptr, "ansatz is NULL");
    if (workspace == nullptr || workspace_bytes < need)
        return fail(DVQ_ECAPACITY, "grad_shift workspace %zu B < %zu B", workspace_bytes, need);
    const int P = ansatz->n * ansatz->layers, R = 2 * P + 1;
    return enqueue_shift(ansatz, theta, precision, coeffs, strings, L, b_kind, b, cost_kind, C, grad,
                         static_cast<char*>(workspace), R, stream_of(stream));
}

size_t dvq_grad_shift_noalloc_max_bytes(void) { return kShiftScratchBytes; }

dvq_status dvq_vqls_grad_shift_noalloc(const dvq_ansatz* ansatz, const double* theta, int32_t precision,
                                       const dvq_c128* coeffs, const dvq_pauli* strings, int32_t L,
                                       int32_t b_kind, const double* b, int32_t cost_kind, double* C,
                                       double* grad, dvq_stream stream) {
    dvq_status st = check_ansatz(ansatz, precision == DVQ_F32 ? 13 : 12);
    if (st != DVQ_OK) return st;
    DVQ_REQUIRE(coeffs && C && grad, "null device pointer");
    DVQ_REQUIRE(L >= 1 && L <= 65536, "L=%d outside 1..65536", L);
    const int64_t P = (int64_t)ansatz->n * ansatz->layers, R = 2 * P + 1;
    const size_t fixed = shift_fixed_bytes(P), row = shift_row_bytes(ansatz->n, L, cost_kind);
    if (fixed + row > kShiftScratchBytes)
        return fail(DVQ_ECAPACITY,
                    "grad_shift_noalloc: %zu B of shift rows + %zu B of terms per row exceed the %zu B "
                    "device scratch (use dvq_vqls_grad_shift with a workspace)",
                    fixed, row, kShiftScratchBytes);
    const int64_t fit = (int64_t)((kShiftScratchBytes - fixed) / row);
    const int chunk = (int)(fit < R ? fit : R);
    hipStream_t s = stream_of(stream);
    char* base = nullptr;
    st = shift_scratch(s, &base);
    if (st != DVQ_OK) return st;
    return enqueue_shift(ansatz, theta, precision, coeffs, strings, L, b_kind, b, cost_kind, C, grad, base,
                         chunk, s);
}

dvq_status dvq_gd_step(double* theta, const double* grad, int64_t count, double lr,
                       dvq_stream stream) {
    DVQ_REQUIRE(theta && grad, "null device pointer");
    DVQ_REQUIRE(count >= 0, "count < 0");
    if (count == 0) return DVQ_OK;
    const int64_t blocks = (count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024;
    hipLaunchKernelGGL(k_gd_step, dim3((unsigned)blocks), dim3(256), 0, stream_of(stream), theta, grad,
                       count, lr);
    DVQ_CHECK_LAUNCH("k_gd_step");
    return DVQ_OK;
}

dvq_status dvq_fidelity(const dvq_ansatz* ansatz, const double* theta, int32_t B,
                        const dvq_c128* target, double* F, dvq_stream stream) {
    dvq_status st = check_ansatz(ansatz, 12);
    if (st != DVQ_OK) return st;
    DVQ_REQUIRE(theta && target && F, "null device pointer");
    DVQ_REQUIRE(B >= 1, "B=%d < 1", B);
    const int n = ansatz->n, P = n * ansatz->layers;
    const size_t lds = (size_t(1) << n) * sizeof(cplx<double>) + (2 * P + 8) * sizeof(double);
    DVQ_TRY_HIP(allow_lds((const void*)k_fidelity, lds));
    hipLaunchKernelGGL(k_fidelity, dim3(B), dim3(256), lds, stream_of(stream), theta, n,
                       ansatz->layers, ansatz->entangler, target, F);
    DVQ_CHECK_LAUNCH("k_fidelity");
    return DVQ_OK;
}

}  // extern "C"
