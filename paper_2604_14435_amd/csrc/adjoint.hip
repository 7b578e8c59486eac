// Adjoint gradient of the VQLS cost over the ansatz (project form of the
// method's gradient: the paper leaves its gradient method unstated).
//
// C is a function of two expectation values of |x> = V(theta)|0>:
//   local  (Section II-C stage iii): C = 1/2 - E / (2 n Psi),
//          E = <x|A^dag U_b (sum_j Z_j) U_b^dag A|x>, Psi = <x|A^dag A|x>;
//   global (Eq. (1)): C = 1 - G / Psi, G = |<b|A|x>|^2,
// with A = sum_l c_l P_l the pruned Pauli sum.  For a Hermitian M,
// d<x|M|x>/dtheta_k = 2 Re <d_k x|M|x>, so dC/dtheta_k = 2 Re <d_k x|lambda>
// with lambda = (dC/dE) M_E |x> + (dC/dPsi) A^dag A |x> (or the G analogue).
// RY(t) = exp(-i t Y/2) has dRY/dt = (1/2) K RY, K = [[0,-1],[1,0]], so
// dC/dtheta_k = Re <K_q x_k | lambda_k>, where x_k and lambda_k are the two
// vectors with every gate after gate k undone.  The sweep undoes the gates
// one at a time on both vectors (inverse gates, no stored states).
//
// One workgroup per parameter row; the three 2^n-amplitude vectors live in
// LDS; all reductions are float64 with a fixed order.
#include "circuits.h"
#include "gates_lds.h"

namespace dvq {

// Threads per row: 512 covers the 512 amplitude pairs of an n = 10 gate
// pass in one step (one row runs at a time in an L-BFGS evaluation, so its
// latency is the evaluation's; 256 threads took 1.4-1.6x longer).
constexpr int kAdjThreads = 512;

template <typename T>
__host__ __device__ constexpr size_t adjoint_lds_bytes(int n, int layers, int L) {
    return 3 * (size_t(1) << n) * sizeof(cplx<T>)            // psi, b1, b2
           + (size_t)L * (sizeof(dvq_pauli) + sizeof(dvq_c128))  // strings, coeffs
           + ((2 * sizeof(T) * n * layers + 15) / 16) * 16         // trig
           + (kAdjThreads / 64) * sizeof(double);                 // reduction scratch
}

// out[k] = sum_l w_l (P_l in)[k] with w_l = c_l or conj(c_l).
template <typename T>
__device__ void lds_pauli_sum(cplx<T>* __restrict__ out, const cplx<T>* __restrict__ in, int n,
                              const dvq_pauli* sp, const dvq_c128* cp, int L, bool conj_coeffs) {
    const int N = 1 << n;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        double ar = 0.0, ai = 0.0;
        for (int l = 0; l < L; ++l) {
            const uint32_t x = sp[l].x, z = sp[l].z;
            const int kk = k ^ (int)x;
            const cplx<T> v = mul_ipow(in[kk], __popc(x & z) + 2 * parity(z & (uint32_t)kk));
            const double cr = cp[l].re, ci = conj_coeffs ? -cp[l].im : cp[l].im;
            ar += cr * (double)v.re - ci * (double)v.im;
            ai += cr * (double)v.im + ci * (double)v.re;
        }
        out[k] = {(T)ar, (T)ai};
    }
    __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(kAdjThreads)
k_adjoint(const double* __restrict__ theta, int n, int layers, int ent,
          const dvq_c128* __restrict__ coeffs, const dvq_pauli* __restrict__ strings, int L,
          int per_row_system, int bkind, const double* __restrict__ bvec, int kind,
          double* __restrict__ Cout, double* __restrict__ grad) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = 1 << n, P = n * layers;
    cplx<T>* psi = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* b1 = psi + N;
    cplx<T>* b2 = b1 + N;
    dvq_pauli* sp = reinterpret_cast<dvq_pauli*>(b2 + N);
    dvq_c128* cp = reinterpret_cast<dvq_c128*>(sp + L);
    T* trig = reinterpret_cast<T*>(cp + L);
    double* red = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(trig) +
                                            ((2 * sizeof(T) * P + 15) / 16) * 16);
    const int64_t row = blockIdx.x;
    const int64_t sys = per_row_system ? row * L : 0;
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
        sp[l] = strings[sys + l];
        cp[l] = coeffs[sys + l];
    }
    lds_trig<T>(trig, theta + row * P, P);  // ends with a barrier

    // forward: psi = V(theta)|0>
    for (int i = threadIdx.x; i < N; i += blockDim.x) psi[i] = {(T)(i == 0 ? 1 : 0), (T)0};
    __syncthreads();
    lds_ansatz<T>(psi, n, n, layers, ent, trig, -1);

    // y = A psi -> b2 ; Psi = <y|y>
    lds_pauli_sum<T>(b2, psi, n, sp, cp, L, false);
    double ps = 0.0;
    for (int k = threadIdx.x; k < N; k += blockDim.x)
        ps += (double)b2[k].re * b2[k].re + (double)b2[k].im * b2[k].im;
    const double Psi = block_sum(ps, red);

    double cost;
    if (kind == DVQ_COST_LOCAL) {
        // u = U_b^dag y -> b1 ; E = sum_k |u_k|^2 (n - 2 popcount(k))
        for (int k = threadIdx.x; k < N; k += blockDim.x) b1[k] = b2[k];
        __syncthreads();
        if (bkind == DVQ_B_PLUS)
            for (int q = 0; q < n; ++q) lds_h<T>(b1, n, q, -1);
        else
            lds_householder<T>(b1, n, bvec, red);
        double es = 0.0;
        for (int k = threadIdx.x; k < N; k += blockDim.x)
            es += ((double)b1[k].re * b1[k].re + (double)b1[k].im * b1[k].im) * (n - 2 * (int)__popc(k));
        const double E = block_sum(es, red);
        cost = 0.5 - 0.5 * E / (n * Psi);
        const double aE = -0.5 / (n * Psi), aPsi = 0.5 * E / (n * Psi * Psi);
        // b1 = U_b D u, then b1 = aE b1 + aPsi y
        for (int k = threadIdx.x; k < N; k += blockDim.x) {
            const T d = (T)(n - 2 * (int)__popc(k));
            b1[k] = {b1[k].re * d, b1[k].im * d};
        }
        __syncthreads();
        if (bkind == DVQ_B_PLUS)
            for (int q = 0; q < n; ++q) lds_h<T>(b1, n, q, -1);
        else
            lds_householder<T>(b1, n, bvec, red);
        for (int k = threadIdx.x; k < N; k += blockDim.x)
            b1[k] = {(T)(aE * b1[k].re + aPsi * b2[k].re), (T)(aE * b1[k].im + aPsi * b2[k].im)};
        __syncthreads();
    } else {
        // g = <b|y>, G = |g|^2 ; b1 = aG g b + aPsi y
        const double invs = 1.0 / sqrt((double)N);
        double gr = 0.0, gi = 0.0;
        for (int k = threadIdx.x; k < N; k += blockDim.x) {
            const double bk = bkind == DVQ_B_PLUS ? invs : bvec[k];
            gr += bk * b2[k].re;
            gi += bk * b2[k].im;
        }
        gr = block_sum(gr, red);
        gi = block_sum(gi, red);
        const double G = gr * gr + gi * gi;
        cost = 1.0 - G / Psi;
        const double aG = -1.0 / Psi, aPsi = G / (Psi * Psi);
        for (int k = threadIdx.x; k < N; k += blockDim.x) {
            const double bk = bkind == DVQ_B_PLUS ? invs : bvec[k];
            b1[k] = {(T)(aG * gr * bk + aPsi * b2[k].re), (T)(aG * gi * bk + aPsi * b2[k].im)};
        }
        __syncthreads();
    }
    // lambda = A^dag b1 -> b2
    lds_pauli_sum<T>(b2, b1, n, sp, cp, L, true);
    cplx<T>* lam = b2;

    // reverse sweep
    for (int l = layers - 1; l >= 0; --l) {
        if (ent == DVQ_ENT_CZ_LADDER) {
            if (n > 1) {
                lds_cz_ladder<T>(psi, n, n, -1);
                lds_cz_ladder<T>(lam, n, n, -1);
            }
        } else {
            for (int q = n - 2; q >= 0; --q) {
                lds_cx<T>(psi, n, q, q + 1, -1);
                lds_cx<T>(lam, n, q, q + 1, -1);
            }
        }
        for (int q = n - 1; q >= 0; --q) {
            const int k = l * n + q;
            const T c = trig[2 * k], s = trig[2 * k + 1];
            double acc = 0.0;
            for (int p = threadIdx.x; p < N / 2; p += blockDim.x) {
                const int i0 = insert0(p, q), i1 = i0 | (1 << q);
                const cplx<T> x0 = psi[i0], x1 = psi[i1], y0 = lam[i0], y1 = lam[i1];
                // Re[ conj(-x1) y0 + conj(x0) y1 ]
                acc += -((double)x1.re * y0.re + (double)x1.im * y0.im) +
                       ((double)x0.re * y1.re + (double)x0.im * y1.im);
                // undo RY: RY(-t) = [[c, s], [-s, c]]
                psi[i0] = {c * x0.re + s * x1.re, c * x0.im + s * x1.im};
                psi[i1] = {c * x1.re - s * x0.re, c * x1.im - s * x0.im};
                lam[i0] = {c * y0.re + s * y1.re, c * y0.im + s * y1.im};
                lam[i1] = {c * y1.re - s * y0.re, c * y1.im - s * y0.im};
            }
            const double gk = block_sum(acc, red);  // contains barriers
            if (threadIdx.x == 0) grad[row * P + k] = gk;
        }
    }
    if (threadIdx.x == 0) Cout[row] = cost;
}

template <typename T>
static dvq_status launch_adjoint(const dvq_ansatz* an, const double* theta, int B,
                                 const dvq_c128* coeffs, const dvq_pauli* strings, int L,
                                 int per_row_system, int bkind, const double* b, int kind,
                                 double* C, double* grad, hipStream_t s) {
    const size_t lds = adjoint_lds_bytes<T>(an->n, an->layers, L);
    if (lds > kMaxLdsBytes)
        return fail(DVQ_EUNSUPPORTED, "adjoint: n=%d, L=%d needs %zu B of LDS", an->n, L, lds);
    DVQ_TRY_HIP(allow_lds((const void*)k_adjoint<T>, lds));
    hipLaunchKernelGGL(k_adjoint<T>, dim3(B), dim3(kAdjThreads), lds, s, theta, an->n, an->layers,
                       an->entangler, coeffs, strings, L, per_row_system, bkind, b, kind, C, grad);
    DVQ_CHECK_LAUNCH("k_adjoint");
    return DVQ_OK;
}

}  // namespace dvq

using namespace dvq;

extern "C" dvq_status dvq_vqls_grad_adjoint(const dvq_ansatz* ansatz, const double* theta, int32_t B,
                                            int32_t precision, const dvq_c128* coeffs,
                                            const dvq_pauli* strings, int32_t L,
                                            int32_t per_row_system, int32_t b_kind, const double* b,
                                            int32_t cost_kind, double* C, double* grad,
                                            dvq_stream stream) {
    dvq_status st = check_ansatz(ansatz, 12);
    if (st != DVQ_OK) return st;
    DVQ_REQUIRE(theta && coeffs && strings && C && grad, "null device pointer");
    DVQ_REQUIRE(B >= 1, "B=%d < 1", B);
    DVQ_REQUIRE(L >= 1 && L <= 65536, "L=%d outside 1..65536", L);
    DVQ_REQUIRE(per_row_system == 0 || per_row_system == 1, "per_row_system must be 0 or 1");
    DVQ_REQUIRE(b_kind == DVQ_B_PLUS || (b_kind == DVQ_B_VECTOR && b != nullptr), "bad b_kind / b");
    DVQ_REQUIRE(cost_kind == DVQ_COST_GLOBAL || cost_kind == DVQ_COST_LOCAL, "unknown cost kind");
    DVQ_REQUIRE(precision == DVQ_F32 || precision == DVQ_F64, "unknown precision %d", precision);
    hipStream_t s = stream_of(stream);
    st = launch_adjoint_fast(ansatz, theta, B, precision, coeffs, strings, L, per_row_system, b_kind, b,
                             cost_kind, C, grad, s);
    if (st != DVQ_EUNSUPPORTED) return st;
    return precision == DVQ_F32
               ? launch_adjoint<float>(ansatz, theta, B, coeffs, strings, L, per_row_system, b_kind,
                                       b, cost_kind, C, grad, s)
               : launch_adjoint<double>(ansatz, theta, B, coeffs, strings, L, per_row_system,
                                        b_kind, b, cost_kind, C, grad, s);
}
