// Block-wide gate operations on a state vector held in LDS.
//
// Every function is called by all threads of the workgroup, updates the
// amplitudes a[0 .. 2^nb) in place and ends with a barrier.  `ctrl` is the
// bit index of a control qubit (the gate acts only where that bit is 1) or -1.
#pragma once

#include "common.h"

namespace dvq {

// Insert a zero bit at position q into p.
__device__ __forceinline__ int insert0(int p, int q) {
    const int low = p & ((1 << q) - 1);
    return ((p - low) << 1) | low;
}

// Real 2x2 matrix [[u00, u01], [u10, u11]] on qubit q.
template <typename T>
__device__ void lds_real_1q(cplx<T>* a, int nb, int q, T u00, T u01, T u10, T u11, int ctrl) {
    const int half = 1 << (nb - 1);
    for (int p = threadIdx.x; p < half; p += blockDim.x) {
        const int i0 = insert0(p, q), i1 = i0 | (1 << q);
        if (ctrl >= 0 && !((i0 >> ctrl) & 1)) continue;
        const cplx<T> x0 = a[i0], x1 = a[i1];
        a[i0] = {u00 * x0.re + u01 * x1.re, u00 * x0.im + u01 * x1.im};
        a[i1] = {u10 * x0.re + u11 * x1.re, u10 * x0.im + u11 * x1.im};
    }
    __syncthreads();
}

// RY(t) with c = cos(t/2), s = sin(t/2).
template <typename T>
__device__ __forceinline__ void lds_ry(cplx<T>* a, int nb, int q, T c, T s, int ctrl) {
    lds_real_1q<T>(a, nb, q, c, -s, s, c, ctrl);
}

template <typename T>
__device__ __forceinline__ void lds_h(cplx<T>* a, int nb, int q, int ctrl) {
    const T r = (T)0.70710678118654752440;
    lds_real_1q<T>(a, nb, q, r, r, r, -r, ctrl);
}

// CZ(q1, q2), optionally controlled (then a CCZ).
template <typename T>
__device__ void lds_cz(cplx<T>* a, int nb, int q1, int q2, int ctrl) {
    const int na = 1 << nb;
    const int need = (1 << q1) | (1 << q2) | (ctrl >= 0 ? (1 << ctrl) : 0);
    for (int i = threadIdx.x; i < na; i += blockDim.x)
        if ((i & need) == need) a[i] = {-a[i].re, -a[i].im};
    __syncthreads();
}

// The whole CZ ladder CZ(0,1) CZ(1,2) ... CZ(n-2,n-1) as one diagonal pass:
// the sign of basis state i is (-1)^{sum_q i_q i_{q+1}} (optionally only
// where bit ctrl is 1).
template <typename T>
__device__ void lds_cz_ladder(cplx<T>* a, int nb, int n, int ctrl) {
    const int na = 1 << nb;
    const uint32_t ladder = (1u << (n - 1)) - 1u;
    for (int i = threadIdx.x; i < na; i += blockDim.x) {
        if (ctrl >= 0 && !((i >> ctrl) & 1)) continue;
        if (parity((uint32_t)i & ((uint32_t)i >> 1) & ladder)) a[i] = {-a[i].re, -a[i].im};
    }
    __syncthreads();
}

// CNOT(control c, target t), optionally controlled (then a Toffoli).
template <typename T>
__device__ void lds_cx(cplx<T>* a, int nb, int c, int t, int ctrl) {
    const int half = 1 << (nb - 1);
    const int need = (1 << c) | (ctrl >= 0 ? (1 << ctrl) : 0);
    for (int p = threadIdx.x; p < half; p += blockDim.x) {
        const int i0 = insert0(p, t), i1 = i0 | (1 << t);
        if ((i0 & need) != need) continue;
        const cplx<T> x0 = a[i0];
        a[i0] = a[i1];
        a[i1] = x0;
    }
    __syncthreads();
}

// Pauli string (x, z) on the system bits [0, n) of the half selected by the
// ancilla bit n (ancilla-controlled when `controlled`, else on the whole
// register with n = nb).  (P psi)[k] = i^{|x&z|} (-1)^{|z & (k^x)|} psi[k^x].
template <typename T>
__device__ void lds_pauli(cplx<T>* a, int n, uint32_t x, uint32_t z, bool controlled) {
    const int N = 1 << n;
    cplx<T>* v = controlled ? a + N : a;
    const int ph = __popc(x & z);
    if (x == 0) {
        for (int k = threadIdx.x; k < N; k += blockDim.x)
            if (parity(z & (uint32_t)k)) v[k] = {-v[k].re, -v[k].im};
    } else {
        const int hb = 31 - __clz(x);  // pairs (k, k^x) with bit hb of k clear
        for (int p = threadIdx.x; p < N / 2; p += blockDim.x) {
            const int k0 = insert0(p, hb), k1 = k0 ^ (int)x;
            const cplx<T> v0 = v[k0], v1 = v[k1];
            // new[k0] = phase(k0) * old[k1], phase(k) = i^ph (-1)^{|z & (k^x)|}
            v[k0] = mul_ipow(v1, ph + 2 * parity(z & (uint32_t)k1));
            v[k1] = mul_ipow(v0, ph + 2 * parity(z & (uint32_t)k0));
        }
    }
    __syncthreads();
}

// Householder state preparation U_b = s (I - 2 w w^T / w^T w), w = e_0 - s b,
// applied to one n-qubit vector v (U_b is real symmetric: its own adjoint).
// `red` >= blockDim.x/64 doubles.
template <typename T>
__device__ void lds_householder(cplx<T>* v, int n, const double* __restrict__ b, double* red) {
    const int N = 1 << n;
    const double s = (b[0] > 0.0) ? -1.0 : 1.0;
    double ww = 0.0, dre = 0.0, dim = 0.0;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const double w = (k == 0 ? 1.0 : 0.0) - s * b[k];
        ww += w * w;
        dre += w * (double)v[k].re;
        dim += w * (double)v[k].im;
    }
    ww = block_sum(ww, red);
    dre = block_sum(dre, red);
    dim = block_sum(dim, red);
    const double fr = 2.0 * dre / ww, fi = 2.0 * dim / ww;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const double w = (k == 0 ? 1.0 : 0.0) - s * b[k];
        v[k] = {(T)(s * ((double)v[k].re - w * fr)), (T)(s * ((double)v[k].im - w * fi))};
    }
    __syncthreads();
}

// The ansatz V(theta) on the system bits of an nb-qubit register; trig[2k],
// trig[2k+1] = cos, sin of theta_k / 2.
template <typename T>
__device__ void lds_ansatz(cplx<T>* a, int nb, int n, int layers, int ent, const T* trig, int ctrl) {
    for (int l = 0; l < layers; ++l) {
        for (int q = 0; q < n; ++q) {
            const int k = l * n + q;
            lds_ry<T>(a, nb, q, trig[2 * k], trig[2 * k + 1], ctrl);
        }
        if (ent == DVQ_ENT_CZ_LADDER) {
            if (n > 1) lds_cz_ladder<T>(a, nb, n, ctrl);
        } else {
            for (int q = 0; q + 1 < n; ++q) lds_cx<T>(a, nb, q, q + 1, ctrl);
        }
    }
}

// cos / sin of theta_k / 2 for k < P into trig (computed in float64).
template <typename T>
__device__ void lds_trig(T* trig, const double* __restrict__ theta, int P) {
    for (int k = threadIdx.x; k < P; k += blockDim.x) {
        double s, c;
        sincos(0.5 * theta[k], &s, &c);
        trig[2 * k] = (T)c;
        trig[2 * k + 1] = (T)s;
    }
    __syncthreads();
}

}  // namespace dvq
