// Circuit enumeration and launch plumbing shared by the Hadamard-test kernels.
#pragma once

#include "common.h"

namespace dvq {

enum TermType { kBeta = 0, kDelta = 1, kGamma = 2 };

struct Term {
    int part;  // 0: real-part circuit, 1: imaginary-part circuit (S^dagger)
    int type;  // kBeta / kDelta / kGamma
    int j;     // qubit of Z_j (delta only)
    int l, m;  // term indices (m unused for gamma)
};

// Arguments of one dvq_vqls_terms launch (passed by value to the kernels).
struct TermsArgs {
    const double* theta;
    const dvq_pauli* strings;
    const double* b;
    dvq_c128* beta;
    dvq_c128* other;
    int n, layers, ent, L, kind, bkind, B;
    int64_t c0;       // first circuit (in decode_term order) of each row's range
    int64_t per_row;  // circuits per row in this launch: c0 .. c0 + per_row - 1
    int64_t total;    // per_row * B
};

// The same launch restricted to circuits first .. first + count - 1 of each
// row (first and count even: whole Re/Im pairs).
inline TermsArgs sub_range(const TermsArgs& g, int64_t first, int64_t count) {
    TermsArgs r = g;
    r.c0 = first;
    r.per_row = count;
    r.total = count * g.B;
    return r;
}

// Circuit c of one theta row.  Order: consecutive pairs (Re, Im) of one term;
// local: terms t = jj*L^2 + l*L + m with jj = 0 for beta and jj = j+1 for
// delta^j; global: beta terms l*L + m, then gamma_l at L^2 + l.
__host__ __device__ __forceinline__ Term decode_term(int64_t c, int L, int n, int kind) {
    Term t;
    t.part = (int)(c & 1);
    const int64_t u = c >> 1;
    const int64_t L2 = (int64_t)L * L;
    if (kind == DVQ_COST_LOCAL) {
        const int64_t jj = u / L2;
        const int64_t lm = u - jj * L2;
        t.type = jj == 0 ? kBeta : kDelta;
        t.j = (int)jj - 1;
        t.l = (int)(lm / L);
        t.m = (int)(lm - (int64_t)t.l * L);
    } else if (u < L2) {
        t.type = kBeta;
        t.j = -1;
        t.l = (int)(u / L);
        t.m = (int)(u - (int64_t)t.l * L);
    } else {
        t.type = kGamma;
        t.j = -1;
        t.l = (int)(u - L2);
        t.m = 0;
    }
    (void)n;
    return t;
}

__device__ __forceinline__ void store_term(const TermsArgs& g, int64_t row, const Term& t, double z) {
    const int64_t L2 = (int64_t)g.L * g.L;
    dvq_c128* dst;
    if (t.type == kBeta)
        dst = g.beta + row * L2 + (int64_t)t.l * g.L + t.m;
    else if (t.type == kDelta)
        dst = g.other + row * (int64_t)g.n * L2 + (int64_t)t.j * L2 + (int64_t)t.l * g.L + t.m;
    else
        dst = g.other + row * (int64_t)g.L + t.l;
    reinterpret_cast<double*>(dst)[t.part] = z;
}

// 2-D grid of at least `total` workgroups (x at most 65536), as few extra
// (immediately exiting) workgroups as possible: gy rows of gx.
inline dim3 grid_for(int64_t total) {
    const int64_t gy = (total + 65535) / 65536;
    const int64_t gx = (total + gy - 1) / gy;
    return dim3((unsigned)gx, (unsigned)gy);
}

template <typename T>
__host__ __device__ constexpr size_t generic_trig_offset(int n, int layers) {
    // amplitudes, then 2P trig values, rounded up to 16 B
    return (((size_t(1) << (n + 1)) * sizeof(cplx<T>) + 2 * sizeof(T) * n * layers) + 15) / 16 * 16;
}

template <typename T>
inline size_t generic_lds_bytes(int n, int layers) {
    return generic_trig_offset<T>(n, layers) + 8 * sizeof(double);
}

dvq_status check_ansatz(const dvq_ansatz* an, int max_n);
dvq_status make_terms_args(TermsArgs& g, const dvq_ansatz* an, const double* theta, int B,
                           int precision, const dvq_pauli* strings, int L, int b_kind,
                           const double* b, int cost_kind, dvq_c128* beta, dvq_c128* other);
dvq_status launch_terms(const TermsArgs& g, int precision, int exec, hipStream_t s);
// Register-resident production kernels; DVQ_EUNSUPPORTED when the shape has none.
dvq_status launch_terms_fast(const TermsArgs& g, int precision, hipStream_t s);
dvq_status launch_terms_shared(const TermsArgs& g, int precision, hipStream_t s);
// Register-resident adjoint (one wavefront per row); DVQ_EUNSUPPORTED when
// the shape has none.
dvq_status launch_adjoint_fast(const dvq_ansatz* an, const double* theta, int B, int precision,
                               const dvq_c128* coeffs, const dvq_pauli* strings, int L,
                               int per_row_system, int bkind, const double* b, int kind, double* C,
                               double* grad, hipStream_t s);

}  // namespace dvq
