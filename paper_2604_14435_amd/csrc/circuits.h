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

// floor(n / d) for 0 <= n < 2^31 as one 64-bit multiply and shift.  With
// s = ceil(log2 d) and m = floor(2^(31+s) / d) + 1, 2^(31+s) < m d <=
// 2^(31+s) + 2^s, so floor(m n / 2^(31+s)) = floor(n / d) for every such n
// (Granlund and Montgomery, division by invariant integers); m < 2^33 and
// m n < 2^64.  The kernels' circuit indices are wave-uniform, so this runs on
// the scalar unit instead of a 64-bit division expansion on the vector unit.
struct DivBy {
    uint64_t m;
    int shift;  // 31 + s
};

inline DivBy div_by(uint32_t d) {
    int s = 0;
    while ((uint64_t(1) << s) < d) ++s;
    return {(uint64_t(1) << (31 + s)) / d + 1, 31 + s};
}

__device__ __forceinline__ uint32_t div_fast(uint32_t n, const DivBy& D) {
    return (uint32_t)(((uint64_t)n * D.m) >> D.shift);
}

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
    // divisors of the index decode when c0 + per_row and total are below
    // 2^31 (fast_div = 1; set by with_fast_div just before a launch)
    DivBy div_row, div_L2, div_L;
    int fast_div;
};

// g with the decode divisors filled in (fast_div = 0 past 2^31 circuits).
inline TermsArgs with_fast_div(TermsArgs g) {
    const int64_t lim = int64_t(1) << 31;
    g.fast_div = (g.total < lim && g.c0 + g.per_row < lim && g.per_row > 0) ? 1 : 0;
    if (g.fast_div) {
        g.div_row = div_by((uint32_t)g.per_row);
        g.div_L2 = div_by((uint32_t)((int64_t)g.L * g.L));
        g.div_L = div_by((uint32_t)g.L);
    }
    return g;
}

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

// decode_term for c < 2^31 with the launch's divisors (same order).
__device__ __forceinline__ Term decode_term_fast(uint32_t c, const TermsArgs& g) {
    Term t;
    t.part = (int)(c & 1u);
    const uint32_t u = c >> 1;
    const uint32_t L = (uint32_t)g.L, L2 = L * L;
    if (g.kind == DVQ_COST_LOCAL) {
        const uint32_t jj = div_fast(u, g.div_L2);
        const uint32_t lm = u - jj * L2;
        t.type = jj == 0 ? kBeta : kDelta;
        t.j = (int)jj - 1;
        t.l = (int)div_fast(lm, g.div_L);
        t.m = (int)(lm - (uint32_t)t.l * L);
    } else if (u < L2) {
        t.type = kBeta;
        t.j = -1;
        t.l = (int)div_fast(u, g.div_L);
        t.m = (int)(u - (uint32_t)t.l * L);
    } else {
        t.type = kGamma;
        t.j = -1;
        t.l = (int)(u - L2);
        t.m = 0;
    }
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

// Both parts of term t (the real-part and imaginary-part circuits) in one
// 16-byte store.
__device__ __forceinline__ void store_term_pair(const TermsArgs& g, int64_t row, const Term& t, double re_part,
                                                double im_part) {
    const int64_t L2 = (int64_t)g.L * g.L;
    dvq_c128* dst;
    if (t.type == kBeta)
        dst = g.beta + row * L2 + (int64_t)t.l * g.L + t.m;
    else if (t.type == kDelta)
        dst = g.other + row * (int64_t)g.n * L2 + (int64_t)t.j * L2 + (int64_t)t.l * g.L + t.m;
    else
        dst = g.other + row * (int64_t)g.L + t.l;
    *dst = dvq_c128{re_part, im_part};
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
