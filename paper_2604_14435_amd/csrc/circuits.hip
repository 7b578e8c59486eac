// Hadamard-test circuits of one VQLS cost evaluation (Section II-A, II-C,
// Eq. (4)): the generic kernel (one workgroup per circuit, amplitudes in LDS,
// one pass per gate), circuit enumeration, and the dvq_vqls_terms entry point.
#include "circuits.h"
#include "gates_lds.h"

namespace dvq {

// ---------------------------------------------------------------- generic kernel

template <typename T>
__global__ void __launch_bounds__(256) k_terms_generic(TermsArgs g) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = g.n, nb = n + 1, na = 1 << nb, P = n * g.layers, anc = n;
    cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
    T* trig = reinterpret_cast<T*>(a + na);
    double* red = reinterpret_cast<double*>(smem + generic_trig_offset<T>(n, g.layers));

    const int64_t gid = (int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
    if (gid >= g.total) return;
    const int64_t row = gid / g.per_row;
    const Term t = decode_term(g.c0 + gid - row * g.per_row, g.L, n, g.kind);

    lds_trig<T>(trig, g.theta + row * P, P);
    for (int i = threadIdx.x; i < na; i += blockDim.x) a[i] = {(T)(i == 0 ? 1 : 0), (T)0};
    __syncthreads();

    lds_h<T>(a, nb, anc, -1);
    const int vctrl = (t.type == kGamma) ? anc : -1;
    lds_ansatz<T>(a, nb, n, g.layers, g.ent, trig, vctrl);
    const dvq_pauli pl = g.strings[t.l];
    if (t.type == kBeta) {
        const dvq_pauli pm = g.strings[t.m];
        lds_pauli<T>(a, n, pm.x, pm.z, true);
        lds_pauli<T>(a, n, pl.x, pl.z, true);
    } else if (t.type == kDelta) {
        const dvq_pauli pm = g.strings[t.m];
        lds_pauli<T>(a, n, pm.x, pm.z, true);
        if (g.bkind == DVQ_B_PLUS) {
            for (int q = 0; q < n; ++q) lds_h<T>(a, nb, q, -1);
        } else {
            lds_householder<T>(a, n, g.b, red);
            lds_householder<T>(a + (1 << n), n, g.b, red);
        }
        lds_cz<T>(a, nb, anc, t.j, -1);
        if (g.bkind == DVQ_B_PLUS) {
            for (int q = 0; q < n; ++q) lds_h<T>(a, nb, q, -1);
        } else {
            lds_householder<T>(a, n, g.b, red);
            lds_householder<T>(a + (1 << n), n, g.b, red);
        }
        lds_pauli<T>(a, n, pl.x, pl.z, true);
    } else {
        lds_pauli<T>(a, n, pl.x, pl.z, true);
        if (g.bkind == DVQ_B_PLUS) {
            for (int q = 0; q < n; ++q) lds_h<T>(a, nb, q, anc);
        } else {
            lds_householder<T>(a + (1 << n), n, g.b, red);
        }
    }
    if (t.part) {  // S^dagger on the ancilla: |1> -> -i |1>
        const int N = 1 << n;
        for (int k = threadIdx.x; k < N; k += blockDim.x) a[N + k] = mul_ipow(a[N + k], 3);
        __syncthreads();
    }
    lds_h<T>(a, nb, anc, -1);

    // <Z_ancilla> = sum_{anc=0} |a|^2 - sum_{anc=1} |a|^2
    T zacc = 0;
    for (int i = threadIdx.x; i < na; i += blockDim.x) {
        const T p = a[i].re * a[i].re + a[i].im * a[i].im;
        zacc += (i >> anc) & 1 ? -p : p;
    }
    const T z = block_sum<T>(zacc, reinterpret_cast<T*>(red));
    if (threadIdx.x == 0) store_term(g, row, t, (double)z);
}

template <typename T>
static dvq_status launch_generic(const TermsArgs& g, hipStream_t s) {
    const size_t lds = generic_lds_bytes<T>(g.n, g.layers);
    if (lds > kMaxLdsBytes)
        return fail(DVQ_EUNSUPPORTED, "generic circuit kernel: n=%d needs %zu B of LDS", g.n, lds);
    DVQ_TRY_HIP(allow_lds((const void*)k_terms_generic<T>, lds));
    const dim3 grid = grid_for(g.total);
    hipLaunchKernelGGL(k_terms_generic<T>, grid, dim3(256), lds, s, g);
    DVQ_CHECK_LAUNCH("k_terms_generic");
    return DVQ_OK;
}

static dvq_status launch_generic_p(const TermsArgs& g, int precision, hipStream_t s) {
    return precision == DVQ_F32 ? launch_generic<float>(g, s) : launch_generic<double>(g, s);
}

// Global cost: the beta circuits (the first 2 L^2 of a row) go to the
// register-resident kernels where the shape has them, the gamma circuits
// (controlled V(theta), 2 L per row) to the generic kernel.
dvq_status launch_terms(const TermsArgs& g, int precision, int exec, hipStream_t s) {
    if (exec == DVQ_EXEC_LITERAL || exec == DVQ_EXEC_SHARED) {
        auto fast = [&](const TermsArgs& a) {
            return exec == DVQ_EXEC_LITERAL ? launch_terms_fast(a, precision, s) : launch_terms_shared(a, precision, s);
        };
        const int64_t nbeta = 2 * (int64_t)g.L * g.L, end = g.c0 + g.per_row;
        if (g.kind == DVQ_COST_GLOBAL && g.c0 < nbeta) {
            const int64_t bend = end < nbeta ? end : nbeta;
            dvq_status st = fast(sub_range(g, g.c0, bend - g.c0));
            if (st == DVQ_OK)
                return end > nbeta ? launch_generic_p(sub_range(g, nbeta, end - nbeta), precision, s) : DVQ_OK;
            if (st != DVQ_EUNSUPPORTED) return st;
        } else if (g.kind == DVQ_COST_LOCAL) {
            dvq_status st = fast(g);
            if (st != DVQ_EUNSUPPORTED) return st;
        }
    }
    return launch_generic_p(g, precision, s);
}

dvq_status check_ansatz(const dvq_ansatz* an, int max_n) {
    DVQ_REQUIRE(an != nullptr, "ansatz is NULL");
    DVQ_REQUIRE(an->n >= 1 && an->n <= max_n, "ansatz n=%d outside 1..%d", an->n, max_n);
    DVQ_REQUIRE(an->layers >= 1 && an->layers <= 64, "ansatz layers=%d outside 1..64", an->layers);
    DVQ_REQUIRE(an->entangler == DVQ_ENT_CZ_LADDER || an->entangler == DVQ_ENT_CNOT_LADDER,
                "unknown entangler %d", an->entangler);
    return DVQ_OK;
}

dvq_status make_terms_args(TermsArgs& g, const dvq_ansatz* an, const double* theta, int B,
                           int precision, const dvq_pauli* strings, int L, int b_kind,
                           const double* b, int cost_kind, dvq_c128* beta, dvq_c128* other) {
    dvq_status st = check_ansatz(an, precision == DVQ_F32 ? 13 : 12);
    if (st != DVQ_OK) return st;
    DVQ_REQUIRE(precision == DVQ_F32 || precision == DVQ_F64, "unknown precision %d", precision);
    DVQ_REQUIRE(theta && strings && beta && other, "null device pointer");
    DVQ_REQUIRE(B >= 1, "B=%d < 1", B);
    DVQ_REQUIRE(L >= 1 && L <= 65536, "L=%d outside 1..65536", L);
    DVQ_REQUIRE(b_kind == DVQ_B_PLUS || b_kind == DVQ_B_VECTOR, "unknown b_kind %d", b_kind);
    DVQ_REQUIRE(b_kind == DVQ_B_PLUS || b != nullptr, "b is NULL for DVQ_B_VECTOR");
    DVQ_REQUIRE(cost_kind == DVQ_COST_GLOBAL || cost_kind == DVQ_COST_LOCAL, "unknown cost kind %d",
                cost_kind);
    const int64_t per_row = dvq_circuit_count(an->n, L, cost_kind);
    DVQ_REQUIRE(per_row * (int64_t)B < (int64_t(1) << 31), "B * circuits = %lld too large",
                (long long)(per_row * B));
    g.theta = theta;
    g.strings = strings;
    g.b = b;
    g.beta = beta;
    g.other = other;
    g.n = an->n;
    g.layers = an->layers;
    g.ent = an->entangler;
    g.L = L;
    g.kind = cost_kind;
    g.bkind = b_kind;
    g.c0 = 0;
    g.per_row = per_row;
    g.total = per_row * B;
    g.B = B;
    return DVQ_OK;
}

}  // namespace dvq

using namespace dvq;

extern "C" dvq_status dvq_vqls_terms(const dvq_ansatz* ansatz, const double* theta, int32_t B,
                                     int32_t precision, const dvq_pauli* strings, int32_t L,
                                     int32_t b_kind, const double* b, int32_t cost_kind,
                                     int32_t exec, dvq_c128* beta, dvq_c128* other,
                                     dvq_stream stream) {
    TermsArgs g;
    dvq_status st = make_terms_args(g, ansatz, theta, B, precision, strings, L, b_kind, b,
                                    cost_kind, beta, other);
    if (st != DVQ_OK) return st;
    DVQ_REQUIRE(exec == DVQ_EXEC_LITERAL || exec == DVQ_EXEC_GENERIC || exec == DVQ_EXEC_SHARED,
                "unknown exec %d", exec);
    return launch_terms(g, precision, exec, stream_of(stream));
}

extern "C" dvq_status dvq_vqls_terms_rhs(const dvq_ansatz* ansatz, const double* theta, int32_t B,
                                         int32_t precision, const dvq_pauli* strings, int32_t L, int32_t R,
                                         const double* b, int32_t cost_kind, int32_t exec, dvq_c128* beta,
                                         dvq_c128* other, dvq_stream stream) {
    DVQ_REQUIRE(R >= 1 && R <= 65536, "R=%d outside 1..65536", R);
    DVQ_REQUIRE(b != nullptr, "b is NULL");
    TermsArgs g;
    dvq_status st = make_terms_args(g, ansatz, theta, B, precision, strings, L, DVQ_B_VECTOR, b, cost_kind,
                                    beta, other);
    if (st != DVQ_OK) return st;
    DVQ_REQUIRE(exec == DVQ_EXEC_LITERAL || exec == DVQ_EXEC_GENERIC || exec == DVQ_EXEC_SHARED,
                "unknown exec %d", exec);
    const hipStream_t s = stream_of(stream);
    const int64_t N = int64_t(1) << g.n, nbeta = 2 * (int64_t)L * L;
    const int64_t other_row = cost_kind == DVQ_COST_LOCAL ? (int64_t)g.n * L * L : (int64_t)L;
    // beta does not involve b: once
    if ((st = launch_terms(sub_range(g, 0, nbeta), precision, exec, s)) != DVQ_OK) return st;
    // the b-dependent circuits, once per right-hand side
    for (int r = 0; r < R; ++r) {
        TermsArgs gr = sub_range(g, nbeta, g.per_row - nbeta);
        gr.b = b + r * N;
        gr.other = other + (int64_t)r * B * other_row;
        if ((st = launch_terms(gr, precision, exec, s)) != DVQ_OK) return st;
    }
    return DVQ_OK;
}
