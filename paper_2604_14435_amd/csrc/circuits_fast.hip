// Register-resident Hadamard-test kernels (one wavefront per circuit).
#include "circuits.h"

namespace dvq {

dvq_status launch_terms_fast(const TermsArgs& g, int precision, hipStream_t s) {
    (void)g;
    (void)precision;
    (void)s;
    return DVQ_EUNSUPPORTED;
}

}  // namespace dvq
