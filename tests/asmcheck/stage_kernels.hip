// Instantiates every stage kernel so that its gfx950 assembly can be checked
// (tests/test_stage_waits.py); never linked into the library.
#include <hip/hip_runtime.h>
#include "rmhd_kernels.hpp"
using namespace rmhd;
template <int S, bool C, bool K> void inst(const Params& p, double* a, unsigned long long* c, int* s) {
    k_stage<S, C, K><<<1, 64>>>(p, 0.1, a, a, a, a, a, a, a, a, a, a, s, 1L, c);
}
void all(const Params& p, double* a, unsigned long long* c, int* s) {
    inst<1, false, false>(p, a, c, s); inst<1, true, false>(p, a, c, s); inst<1, true, true>(p, a, c, s);
    inst<2, false, false>(p, a, c, s); inst<2, true, false>(p, a, c, s); inst<2, true, true>(p, a, c, s);
    inst<3, false, false>(p, a, c, s); inst<3, true, false>(p, a, c, s); inst<3, true, true>(p, a, c, s);
}
