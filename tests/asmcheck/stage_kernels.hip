// Instantiates every stage kernel (the fused final update + stage 1 too),
// the FP64 x-flux kernels and y/z window kernels (general and diagonal
// metric; the z window with the stage-2 update too) so that their gfx950
// assembly can be checked (tests/test_stage_waits.py); never linked into the
// library.
#include <hip/hip_runtime.h>
#include "rmhd_kernels.hpp"
using namespace rmhd;
template <int S, bool C, bool K, bool DG> void inst(const Params& p, double* a, unsigned long long* c, int* s) {
    k_stage<S, C, K, DG><<<1, 64>>>(p, 0.1, a, a, a, a, a, a, a, a, a, a, a, s, 1L, c);
}
template <int RC, bool C, bool DG> void inst_x(const Params& p, double* a) {
    k_flux_p<0, RC, C, double, false, DG><<<8, 256>>>(p, a, a, a, 1, 1L);
}
template <int D, int RC, bool C, class R, bool SH, bool DG> void inst_w(const Params& p, double* a) {
    k_flux_w<D, RC, C, R, SH, DG><<<8, 64>>>(p, a, a, a, 32, 1, 1);
}
void all_w(const Params& p, double* a) {
    inst_w<1, 2, true, double, false, false>(p, a); inst_w<2, 2, true, double, false, false>(p, a);
    inst_w<1, 1, true, double, false, false>(p, a); inst_w<2, 0, false, double, false, false>(p, a);
    inst_w<1, 2, true, float, false, false>(p, a); inst_w<2, 2, true, float, false, false>(p, a);
    inst_w<1, 2, true, double, true, false>(p, a); inst_w<2, 1, true, float, true, false>(p, a);
    inst_w<1, 2, true, double, false, true>(p, a); inst_w<2, 2, true, double, false, true>(p, a);
    inst_w<1, 2, true, float, false, true>(p, a); inst_w<2, 1, true, double, true, true>(p, a);
}
template <int S> void stages(const Params& p, double* a, unsigned long long* c, int* s) {
    inst<S, false, false, false>(p, a, c, s);
    inst<S, true, false, false>(p, a, c, s); inst<S, true, true, false>(p, a, c, s);
    inst<S, true, false, true>(p, a, c, s); inst<S, true, true, true>(p, a, c, s);
}
void all(const Params& p, double* a, unsigned long long* c, int* s) {
    inst_x<0, false, false>(p, a); inst_x<1, false, false>(p, a); inst_x<2, false, false>(p, a);
    inst_x<0, true, false>(p, a); inst_x<1, true, false>(p, a); inst_x<2, true, false>(p, a);
    inst_x<0, true, true>(p, a); inst_x<1, true, true>(p, a); inst_x<2, true, true>(p, a);
    stages<1>(p, a, c, s); stages<2>(p, a, c, s); stages<3>(p, a, c, s); stages<4>(p, a, c, s);
}
template <int RC, bool C, bool DG> void inst_f(const Params& p, double* a) {
    k_flux_w<2, RC, C, double, false, DG, true><<<8, 64>>>(p, a, a, a, 32, 1, 1, FuseArgs{});
}
void all_f(const Params& p, double* a) {
    inst_f<1, true, true>(p, a); inst_f<0, true, true>(p, a); inst_f<1, false, false>(p, a);
}
