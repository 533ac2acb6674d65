/*
 * Memory and undefined-behaviour check of the oracle (test infrastructure).
 *
 * Built by oracle.build_sanitized() with g++ -fsanitize=address,undefined
 * and run by the CPU tests: it includes the oracle's single source, fills a
 * few small grids with smooth physical data (a curved metric with shift and
 * extrinsic curvature, periodic and copy boundaries, 1D, 2D and 3D), and
 * calls every grid entry point once -- the step, its dual-number tangent,
 * the stages, the plain recovery, the explicit operator, the conductivity
 * models and the atmosphere.  Any invalid access or undefined operation
 * aborts with the sanitizer's report; a failed recovery returns 1.
 */
#include "rmhd_oracle.cpp"

#include <cstdio>

namespace {

struct Case {
    int n[3], active, bc;
    bool curved;
    int sigma_model;
    double rho_atmo;
};

double wave(double x, double y, double z, double a, double b, double c) {
    return std::sin(6.283185307179586 * (a * x + b * y + c * z));
}

int run(const Case& cs) {
    Grid gr;
    std::memset(&gr, 0, sizeof gr);
    for (int d = 0; d < 3; ++d) {
        gr.n[d] = cs.n[d];
        gr.bc[d] = cs.bc;
        gr.dx[d] = 1.0 / cs.n[d];
        gr.x0[d] = 0.5 * gr.dx[d];
    }
    gr.active = cs.active;
    gr.ng = 3;
    gr.recon = 2;
    gr.c2p_maxit = 500;
    gr.speed_mode = 0;
    gr.gamma_ad = 4.0 / 3.0;
    gr.kappa = 1.0;
    gr.c2p_tol = 1e-14;
    gr.sigma_model = cs.sigma_model;
    gr.sigma0 = 50.0;
    gr.sigma_exp = 2.0;
    gr.sigma_Datmo = 0.2;
    gr.rho_atmo = cs.rho_atmo;
    gr.K_atmo = 0.5;
    Geo ge(gr);
    const long Np = ge.Np;
    std::vector<double> P((size_t)NF * Np), U((size_t)NF * Np), met((size_t)NM * Np), sig((size_t)Np);
    for (int k = 0; k < ge.np[2]; ++k)
        for (int j = 0; j < ge.np[1]; ++j)
            for (int i = 0; i < ge.np[0]; ++i) {
                const long o = ge.idx(i, j, k);
                const double x = gr.x0[0] + (i - ge.g[0]) * gr.dx[0];
                const double y = gr.x0[1] + (j - ge.g[1]) * gr.dx[1];
                const double z = gr.x0[2] + (k - ge.g[2]) * gr.dx[2];
                const double w1 = wave(x, y, z, 1, 1, 0), w2 = wave(x, y, z, 0, 1, 1), w3 = wave(x, y, z, 1, 0, 1);
                double* p = P.data();
                p[(long)P_RHO * Np + o] = 1.0 + 0.3 * w1;
                p[(long)P_PRS * Np + o] = 0.6 + 0.2 * w2;
                p[(long)(P_V + 0) * Np + o] = 0.2 * w3;
                p[(long)(P_V + 1) * Np + o] = -0.15 * w1;
                p[(long)(P_V + 2) * Np + o] = 0.1 * w2;
                p[(long)(P_B + 0) * Np + o] = 0.4 + 0.1 * w2;
                p[(long)(P_B + 1) * Np + o] = 0.3 * w3;
                p[(long)(P_B + 2) * Np + o] = -0.2 * w1;
                for (int c = 0; c < 3; ++c) p[(long)(P_E + c) * Np + o] = 0.05 * (c + 1) * w1;
                p[(long)P_PHI * Np + o] = 0.01 * w2;
                p[(long)P_PSI * Np + o] = -0.01 * w3;
                p[(long)P_Q * Np + o] = 0.02 * w1;
                sig[(size_t)o] = 10.0 + 5.0 * w2;
                double f[NM];
                flat_fields(f);
                if (cs.curved) {
                    f[M_ALP] = 1.0 - 0.05 * w1;
                    for (int b = 0; b < 3; ++b) f[M_BET + b] = 0.02 * (b + 1) * w2;
                    const double psi4 = 1.0 + 0.1 * w3;
                    f[M_G + 0] = f[M_G + 3] = f[M_G + 5] = psi4;
                    f[M_G + 1] = 0.01 * w1;
                    for (int b = 0; b < 6; ++b) f[M_K + b] = 0.03 * w2 * (b % 3 == 0 ? 1.0 : 0.5);
                }
                for (int a = 0; a < NM; ++a) met[(size_t)a * Np + o] = f[a];
            }
    const double* mp = cs.curved ? met.data() : nullptr;
    orc_prim2con(&gr, mp, P.data(), U.data());
    const double dt = 0.2 * gr.dx[0];
    long nf = 0;
    // explicit operator, recovery, stages, step, tangent
    std::vector<double> L((size_t)NF * Np), Pr((size_t)NF * Np);
    std::vector<int32_t> st((size_t)Np), it((size_t)Np);
    orc_explicit_rhs(&gr, mp, P.data(), sig.data(), L.data());
    nf += orc_con2prim(&gr, mp, U.data(), P.data(), Pr.data(), st.data(), it.data());
    std::vector<double> P1(P), U1(U), R1((size_t)3 * Np), U2(U), P2(P), R2((size_t)3 * Np), F1((size_t)NF * Np),
        U3(U), P3(P);
    const double* sp = cs.sigma_model ? nullptr : sig.data();
    nf += orc_stage1(&gr, mp, dt, sp, U.data(), P.data(), P1.data(), R1.data(), U1.data(), st.data(), it.data());
    nf += orc_stage2(&gr, mp, dt, sp, U.data(), P1.data(), R1.data(), U2.data(), P2.data(), R2.data(), F1.data(),
                     st.data(), it.data());
    nf += orc_final(&gr, mp, dt, sp, U.data(), F1.data(), P2.data(), R1.data(), R2.data(), U3.data(), P3.data(),
                    st.data(), it.data());
    std::vector<double> Us(U), Ps(P);
    nf += orc_step(&gr, mp, dt, sp, Us.data(), Ps.data(), st.data());
    std::vector<double> Ut(U), dU((size_t)NF * Np, 1e-3), Pt(P), dP((size_t)NF * Np), ds((size_t)Np, 0.1);
    nf += orc_step_tangent(&gr, mp, dt, sig.data(), ds.data(), Ut.data(), dU.data(), Pt.data(), dP.data());
    const double smax = orc_max_signal_speed(&gr, mp);
    std::printf("case n=%dx%dx%d active=%d bc=%d curved=%d model=%d atmo=%g: failed %ld, max speed %.4g\n",
                cs.n[0], cs.n[1], cs.n[2], cs.active, cs.bc, (int)cs.curved, cs.sigma_model, cs.rho_atmo, nf, smax);
    return nf == 0 ? 0 : 1;
}

}  // namespace

int main() {
    const Case cases[] = {
        {{7, 5, 4}, 7, BC_PERIODIC, true, 0, 0.0},
        {{6, 5, 1}, 3, BC_COPY, true, 1, 0.0},
        {{9, 1, 1}, 1, BC_COPY, false, 2, 0.0},
        {{5, 4, 6}, 7, BC_COPY, true, 2, 1.05},
        {{8, 3, 1}, 1, BC_PERIODIC, false, 0, 0.0},
    };
    int bad = 0;
    for (const Case& c : cases) bad |= run(c);
    return bad;
}
