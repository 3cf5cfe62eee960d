// Host check of the complex64 step tables (no GPU): the rounding the library uploads,
// compiled from its own source with g++.  For long runs of small and large steps:
//  - rounding the phase rows in pieces (as a run is pipelined) equals rounding them whole;
//  - per phase entry, the product of the rows' squared magnitudes undoes the product of the
//    link layers' norm gains to within 5e-7 (relative), however many rows;
//  - every row is either of unit magnitude within a few ulps or at least 2^-14 away from
//    it (a row that undoes gathered gains), apart from the last;
//  - every entry keeps the FP64 phase angle within 1e-6.
#include <cmath>
#include <cstdio>
#include <vector>

#include "lgt_internal.hpp"

using namespace lgt;

static int failures = 0;

static void check(bool ok, const char *what, const char *name)
{
    if (!ok) {
        std::printf("%s: FAILED %s\n", name, what);
        ++failures;
    }
}

static void run(const char *name, int n_links, int n_plaq, double dt, const std::vector<double> &cx,
                const std::vector<double> &cz, int order)
{
    const int n = (int)cx.size(), np1 = n_plaq + 1;
    StepTables st;
    build_step_tables(n_links, n_plaq, dt, cx.data(), cz.data(), n, order, st);
    std::vector<RotParam<float>> rot;
    std::vector<Cplx<float>> whole;
    round_tables_f32(st, n_links, n_plaq, rot, whole);
    // in pieces of 32, 64, 128, ... rows
    std::vector<long double> gain;
    std::vector<RotParam<float>> rot2;
    round_rot_f32(st, n_links, rot2, gain);
    std::vector<Cplx<float>> parts((size_t)st.n_phase * np1);
    PhaseRounding pr;
    for (int k0 = 0, len = 32; k0 < st.n_phase; k0 += len, len *= 2)
        round_phase_f32(st, n_plaq, gain, k0, std::min(st.n_phase, k0 + len), parts, pr);
    bool same = rot.size() == rot2.size();
    for (size_t i = 0; same && i < rot.size(); ++i) same = rot[i].u == rot2[i].u && rot[i].v == rot2[i].v;
    for (size_t i = 0; same && i < whole.size(); ++i) same = whole[i].re == parts[i].re && whole[i].im == parts[i].im;
    check(same, "pieces differ from the whole table", name);
    long double log_gain = 0;
    for (int j = 0; j < n; ++j) log_gain += std::log(gain[j]);
    double worst = 0, worst_angle = 0;
    int folds = 0, between = 0;
    for (int m = 0; m < np1; ++m) {
        long double log_mag = 0;
        for (int k = 0; k < st.n_phase; ++k) {
            const Cplx<float> p = whole[(size_t)k * np1 + m];
            const long double a2 = (long double)p.re * p.re + (long double)p.im * p.im;
            log_mag += std::log(a2);
            const double d = std::fabs((double)a2 - 1.0);
            if (m == 0 && k + 1 < st.n_phase) {
                if (d > 1.0 / 16384) ++folds;
                else if (d > 8.0 * 0x1p-24) ++between;
            }
            const size_t i = (size_t)k * np1 + m;
            const double want = std::atan2(st.ph_im[i], st.ph_re[i]);
            double got = std::atan2((double)p.im, (double)p.re) - want;
            got = std::remainder(got, 2 * M_PI);
            worst_angle = std::max(worst_angle, std::fabs(got));
        }
        worst = std::max(worst, (double)std::fabs(log_mag + log_gain));
    }
    check(worst < 5e-7, "magnitudes do not undo the gains", name);
    check(between == 0, "a row is neither unit nor a gathered correction", name);
    check(worst_angle < 1e-6, "phase angle moved", name);
    std::printf("%s: rows %d, folded rows %d, |log prod| %.2e, angle %.1e: %s\n", name, st.n_phase,
                folds, worst, worst_angle, failures ? "FAILED" : "ok");
}

int main()
{
    {   // the paper's scan: 2 x 10^5 substeps of 4e-5, coupling ramped from 0 (3x3)
        const int n = 200000;
        std::vector<double> g(n), one(n, 1.0);
        for (int j = 0; j < n; ++j) g[j] = 2.0 * (j + 1) / n;
        run("ramp first order", 18, 9, 4e-5, g, one, LGT_ORDER_TROTTER);
        run("ramp symmetric", 18, 9, 4e-5, g, one, LGT_ORDER_SYMMETRIC);
        run("constant coupling", 18, 9, 4e-5, one, one, LGT_ORDER_TROTTER);
    }
    {   // the benchmark's steps (2x2x2, dt = 0.05): gains folded every row; tan and cot forms
        const int n = 2000;
        for (double hx : {0.2, 1.0, 25.0}) {
            std::vector<double> cx(n, hx), cz(n);
            for (int j = 0; j < n; ++j) cz[j] = (j + 1.0) / n;
            char name[64];
            std::snprintf(name, sizeof name, "2x2x2 h_x=%g", hx);
            run(name, 24, 24, 0.05, cx, cz, LGT_ORDER_SYMMETRIC);
        }
    }
    std::printf("failures: %d\n", failures);
    return failures ? 1 : 0;
}
