// Host FP64 schedule and per-step tables (Sec. 2.2 of arXiv:1910.08020).
//
// Step j of a run of n substeps of length dt = T/n uses the coupling at the
// substep's right end, f_j = (j+1)/n, as in g_{k,m} = (k-1) g_s + m delta.
// First order (eq. (a)) applies the link layer, then the plaquette phase.
// The symmetric order (eq. (s)) brackets the link layer with two half phases;
// inside one call the half phases of neighbouring substeps are merged into a
// single phase table, as in the rewritten product that follows eq. (s).
#include <cmath>
#include <limits>

#include "lgt_internal.hpp"

namespace lgt {

std::string schedule_coeffs(const lgt_schedule *s, int64_t first, int64_t count, double &dt,
                            std::vector<double> &cx, std::vector<double> &cz)
{
    if (!s) return "null schedule";
    if (s->n_steps < 1) return "schedule needs n_steps >= 1";
    if (!std::isfinite(s->T) || s->T == 0.0) return "schedule T must be finite and nonzero";
    if (first < 0 || count < 0 || first + count > s->n_steps)
        return "step range outside [0, n_steps)";
    if (count > (int64_t)1 << 30) return "too many steps in one call";
    if (s->s_rule != 0 && s->s_rule != 1) return "s_rule must be 0 or 1";
    dt = s->T / (double)s->n_steps;
    cx.resize(count);
    cz.resize(count);
    const double n = (double)s->n_steps;
    for (int64_t i = 0; i < count; ++i) {
        const int64_t j = first + i;
        const double f = s->s_rule == 0 ? (double)(j + 1) / n : ((double)j + 0.5) / n;
        switch (s->ramp) {
        case LGT_RAMP_PLAQ:
            cx[i] = s->h_x;
            cz[i] = f * s->h_p;
            break;
        case LGT_RAMP_COUPLING:
            cx[i] = s->g0 + (s->g1 - s->g0) * f;
            cz[i] = 1.0;
            break;
        case LGT_RAMP_EXPLICIT:
            if (!s->cx || !s->cz) return "explicit schedule needs cx and cz arrays";
            cx[i] = s->cx[j];
            cz[i] = s->cz[j];
            break;
        default:
            return "unknown ramp";
        }
        if (!std::isfinite(cx[i]) || !std::isfinite(cz[i])) return "non-finite coefficient";
    }
    return "";
}

void build_step_tables(int n_links, int n_plaq, double dt, const double *cx, const double *cz,
                       int n_steps, int order, StepTables &out)
{
    out.n_steps = n_steps;
    out.pre_phase = (order == LGT_ORDER_SYMMETRIC) ? 1 : 0;
    out.n_phase = n_steps + out.pre_phase;
    out.rot_u.resize(n_steps);
    out.rot_v.resize(n_steps);
    std::vector<double> scale(n_steps);
    for (int j = 0; j < n_steps; ++j) {
        // exp(+i a sigma^x) = cos a + i sin a sigma^x, a = dt cx_j  (R_x(-2 a))
        const double a = dt * cx[j];
        const double c = std::cos(a), s = std::sin(a);
        if (std::fabs(c) >= std::fabs(s)) {
            out.rot_u[j] = 1.0;
            out.rot_v[j] = s / c;
            scale[j] = std::pow(c, n_links);
        } else {
            out.rot_u[j] = c / s;
            out.rot_v[j] = 1.0;
            scale[j] = std::pow(s, n_links);
        }
    }
    const int np1 = n_plaq + 1;
    out.ph_re.assign((size_t)out.n_phase * np1, 0.0);
    out.ph_im.assign((size_t)out.n_phase * np1, 0.0);
    auto fill = [&](int k, double theta, double sc) {
        // exp(-i t Hz) with Hz = -cz sum U_p: phase e^{i theta (n_plaq - 2m)} for m odd plaquettes
        for (int m = 0; m <= n_plaq; ++m) {
            const double ang = theta * (double)(n_plaq - 2 * m);
            out.ph_re[(size_t)k * np1 + m] = sc * std::cos(ang);
            out.ph_im[(size_t)k * np1 + m] = sc * std::sin(ang);
        }
    };
    if (order == LGT_ORDER_TROTTER) {
        for (int j = 0; j < n_steps; ++j) fill(j, dt * cz[j], scale[j]);
    } else {
        if (n_steps > 0) fill(0, 0.5 * dt * cz[0], 1.0);
        for (int j = 0; j < n_steps; ++j) {
            const double th = (j + 1 < n_steps) ? 0.5 * dt * (cz[j] + cz[j + 1]) : 0.5 * dt * cz[j];
            fill(j + 1, th, scale[j]);
        }
    }
}

// Nearest float, then the +-2 ulp neighbourhood searched for the pair whose relative
// squared-magnitude error, added to `carry` (the error of the same entry summed over the
// rows before it), is smallest in magnitude (ties: closest to the value).  Returns the
// chosen pair's error.  Choosing for the running sum rather than for each row alone keeps
// the product of a run's magnitudes within about one ulp of its target: for slowly varying
// couplings the nearest magnitude misses its target by the same amount, with the same
// sign, for thousands of rows, and over 10^6 rows those misses sum to 1e-2.
static double round_pair_norm(double x, double y, double target2, double carry, float &fx,
                              float &fy)
{
    const float x0 = (float)x, y0 = (float)y;
    float cx[5], cy[5];
    cx[2] = x0;
    cy[2] = y0;
    cx[1] = std::nextafter(x0, -INFINITY); cx[0] = std::nextafter(cx[1], -INFINITY);
    cx[3] = std::nextafter(x0, INFINITY);  cx[4] = std::nextafter(cx[3], INFINITY);
    cy[1] = std::nextafter(y0, -INFINITY); cy[0] = std::nextafter(cy[1], -INFINITY);
    cy[3] = std::nextafter(y0, INFINITY);  cy[4] = std::nextafter(cy[3], INFINITY);
    // a float squared is exact in double (24-bit significands), so a*a + b*b carries one
    // rounding at most: far below the spacing of the candidates' magnitudes (~1e-7)
    double best = std::numeric_limits<double>::infinity(), bestd = best, beste = 0;
    fx = x0;
    fy = y0;
    for (int i = 0; i < 5; ++i)
        for (int k = 0; k < 5; ++k) {
            const double a = cx[i], b = cy[k];
            const double rel = (a * a + b * b) / target2 - 1.0;
            const double e = std::fabs(carry + rel);
            const double dd = (a - x) * (a - x) + (b - y) * (b - y);
            if (e < best || (e == best && dd < bestd)) {
                best = e;
                bestd = dd;
                beste = rel;
                fx = cx[i];
                fy = cy[k];
            }
        }
    return beste;
}

void round_rot_f32(const StepTables &in, int n_links, std::vector<RotParam<float>> &rot,
                   std::vector<long double> &gain)
{
    rot.resize(in.n_steps);
    gain.resize(in.n_steps);   // norm gain of the float link layer
    for (int j = 0; j < in.n_steps; ++j) {
        rot[j].u = (float)in.rot_u[j];
        rot[j].v = (float)in.rot_v[j];
        long double g = (long double)rot[j].u * rot[j].u + (long double)rot[j].v * rot[j].v;
        gain[j] = std::pow(g, (long double)n_links);
    }
}

void round_phase_f32(const StepTables &in, int n_plaq, const std::vector<long double> &gain,
                     int k0, int k1, std::vector<Cplx<float>> &ph, PhaseRounding &pr)
{
    // Norm gains of the link layers smaller than this are carried to a later phase row:
    // a phase entry whose magnitude is within a few ulps of 1 is applied as a whole ulp or
    // not at all (the same way every row), while one at least this far from 1 is applied
    // to the nearest ulp.  Every call's last row takes what is left, so a call ends with
    // the norm it started with.
    constexpr long double kFoldLog = 1.0L / 4096;
    const int np1 = n_plaq + 1;
    if (ph.size() < (size_t)in.n_phase * np1) ph.resize((size_t)in.n_phase * np1);
    if (pr.carry.size() != (size_t)np1) pr.carry.assign(np1, 0.0);
    for (int k = k0; k < k1; ++k) {
        // the phase after link layer j undoes that layer's gain, now or at a later row
        const int j = k - in.pre_phase;
        if (j >= 0) pr.gain *= gain[j];
        long double target2 = 1.0L;
        if (k == in.n_phase - 1 || std::fabs(std::log(pr.gain)) > kFoldLog) {
            target2 = 1.0L / pr.gain;
            pr.gain = 1.0L;
        }
        // sign of the folded cos^N / sin^N factor, from the FP64 table
        double mag = 0;
        for (int m = 0; m < np1; ++m)
            mag = std::max(mag, std::hypot(in.ph_re[(size_t)k * np1 + m],
                                           in.ph_im[(size_t)k * np1 + m]));
        const double rescale = (mag > 0) ? std::sqrt((double)target2) / mag : 1.0;
        for (int m = 0; m < np1; ++m) {
            const size_t i = (size_t)k * np1 + m;
            pr.carry[m] += round_pair_norm(in.ph_re[i] * rescale, in.ph_im[i] * rescale,
                                           (double)target2, pr.carry[m], ph[i].re, ph[i].im);
        }
    }
}

void round_tables_f32(const StepTables &in, int n_links, int n_plaq,
                      std::vector<RotParam<float>> &rot, std::vector<Cplx<float>> &ph)
{
    std::vector<long double> gain;
    round_rot_f32(in, n_links, rot, gain);
    ph.assign((size_t)in.n_phase * (n_plaq + 1), Cplx<float>{});
    PhaseRounding pr;
    round_phase_f32(in, n_plaq, gain, 0, in.n_phase, ph, pr);
}

void round_tables_f64(const StepTables &in, int n_plaq, std::vector<RotParam<double>> &rot,
                      std::vector<Cplx<double>> &ph)
{
    const int np1 = n_plaq + 1;
    rot.resize(in.n_steps);
    for (int j = 0; j < in.n_steps; ++j) {
        rot[j].u = in.rot_u[j];
        rot[j].v = in.rot_v[j];
    }
    ph.resize((size_t)in.n_phase * np1);
    for (size_t i = 0; i < ph.size(); ++i) {
        ph[i].re = in.ph_re[i];
        ph[i].im = in.ph_im[i];
    }
}

}  // namespace lgt
