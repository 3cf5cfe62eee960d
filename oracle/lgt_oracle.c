/*
 * lgt_oracle.c -- plain FP64 CPU reference for the Trotterized adiabatic
 * evolution of quantum Z2 lattice gauge theory (Cui, Shi, Yang,
 * arXiv:1910.08020, JHEP 2020).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header or table with the
 * GPU library: everything here is written out directly from the paper's
 * definitions, with plain loops and no blocking, fusion or lookup tables.
 *
 * Conventions (paper Sec. 2.1):
 *   sigma^z |0> = |0>, sigma^z |1> = -|1>.  Bit q of an amplitude index is
 *   the state of link qubit q (bit = 1 <=> link in |1>).
 *   State vectors are arrays of 2^N "double complex" (re, im interleaved).
 *
 * Lattice numbering.  Fig. 1 of the paper is missing from the available
 * text; only its caption survives.  The numbering used here is the reading
 * that reproduces every plaquette quoted in that caption:
 *   site   s = sum_mu x_mu * prod_{nu<mu} L_nu        (x direction fastest)
 *   link   l(s, mu) = d*s + (d-1-mu)                  (mu = 0 is x, 0-based)
 *   plaquette (s; mu<nu) = { l(s,mu), l(s+e_mu,nu), l(s+e_nu,mu), l(s,nu) }
 *   star(s) = { l(s,mu), l(s-e_mu,mu) : mu = 0..d-1 }  (Gauss law, Sec. 2.1)
 * Plaquettes are listed site by site, and inside a site by (mu,nu) pairs in
 * lexicographic order.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXD 3

/* ------------------------------------------------------------------ */
/* lattice geometry (Sec. 2.1: N_l = d L^d, N_p = N_l (d-1)/2)          */
/* ------------------------------------------------------------------ */

static int wrap(int v, int L) { return ((v % L) + L) % L; }

static int site_of(int d, const int *L, const int *x)
{
    int s = 0, stride = 1;
    for (int mu = 0; mu < d; ++mu) {
        s += wrap(x[mu], L[mu]) * stride;
        stride *= L[mu];
    }
    return s;
}

static void coords_of(int d, const int *L, int s, int *x)
{
    for (int mu = 0; mu < d; ++mu) {
        x[mu] = s % L[mu];
        s /= L[mu];
    }
}

static int link_of(int d, const int *L, const int *x, int mu)
{
    return d * site_of(d, L, x) + (d - 1 - mu);
}

static int check_lattice(int d, const int *L)
{
    if (d < 2 || d > ORC_MAXD) return -1;
    for (int mu = 0; mu < d; ++mu)
        if (L[mu] < 2) return -1;
    return 0;
}

int orc_counts(int d, const int *L, int *n_sites, int *n_links, int *n_plaq)
{
    if (check_lattice(d, L)) return -1;
    int V = 1;
    for (int mu = 0; mu < d; ++mu) V *= L[mu];
    *n_sites = V;
    *n_links = d * V;
    *n_plaq = V * d * (d - 1) / 2;
    return 0;
}

/* out: n_plaq rows of 4 link indices, in the order described above */
int orc_plaquettes(int d, const int *L, int *out)
{
    if (check_lattice(d, L)) return -1;
    int ns, nl, np;
    orc_counts(d, L, &ns, &nl, &np);
    int k = 0;
    for (int s = 0; s < ns; ++s) {
        int x[ORC_MAXD], y[ORC_MAXD];
        coords_of(d, L, s, x);
        for (int mu = 0; mu < d; ++mu)
            for (int nu = mu + 1; nu < d; ++nu) {
                out[4 * k + 0] = link_of(d, L, x, mu);
                memcpy(y, x, sizeof y); y[mu] += 1;
                out[4 * k + 1] = link_of(d, L, y, nu);
                memcpy(y, x, sizeof y); y[nu] += 1;
                out[4 * k + 2] = link_of(d, L, y, mu);
                out[4 * k + 3] = link_of(d, L, x, nu);
                ++k;
            }
    }
    return k;
}

/* out: n_sites rows of 2d link indices: the links ending at each site */
int orc_stars(int d, const int *L, int *out)
{
    if (check_lattice(d, L)) return -1;
    int ns, nl, np;
    orc_counts(d, L, &ns, &nl, &np);
    for (int s = 0; s < ns; ++s) {
        int x[ORC_MAXD], y[ORC_MAXD];
        coords_of(d, L, s, x);
        for (int mu = 0; mu < d; ++mu) {
            out[2 * d * s + 2 * mu] = link_of(d, L, x, mu);
            memcpy(y, x, sizeof y); y[mu] -= 1;
            out[2 * d * s + 2 * mu + 1] = link_of(d, L, y, mu);
        }
    }
    return ns;
}

/*
 * Links traversed by a closed walk on the direct lattice (a Wegner-Wilson
 * contour, Sec. 2.1).  moves[i] = +(mu+1) steps along +mu, -(mu+1) along
 * -mu.  A link traversed twice cancels (sigma^z squared is one), so the
 * result is the set of links crossed an odd number of times.  Returns the
 * number of links written to out (at most n_moves), or -1.
 */
int orc_walk_links(int d, const int *L, int start_site, const int *moves,
                   int n_moves, int *out)
{
    if (check_lattice(d, L)) return -1;
    int ns, nl, np;
    orc_counts(d, L, &ns, &nl, &np);
    unsigned char *odd = calloc((size_t)nl, 1);
    if (!odd) return -1;
    int x[ORC_MAXD];
    coords_of(d, L, start_site, x);
    for (int i = 0; i < n_moves; ++i) {
        int m = moves[i];
        int mu = (m > 0 ? m : -m) - 1;
        if (mu < 0 || mu >= d) { free(odd); return -1; }
        if (m > 0) {
            odd[link_of(d, L, x, mu)] ^= 1;
            x[mu] = wrap(x[mu] + 1, L[mu]);
        } else {
            x[mu] = wrap(x[mu] - 1, L[mu]);
            odd[link_of(d, L, x, mu)] ^= 1;
        }
    }
    int k = 0;
    for (int l = 0; l < nl; ++l)
        if (odd[l]) out[k++] = l;
    free(odd);
    return k;
}

/* ------------------------------------------------------------------ */
/* state preparation                                                    */
/* ------------------------------------------------------------------ */

/* |+>^N: every link qubit in (|0>+|1>)/sqrt 2 (Sec. 2.3, after the Hadamards) */
void orc_init_plus(double complex *psi, int N)
{
    uint64_t dim = 1ull << N;
    double a = 1.0 / sqrt((double)dim);
    for (uint64_t b = 0; b < dim; ++b) psi[b] = a;
}

/* computational basis state |b0> */
void orc_init_basis(double complex *psi, int N, uint64_t b0)
{
    uint64_t dim = 1ull << N;
    for (uint64_t b = 0; b < dim; ++b) psi[b] = 0;
    psi[b0] = 1;
}

/* ------------------------------------------------------------------ */
/* evolution operators                                                  */
/* ------------------------------------------------------------------ */

/*
 * exp(+i alpha sigma^x_q) on link q, i.e. R_x(-2 alpha) with
 * R_x(phi) = exp(-i sigma^x phi / 2) (Sec. 2.2, link layer).
 */
void orc_rx_link(double complex *psi, int N, int q, double alpha)
{
    uint64_t dim = 1ull << N, bit = 1ull << q;
    double c = cos(alpha), s = sin(alpha);
    long long nb = (long long)dim;
#pragma omp parallel for schedule(static)
    for (long long bb = 0; bb < nb; ++bb) {
        uint64_t b = (uint64_t)bb;
        if (b & bit) continue;
        double complex a0 = psi[b], a1 = psi[b | bit];
        psi[b] = c * a0 + I * s * a1;
        psi[b | bit] = I * s * a0 + c * a1;
    }
}

/* the whole link layer exp(-i t (-h_x sum_l sigma^x_l)) with alpha = t h_x */
void orc_x_layer(double complex *psi, int N, double alpha)
{
    for (int q = 0; q < N; ++q) orc_rx_link(psi, N, q, alpha);
}

/*
 * Plaquette layer: exp(+i theta sum_p U_p) with U_p = prod_{l in p} sigma^z_l.
 * This is exp(-i t H_Z) for H_Z = -c_z sum_p U_p and theta = t c_z.  Each
 * amplitude is multiplied by exp(i theta sum_p u_p(b)), the sum evaluated
 * directly from the plaquette link lists.
 */
void orc_plaq_layer(double complex *psi, int N, int n_plaq, const int *plaq,
                    double theta)
{
    uint64_t dim = 1ull << N;
    long long nb = (long long)dim;
#pragma omp parallel for schedule(static)
    for (long long bb = 0; bb < nb; ++bb) {
        uint64_t b = (uint64_t)bb;
        int sum = 0;
        for (int p = 0; p < n_plaq; ++p) {
            int par = 0;
            for (int k = 0; k < 4; ++k) par ^= (int)((b >> plaq[4 * p + k]) & 1u);
            sum += par ? -1 : 1;
        }
        psi[b] *= cexp(I * theta * (double)sum);
    }
}

/*
 * Trotterized evolution with a Hamiltonian that changes every step
 * (Sec. 2.2).  Step j (0-based here) uses
 *     H_j = -cx[j] sum_l sigma^x_l - cz[j] sum_p U_p
 * over a time dt.
 *   order 1 (eq. (a), first order):  psi <- e^{-i dt Hz_j} e^{-i dt Hx_j} psi
 *   order 2 (eq. (s), symmetric):    psi <- e^{-i dt Hz_j/2} e^{-i dt Hx_j} e^{-i dt Hz_j/2} psi
 * The symmetric form is applied unmerged: adjacent half steps are not
 * combined here.
 */
int orc_evolve(double complex *psi, int N, int n_plaq, const int *plaq,
               long long n_steps, const double *cx, const double *cz,
               double dt, int order)
{
    if (order != 1 && order != 2) return -1;
    for (long long j = 0; j < n_steps; ++j) {
        if (order == 1) {
            orc_x_layer(psi, N, dt * cx[j]);
            orc_plaq_layer(psi, N, n_plaq, plaq, dt * cz[j]);
        } else {
            orc_plaq_layer(psi, N, n_plaq, plaq, 0.5 * dt * cz[j]);
            orc_x_layer(psi, N, dt * cx[j]);
            orc_plaq_layer(psi, N, n_plaq, plaq, 0.5 * dt * cz[j]);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* circuit form: one gate at a time (Sec. 2.2, eq. (ara) and the link   */
/* layer), with the ancilla replaced by the last link of the plaquette  */
/* ------------------------------------------------------------------ */

void orc_cnot(double complex *psi, int N, int ctrl, int tgt)
{
    uint64_t dim = 1ull << N, cb = 1ull << ctrl, tb = 1ull << tgt;
    for (uint64_t b = 0; b < dim; ++b) {
        if ((b & cb) && !(b & tb)) {
            double complex t = psi[b];
            psi[b] = psi[b | tb];
            psi[b | tb] = t;
        }
    }
}

/* R_z(phi) = exp(-i sigma^z phi / 2) on qubit q */
void orc_rz(double complex *psi, int N, int q, double phi)
{
    uint64_t dim = 1ull << N, bit = 1ull << q;
    double complex e0 = cexp(-I * phi / 2), e1 = cexp(I * phi / 2);
    for (uint64_t b = 0; b < dim; ++b) psi[b] *= (b & bit) ? e1 : e0;
}

/* R_x(phi) = exp(-i sigma^x phi / 2) on qubit q */
void orc_rx(double complex *psi, int N, int q, double phi)
{
    uint64_t dim = 1ull << N, bit = 1ull << q;
    double c = cos(phi / 2), s = sin(phi / 2);
    for (uint64_t b = 0; b < dim; ++b) {
        if (b & bit) continue;
        double complex a0 = psi[b], a1 = psi[b | bit];
        psi[b] = c * a0 - I * s * a1;
        psi[b | bit] = -I * s * a0 + c * a1;
    }
}

/*
 * exp(+i theta U_p) for one plaquette as a gate sequence: the parity of the
 * four links is collected on the last listed link by a CNOT ladder, a
 * z-rotation R_z(-2 theta) acts on that link, and the ladder is undone.
 * On even parity R_z(-2 theta) multiplies by e^{+i theta}, on odd parity by
 * e^{-i theta}, which is exp(+i theta u_p(b)).
 */
void orc_plaq_gadget(double complex *psi, int N, const int *links, double theta)
{
    int t = links[3];
    orc_cnot(psi, N, links[0], t);
    orc_cnot(psi, N, links[1], t);
    orc_cnot(psi, N, links[2], t);
    orc_rz(psi, N, t, -2.0 * theta);
    orc_cnot(psi, N, links[2], t);
    orc_cnot(psi, N, links[1], t);
    orc_cnot(psi, N, links[0], t);
}

static void circuit_x(double complex *psi, int N, double alpha)
{
    for (int q = 0; q < N; ++q) orc_rx(psi, N, q, -2.0 * alpha);
}

static void circuit_z(double complex *psi, int N, int n_plaq, const int *plaq,
                      double theta)
{
    for (int p = 0; p < n_plaq; ++p) orc_plaq_gadget(psi, N, plaq + 4 * p, theta);
}

/* same schedule and orders as orc_evolve, executed gate by gate */
int orc_evolve_circuit(double complex *psi, int N, int n_plaq, const int *plaq,
                       long long n_steps, const double *cx, const double *cz,
                       double dt, int order)
{
    if (order != 1 && order != 2) return -1;
    for (long long j = 0; j < n_steps; ++j) {
        if (order == 1) {
            circuit_x(psi, N, dt * cx[j]);
            circuit_z(psi, N, n_plaq, plaq, dt * cz[j]);
        } else {
            circuit_z(psi, N, n_plaq, plaq, 0.5 * dt * cz[j]);
            circuit_x(psi, N, dt * cx[j]);
            circuit_z(psi, N, n_plaq, plaq, 0.5 * dt * cz[j]);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* circuits with one ancilla qubit a (Sec. 2.2, eq. (ara); Sec. 2.3;    */
/* the controlled evolution U(t) of Sec. 2.4).  The state has N + 1     */
/* qubits; the callers put the ancilla on bit N.                        */
/* ------------------------------------------------------------------ */

/* controlled-Z: amplitude sign flips where qubits a and b are both |1> */
void orc_cz(double complex *psi, int Ntot, int a, int b)
{
    uint64_t dim = 1ull << Ntot, m = (1ull << a) | (1ull << b);
    for (uint64_t i = 0; i < dim; ++i)
        if ((i & m) == m) psi[i] = -psi[i];
}

/* measurement of qubit q with outcome |0> selected: the |1> half is dropped
   (the caller renormalises) */
void orc_project_zero(double complex *psi, int Ntot, int q)
{
    uint64_t dim = 1ull << Ntot, bit = 1ull << q;
    for (uint64_t i = 0; i < dim; ++i)
        if (i & bit) psi[i] = 0;
}

/*
 * eq. (ara): A^-1 R_z^a(-2 theta) A with A the product of CNOT(l -> a) over the four
 * plaquette links.  A writes the plaquette parity into the ancilla, R_z^a(-2 theta)
 * multiplies ancilla |0> by e^{+i theta} and |1> by e^{-i theta}, and the reversed
 * CNOTs restore the ancilla.  Ancilla |0>: exp(+i theta U_p) = exp(-i theta Z_p);
 * ancilla |1>: the opposite sign, i.e. the time-reversed plaquette evolution.
 */
void orc_anc_gadget(double complex *psi, int Ntot, const int *links, int a, double theta)
{
    for (int k = 0; k < 4; ++k) orc_cnot(psi, Ntot, links[k], a);
    orc_rz(psi, Ntot, a, -2.0 * theta);
    for (int k = 3; k >= 0; --k) orc_cnot(psi, Ntot, links[k], a);
}

/* link layer exp(+i alpha sum sigma^x); with `controlled`, each R_x sits between two
   CZ(a, l), which turns it into R_x of the opposite angle when the ancilla is |1>
   (Z R_x(phi) Z = R_x(-phi)): the direction of time follows the ancilla */
static void anc_x(double complex *psi, int N, int a, double alpha, int controlled)
{
    for (int q = 0; q < N; ++q) {
        if (controlled) orc_cz(psi, N + 1, a, q);
        orc_rx(psi, N + 1, q, -2.0 * alpha);
        if (controlled) orc_cz(psi, N + 1, a, q);
    }
}

static void anc_z(double complex *psi, int N, int a, int n_plaq, const int *plaq, double theta)
{
    for (int p = 0; p < n_plaq; ++p) orc_anc_gadget(psi, N + 1, plaq + 4 * p, a, theta);
}

/* the orders of orc_evolve with the ancilla gadget for every plaquette; the ancilla is
   bit N of the (N+1)-qubit state */
int orc_evolve_ancilla(double complex *psi, int N, int n_plaq, const int *plaq,
                       long long n_steps, const double *cx, const double *cz,
                       double dt, int order, int controlled)
{
    if (order != 1 && order != 2) return -1;
    const int a = N;
    for (long long j = 0; j < n_steps; ++j) {
        if (order == 1) {
            anc_x(psi, N, a, dt * cx[j], controlled);
            anc_z(psi, N, a, n_plaq, plaq, dt * cz[j]);
        } else {
            anc_z(psi, N, a, n_plaq, plaq, 0.5 * dt * cz[j]);
            anc_x(psi, N, a, dt * cx[j], controlled);
            anc_z(psi, N, a, n_plaq, plaq, 0.5 * dt * cz[j]);
        }
    }
    return 0;
}

/*
 * Sec. 2.3: from |+>^N |0>_a, for each plaquette the four CNOT(l -> a) put its parity on
 * the ancilla, the ancilla is measured with outcome |0> (even parity, U_p = +1), and four
 * more CNOTs return it to |0>.  The product of the projections is left unnormalised.
 */
void orc_prepare_ground_circuit(double complex *psi, int N, int n_plaq, const int *plaq)
{
    const int a = N;
    for (int p = 0; p < n_plaq; ++p) {
        const int *l = plaq + 4 * p;
        for (int k = 0; k < 4; ++k) orc_cnot(psi, N + 1, l[k], a);
        orc_project_zero(psi, N + 1, a);
        for (int k = 3; k >= 0; --k) orc_cnot(psi, N + 1, l[k], a);
    }
}

/* ------------------------------------------------------------------ */
/* pseudo-measurement (Sec. 2.4): sums over all basis states            */
/* Sums run sequentially in ascending b with an extended-precision      */
/* (long double) accumulator, so that 2^24-term sums stay far below     */
/* the 1e-10 comparison tolerance.                                      */
/* ------------------------------------------------------------------ */

/* <psi|psi> */
double orc_norm2(const double complex *psi, int N)
{
    uint64_t dim = 1ull << N;
    long double acc = 0;
    for (uint64_t b = 0; b < dim; ++b) {
        double re = creal(psi[b]), im = cimag(psi[b]);
        acc += re * re + im * im;
    }
    return acc;
}

/* <psi| prod_{l in links} sigma^z_l |psi>, not normalized */
double orc_expect_z(const double complex *psi, int N, const int *links, int n)
{
    uint64_t dim = 1ull << N;
    long double acc = 0;
    for (uint64_t b = 0; b < dim; ++b) {
        int par = 0;
        for (int k = 0; k < n; ++k) par ^= (int)((b >> links[k]) & 1u);
        double re = creal(psi[b]), im = cimag(psi[b]);
        double p = re * re + im * im;
        acc += par ? -p : p;
    }
    return acc;
}

/* Re <psi| prod_{l in links} sigma^x_l |psi>, not normalized */
double orc_expect_x(const double complex *psi, int N, const int *links, int n)
{
    uint64_t dim = 1ull << N, flip = 0;
    for (int k = 0; k < n; ++k) flip ^= 1ull << links[k];
    long double acc = 0;
    for (uint64_t b = 0; b < dim; ++b) acc += creal(conj(psi[b]) * psi[b ^ flip]);
    return acc;
}

/*
 * Density of states of Z = -sum_p U_p (Sec. 3.3): out[m] = sum of |psi_b|^2
 * over the basis states with exactly m plaquettes of odd parity, so that the
 * eigenvalue of Z there is z = -(n_plaq - 2m).  out has n_plaq+1 entries.
 */
void orc_zdos(const double complex *psi, int N, int n_plaq, const int *plaq,
              double *out)
{
    uint64_t dim = 1ull << N;
    long double *acc = calloc((size_t)n_plaq + 1, sizeof(long double));
    if (!acc) return;
    for (uint64_t b = 0; b < dim; ++b) {
        int m = 0;
        for (int p = 0; p < n_plaq; ++p) {
            int par = 0;
            for (int k = 0; k < 4; ++k) par ^= (int)((b >> plaq[4 * p + k]) & 1u);
            m += par;
        }
        double re = creal(psi[b]), im = cimag(psi[b]);
        acc[m] += re * re + im * im;
    }
    for (int m = 0; m <= n_plaq; ++m) out[m] = (double)acc[m];
    free(acc);
}

/* ------------------------------------------------------------------ */
/* sampling in the computational basis                                 */
/* ------------------------------------------------------------------ */

/*
 * SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), used as a counter-based
 * generator: draw i is the finalizer applied to seed + (i+1)*golden_gamma.
 * The uniform is the top 53 bits scaled by 2^-53.
 */
static uint64_t splitmix64_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double orc_uniform(uint64_t seed, uint64_t i)
{
    return (double)(splitmix64_at(seed, i) >> 11) * (1.0 / 9007199254740992.0);
}

/*
 * Shot i is the smallest basis index b whose cumulative probability
 * sum_{b' <= b} |psi_b'|^2 exceeds u_i * <psi|psi> (inverse CDF in
 * ascending b).  The cumulative sums are taken in plain sequential order.
 */
int orc_sample(const double complex *psi, int N, uint64_t n_shots,
               uint64_t seed, uint64_t *out)
{
    uint64_t dim = 1ull << N;
    double *cdf = malloc(sizeof(double) * dim);
    if (!cdf) return -1;
    long double acc = 0;
    for (uint64_t b = 0; b < dim; ++b) {
        double re = creal(psi[b]), im = cimag(psi[b]);
        acc += re * re + im * im;
        cdf[b] = acc;
    }
    for (uint64_t i = 0; i < n_shots; ++i) {
        double target = orc_uniform(seed, i) * (double)acc;
        uint64_t lo = 0, hi = dim - 1;
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > target) hi = mid; else lo = mid + 1;
        }
        out[i] = lo;
    }
    free(cdf);
    return 0;
}

/* the cumulative sums themselves, for tests that check a sample's validity */
int orc_cdf(const double complex *psi, int N, double *cdf)
{
    uint64_t dim = 1ull << N;
    long double acc = 0;
    for (uint64_t b = 0; b < dim; ++b) {
        double re = creal(psi[b]), im = cimag(psi[b]);
        acc += re * re + im * im;
        cdf[b] = acc;
    }
    return 0;
}
