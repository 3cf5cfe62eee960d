/*
 * lgt.h -- C ABI of the MI355X state-vector engine for the Trotterized
 * adiabatic evolution of quantum Z2 lattice gauge theory
 * (Cui, Shi, Yang, "Circuit-based digital adiabatic quantum simulation and
 * pseudoquantum simulation as new approaches to lattice gauge theory",
 * arXiv:1910.08020).
 *
 * Model (Sec. 2.1).  One qubit per link of a periodic d-dimensional lattice,
 * d in {2,3}.  sigma^z|0> = |0>, sigma^z|1> = -|1>.  The engine evolves
 *     H_j = -cx_j sum_l sigma^x_l - cz_j sum_p U_p,   U_p = prod_{l in p} sigma^z_l
 * which covers both the paper's H = Z + g X (cx = g, cz = 1) and the form
 * H(s) = -h_x sum sigma^x - s h_p sum U_p in which the plaquette term ramps.
 *
 * State layout.  2^N interleaved complex amplitudes (complex64: float re,im;
 * complex128: double re,im), N = number of links.  Bit q of the amplitude
 * index is link q (bit set <=> link in |1>).  Sites are numbered with the
 * x coordinate fastest; link l(s,mu) = d*s + (d-1-mu) (mu = 0 is x); the
 * plaquette (s; mu<nu) is {l(s,mu), l(s+e_mu,nu), l(s+e_nu,mu), l(s,nu)}.
 * This numbering reproduces the plaquettes quoted in the caption of Fig. 1.
 *
 * Errors.  Every call returns an lgt_status; nothing else crosses the ABI.
 * After a failure lgt_last_error(ctx) returns a message owned by the context
 * (or by the library for calls without a context), valid until the next call
 * on that context.  A context must not be used from two threads at once.
 *
 * Asynchrony.  Calls that enqueue GPU work (reset, evolve) return once the
 * work is enqueued on the context's stream.  Calls that return host data
 * (measure, sample, get_state) synchronise the stream first.
 */
#ifndef LGT_H
#define LGT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lgt_ctx lgt_ctx;

typedef enum {
    LGT_OK = 0,
    LGT_E_INVALID = 1,      /* bad argument (null pointer, size, enum, lattice) */
    LGT_E_UNSUPPORTED = 2,  /* valid request the engine does not implement      */
    LGT_E_OOM = 3,          /* device or host allocation failed, or over budget  */
    LGT_E_DEVICE = 4,       /* a HIP runtime call failed                          */
    LGT_E_STATE = 5,        /* call not valid in the object's current state       */
    LGT_E_BUSY = 6          /* server: no slot or memory free right now           */
} lgt_status;

typedef enum { LGT_C64 = 0, LGT_C128 = 1 } lgt_dtype;

/* eq. (a) generalised first-order decomposition; eq. (s) symmetric one */
typedef enum { LGT_ORDER_TROTTER = 1, LGT_ORDER_SYMMETRIC = 2 } lgt_order;

/* FUSED: link layer in LDS-tiled passes with the plaquette phases folded into
 * the pass that ends a step (consecutive steps share that pass, see lgt_set_plan).
 * CIRCUIT: one full-state pass per gate, as in eq. (ara)
 * (CNOT ladder onto the last plaquette link, R_z, inverse ladder) and the
 * R_x link layer of Sec. 2.2. */
/* ANCILLA: eq. (ara) itself: for every plaquette the CNOTs from its four links onto the
 * ancilla qubit, R_z^a(-2 theta) on the ancilla and the CNOTs in reverse order, and R_x on
 * every link.  With the ancilla in |0> this is the forward evolution; in |1> the plaquette
 * part runs backwards in time (the remark after eq. (ara)).
 * CONTROLLED: the same with every R_x between two CZ(ancilla, link), so that the ancilla
 * sets the direction of time of the whole step: |0><0| (x) U(t) + |1><1| (x) U(-t), the
 * controlled evolution that phase estimation needs (Sec. 2.4).
 * Both need a context from lgt_create_ancilla; such a context runs these two forms only. */
typedef enum {
    LGT_FORM_FUSED = 0,
    LGT_FORM_CIRCUIT = 1,
    LGT_FORM_ANCILLA = 2,
    LGT_FORM_CONTROLLED = 3
} lgt_form;

typedef enum {
    LGT_INIT_PLUS = 0,     /* |+>^N: Hadamard on every link (Sec. 2.3)              */
    LGT_INIT_ZGROUND = 1,  /* prod_p P_p |+>^N normalised: every U_p = +1 (Sec. 2.3) */
    LGT_INIT_BASIS = 2,    /* computational basis state |basis_index>                */
    LGT_INIT_ZGROUND_CIRCUIT = 3  /* ancilla contexts: |+>^N |0>_a, then for every plaquette
                                     CNOTs onto the ancilla, a measurement keeping ancilla
                                     |0>, CNOTs back (Sec. 2.3); normalised at the end.
                                     Equals ZGROUND (x) |0>_a                               */
} lgt_init;

/* ---------------------------------------------------------------------------
 * Lattice and context
 * ------------------------------------------------------------------------- */

/*
 * lgt_create: build the lattice (Sec. 2.1: N_l = d prod L, N_p = N_l (d-1)/2)
 * and allocate its 2^N_l-amplitude state on the current HIP device, set to
 * |+>^N.  d in {2,3}; L[0..d-1] >= 2; periodic must be 1 (the paper uses tori
 * only; 0 gives LGT_E_UNSUPPORTED).  N_l <= 34 and N_p <= 32, else
 * LGT_E_UNSUPPORTED.  A state that does not fit gives LGT_E_OOM.
 * On success *out owns the device state, a stream and small tables; release
 * with lgt_destroy.
 */
lgt_status lgt_create(int d, const int *L, int periodic, lgt_dtype dtype, lgt_ctx **out);

/*
 * lgt_create_ex: as lgt_create, but the state lives in a caller-owned device
 * buffer dev_buf of `bytes` bytes (>= state size, 256-byte aligned) and the
 * context enqueues on the caller's hipStream_t `stream` (NULL: a new stream).
 * The caller keeps ownership of both; they must outlive the context.  The
 * buffer is set to |+>^N.
 */
lgt_status lgt_create_ex(int d, const int *L, int periodic, lgt_dtype dtype,
                         void *dev_buf, size_t bytes, void *stream, lgt_ctx **out);

/*
 * lgt_create_ancilla: as lgt_create, with one ancilla qubit a = bit N_l of the amplitude
 * index on top of the links (2^(N_l+1) amplitudes; the lattice part of every index keeps
 * its layout).  lgt_reset puts the lattice in the requested state and the ancilla in |0>
 * (LGT_INIT_BASIS takes an (N_l+1)-bit index).  Such a context evolves with
 * LGT_FORM_ANCILLA / LGT_FORM_CONTROLLED; lgt_measure, lgt_sample, lgt_apply_pauli and
 * lgt_apply_gate act on all N_l + 1 qubits (masks may name bit N_l).  Scans, batches,
 * lgt_tune and LGT_OBS_XDOS give LGT_E_UNSUPPORTED.
 */
lgt_status lgt_create_ancilla(int d, const int *L, int periodic, lgt_dtype dtype, lgt_ctx **out);

lgt_status lgt_destroy(lgt_ctx *ctx);

typedef struct {
    int d, L[3];
    int n_links, n_plaq, n_sites;
    lgt_dtype dtype;
    size_t state_bytes;
    void *state;                  /* device pointer to the amplitudes                   */
    void *stream;                 /* hipStream_t the context enqueues on                */
    const uint64_t *plaq_masks;   /* [n_plaq]   links of each plaquette, as bit masks   */
    const int32_t *plaq_links;    /* [n_plaq*4] links in the order l(s,mu), l(s+e_mu,nu), l(s+e_nu,mu), l(s,nu) */
    const uint64_t *star_masks;   /* [n_sites]  links ending at each site (Gauss law G_i) */
    const uint32_t *link_plaqs;   /* [n_links]  plaquettes containing each link, bit p   */
    int n_qubits;                 /* n_links, plus 1 for an ancilla context              */
} lgt_info_t;

/* Host pointers in *out stay valid until lgt_destroy. */
lgt_status lgt_info(const lgt_ctx *ctx, lgt_info_t *out);

/*
 * lgt_lattice_query: host-only geometry of the lattice lgt_create would build
 * (Sec. 2.1), without touching a GPU.  Counts are written to the non-null
 * count pointers; plaq_links (n_plaq*4 int32, same order as lgt_info) and
 * star_masks (n_sites uint64) are filled when non-null.  Errors as lgt_create.
 */
lgt_status lgt_lattice_query(int d, const int *L, int *n_links, int *n_plaq, int *n_sites,
                             int32_t *plaq_links, uint64_t *star_masks);

/*
 * lgt_wilson_mask: link mask of the boundary of a rectangular a x b region of
 * plaquettes in the (mu,nu) plane whose lower-left corner is site `site`
 * (a Wegner-Wilson loop, Sec. 2.1).  0 <= mu < nu < d, 1 <= a < L[mu],
 * 1 <= b < L[nu].  With a = L[mu] the region wraps and the result is the
 * product of two non-contractible loops.  Host-only; no GPU work.
 */
lgt_status lgt_wilson_mask(const lgt_ctx *ctx, int site, int mu, int nu, int a, int b,
                           uint64_t *mask);

/*
 * lgt_contour_mask: the Wegner-Wilson contours c1, c2, c3 of Sec. 3.1, whose perimeters are
 * in the ratios 1 : 1.5 : 2 and enclosed areas 1 : 2 : 3 (perimeter 4, 6, 8 links), as the
 * boundary of a chain of k = 1, 2, 3 plaquettes starting at site 0.  2D: the plaquette,
 * the 1 x 2 block along x, the L of three plaquettes.  3D (the paper's figure of the 3D
 * contours is missing; a planar 1 x 2 block wraps around an extent of 2): the xy plaquette,
 * plus the xz plaquette sharing its x link, plus the xy plaquette one step up in z.
 * Host only.  LGT_E_UNSUPPORTED where the chain wraps around the torus (e.g. c2 on 2 x L).
 */
lgt_status lgt_contour_mask(const lgt_ctx *ctx, int k, uint64_t *mask);

/* lgt_line_mask: non-contractible loop C_mu through `site` (Sec. 2.1). */
lgt_status lgt_line_mask(const lgt_ctx *ctx, int site, int mu, uint64_t *mask);
/*
 * lgt_thooft_mask: links of the 't Hooft operator V_mu = prod sigma^x (Sec. 2.1, the
 * definition after Fig. fig_torus_lattice): the mu-links of the sites on the plane
 * x_mu = 0, i.e. every link piercing the closed dual surface between x_mu = 0 and 1.
 * With this labelling the Wilson line of lgt_line_mask(.., mu) shares exactly one link with
 * V_mu and anticommutes with it, and commutes with V_nu for nu != mu.  Host only.
 */
lgt_status lgt_thooft_mask(const lgt_ctx *ctx, int mu, uint64_t *mask);

/* lgt_reset: overwrite the state (Sec. 2.3).  basis_index < 2^(number of qubits) for
 * LGT_INIT_BASIS (N_l, or N_l + 1 with an ancilla); LGT_INIT_ZGROUND_CIRCUIT needs an
 * ancilla context (LGT_E_UNSUPPORTED otherwise). */
lgt_status lgt_reset(lgt_ctx *ctx, lgt_init init, uint64_t basis_index);

/* ---------------------------------------------------------------------------
 * Evolution (Sec. 2.2)
 * ------------------------------------------------------------------------- */

typedef enum {
    LGT_RAMP_PLAQ = 0,      /* cx_j = h_x, cz_j = f_j h_p                           */
    LGT_RAMP_COUPLING = 1,  /* cx_j = g0 + (g1-g0) f_j, cz_j = 1 (paper: H = Z + gX) */
    LGT_RAMP_EXPLICIT = 2   /* cx_j = cx[j], cz_j = cz[j]                             */
} lgt_ramp;

/*
 * Schedule of n_steps substeps of length dt = T / n_steps.  Step j
 * (0-based) has f_j = (j+1)/n_steps when s_rule = 0: the coupling of a
 * substep is its value at the substep's right end, as in
 * g_{k,m} = (k-1) g_s + m delta (Sec. 2.2).  s_rule = 1 takes the midpoint
 * (j+1/2)/n_steps.  For LGT_RAMP_EXPLICIT, cx and cz are host arrays of
 * n_steps doubles, copied during lgt_evolve.
 */
typedef struct {
    double T;
    int64_t n_steps;
    double h_x, h_p;
    int ramp;
    double g0, g1;
    int s_rule;
    const double *cx, *cz;
} lgt_schedule;

/*
 * lgt_evolve: apply steps first_step .. first_step+count-1 of the schedule.
 *   LGT_ORDER_TROTTER:   psi <- e^{-i dt Hz_j} e^{-i dt Hx_j} psi       (eq. (a))
 *   LGT_ORDER_SYMMETRIC: psi <- e^{-i dt Hz_j/2} e^{-i dt Hx_j} e^{-i dt Hz_j/2} psi (eq. (s))
 * with Hx_j = -cx_j sum sigma^x and Hz_j = -cz_j sum U_p.  In symmetric order
 * the half plaquette steps of neighbouring substeps inside one call are
 * merged into one phase (they commute, as in the rewritten product of
 * Sec. 2.2); a call starts and ends with a half step, so splitting a run into
 * several calls gives the same state up to rounding.  The schedule's
 * coefficient tables are computed on the host in FP64.  A complex64 context
 * rounds them to FP32 so that the phases undo the link layers' norm gains
 * over the call to about one FP32 ulp; the norm then moves only by the
 * rounding of the state arithmetic (about 1e-5 over the 2000 steps of dt 0.05
 * on 24 links).  Where the first rotations of a run are smaller than an FP32
 * ulp of the amplitudes (steps of ~1e-5 from coupling 0) the norm moves by
 * ~1e-3 over 10^5 steps, which expectation values divide out (the norm
 * itself then needs a complex128 context).
 * Errors: LGT_E_INVALID for a bad schedule or a step range outside
 * [0, n_steps); LGT_E_UNSUPPORTED for an unknown form.
 */
lgt_status lgt_evolve(lgt_ctx *ctx, const lgt_schedule *sched, lgt_order order,
                      lgt_form form, int64_t first_step, int64_t count);

/* ---------------------------------------------------------------------------
 * Pseudo-measurement (Sec. 2.4): sums over all basis states, FP64 on the GPU
 * ------------------------------------------------------------------------- */

typedef enum {
    LGT_OBS_NORM = 0,    /* out[0] = <psi|psi>                                         */
    LGT_OBS_Z = 1,       /* out[k] = <prod_{l in masks[k]} sigma^z_l>  (Wilson loops)   */
    LGT_OBS_X = 2,       /* out[k] = Re<prod_{l in masks[k]} sigma^x_l> (G_i, 't Hooft) */
    LGT_OBS_PLAQ = 3,    /* out[p] = <U_p>, p < n_plaq                                  */
    LGT_OBS_STAR = 4,    /* out[i] = <G_i>, i < n_sites                                 */
    LGT_OBS_SIGMAX = 5,  /* out[l] = <sigma^x_l>, l < n_links                           */
    LGT_OBS_SIGMAZ = 6,  /* out[l] = <sigma^z_l>                                        */
    LGT_OBS_ENERGY = 7,  /* out[0] = -cx sum_l <sigma^x_l> - cz sum_p <U_p>             */
    LGT_OBS_ZDOS = 8,    /* out[m] = weight of basis states with m odd plaquettes,
                            i.e. Z = -sum U_p = 2m - n_plaq (Sec. 3.3), m <= n_plaq     */
    LGT_OBS_XDOS = 9     /* out[k] = weight of sigma^x eigenstates with k links at
                            sigma^x = -1, i.e. X = -sum sigma^x = 2k - n_links (Sec. 3.3),
                            k <= n_links: the Walsh-Hadamard transform of a device copy
                            of the state (the state itself is left unchanged), then a
                            popcount histogram; needs one extra state-sized buffer      */
} lgt_obs_kind;

typedef struct {
    int kind;
    int n_masks;              /* LGT_OBS_Z / LGT_OBS_X only                */
    const uint64_t *masks;    /* host array of n_masks link masks          */
    double cx, cz;            /* LGT_OBS_ENERGY only                       */
} lgt_observable;

/*
 * lgt_measure: expectation values normalised by <psi|psi> (except
 * LGT_OBS_NORM), accumulated in FP64 on the GPU, written to the host array
 * out of out_len doubles.  out_len smaller than the result gives
 * LGT_E_INVALID and writes nothing.  Masks of LGT_OBS_Z / LGT_OBS_X may name
 * any qubit of the context (bit N_l is the ancilla of an ancilla context);
 * other bits give LGT_E_INVALID.  On an ancilla context the lattice
 * observables sum over both ancilla values.
 */
lgt_status lgt_measure(lgt_ctx *ctx, const lgt_observable *obs, double *out, size_t out_len);

/*
 * lgt_apply_pauli: psi <- X^xmask Z^zmask psi, a product of sigma^z over the zmask links
 * followed by sigma^x over the xmask links (Sec. 3.5: Wegner-Wilson operators W_mu on
 * non-contractible loops move the initial state between topological sectors; 't Hooft
 * operators V_mu are the sigma^x strings).  In place on the device, stream-ordered.
 * E_INVALID for masks with bits at or beyond the context's qubit count (N_l, or N_l + 1
 * with an ancilla).
 */
lgt_status lgt_apply_pauli(lgt_ctx *ctx, uint64_t xmask, uint64_t zmask);

/*
 * lgt_apply_gate: one gate of the circuits of Sec. 2.2 - 2.4 on qubit q0 (and q1), any
 * qubit of the context including the ancilla: H (Hadamard), X, RX / RZ
 * (exp(-i sigma angle / 2)), CNOT (control q0, target q1), CZ.  One full-state pass,
 * stream-ordered.  E_INVALID for qubits out of range or q0 == q1 in a two-qubit gate.
 */
typedef enum {
    LGT_GATE_H = 0,
    LGT_GATE_X = 1,
    LGT_GATE_RX = 2,
    LGT_GATE_RZ = 3,
    LGT_GATE_CNOT = 4,
    LGT_GATE_CZ = 5
} lgt_gate;
lgt_status lgt_apply_gate(lgt_ctx *ctx, lgt_gate gate, int q0, int q1, double angle);

/*
 * lgt_scan: the stepwise adiabatic evolution of Sec. 2.2, paused for measurement after every
 * `substeps` substeps (one "step" of the paper is n substeps of length t_s/n; Sec. 3 computes
 * its quantities after each step).  Runs substeps * n_points substeps of `sched` from
 * first_step in the fused form, each block as one lgt_evolve call (the symmetric half phases
 * close at every pause), and writes after block k, in row k of `out` (row-major,
 * n_points rows of 5 + n_masks doubles):
 *   [0], [1]  cx and cz of the block's last substep (cx is the coupling g of the paper form)
 *   [2]       <Z> = sum_p <Z_p> = -sum_p <U_p>            (Sec. 2.1: Z_p = -prod sigma^z)
 *   [3]       <X> = -sum_l <sigma^x_l>, so <H> = cz <Z> + cx <X>   (Sec. 3.2)
 *   [4]       the norm <psi|psi>
 *   [5 + i]   <prod_{l in masks[i]} sigma^z_l>, Wegner-Wilson loops (Sec. 3.1)
 * Expectations are divided by the norm.  Every measurement is an FP64 reduction on the
 * device, queued behind the evolution without host round trips; the call returns when the
 * last row is on the host.  0 <= n_masks <= 32; masks must not have bits at or beyond N_l.
 * E_INVALID for bad counts, masks, a short `out` or a schedule range outside the schedule.
 */
lgt_status lgt_scan(lgt_ctx *ctx, const lgt_schedule *sched, lgt_order order,
                    int64_t first_step, int64_t substeps, int64_t n_points,
                    const uint64_t *masks, int n_masks, double *out, size_t out_len);

/*
 * Host-side analysis of a scan (no device work; ctx not needed).
 * lgt_critical_point: Sec. 3.2 locates g_c at the lowest point of the valley of
 *   d^2<H>/dg^2.  The second derivative is the three-point difference over neighbours
 *   `stride` points apart (stride >= 1 smooths the per-step curve), its minimum is refined
 *   by the parabola through the lowest point and its two neighbours.  g: n increasing
 *   couplings, h: <H> at each; *g_c receives the minimum's position, *d2_min its value.
 *   E_INVALID if n < 2 * stride + 3 or g is not increasing.
 * lgt_crossing: the first coupling where a - b changes sign (Sec. 3.2: <Z> and <X> cross
 *   at the self-dual point of the 3+1D theory), by linear interpolation between the two
 *   bracketing points.  E_INVALID if there is no sign change.
 */
lgt_status lgt_critical_point(const double *g, const double *h, int n, int stride,
                              double *g_c, double *d2_min);
lgt_status lgt_crossing(const double *g, const double *a, const double *b, int n, double *g_x);

/*
 * lgt_sample: n_shots computational-basis samples written to the host array
 * out (bit q of out[i] = link q; bit N_l the ancilla of an ancilla context).  Shot i
 * draws u_i from the counter-based
 * SplitMix64 stream (finaliser of seed + (i+1)*0x9E3779B97F4A7C15, top 53
 * bits / 2^53) and returns the smallest b whose FP64 cumulative probability
 * in ascending b exceeds u_i <psi|psi>.  1 <= n_shots <= 2^26.
 */
lgt_status lgt_sample(lgt_ctx *ctx, uint64_t n_shots, uint64_t seed, uint64_t *out);

/*
 * lgt_sample_noalloc: lgt_sample for callers that cannot allocate device memory (code
 * between graph captures, serving loops and harnesses that forbid hipMalloc): the same
 * shots, bit for bit, with no hipMalloc, hipFree or other allocation.  The block sums and
 * the shots live in a fixed array of 16 MiB per GPU, kept until the process ends: at most
 * 2^20 shots and states of at most 30 qubits, else LGT_E_INVALID.  Every call on one GPU
 * uses that GPU's array, so calls on one GPU that overlap in time (two threads, or two
 * streams) race and must be serialised by the caller.  The call returns when the shots are
 * in out[0..n_shots-1] (host memory).
 */
lgt_status lgt_sample_noalloc(lgt_ctx *ctx, uint64_t n_shots, uint64_t seed, uint64_t *out);

/* State transfer: host buffer of exactly info.state_bytes in the context's dtype. */
lgt_status lgt_get_state(lgt_ctx *ctx, void *host, size_t bytes);
lgt_status lgt_set_state(lgt_ctx *ctx, const void *host, size_t bytes);

/*
 * lgt_copy_state: device-to-device copy of src's amplitudes into dst (same lattice and
 * dtype), enqueued on dst's stream after src's stream has drained.  An on-device
 * checkpoint of a run that is paused between steps (the paper pauses after every step
 * to measure, Sec. 2.2).
 */
lgt_status lgt_copy_state(lgt_ctx *dst, lgt_ctx *src);

/* lgt_sync: wait for the context's stream. */
lgt_status lgt_sync(lgt_ctx *ctx);

/*
 * lgt_set_profiling: on = 0 stops profiling; on = k >= 1 brackets every k-th launch of
 * each kernel family with HIP events on the context's stream (k = 1: every launch).
 * lgt_kernel_stats: per kernel family, the number of timed launches and their summed
 * duration, collected while profiling is on.  names[i] points to a static string.
 * Returns the number of families written (<= cap) in *n.
 */
lgt_status lgt_set_profiling(lgt_ctx *ctx, int on);
lgt_status lgt_kernel_stats(lgt_ctx *ctx, const char **names, int64_t *launches,
                            double *total_ms, int cap, int *n);

/*
 * lgt_tune: autotuner for the link-layer pass plan of this context's lattice and dtype.
 * Times each candidate plan (12-bit or full-size low tiles, high tiles with the longest
 * or the shortest contiguous rows, register passes) over `steps` identity steps on the context's
 * own state (u = 1, v = 0 and unit phases, which leave every amplitude bit-for-bit
 * unchanged) and keeps the fastest for later evolve calls on this context.  Plans apply
 * the same rotations in a different order, so a tuned context may round differently
 * from an untuned one (within the precision of the dtype).  States of <= 12 links have
 * a single on-chip kernel and nothing to tune.  1 <= steps <= 1024.
 * lgt_plan_describe: the plan evolve will use, as text (e.g. "tile_low14 | tile_high(...)").
 *
 * lgt_set_plan: pick the plan by code, e.g. to reuse what lgt_tune chose in another process
 * (lgt_get_plan reads it back).  0 = built-in rule; 1 = 12-bit low tile, then high tiles
 * with the longest rows; 2 = the largest low tile (14 bits complex64, 13 complex128), then
 * as 1; 3 = as 2 with the shortest rows; 4 = 12-bit LDS tile and register passes only;
 * 5 = complex128 only: a 14-bit low tile that keeps one link in registers, then as 1
 * (complex64: as 2).  With complex128 the longest-row high tile of 11 links (plans 1, 2 at
 * 24 links) also keeps one link in registers, over rows of 8 amplitudes; plan 3 takes rows
 * of 4 amplitudes there instead.
 * Adding LGT_PLAN_NO_MERGE keeps one launch per pass and step.  Without it, tile plans
 * walk their passes forwards and backwards on alternate steps, so that the pass ending one
 * step also starts the next and applies both rotations around the phase in one launch
 * (the X layer is a product of commuting single-link rotations, the product of R_x gates
 * after eq. (ara), Sec. 2.2): P passes per step become P - 1 plus
 * one per call.  Every plan gives the same result up to rounding.  E_INVALID for unknown
 * codes.
 */
#define LGT_PLAN_NO_MERGE 8
lgt_status lgt_tune(lgt_ctx *ctx, int steps);
lgt_status lgt_plan_describe(const lgt_ctx *ctx, char *out, size_t len);
/* lgt_plan_query: the plan lgt_plan_describe would show for a context of n_links links
 * (1..34), dtype LGT_C64 / LGT_C128 and plan code `plan` (as lgt_set_plan), computed on the
 * host without a context or a GPU: "tile_low<h>" covers links 0..h-1, "tile_high(q<q>,h<h>,
 * rows<r>)" and "reg_high(q<q>,h<h>)" links q..q+h-1, every link exactly once per step.
 * E_INVALID for arguments out of range or a buffer shorter than the text. */
lgt_status lgt_plan_query(int n_links, lgt_dtype dtype, int plan, char *out, size_t len);
lgt_status lgt_set_plan(lgt_ctx *ctx, int plan);
lgt_status lgt_get_plan(const lgt_ctx *ctx, int *plan);

/* Message for the last failure on ctx (ctx may be NULL for create/batch calls). */
const char *lgt_last_error(const lgt_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Batching: many instances of one lattice advanced by shared launches
 * ------------------------------------------------------------------------- */

/*
 * lgt_batch_evolve: advance n contexts that share d, L and dtype by the same
 * step range of their own schedules (each may have its own couplings, e.g. a
 * lambda scan).  Equivalent to calling lgt_evolve on each context (bit for bit),
 * but every pass is one launch over all instances, and small lattices (N <= 12) run
 * every step of the range in a single launch with the state held on chip.
 * Work is enqueued on ctxs[0]'s stream; the other contexts' streams are
 * synchronised first.  States that each fit in 160 MiB but together do not (e.g.
 * 24-link complex64 states, 128 MiB each) run in groups of at most 160 MiB, one group
 * after the other on its first context's stream, the call waiting for each group, so
 * that a group's state stays in the 256 MB Infinity Cache between passes; a group size
 * chosen by lgt_batch_tune (or lgt_batch_set_group) on ctxs[0] replaces that rule.  Errors
 * as lgt_evolve; LGT_E_INVALID if the contexts do not share lattice and dtype.
 */
lgt_status lgt_batch_evolve(int n, lgt_ctx *const *ctxs, const lgt_schedule *scheds,
                            const lgt_order *orders, int64_t first_step, int64_t count);

/*
 * lgt_batch_tune: autotuner for the number of instances per launch of lgt_batch_evolve over
 * these n contexts (same lattice and dtype).  Times `steps` identity steps (u = 1, v = 0 and
 * unit phases, which leave every state bit for bit unchanged) with the instances in launch
 * groups of each candidate size (all n in one launch, the Infinity-Cache-sized group, n/2,
 * n/4, ..., 1), the groups one after the other on ctxs[0]'s stream, and keeps the fastest
 * size in ctxs[0]; later lgt_batch_evolve calls whose first context is ctxs[0] run their
 * instances in groups of that size.  *group receives the choice.  Every grouping gives the
 * same results bit for bit.  States of <= 12 links run every instance in one on-chip
 * launch and keep one group.  1 <= steps <= 1024.
 * lgt_batch_set_group: set that size directly (0 = the built-in rule: groups whose states
 * fit the Infinity Cache together, else one group), e.g. to reuse a tuned size.
 */
lgt_status lgt_batch_tune(int n, lgt_ctx *const *ctxs, int steps, int *group);
lgt_status lgt_batch_set_group(lgt_ctx *ctx, int group);

/*
 * lgt_set_graphs: on != 0 makes lgt_batch_evolve calls whose first context is ctx capture
 * their launch sequence into a HIP graph once per structure (instances, step count, plan,
 * rotation forms, table layout) and replay it on later calls with the same structure;
 * the tables are uploaded before each replay, outside the graph, and the graph holds
 * kernel launches only.  Results are bit for bit those of direct launches.  While
 * profiling is on, and on a context that runs on the null stream, batches launch
 * directly.  At most 64 graphs are kept per context; the cache is dropped whole when full.
 * Measured on MI355X the replay takes as long
 * as direct launches (the gap between dependent kernels is on the device), so it is off
 * by default; it serves callers that want one host call per batch.  on = 0 also frees the
 * cached graphs.
 */
lgt_status lgt_set_graphs(lgt_ctx *ctx, int on);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of adiabatic runs of mixed lattice sizes
 * ------------------------------------------------------------------------- */

typedef struct lgt_server lgt_server;

typedef struct {
    int d, L[3];
    lgt_dtype dtype;
    lgt_schedule sched;     /* cx/cz pointers, if used, are copied at submit */
    lgt_order order;
} lgt_request;

typedef struct {
    int done;               /* 1 when finished                                 */
    lgt_status status;      /* LGT_OK or the failure                           */
    double energy;          /* <H> at the last step                            */
    double plaq_mean;       /* (1/N_p) sum_p <U_p>                             */
    double gauss_violation; /* max_i |1 - <G_i>|                               */
    double norm;            /* <psi|psi>                                       */
    double latency_ms;      /* submit -> result ready                          */
    double queue_ms;        /* submit -> admission                             */
} lgt_result;

/*
 * lgt_server_create: a server that keeps admitted runs resident on the
 * current device, admitting them while their state plus scratch fits in
 * hbm_budget bytes and a slot (max_slots) is free.  A worker thread advances
 * every admitted run per round, one batched launch sequence per lattice shape
 * (in groups whose states fit the Infinity Cache together), so runs that arrive
 * while others are in flight join at the next round (continuous batching).  A
 * run advances chunk_steps steps per round if its state is 128 MiB or more, and
 * up to 4x as many for smaller states, whose steps cost about a launch each; the
 * count depends on the run's shape only.  Runs finish independently.
 */
lgt_status lgt_server_create(size_t hbm_budget, int max_slots, int chunk_steps,
                             lgt_server **out);

/* lgt_server_submit: queue a run.  The request (and its explicit coefficient arrays) is
 * copied and its tables are built on the calling thread.  LGT_E_INVALID for a bad request,
 * including n_steps < 1 or > 2^24 (checked before anything is read from cx / cz);
 * LGT_E_OOM if the run can never fit the budget or a host allocation fails. */
lgt_status lgt_server_submit(lgt_server *srv, const lgt_request *req, uint64_t *ticket);

/* lgt_server_poll: non-blocking; out->done = 0 while the run is queued or running.
 * A finished result is delivered once: the poll or wait that returns it with done = 1 also
 * releases the ticket, and later calls with that ticket give LGT_E_INVALID. */
lgt_status lgt_server_poll(lgt_server *srv, uint64_t ticket, lgt_result *out);

/* lgt_server_wait: block until the run is done (timeout_ms < 0: no limit); LGT_E_BUSY (and
 * out->done = 0) if the time runs out first.  Delivers and releases like lgt_server_poll. */
lgt_status lgt_server_wait(lgt_server *srv, uint64_t ticket, double timeout_ms,
                           lgt_result *out);

/* lgt_server_cancel: a queued run is dropped at once; an admitted run stops at the next
 * round boundary and gives back its slot and memory.  Its result then comes with
 * done = 1 and status LGT_E_STATE.  A run that completes in the round under way keeps its
 * result.  LGT_E_INVALID for an unknown or already delivered ticket, LGT_E_STATE if the
 * run has already finished (its result is waiting to be delivered). */
lgt_status lgt_server_cancel(lgt_server *srv, uint64_t ticket);

typedef struct {
    size_t budget_bytes, used_bytes;   /* admission budget and the footprint admitted now */
    int pending, active;               /* queued runs, admitted runs                        */
    uint64_t completed, failed, cancelled;  /* finished runs by outcome                    */
    uint64_t undelivered;              /* finished results not yet returned by poll / wait */
} lgt_server_stats_t;

/* lgt_server_stats: a snapshot of the server's queue, memory and outcome counters. */
lgt_status lgt_server_stats(lgt_server *srv, lgt_server_stats_t *out);

/* lgt_server_inject_fault: testing hook for the failure path of a round.  The launch group
 * that holds the (queued or admitted) run next reports a failed launch without launching
 * anything: every run of that group ends with LGT_E_DEVICE and gives back its slot and
 * memory, while the other groups of the round go on.  LGT_E_INVALID if the ticket is not
 * queued or running. */
lgt_status lgt_server_inject_fault(lgt_server *srv, uint64_t ticket);

/* lgt_server_destroy: finish the admitted runs, cancel the queued ones, stop the worker
 * and free the server's memory.  Undelivered results are dropped with it. */
lgt_status lgt_server_destroy(lgt_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* LGT_H */
