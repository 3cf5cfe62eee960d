// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lgt.h"

namespace lgt {

constexpr int kMaxLinks = 34;     // 2^34 complex64 = 128 GiB: fits one 288 GB GPU
constexpr int kMaxPlaq = 32;      // syndrome of all plaquettes fits a 32-bit word
constexpr int kParityBytes = 5;   // byte tables cover 40 index bits

// Periodic lattice (Sec. 2.1).  Sites numbered x-fastest; link l(s,mu) = d s + d-1-mu.
struct Lattice {
    int d = 0;
    int L[3] = {1, 1, 1};
    int n_sites = 0, n_links = 0, n_plaq = 0;
    std::vector<int32_t> plaq_links;    // n_plaq * 4
    std::vector<uint64_t> plaq_mask;    // n_plaq
    std::vector<uint64_t> star_mask;    // n_sites
    std::vector<uint32_t> link_plaqs;   // n_links: plaquettes touching each link
    std::vector<int> fwd, bwd;          // neighbour tables [s * d + mu]

    int link(int s, int mu) const { return d * s + (d - 1 - mu); }
};

// returns an empty string on success, else the reason
std::string build_lattice(int d, const int *L, Lattice &out);
uint64_t region_mask(const Lattice &lat, int site, int mu, int nu, int a, int b);
uint64_t line_mask(const Lattice &lat, int site, int mu);
uint64_t contour_mask(const Lattice &lat, int k);   // c1..c3 of Sec. 3.1, 0 if degenerate
uint64_t thooft_mask(const Lattice &lat, int mu);

// Plaquette syndrome tables: P(b) = XOR_k tab[k][(b >> 8k) & 255], bit p of P(b)
// is the parity of plaquette p on basis state b.  P is linear over GF(2).
void build_parity_tables(const Lattice &lat, uint32_t tab[kParityBytes][256]);

// ---------------------------------------------------------------------------
// Per-step device tables (Sec. 2.2 schedule, computed in FP64 on the host)
// ---------------------------------------------------------------------------
// The link layer prod_l exp(i a sigma^x_l) factors as scale * prod_l (u + i v sigma^x_l)
// with (u, v) = (1, tan a) when |tan a| <= 1 and (cot a, 1) otherwise; each pair
// update is then two FMAs per real component.  The scale (cos a)^N or (sin a)^N
// is folded into the plaquette phase table applied right after the layer.
template <typename T>
struct RotParam {
    T u, v;
};

template <typename T>
struct Cplx {
    T re, im;
};

struct StepTables {
    int n_steps = 0;          // link layers in the call
    int n_phase = 0;          // phase applications (n_steps, or n_steps+1 if symmetric)
    int pre_phase = 0;        // 1: phase[0] is applied before the first link layer
    std::vector<double> rot_u, rot_v;          // [n_steps]
    std::vector<double> ph_re, ph_im;          // [n_phase * (n_plaq+1)]
};

// cx/cz: per-step coefficients of the steps in the call, dt the substep length.
void build_step_tables(int n_links, int n_plaq, double dt, const double *cx, const double *cz,
                       int n_steps, int order, StepTables &out);

// Round to complex64 tables: the float (u, v) to nearest; the phase rows undo the link
// layers' norm gains, each gain at its own row once the gains not yet undone reach 2^-12
// (else at a later row, at the latest the call's last), and each entry is chosen among
// nearby floats so that its magnitudes multiply to their targets within about one FP32
// ulp over the whole run (the entry's magnitude error is carried from row to row).
void round_tables_f32(const StepTables &in, int n_links, int n_plaq,
                      std::vector<RotParam<float>> &rot, std::vector<Cplx<float>> &ph);
// What the phase rounding carries from row to row: per entry, the magnitude error so far;
// the link layers' gain not yet undone.
struct PhaseRounding {
    std::vector<double> carry;
    long double gain = 1.0L;
};
// The same rounding in pieces: every link layer (with its norm gain), then phase rows
// [k0, k1) into a table sized for all rows, in increasing order, with one PhaseRounding
// (fresh at the first row) passed on from piece to piece.  Rows come out identical to the
// whole-table call.
void round_rot_f32(const StepTables &in, int n_links, std::vector<RotParam<float>> &rot,
                   std::vector<long double> &gain);
void round_phase_f32(const StepTables &in, int n_plaq, const std::vector<long double> &gain,
                     int k0, int k1, std::vector<Cplx<float>> &ph, PhaseRounding &pr);
void round_tables_f64(const StepTables &in, int n_plaq,
                      std::vector<RotParam<double>> &rot, std::vector<Cplx<double>> &ph);

// Expand an lgt_schedule into per-step coefficients for steps [first, first+count).
std::string schedule_coeffs(const lgt_schedule *s, int64_t first, int64_t count, double &dt,
                            std::vector<double> &cx, std::vector<double> &cz);

// ---------------------------------------------------------------------------
// Device-side instance description used by every pass kernel.  Batched
// launches read instance blockIdx.y from an array of these.
// ---------------------------------------------------------------------------
struct DevInst {
    void *psi;                 // amplitudes
    const void *rot;           // RotParam<T>[n_total]
    const void *phase;         // Cplx<T>[n_phase][n_plaq+1]
    const uint32_t *ptab;      // [kParityBytes][256] syndrome byte tables
    int step0;                 // link layer step0 + step of a launch uses rot[step0 + step]
    int ph0;                   // phase index idx of a launch reads phase[ph0 + idx]
    int n_total;               // steps in rot; launches past the end leave the instance alone
    int pad;
};

// kernel launch plan for one link layer of an N-link state
enum PassKind { PASS_LOW12 = 0, PASS_HIGH_REG = 1, PASS_TILE_LOW = 2, PASS_TILE_HIGH = 3 };
struct Pass {
    int kind = 0;
    int q0 = 0;                // first rotated index bit (high passes)
    int h = 0;                 // rotated bits (high passes)
    int cb = 0;                // contiguous row bits (tile high passes)
};
struct PassPlan {
    int n_passes = 0;
    Pass pass[8];
    // consecutive steps run their passes in alternating order, and the pass that ends one
    // step and starts the next applies both rotations around the phase in one launch
    bool merge = false;
};
// plan code flag: keep one launch per pass and step (no merged steps)
constexpr int kPlanNoMerge = 8;
// plan = 0: built-in rule (2 when the big low tile gives >= 64 workgroups, else 1);
// 1: 12-bit low tile + high tiles; 2: big low tile + high tiles with the longest rows;
// 3: big low tile, shortest rows; 4: 12-bit LDS tile + register passes
PassPlan plan_passes(int n_links, int dtype, int plan = 0, int n_inst = 1);
std::string describe_plan(const PassPlan &p, int n_links);

// ---------------------------------------------------------------------------
// Kernel launchers (kernels.hip).  All return hipSuccess or the HIP error.
// ---------------------------------------------------------------------------
enum KernelFamily {
    KF_INIT = 0, KF_LOW, KF_HIGH, KF_PHASE, KF_SMALL, KF_GATE_RX, KF_GATE_RZ, KF_GATE_CNOT,
    KF_RED_DIAG, KF_RED_FLIP, KF_RED_DOS, KF_SAMPLE, KF_TILE_LOW, KF_TILE_HIGH, KF_GATE_H,
    KF_GATE_CZ, KF_PROJECT, KF_COUNT
};
const char *kernel_family_name(int kf);

hipError_t launch_init(int dtype, void *psi, int n, int init, uint64_t basis, double amp,
                       const uint32_t *ptab_dev, hipStream_t st);
// one link layer pass over n_inst instances (pointers in dev_inst, device memory)
hipError_t launch_low(int dtype, const DevInst *dev_inst, int n_inst, int n, int low_bits,
                      int step, int pre_phase_idx, int post_phase_idx, int n_plaq,
                      hipStream_t st);
hipError_t launch_high(int dtype, const DevInst *dev_inst, int n_inst, int n, int q0, int h,
                       int step, int post_phase_idx, int n_plaq, hipStream_t st);
// persistent tile pass; forms: bit 0 = launch for tan-form steps, bit 1 = cot-form steps.
// High passes keep rows of 2^cb amplitudes contiguous (cb = 4 or 5 for complex64,
// 3 or 4 for complex128) and rotate index bits [hb, hb+h).
// merge = 1: rotation of `step`, the phase `post`, then the rotation of step + 1 (pre = -1);
// forms then holds the forms of step + 1 in bits 2-3.
// Kernel-level timing of the tile launchers: while set, the launcher's first kernel
// records `start` as it begins and every kernel records `stop` as it ends (timestamps of
// the dispatch itself, so no extra stream packets sit between the kernels).
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
    bool used = false;
};
extern thread_local LaunchTiming *g_launch_timing;

hipError_t launch_tile(int dtype, const DevInst *dev_inst, int n_inst, int n, int low, int hb,
                       int h, int cb, int step, int pre, int post, int n_plaq, int forms,
                       int merge, hipStream_t st);
// wave bits of the tile pass rotating h bits with rows of 2^cb, -1 if no such pass
int pass_wave_bits(int dtype, int low, int h, int cb);
bool pass_offsets_fit(int dtype, int n, int low, int hb, int h, int cb);
hipError_t launch_phase(int dtype, const DevInst *dev_inst, int n_inst, int n, int phase_idx,
                        int n_plaq, hipStream_t st);
// whole evolution of small states, one workgroup per instance: n <= 8 in one wavefront's
// registers, 9 <= n <= 12 in LDS
hipError_t launch_small(int dtype, const DevInst *dev_inst, int n_inst, int n, int n_steps,
                        int pre_phase, int n_plaq, hipStream_t st);
// enqueue `count` fused substeps for n_inst instances (api.cpp); pre_first: phase index
// applied before the first link layer or -1; the phase after layer j is post_off + j
// forms[j]: kFormTan if some instance's link layer j uses the tan form, kFormCot the cot form
constexpr uint8_t kFormTan = 1, kFormCot = 2;
hipError_t enqueue_fused_steps(int dtype, int n_links, int n_plaq, const DevInst *dev_inst,
                               int n_inst, int count, int pre_first, int post_off,
                               const uint8_t *forms, int plan, hipStream_t st, void *prof_ctx);
// The same launches for steps [j_begin, j_end) of a count-step call, continued across
// calls through `cur` (the pass order and whether the range starts inside a merged launch).
struct FusedCursor {
    bool fwd = true, merged_in = false;
};
hipError_t enqueue_fused_range(int dtype, int n, int n_plaq, const DevInst *dev_inst, int n_inst,
                               int count, int j_begin, int j_end, int pre_first, int post_off,
                               const uint8_t *forms, int plan_sel, hipStream_t st,
                               void *prof_ctx, FusedCursor &cur);
bool small_supported(int dtype, int n);
// circuit-form gates
hipError_t launch_gate_rx(int dtype, void *psi, int n, int q, double phi, hipStream_t st);
hipError_t launch_gate_rz(int dtype, void *psi, int n, int q, double phi, hipStream_t st);
hipError_t launch_gate_cnot(int dtype, void *psi, int n, int c, int t, hipStream_t st);
// reductions: partial sums per block, FP64
int reduce_blocks(int n);
int reduce_diag_blocks(int n);   // partial rows written by launch_reduce_diag
hipError_t launch_reduce_diag(int dtype, const void *psi, int n, const uint64_t *masks_dev,
                              int n_masks, double *partials, hipStream_t st);
hipError_t launch_reduce_flip(int dtype, const void *psi, int n, const uint64_t *masks_dev,
                              int n_masks, double *partials, hipStream_t st);
// out[c] = sum of partials[row][c] over rows (device-side final sum of a reduction)
hipError_t launch_sum_cols(const double *partials, int rows, int width, int ncols, double *out,
                           hipStream_t st);
// histogram of |psi_b|^2 over popcount(b), bins 0..n (n <= kMaxPlaq)
hipError_t launch_reduce_popcount(int dtype, const void *psi, int n, const uint32_t *ptab_dev,
                                  double *partials, hipStream_t st);
hipError_t launch_gate_h(int dtype, void *psi, int n, int q, hipStream_t st);
hipError_t launch_gate_cz(int dtype, void *psi, int n, int a, int b, hipStream_t st);
// amplitudes with a bit of zero_mask set become 0, the others are multiplied by scale
hipError_t launch_project_scale(int dtype, void *psi, int n, uint64_t zero_mask, double scale,
                                hipStream_t st);
// psi <- X^xmask Z^zmask psi (Pauli string: Z on the zmask links, then X on the xmask links)
hipError_t launch_pauli(int dtype, void *psi, int n, uint64_t xmask, uint64_t zmask, hipStream_t st);
hipError_t launch_reduce_dos(int dtype, const void *psi, int n, const uint32_t *ptab_dev,
                             int n_plaq, double *partials, hipStream_t st);
// sampling: block sums -> prefix -> inverse CDF
int sample_block_bits(int n);
// Allocation-free sampling: a static device array per GPU holds the block sums
// (kScratchSums doubles: states of up to 30 qubits at 2^10 amplitudes per block) and the
// shots (kScratchShots words).  scratch_address gives its device address on `device`,
// taken once per device with hipGetSymbolAddress.  launch_sample_scratch runs the same
// kernels as launch_sample with the prefix on the device (same additions, same order) and
// leaves the shots at word kScratchSums of the array.
constexpr int kScratchSums = 1 << 20;
constexpr int kScratchShots = 1 << 20;
constexpr int kMaxDevices = 64;
hipError_t scratch_address(int device, void **out);
hipError_t launch_sample_scratch(int dtype, const void *psi, int n, uint64_t n_shots,
                                 uint64_t seed, void *scratch_dev, hipStream_t st);
hipError_t launch_sample(int dtype, const void *psi, int n, uint64_t n_shots, uint64_t seed,
                         double *block_sums, double *block_prefix, uint64_t *out_dev,
                         hipStream_t st);

}  // namespace lgt
