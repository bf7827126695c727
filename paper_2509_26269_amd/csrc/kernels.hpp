// kernels.hpp -- internal launch interface between the host API and the HIP
// kernels of the bilayer minimum-mode kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace moto {

// Slots of the per-block partial sums of the energy-type reductions.
constexpr int NPART = 11;

// Stencil coefficients in FP64 (cast to the kernel precision at launch).
// Shell table of a Hamiltonian with more than three exchange shells: the
// lattice offsets of every shell (sorted by distance, shell s = offsets
// [start[s], start[s+1])), the largest |dx|, |dy| (the tile halo) and the
// stencil coefficients cJ[s] = -2 J_s.  Passed by value as a kernel argument.
constexpr int GEN_MAX_SHELLS = MOTO_MAX_SHELLS;
constexpr int GEN_MAX_OFF = 448;
constexpr int GEN_RMAX = 12;
struct GenShells {
    int ns, n_off, R;
    int start[GEN_MAX_SHELLS + 1];
    signed char dx[GEN_MAX_OFF], dy[GEN_MAX_OFF];
    double cJ[GEN_MAX_SHELLS];
};

// The same offsets as a compile-time table (the shell geometry is fixed;
// only the couplings vary), so that the general-shell kernels address LDS
// with immediate offsets.  Shell s: squared length = the s-th smallest
// value of dx^2 + dx dy + dy^2 > 0 over |dx|, |dy| <= GEN_RMAX.
struct ShellGeom {
    int n_off;
    int start[GEN_MAX_SHELLS + 1];
    signed char dx[GEN_MAX_OFF], dy[GEN_MAX_OFF];
};

constexpr ShellGeom make_shell_geom() {
    ShellGeom t{};
    int len[GEN_MAX_SHELLS] = {};
    int last = 0;
    for (int s = 0; s < GEN_MAX_SHELLS; ++s) {
        int best = 1 << 30;
        for (int dy = -GEN_RMAX; dy <= GEN_RMAX; ++dy)
            for (int dx = -GEN_RMAX; dx <= GEN_RMAX; ++dx) {
                const int d2 = dx * dx + dx * dy + dy * dy;
                if (d2 > last && d2 < best) best = d2;
            }
        len[s] = best;
        last = best;
    }
    int n = 0;
    for (int s = 0; s < GEN_MAX_SHELLS; ++s) {
        t.start[s] = n;
        for (int dy = -GEN_RMAX; dy <= GEN_RMAX; ++dy)
            for (int dx = -GEN_RMAX; dx <= GEN_RMAX; ++dx)
                if (dx * dx + dx * dy + dy * dy == len[s] && n < GEN_MAX_OFF) {
                    t.dx[n] = (signed char)dx;
                    t.dy[n] = (signed char)dy;
                    ++n;
                }
    }
    t.start[GEN_MAX_SHELLS] = n;
    t.n_off = n;
    return t;
}
constexpr ShellGeom kShellGeom = make_shell_geom();
static_assert(kShellGeom.n_off < GEN_MAX_OFF, "shell table capacity");
static_assert(kShellGeom.start[35] == 360, "the 35 shells of the Pd/Fe/Ir(111) table hold 360 bonds");

struct CoefD {
    double cJ[3];
    double cD;
    double cK;
    double B[3];
    const GenShells* gen = nullptr;  // set for more than three shells
};

template <class T>
inline Coef<T> coef_cast(const CoefD& d) {
    Coef<T> k;
    for (int s = 0; s < 3; ++s) k.cJ[s] = (T)d.cJ[s];
    k.cD = (T)d.cD;
    k.cK = (T)d.cK;
    for (int a = 0; a < 3; ++a) k.B[a] = (T)d.B[a];
    return k;
}

// ---- stencil.hip ----
hipError_t launch_energy_grad(const Geo& g, const CoefD& k, bool f64, int batch, const void* m,
                              const uint8_t* mask, void* grad, void* c, void* F, double* part,
                              hipStream_t st);
hipError_t launch_param_mixed(const Geo& g, bool f64, int batch, const void* m, const void* U, double* part,
                              hipStream_t st);
hipError_t launch_param_grad_apply(const Geo& g, int ns, bool f64, int batch, const void* m, const double* w,
                                  void* out, hipStream_t st);
hipError_t launch_reduce_partials(const double* part, int batch, int tiles, int ns, double* E, double* dth,
                                  hipStream_t st);
// Device address of this GPU's copy of the energy scratch array (looked up once
// per device with that device current); ENERGY_SCRATCH_BYTES long.
constexpr size_t ENERGY_SCRATCH_BYTES = MOTO_NOALLOC_SCRATCH_BYTES;
hipError_t energy_scratch(double** out);
// variant: frame-layout kernel variant (-1 = default choice), see hvp.hip;
// vbs: elements from one lattice's vector block to the next (0 = nvec
// vectors back to back)
hipError_t launch_tangent_hvp(const Geo& g, const CoefD& k, bool f64, bool frame, int batch, const void* m,
                              const void* c, const uint8_t* mask, int nvec, const void* V, void* W,
                              const int* done, hipStream_t st, int variant = -1, long long vbs = 0);

// ---- shells.hip: general-shell lattice kernels (more than three shells) ----
hipError_t launch_energy_grad_gen(const Geo& g, const CoefD& k, bool f64, int batch, const void* m,
                                  const uint8_t* mask, void* grad, void* c, void* F, double* part, hipStream_t st);
hipError_t launch_tangent_hvp_gen(const Geo& g, const CoefD& k, bool f64, bool frame, int batch, const void* m,
                                  const void* c, const uint8_t* mask, int nvec, long long vbs, const void* V, void* W,
                                  const int* done, hipStream_t st);

// ---- hvp.hip: frame-layout tangent HVP variants (tile shapes / staging) ----
constexpr int HVP_NVARIANTS = 12;
bool hvp_variant_ok(int variant, const Geo& g, bool f64);
int hvp_default_variant(const Geo& g, bool f64);
const char* hvp_variant_name(int variant);
hipError_t launch_hvp_frame(int variant, const Geo& g, const CoefD& k, bool f64, int batch, const void* m,
                            const void* c, const uint8_t* mask, int nvec, const void* V, void* W, const int* done,
                            hipStream_t st, long long vbs = 0);
hipError_t launch_hessian_apply(const Geo& g, const CoefD& k, bool f64, int batch, int nvec, const void* V,
                                void* W, hipStream_t st);
hipError_t launch_topo_charge(const Geo& g, int batch, const double* m, double* part, hipStream_t st);

// ---- lobpcg.hip ----
// Control block of one eigen-solve, resident in device memory.
constexpr int MAXB = 16;        // max block width (k + guard)
constexpr int MAXS = 3 * MAXB;  // max Rayleigh-Ritz basis size
struct EigCtrl {
    int done;         // 1 once converged / capped / failed: later launches are no-ops
    int status;       // MOTO_CONVERGED, MOTO_NOT_CONVERGED, MOTO_NAN, MOTO_BREAKDOWN
    int iters;        // LOBPCG iterations taken
    int np;           // columns of P in the current basis (0 or mb)
    long long n_hvp;  // HVP columns applied
    int rank;         // basis rank kept by the last Rayleigh-Ritz
    int orth_skip;    // 1: the first orthonormalisation pass of W settled it (the second is a no-op)
    double lam[MAXB];
    double resid[MAXB];
    double C[MAXS * MAXB];       // Ritz coefficients of X, column-major [ns][mb]
    double Cp[MAXS * MAXB];      // orthonormal complement spanning the new P, [ns][mb]
    double Bw[2 * MAXB * MAXB];  // [X P]^T W projection coefficients, [2mb][mb]
    double Tw[MAXB * MAXB];      // orthonormalising transform of the projected block, [mb][mb]
};

struct EigArgs {
    int n2;        // rows of the frame-coordinate vectors (2N)
    int mb;        // block width
    int k;         // wanted pairs
    int max_iter;
    double tol_abs;
    double drop;   // rank threshold of the orthonormalisations (relative)
    // Population of P independent solves on lattices of one geometry: member
    // y = blockIdx.y owns S, HS at + y s_ms elements, partial rows at
    // + y part_ms doubles, Grams at + y g_ms doubles and control block y.
    int P = 1;
    long long s_ms = 0, part_ms = 0, g_ms = 0;
    // masked solve: site activity (member y at mask + y mask_ms) of the
    // Nsite sites; row r of a block column belongs to site r mod Nsite
    const uint8_t* mask = nullptr;
    int Nsite = 0;
    long long mask_ms = 0;
};

// ---- lanczos.hip ----
constexpr int LZ_MAXM = 64;                 // max Krylov depth
constexpr int LZ_MAXBLK = 4;                // max start-block size of the band Lanczos
constexpr int LZ_NCOL = LZ_MAXM + LZ_MAXBLK;  // basis columns (depth + residual block)
constexpr int LZ_LDT = LZ_NCOL;             // leading dimension of the projected matrix
// Control block of one thick-restart band-Lanczos solve, resident in device memory.
struct LzCtrl {
    int done;        // 1 once stopped: later step launches are no-ops
    int status;      // MOTO_CONVERGED, MOTO_NOT_CONVERGED, MOTO_NAN, MOTO_BREAKDOWN
    int restarts;    // thick restarts taken
    int m_eff;       // Krylov depth of the current cycle (smaller after a breakdown)
    int m_max;       // Krylov depth asked for
    int nkeep;       // Ritz vectors formed by the last restart
    int blk;         // start-block size b
    int brk;         // 1: the cycle ended on a breakdown (dependent new column)
    long long n_hvp; // HVP columns applied
    double beta;     // |w| of the last orthogonalisation
    double w0sq;     // |w|^2 of a start/residual column before its projection
    double h[LZ_NCOL];               // reorthogonalisation coefficients of the current pass
    double T[LZ_LDT * LZ_LDT];       // projected matrix Q^T H Q and the residual rows below it
    double Y[LZ_MAXM * LZ_MAXM];     // Ritz vectors of T, vector i at [i * LZ_MAXM]
    double theta[LZ_MAXM], resid[LZ_MAXM];
    EigCtrl out;     // eigenvalues, residuals and counters in the eigen-solve layout
};
// NaN or infinite spins or Weingarten scalars: the solve ends at once with
// MOTO_NAN (P members of the LOBPCG population, or one Lanczos solve).
hipError_t launch_check_finite(const double* m, const double* c, int N, int P, EigCtrl* ctrl, hipStream_t st);
hipError_t launch_check_finite(const double* m, const double* c, int N, LzCtrl* ctrl, hipStream_t st);
int lz_blocks(int n2);
// Start block: column 0 = sum of the nwarm warm vectors (or SplitMix64 entries),
// columns 1..b-1 SplitMix64 entries; masked sites zero.  Resets the control block.
hipError_t launch_lz_init(bool f64, int N, int b, void* Q, const double* m, const double* Vwarm, int nwarm,
                          const uint8_t* mask, uint64_t seed, LzCtrl* ctrl, int m_max, hipStream_t st);
// Orthogonalise column c against columns 0..c-1 twice and normalise it.  tj >= 0:
// column c is the image of column tj (c = tj + b): the coefficients of both
// passes fill column tj of T and |w| goes to T[c][tj]; a negligible |w| ends the
// cycle (m_eff = tj + 1).  tj < 0: no T entries (start and residual blocks).
hipError_t launch_lz_orth(bool f64, int n2, void* Q, int c, int tj, double* part, int nblk, LzCtrl* ctrl,
                          hipStream_t st);
hipError_t launch_lz_rr_restart(bool f64, int n2, int b, void* Q, int k, int keep, double tol_abs, int max_restarts,
                                int m_max, int nblk, const uint8_t* mask, int N, uint64_t seed, LzCtrl* ctrl,
                                hipStream_t st);

// ---- explorer.hip ----
int l1_chunks(long long n3);
hipError_t launch_candidates(int N, int P, const double* x0, const uint8_t* mask, const double* delta, double* X,
                             uint8_t* mask_rep, hipStream_t st);
// part: l1_chunks(3N) * P * (P + A) doubles; D: P * (P + A)
hipError_t launch_l1(long long n3, int P, int A, const double* X, const double* Arch, double* part, double* D,
                     hipStream_t st);
hipError_t launch_explorer_finish(int P, int A, int k, const double* D, const double* E, const double* evals,
                                  const double* Qc, const double* Qx0, double Q_target, const EigCtrl* ctrl,
                                  moto_explorer_result* res, hipStream_t st);

hipError_t launch_eig_init(bool f64, const EigArgs& a, void* S, const double* m, const double* Vwarm, int nwarm,
                           const void* Xsave, int use_save, const uint8_t* mask, int N, uint64_t seed,
                           EigCtrl* ctrl, hipStream_t st);
// Orthonormalise the X block (target 0, start) or the W block against [X P]
// and itself (target 1: first pass, target 2: second pass, a no-op when the
// first was well conditioned), in place.
hipError_t launch_orth(bool f64, const EigArgs& a, int target, void* S, double* part, int nblk, double* G,
                       EigCtrl* ctrl, hipStream_t st);
hipError_t launch_gram(bool f64, const EigArgs& a, int ns, const void* S, const void* HS, double* part, int nblk,
                       double* G, const EigCtrl* ctrl, hipStream_t st);
int gram_blocks(int n2);
hipError_t launch_rr(const EigArgs& a, int ns, const double* G, EigCtrl* ctrl, hipStream_t st);
hipError_t launch_update(bool f64, const EigArgs& a, int ns, void* S, void* HS, double* part, int nblk,
                         EigCtrl* ctrl, hipStream_t st);
int update_blocks(int n2, bool f64, int mb);  // row-update workgroups (same rule as the launchers)
bool rows_on_matrix_cores(bool f64, int mb);  // FP32 block widths from 5
hipError_t launch_eig_control(const EigArgs& a, const double* part, int nblk, EigCtrl* ctrl, int first,
                              hipStream_t st);
hipError_t launch_eig_gather_info(int P, const EigCtrl* ctrl, moto_info* out, hipStream_t st);
// all_done = 1 once every member's control block says done (P > 1 only).
hipError_t launch_eig_all_done(const EigArgs& a, const EigCtrl* ctrl, int* all_done, hipStream_t st);
hipError_t launch_eig_output(bool f64, const EigArgs& a, const void* S, const double* m, int N, double* V,
                             double* part, const EigCtrl* ctrl, double* evals, double* resid, void* Xsave,
                             hipStream_t st);

// ---- step.hip ----
struct StepArgs {
    int N;
    int mem;
    int rule;  // 0 lbfgs, 1 fixed
    int k_reflect;
    double theta_max;
    double alpha0;
    double sy_min;
    double tau_F;
};
size_t step_state_bytes(int N, int mem);
hipError_t launch_step(const StepArgs& a, double* m, const double* F, const double* V, void* state, double* out,
                       hipStream_t st);
hipError_t launch_step_population(const StepArgs& a, int P, int k, double* m, const double* F, const double* V,
                                  void* state, size_t state_bytes, double* out, hipStream_t st);
hipError_t launch_step_stop(void* state, int N, int mem, size_t state_bytes, int y, hipStream_t st);
hipError_t launch_seed_rotate(int N, double* m, const double* v1, double scale_sign_eta, double* part,
                              hipStream_t st);
hipError_t launch_f64_to_f32(const double* src, float* dst, size_t n, hipStream_t st);
hipError_t launch_mask_zero(double* v, const uint8_t* mask, int N, int ncomp, hipStream_t st);
// zero `bytes` (a multiple of 16) at a 16-byte aligned device address (a
// kernel, not a memset node: the drivers stay graph-capturable)
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
// moto_descend_result from device values (MOTO_ASYNC descent)
hipError_t launch_descend_result(void* state, int N, int mem, const double* out, const double* Eo, const double* Q,
                                 moto_descend_result* res, hipStream_t st);

// ---- batched.hip ----
struct BatchArgs {
    CoefD k;
    double hest, tau_F, tau_lam, theta_max, alpha0, sy_min, eig_tol_abs, drop;
    int kk, k_cert, mem, max_outer, eig_max_iter, n;
    unsigned long long seed;
};
size_t batch_search_bytes(int N, int mem);
// tile shapes of the batched searches' lattice loops
constexpr int BATCH_TILE_32x8 = MOTO_TILE_32x8, BATCH_TILE_16x16 = MOTO_TILE_16x16, BATCH_TILE_64x4 = MOTO_TILE_64x4;
hipError_t launch_batched_search(const BatchArgs& a, double* m_all, const uint8_t* mask_all, const int* Ls,
                                 const int* tiles, const int* order, const long long* m_off,
                                 const long long* ws_off, char* ws, moto_search_result* res, int grid,
                                 hipStream_t st);

}  // namespace moto
