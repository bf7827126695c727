// lanczos.hip -- the second inner solver: thick-restart band Lanczos with
// full reorthogonalisation on the (masked) tangent Hessian in frame
// coordinates (the paper's HVP-Lanczos operator mode; Krylov depth and
// reorthogonalisation are its named hyperparameters).
//
// The Krylov space grows from a start block of b orthonormal vectors (band
// Lanczos, Ruhe 1979).  Step j:
//   w = H q_j                       (the HVP kernel, one vector)
//   h = Q_{0..j+b-1}^T w, w -= Q h  (classical Gram-Schmidt, twice; the
//                                    coefficients of both passes summed are
//                                    column j of Q^T H Q)
//   beta = |w|, q_{j+b} = w / beta
// so H Q_m = Q_m T_m + Q_{m..m+b-1} T[m..m+b-1][0..m): a Ritz pair (theta, y)
// of T_m has the residual norm |T[m..m+b-1][0..m) y|.  A single start vector
// (b = 1) can keep the second member of a close eigenvalue pair out of the
// space long after the first has met the stopping rule; a block of b
// directions brings such a pair in together.
// Q lives in one [m_max + b][2N] array; w is written straight into its
// column.  At the end of a cycle one workgroup takes the `keep` lowest
// eigenpairs of T (FP64, symeig_low), tests the residuals and
// either stops or restarts from the `keep` lowest Ritz vectors plus the
// residual block (Wu & Simon 2000), which is re-orthonormalised before the
// next cycle; the steps of that cycle fill the couplings of T.  A breakdown
// (a new column with negligible norm) ends the cycle early; the residual rows
// stay exact, and the restart puts a fresh SplitMix64 direction in place of
// the dependent column.  All reductions are FP64 with a fixed order.
#include <type_traits>

#include "dense_wg.hpp"
#include "kernels.hpp"

namespace moto {

constexpr int LZP = LZ_NCOL + 1;  // doubles per block partial row (columns, then |w|^2)

__device__ __forceinline__ int lz_rows_per_block(int n2, int nblk) {
    const int per = (n2 + nblk - 1) / nblk;
    return (per + 63) & ~63;
}

// Start block: column 0 is the sum of the warm vectors (ambient, FP64) in
// frame coordinates, or SplitMix64 entries; columns 1..b-1 SplitMix64 entries
// of their own; masked sites zero.  Resets the control block.
template <class T>
__global__ __launch_bounds__(NT) void k_lz_init(int N, int b, T* __restrict__ Q, const double* __restrict__ m,
                                                const double* __restrict__ Vwarm, int nwarm,
                                                const uint8_t* __restrict__ mask, uint64_t seed,
                                                LzCtrl* __restrict__ ctrl, int m_max) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->done = 0;
        ctrl->status = MOTO_NOT_CONVERGED;
        ctrl->restarts = 0;
        ctrl->m_eff = m_max;
        ctrl->m_max = m_max;
        ctrl->nkeep = 0;
        ctrl->blk = b;
        ctrl->brk = 0;
        ctrl->n_hvp = 0;
        ctrl->out.status = MOTO_NOT_CONVERGED;
        ctrl->out.iters = 0;
        ctrl->out.n_hvp = 0;
    }
    // entries of T below the band are never written by a step: start from zero
    for (int i = blockIdx.x * NT + threadIdx.x; i < LZ_LDT * LZ_LDT; i += gridDim.x * NT) ctrl->T[i] = 0.0;
    const size_t n2 = 2 * (size_t)N;
    for (int s = blockIdx.x * NT + threadIdx.x; s < N; s += gridDim.x * NT) {
        const bool on = mask == nullptr || mask[s] != 0;
        for (int l = 0; l < b; ++l) {
            double a = 0.0, bb = 0.0;
            if (on) {
                if (l == 0 && nwarm > 0) {
                    double e1[3], e2[3];
                    onb(m[s], m[N + s], m[2 * N + s], e1, e2);
                    for (int j = 0; j < nwarm; ++j) {
                        const double* v = Vwarm + (size_t)j * 3 * N;
                        a += e1[0] * v[s] + e1[1] * v[N + s] + e1[2] * v[2 * N + s];
                        bb += e2[0] * v[s] + e2[1] * v[N + s] + e2[2] * v[2 * N + s];
                    }
                } else {
                    a = splitmix_uniform(seed, (uint64_t)l * n2 + s);
                    bb = splitmix_uniform(seed, (uint64_t)l * n2 + N + s);
                }
            }
            Q[(size_t)l * n2 + s] = (T)a;
            Q[(size_t)l * n2 + N + s] = (T)bb;
        }
    }
}

// the kernels of step tj (tj >= 0) do nothing once the cycle has ended
__device__ __forceinline__ bool lz_skip(const LzCtrl* ctrl, int tj) {
    return ctrl->done || (tj >= 0 && tj >= ctrl->m_eff);
}

// Partial dots of w = Q[c] with Q[0..c): blockIdx.x picks the rows, wave w of
// block (x, y) the column q = 4 y + w, so every column's rows are read by its
// own wave in parallel; lane l takes the rows start + l, start + l + 64, ...
// into two alternating partial sums (fixed order).
template <class T>
__global__ __launch_bounds__(NT) void k_lz_dots(int n2, const T* __restrict__ Q, int c, int tj, int self,
                                                double* __restrict__ part, const LzCtrl* __restrict__ ctrl) {
    if (lz_skip(ctrl, tj)) return;
    const int col = blockIdx.y * (NT / 64) + (threadIdx.x >> 6);
    if (col >= c + self) return;  // self = 1: also |w|^2 before the projection (slot c)
    const int per = lz_rows_per_block(n2, gridDim.x);
    const int r0 = blockIdx.x * per, r1 = min(n2, r0 + per);
    const int lane = threadIdx.x & 63;
    const T* __restrict__ w = Q + (size_t)c * n2;
    const T* __restrict__ q = Q + (size_t)col * n2;
    double s0 = 0.0, s1 = 0.0;
    int r = r0 + lane;
    for (; r + 64 < r1; r += 128) {
        s0 += (double)q[r] * (double)w[r];
        s1 += (double)q[r + 64] * (double)w[r + 64];
    }
    if (r < r1) s0 += (double)q[r] * (double)w[r];
    const double s = wave_sum(s0 + s1);
    if (lane == 0) part[(size_t)blockIdx.x * LZP + col] = s;
}

// h_q = sum_b part[b][q] for q < c (one wavefront per column).  With tj >= 0,
// pass 0 sets column tj of T to h and pass 1 adds h to it.
__global__ __launch_bounds__(NT) void k_lz_reduce(const double* __restrict__ part, int nblk, int c, int tj, int pass,
                                                  int self, LzCtrl* __restrict__ ctrl) {
    if (lz_skip(ctrl, tj)) return;
    const int lane = threadIdx.x & 63;
    for (int q = blockIdx.x * (NT / 64) + (threadIdx.x >> 6); q < c + self; q += gridDim.x * (NT / 64)) {
        double s = 0.0;
#pragma unroll 4  // several loads in flight per lane
        for (int b = lane; b < nblk; b += 64) s += part[(size_t)b * LZP + q];
        s = wave_sum(s);
        if (q == c) {  // |w|^2 before the projection
            if (lane == 0) ctrl->w0sq = s;
            continue;
        }
        if (lane == 0) {
            ctrl->h[q] = s;
            if (tj >= 0) {
                const double t = pass == 0 ? s : ctrl->T[q * LZ_LDT + tj] + s;
                ctrl->T[q * LZ_LDT + tj] = t;
                ctrl->T[tj * LZ_LDT + q] = t;
            }
        }
    }
}

// w -= Q[0..c) h; on the last pass also the partial |w|^2.
template <class T>
__global__ __launch_bounds__(NT) void k_lz_update(int n2, T* __restrict__ Q, int c, int tj, int want_norm,
                                                  double* __restrict__ part, const LzCtrl* __restrict__ ctrl) {
    if (lz_skip(ctrl, tj)) return;
    __shared__ double h[LZ_NCOL];
    __shared__ double red[NT / 64];
    for (int q = threadIdx.x; q < c; q += NT) h[q] = ctrl->h[q];
    __syncthreads();
    T* __restrict__ w = Q + (size_t)c * n2;
    double s2 = 0.0;
    for (int r = blockIdx.x * NT + threadIdx.x; r < n2; r += gridDim.x * NT) {
        double v = (double)w[r];
        for (int q = 0; q < c; ++q) v -= h[q] * (double)Q[(size_t)q * n2 + r];
        const T tv = (T)v;
        w[r] = tv;
        s2 += (double)tv * tv;
    }
    if (!want_norm) return;
    s2 = wave_sum(s2);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s2;
    __syncthreads();
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * LZP + LZ_NCOL] = red[0] + red[1] + red[2] + red[3];
}

// beta = |w| from the partials (one workgroup).  tj >= 0: one HVP counted,
// T[c][tj] = beta, and a negligible beta ends the cycle after column tj.
// tj < 0 (start or residual block): a column that the projection reduces to
// rounding noise means no independent direction is left (MOTO_BREAKDOWN).
__global__ __launch_bounds__(NT) void k_lz_beta(const double* __restrict__ part, int nblk, int c, int tj,
                                                double rel_dep, LzCtrl* __restrict__ ctrl) {
    if (lz_skip(ctrl, tj)) return;
    __shared__ double red[NT / 64];
    double s = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x; b < nblk; b += NT) s += part[(size_t)b * LZP + LZ_NCOL];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double beta = sqrt(red[0] + red[1] + red[2] + red[3]);
    ctrl->beta = beta;
    if (!isfinite(beta)) {
        ctrl->status = MOTO_NAN;
        ctrl->done = 1;
        return;
    }
    if (tj < 0) {
        // dependent: what is left after the projection is rounding of the
        // column's own size (relative rel_dep: about 1e3 units of the basis
        // precision)
        if (!(beta > rel_dep * sqrt(ctrl->w0sq))) {
            ctrl->status = MOTO_BREAKDOWN;
            ctrl->done = 1;
        }
        return;
    }
    ctrl->n_hvp += 1;
    ctrl->T[c * LZ_LDT + tj] = beta;
    ctrl->T[tj * LZ_LDT + c] = beta;
    if (beta <= 1e-14 * fmax(1.0, fabs(ctrl->T[tj * LZ_LDT + tj]))) {
        ctrl->m_eff = tj + 1;
        ctrl->brk = 1;
    }
}

// q_c = w / beta (not after a breakdown: the restart replaces that column)
template <class T>
__global__ __launch_bounds__(NT) void k_lz_scale(int n2, T* __restrict__ Q, int c, int tj,
                                                 const LzCtrl* __restrict__ ctrl) {
    if (ctrl->done || (tj >= 0 && (tj >= ctrl->m_eff || (ctrl->brk && tj + 1 == ctrl->m_eff)))) return;
    const double beta = ctrl->beta;
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    T* __restrict__ q = Q + (size_t)c * n2;
    for (int r = blockIdx.x * NT + threadIdx.x; r < n2; r += gridDim.x * NT) q[r] = (T)((double)q[r] * inv);
}

// Rayleigh-Ritz on T[0..m) (wave 0; all waves in the eigen-solve's
// multisection): eigenpairs in ascending order, residual norms
// |T[m..m+b)[0..m) y_i|, stop test.
constexpr int LZ_RR_WAVES = 4;  // waves of the multisection (the rest runs on wave 0)
__global__ __launch_bounds__(LZ_RR_WAVES * WL) void k_lz_rr(int k, int keep, double tol_abs, int max_restarts,
                                                            LzCtrl* __restrict__ ctrl) {
    constexpr int LD = LZ_MAXM + 1;
    __shared__ double A[LD * LD], Z[LD * LD];
    __shared__ double ev[LZ_MAXM];
    const int lane = wlane();
    const bool w0 = threadIdx.x < WL;
    if (ctrl->done) {  // stopped inside the cycle (NaN, no direction left)
        if (threadIdx.x == 0) {
            ctrl->out.status = ctrl->status;
            ctrl->out.iters = ctrl->restarts;
            ctrl->out.n_hvp = ctrl->n_hvp;
        }
        return;
    }
    const int m = ctrl->m_eff;
    const int b = ctrl->blk;
    if (w0) for2(m, m, [&](int r, int c) { A[r * LD + c] = 0.5 * (ctrl->T[r * LZ_LDT + c] + ctrl->T[c * LZ_LDT + r]); });
    __syncthreads();
    // the kk lowest Ritz pairs, ascending (column i of Z)
    const int kk = keep < m ? keep : m;
    symeig_low<LD, 32, ((LD - 1 + 15) / 16) * 16, LZ_RR_WAVES>(A, Z, m, kk, ev);
    if (!w0) return;
    for2(kk, m, [&](int i, int r) { ctrl->Y[i * LZ_MAXM + r] = Z[r * LD + i]; });
    for (int i = lane; i < kk; i += WL) {
        double r2 = 0.0;
        for (int l = 0; l < b; ++l) {
            double t = 0.0;
            for (int c = 0; c < m; ++c) t += ctrl->T[(m + l) * LZ_LDT + c] * Z[c * LD + i];
            r2 += t * t;
        }
        const double th = ev[i];
        const double rn = sqrt(r2);
        ctrl->theta[i] = th;
        ctrl->resid[i] = rn;
        if (i < MAXB) {
            ctrl->out.lam[i] = th;
            ctrl->out.resid[i] = rn;
        }
    }
    wsync();
    if (lane != 0) return;
    bool conv = m >= k, bad = false;
    for (int i = 0; i < k && i < kk; ++i) {
        if (!isfinite(ctrl->theta[i]) || !isfinite(ctrl->resid[i])) bad = true;
        if (!(ctrl->resid[i] <= tol_abs)) conv = false;
    }
    ctrl->nkeep = kk;
    if (bad) {
        ctrl->status = MOTO_NAN;
        ctrl->done = 1;
    } else if (conv) {
        ctrl->status = MOTO_CONVERGED;
        ctrl->done = 1;
    } else if (ctrl->restarts >= max_restarts) {
        ctrl->status = MOTO_NOT_CONVERGED;
        ctrl->done = 1;
    } else {
        ctrl->restarts += 1;
    }
    ctrl->out.status = ctrl->status;
    ctrl->out.iters = ctrl->restarts;
    ctrl->out.n_hvp = ctrl->n_hvp;
}

// After k_lz_rr: Q[:, 0..kk) = Q[:, 0..m) Y (rows in place); when going on,
// Q[:, kk + l] = Q[:, m + l] (l < b; after a breakdown the dependent last
// column becomes fresh SplitMix64 entries) and T = diag(theta).  The product
// runs on the matrix cores: a wave takes 16 rows at a time, reads all m
// basis columns of them into FP64 16x16x4 products against Y (in LDS,
// zero-padded to 64 x 64) and writes its rows only after that, so the update
// is in place; the residual columns of the same rows move last.  The
// product is formed transposed (Y^T Q^T): lane l supplies Y[4 t + l / 16]
// [col l % 16] and Q[4 t + l / 16][row l % 16] and receives row l % 16 of
// column l / 16 + 4 e, so every store writes 16 consecutive rows.
typedef double lz_d4 __attribute__((ext_vector_type(4)));

template <class T>
__global__ __launch_bounds__(NT) void k_lz_restart(int n2, T* __restrict__ Q, const uint8_t* __restrict__ mask,
                                                   int N, uint64_t seed, LzCtrl* __restrict__ ctrl) {
    __shared__ double Yt[LZ_MAXM][LZ_MAXM];  // Yt[c][i]: component c of Ritz vector i
    if (ctrl->status == MOTO_NAN || ctrl->status == MOTO_BREAKDOWN) return;
    const int m = ctrl->m_eff, kk = ctrl->nkeep, b = ctrl->blk;
    const bool brk = ctrl->brk != 0;
    for (int e = threadIdx.x; e < LZ_MAXM * LZ_MAXM; e += NT) {
        const int c = e / LZ_MAXM, i = e - c * LZ_MAXM;
        Yt[c][i] = (c < m && i < kk) ? ctrl->Y[i * LZ_MAXM + c] : 0.0;
    }
    __syncthreads();
    const bool go_on = ctrl->done == 0;
    const uint64_t fseed = seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(ctrl->restarts + 1));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ln = lane & 15, lg = lane >> 4;
    const int ks = (m + 3) >> 2, nt = (kk + 15) >> 4;
    const int ntiles = (n2 + 15) >> 4, nwv = gridDim.x * (NT / 64);
    for (int tile = blockIdx.x * (NT / 64) + wv; tile < ntiles; tile += nwv) {
        const int r0 = tile * 16, ra = r0 + ln;
        lz_d4 acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = lz_d4{0.0, 0.0, 0.0, 0.0};
        for (int t = 0; t < ks; ++t) {
            const int c = 4 * t + lg;
            const double av = (c < m && ra < n2) ? (double)Q[(size_t)c * n2 + ra] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (q < nt) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(Yt[c][16 * q + ln], av, acc[q], 0, 0, 0);
        }
        // transposed product: lane (ln, lg) holds row r0 + ln of columns
        // 16 q + lg + 4 e (16 consecutive rows per store)
        if (ra < n2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q < nt) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int col = 16 * q + lg + 4 * e;
                        if (col < kk) Q[(size_t)col * n2 + ra] = (T)acc[q][e];
                    }
                }
            }
        }
        if (go_on && lg < b && ra < n2) {
            T v;
            if (brk && lg == b - 1) {
                const int site = ra < N ? ra : ra - N;
                v = (mask == nullptr || mask[site] != 0) ? (T)splitmix_uniform(fseed, (uint64_t)ra) : T(0);
            } else {
                v = Q[(size_t)(m + lg) * n2 + ra];
            }
            Q[(size_t)(kk + lg) * n2 + ra] = v;
        }
    }
}

// A launch of its own, after every block of k_lz_restart has read m_eff and brk.
__global__ __launch_bounds__(NT) void k_lz_restart_ctrl(LzCtrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    const int kk = ctrl->nkeep;
    for (int i = threadIdx.x; i < LZ_LDT * LZ_LDT; i += NT) {
        const int r = i / LZ_LDT, c = i - r * LZ_LDT;
        ctrl->T[i] = (r == c && r < kk) ? ctrl->theta[r] : 0.0;
    }
    if (threadIdx.x == 0) {
        ctrl->m_eff = ctrl->m_max;
        ctrl->brk = 0;
    }
}

// --------------------------------------------------------------------------
// one row per thread up to 1024 workgroups: the row kernels walk the basis
// columns with one load each, so their time grows with the rows a thread has
int lz_blocks(int n2) {
    const int nb = (n2 + NT - 1) / NT;
    return nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
}

hipError_t launch_lz_init(bool f64, int N, int b, void* Q, const double* m, const double* Vwarm, int nwarm,
                          const uint8_t* mask, uint64_t seed, LzCtrl* ctrl, int m_max, hipStream_t st) {
    const int nb = lz_blocks(N);
    if (f64)
        hipLaunchKernelGGL(k_lz_init<double>, dim3(nb), dim3(NT), 0, st, N, b, (double*)Q, m, Vwarm, nwarm, mask,
                           seed, ctrl, m_max);
    else
        hipLaunchKernelGGL(k_lz_init<float>, dim3(nb), dim3(NT), 0, st, N, b, (float*)Q, m, Vwarm, nwarm, mask,
                           seed, ctrl, m_max);
    return hipGetLastError();
}

hipError_t launch_lz_orth(bool f64, int n2, void* Q, int c, int tj, double* part, int nblk, LzCtrl* ctrl,
                          hipStream_t st) {
    for (int pass = 0; pass < 2; ++pass) {
        // the start and residual columns (tj < 0) also measure their own
        // norm in the first pass, the scale of the dependence test
        const int self = (tj < 0 && pass == 0) ? 1 : 0;
        const int rb = (c + self + NT / 64 - 1) / (NT / 64);
        const int cg = rb < 1 ? 1 : rb;  // column groups of the dot kernel (one column per wave)
        if (f64)
            hipLaunchKernelGGL(k_lz_dots<double>, dim3(nblk, cg), dim3(NT), 0, st, n2, (const double*)Q, c, tj, self,
                               part, ctrl);
        else
            hipLaunchKernelGGL(k_lz_dots<float>, dim3(nblk, cg), dim3(NT), 0, st, n2, (const float*)Q, c, tj, self,
                               part, ctrl);
        hipLaunchKernelGGL(k_lz_reduce, dim3(cg), dim3(NT), 0, st, part, nblk, c, tj, pass, self, ctrl);
        if (f64)
            hipLaunchKernelGGL(k_lz_update<double>, dim3(nblk), dim3(NT), 0, st, n2, (double*)Q, c, tj, pass, part,
                               ctrl);
        else
            hipLaunchKernelGGL(k_lz_update<float>, dim3(nblk), dim3(NT), 0, st, n2, (float*)Q, c, tj, pass, part,
                               ctrl);
    }
    hipLaunchKernelGGL(k_lz_beta, dim3(1), dim3(NT), 0, st, part, nblk, c, tj, f64 ? 1e-12 : 1e-4, ctrl);
    if (f64)
        hipLaunchKernelGGL(k_lz_scale<double>, dim3(nblk), dim3(NT), 0, st, n2, (double*)Q, c, tj, ctrl);
    else
        hipLaunchKernelGGL(k_lz_scale<float>, dim3(nblk), dim3(NT), 0, st, n2, (float*)Q, c, tj, ctrl);
    return hipGetLastError();
}

hipError_t launch_lz_rr_restart(bool f64, int n2, int b, void* Q, int k, int keep, double tol_abs, int max_restarts,
                                int m_max, int nblk, const uint8_t* mask, int N, uint64_t seed, LzCtrl* ctrl,
                                hipStream_t st) {
    (void)b;
    hipLaunchKernelGGL(k_lz_rr, dim3(1), dim3(LZ_RR_WAVES * WL), 0, st, k, keep, tol_abs, max_restarts, ctrl);
    (void)m_max;
    if (f64)
        hipLaunchKernelGGL(k_lz_restart<double>, dim3(nblk), dim3(NT), 0, st, n2, (double*)Q, mask, N, seed, ctrl);
    else
        hipLaunchKernelGGL(k_lz_restart<float>, dim3(nblk), dim3(NT), 0, st, n2, (float*)Q, mask, N, seed, ctrl);
    hipLaunchKernelGGL(k_lz_restart_ctrl, dim3(1), dim3(NT), 0, st, ctrl);
    return hipGetLastError();
}

}  // namespace moto
