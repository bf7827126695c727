// lanczos.hip -- the second inner solver: thick-restart Lanczos with full
// reorthogonalisation on the (masked) tangent Hessian in frame coordinates
// (the paper's HVP-Lanczos operator mode; Krylov depth and
// reorthogonalisation are its named hyperparameters).  One step j:
//   w = H q_j                       (the HVP kernel, one vector)
//   h = Q_{0..j}^T w, w -= Q h      (classical Gram-Schmidt, twice; the
//                                    coefficients of both passes summed are
//                                    column j of Q^T H Q)
//   beta = |w|, q_{j+1} = w / beta
// Q lives in one [m_max + 1][2N] array; w is written straight into column
// j + 1.  At the end of a cycle one wavefront diagonalises the projected
// matrix T (FP64, Householder tridiagonalisation and implicit QL), tests the
// residual estimates |beta_m y_m,i| and either stops or restarts from the
// `keep` lowest Ritz vectors plus the residual direction (Wu & Simon 2000):
// T becomes diag(theta) bordered by beta_m y_m.  All reductions are FP64 with a fixed order.
#include <type_traits>

#include "dense_wg.hpp"
#include "kernels.hpp"

namespace moto {

constexpr int LZP = LZ_MAXM + 2;  // doubles per block partial row (columns, then |w|^2)

__device__ __forceinline__ int lz_rows_per_block(int n2, int nblk) {
    const int per = (n2 + nblk - 1) / nblk;
    return (per + 63) & ~63;
}

// Start vector: the sum of the warm vectors (ambient, FP64) in frame
// coordinates, else SplitMix64 entries; masked sites zero.  Partial |q|^2.
template <class T>
__global__ __launch_bounds__(NT) void k_lz_init(int N, T* __restrict__ Q, const double* __restrict__ m,
                                                const double* __restrict__ Vwarm, int nwarm,
                                                const uint8_t* __restrict__ mask, uint64_t seed,
                                                double* __restrict__ part, LzCtrl* __restrict__ ctrl, int m_max) {
    __shared__ double red[NT / 64];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->done = 0;
        ctrl->status = MOTO_NOT_CONVERGED;
        ctrl->restarts = 0;
        ctrl->m_eff = m_max;
        ctrl->m_max = m_max;
        ctrl->n_hvp = 0;
    }
    double s2 = 0.0;
    for (int s = blockIdx.x * NT + threadIdx.x; s < N; s += gridDim.x * NT) {
        double a = 0.0, b = 0.0;
        const bool on = mask == nullptr || mask[s] != 0;
        if (on) {
            if (nwarm > 0) {
                double e1[3], e2[3];
                onb(m[s], m[N + s], m[2 * N + s], e1, e2);
                for (int j = 0; j < nwarm; ++j) {
                    const double* v = Vwarm + (size_t)j * 3 * N;
                    a += e1[0] * v[s] + e1[1] * v[N + s] + e1[2] * v[2 * N + s];
                    b += e2[0] * v[s] + e2[1] * v[N + s] + e2[2] * v[2 * N + s];
                }
            } else {
                a = splitmix_uniform(seed, (uint64_t)s);
                b = splitmix_uniform(seed, (uint64_t)N + s);
            }
        }
        const T ta = (T)a, tb = (T)b;
        Q[s] = ta;
        Q[N + s] = tb;
        s2 += (double)ta * ta + (double)tb * tb;
    }
    s2 = wave_sum(s2);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s2;
    __syncthreads();
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * LZP + LZ_MAXM + 1] = red[0] + red[1] + red[2] + red[3];
}

// Partial dots of w = Q[j + 1] with Q[0..j]: blockIdx.x picks the rows,
// wave w of block (x, y) the column c = 4 y + w, so every column's rows are
// read by its own wave in parallel; lane l takes the rows start + l,
// start + l + 64, ... into two alternating partial sums (fixed order).
template <class T>
__global__ __launch_bounds__(NT) void k_lz_dots(int n2, const T* __restrict__ Q, int j, double* __restrict__ part,
                                                const LzCtrl* __restrict__ ctrl) {
    if (ctrl->done || j >= ctrl->m_eff) return;
    const int c = blockIdx.y * (NT / 64) + (threadIdx.x >> 6);
    if (c > j) return;
    const int per = lz_rows_per_block(n2, gridDim.x);
    const int r0 = blockIdx.x * per, r1 = min(n2, r0 + per);
    const int lane = threadIdx.x & 63;
    const T* __restrict__ w = Q + (size_t)(j + 1) * n2;
    const T* __restrict__ q = Q + (size_t)c * n2;
    double s0 = 0.0, s1 = 0.0;
    int r = r0 + lane;
    for (; r + 64 < r1; r += 128) {
        s0 += (double)q[r] * (double)w[r];
        s1 += (double)q[r + 64] * (double)w[r + 64];
    }
    if (r < r1) s0 += (double)q[r] * (double)w[r];
    const double s = wave_sum(s0 + s1);
    if (lane == 0) part[(size_t)blockIdx.x * LZP + c] = s;
}

// h_c = sum_b part[b][c] for c <= j (one wavefront per column).  pass 0
// stores h and sets column j of T; pass 1 stores h and adds it to T.
__global__ __launch_bounds__(NT) void k_lz_reduce(const double* __restrict__ part, int nblk, int j, int pass,
                                                  LzCtrl* __restrict__ ctrl) {
    if (ctrl->done || j >= ctrl->m_eff) return;
    const int lane = threadIdx.x & 63;
    for (int c = blockIdx.x * (NT / 64) + (threadIdx.x >> 6); c <= j; c += gridDim.x * (NT / 64)) {
        double s = 0.0;
        for (int b = lane; b < nblk; b += 64) s += part[(size_t)b * LZP + c];
        s = wave_sum(s);
        if (lane == 0) {
            ctrl->h[c] = s;
            const double t = pass == 0 ? s : ctrl->T[c * LZ_LDT + j] + s;
            ctrl->T[c * LZ_LDT + j] = t;
            ctrl->T[j * LZ_LDT + c] = t;
        }
    }
}

// w -= Q[0..j] h; on the last pass also the partial |w|^2.
template <class T>
__global__ __launch_bounds__(NT) void k_lz_update(int n2, T* __restrict__ Q, int j, int want_norm,
                                                  double* __restrict__ part, const LzCtrl* __restrict__ ctrl) {
    if (ctrl->done || j >= ctrl->m_eff) return;
    __shared__ double h[LZ_MAXM + 1];
    __shared__ double red[NT / 64];
    for (int c = threadIdx.x; c <= j; c += NT) h[c] = ctrl->h[c];
    __syncthreads();
    T* __restrict__ w = Q + (size_t)(j + 1) * n2;
    double s2 = 0.0;
    for (int r = blockIdx.x * NT + threadIdx.x; r < n2; r += gridDim.x * NT) {
        double v = (double)w[r];
        for (int c = 0; c <= j; ++c) v -= h[c] * (double)Q[(size_t)c * n2 + r];
        const T tv = (T)v;
        w[r] = tv;
        s2 += (double)tv * tv;
    }
    if (!want_norm) return;
    s2 = wave_sum(s2);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s2;
    __syncthreads();
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * LZP + LZ_MAXM + 1] = red[0] + red[1] + red[2] + red[3];
}

// beta = |w| from the partials (one workgroup).  col < 0: the start vector
// (no T entry, no HVP count).  A negligible beta ends the cycle at j + 1.
__global__ __launch_bounds__(NT) void k_lz_beta(const double* __restrict__ part, int nblk, int j,
                                                LzCtrl* __restrict__ ctrl) {
    if (ctrl->done || j >= ctrl->m_eff) return;
    __shared__ double red[NT / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += NT) s += part[(size_t)b * LZP + LZ_MAXM + 1];
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
    if (j < 0) return;
    ctrl->n_hvp += 1;
    ctrl->T[(j + 1) * LZ_LDT + j] = beta;
    ctrl->T[j * LZ_LDT + j + 1] = beta;
    if (beta <= 1e-14 * fmax(1.0, fabs(ctrl->T[j * LZ_LDT + j]))) ctrl->m_eff = j + 1;
}

// q_{j+1} = w / beta (column `col` = j + 1)
template <class T>
__global__ __launch_bounds__(NT) void k_lz_scale(int n2, T* __restrict__ Q, int col, const LzCtrl* __restrict__ ctrl) {
    if (ctrl->done || (col > 0 && col - 1 >= ctrl->m_eff)) return;
    const double beta = ctrl->beta;
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    T* __restrict__ q = Q + (size_t)col * n2;
    for (int r = blockIdx.x * NT + threadIdx.x; r < n2; r += gridDim.x * NT) q[r] = (T)((double)q[r] * inv);
}

// Rayleigh-Ritz on T[0..m) (one wavefront): eigenpairs in ascending order,
// residual estimates, stop test; when going on, the restarted T.
__global__ __launch_bounds__(WL) void k_lz_rr(int k, int keep, double tol_abs, int max_restarts,
                                              LzCtrl* __restrict__ ctrl) {
    constexpr int LD = LZ_MAXM + 1;
    __shared__ double A[LD * LD], Z[LD * LD];
    __shared__ double ev[LZ_MAXM];
    __shared__ int order[LZ_MAXM];
    if (ctrl->status == MOTO_NAN) return;
    const int lane = wlane();
    const int m = ctrl->m_eff;
    const bool full = m == ctrl->m_max;
    const double bm = full ? ctrl->T[m * LZ_LDT + m - 1] : 0.0;
    for2(m, m, [&](int r, int c) { A[r * LD + c] = 0.5 * (ctrl->T[r * LZ_LDT + c] + ctrl->T[c * LZ_LDT + r]); });
    wsync();
    symeig_wg<LD>(A, Z, m);
    for (int i = lane; i < m; i += WL) ev[i] = A[i * LD + i];
    wsync();
    for (int i = lane; i < m; i += WL) {
        const double li = ev[i];
        int rk = 0;
        for (int q = 0; q < m; ++q) rk += (ev[q] < li) || (ev[q] == li && q < i);
        order[rk] = i;
    }
    wsync();
    const int kk = keep < m ? keep : m;
    for2(kk, m, [&](int i, int r) { ctrl->Y[i * LZ_MAXM + r] = Z[r * LD + order[i]]; });
    for (int i = lane; i < kk; i += WL) {
        const double th = ev[order[i]];
        const double rn = fabs(bm * Z[(m - 1) * LD + order[i]]);
        ctrl->theta[i] = th;
        ctrl->resid[i] = rn;
        if (i < MAXB) {
            ctrl->out.lam[i] = th;
            ctrl->out.resid[i] = rn;
        }
    }
    wsync();
    if (lane != 0) return;
    bool conv = true, bad = false;
    for (int i = 0; i < k && i < kk; ++i) {
        if (!isfinite(ctrl->theta[i]) || !isfinite(ctrl->resid[i])) bad = true;
        if (!(ctrl->resid[i] <= tol_abs)) conv = false;
    }
    ctrl->nkeep = kk;
    if (bad) {
        ctrl->status = MOTO_NAN;
        ctrl->done = 1;
    } else if (conv || !full) {
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

// After k_lz_rr: Q[:, 0..keep) = Q[:, 0..m) Y (rows in place), and, when
// going on, Q[:, keep] = Q[:, m] and T = diag(theta) bordered by beta_m y_m.
template <class T, int MM>
__global__ __launch_bounds__(NT) void k_lz_restart(int n2, T* __restrict__ Q, LzCtrl* __restrict__ ctrl) {
    __shared__ double Y[MM * MM];
    const int m = ctrl->m_eff, kk = ctrl->nkeep;
    if (ctrl->status == MOTO_NAN) return;
    for (int i = threadIdx.x; i < kk * m; i += NT) Y[i] = ctrl->Y[(i / m) * LZ_MAXM + (i % m)];
    __syncthreads();
    const bool go_on = ctrl->done == 0;
    for (int r = blockIdx.x * NT + threadIdx.x; r < n2; r += gridDim.x * NT) {
        T q[MM];
#pragma unroll
        for (int c = 0; c < MM; ++c)
            if (c < m) q[c] = Q[(size_t)c * n2 + r];
        for (int i = 0; i < kk; ++i) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < MM; ++c)
                if (c < m) s += (double)q[c] * Y[i * m + c];
            Q[(size_t)i * n2 + r] = (T)s;
        }
        if (go_on) Q[(size_t)kk * n2 + r] = Q[(size_t)m * n2 + r];
    }
    if (go_on && blockIdx.x == 0) {
        __syncthreads();
        // the restarted projected matrix (block 0 only; the next kernels
        // read it after this launch)
        const double bm = ctrl->T[m * LZ_LDT + m - 1];
        __syncthreads();  // every wave holds beta_m before the matrix is cleared
        for (int i = threadIdx.x; i < LZ_LDT * LZ_LDT; i += NT) ctrl->T[i] = 0.0;
        __syncthreads();
        for (int i = threadIdx.x; i < kk; i += NT) {
            ctrl->T[i * LZ_LDT + i] = ctrl->theta[i];
            const double cpl = bm * Y[i * m + m - 1];
            ctrl->T[i * LZ_LDT + kk] = cpl;
            ctrl->T[kk * LZ_LDT + i] = cpl;
        }
        if (threadIdx.x == 0) ctrl->m_eff = ctrl->m_max;
    }
}

// --------------------------------------------------------------------------
// one row per thread up to 1024 workgroups: the row kernels walk the basis
// columns with one load each, so their time grows with the rows a thread has
int lz_blocks(int n2) {
    const int nb = (n2 + NT - 1) / NT;
    return nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
}

hipError_t launch_lz_init(bool f64, int N, void* Q, const double* m, const double* Vwarm, int nwarm,
                          const uint8_t* mask, uint64_t seed, double* part, int nblk, LzCtrl* ctrl, int m_max,
                          hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(k_lz_init<double>, dim3(nblk), dim3(NT), 0, st, N, (double*)Q, m, Vwarm, nwarm, mask,
                           seed, part, ctrl, m_max);
    else
        hipLaunchKernelGGL(k_lz_init<float>, dim3(nblk), dim3(NT), 0, st, N, (float*)Q, m, Vwarm, nwarm, mask,
                           seed, part, ctrl, m_max);
    hipLaunchKernelGGL(k_lz_beta, dim3(1), dim3(NT), 0, st, part, nblk, -1, ctrl);
    if (f64)
        hipLaunchKernelGGL(k_lz_scale<double>, dim3(nblk), dim3(NT), 0, st, 2 * N, (double*)Q, 0, ctrl);
    else
        hipLaunchKernelGGL(k_lz_scale<float>, dim3(nblk), dim3(NT), 0, st, 2 * N, (float*)Q, 0, ctrl);
    return hipGetLastError();
}

// Orthogonalise column j + 1 (already H q_j) against columns 0..j twice,
// normalise it, record beta.
hipError_t launch_lz_orth(bool f64, int n2, void* Q, int j, double* part, int nblk, LzCtrl* ctrl, hipStream_t st) {
    const int rb = (j + 1 + NT / 64 - 1) / (NT / 64);
    const int cg = rb < 1 ? 1 : rb;  // column groups of the dot kernel (one column per wave)
    for (int pass = 0; pass < 2; ++pass) {
        if (f64)
            hipLaunchKernelGGL(k_lz_dots<double>, dim3(nblk, cg), dim3(NT), 0, st, n2, (const double*)Q, j, part, ctrl);
        else
            hipLaunchKernelGGL(k_lz_dots<float>, dim3(nblk, cg), dim3(NT), 0, st, n2, (const float*)Q, j, part, ctrl);
        hipLaunchKernelGGL(k_lz_reduce, dim3(rb < 1 ? 1 : rb), dim3(NT), 0, st, part, nblk, j, pass, ctrl);
        if (f64)
            hipLaunchKernelGGL(k_lz_update<double>, dim3(nblk), dim3(NT), 0, st, n2, (double*)Q, j, pass, part,
                               ctrl);
        else
            hipLaunchKernelGGL(k_lz_update<float>, dim3(nblk), dim3(NT), 0, st, n2, (float*)Q, j, pass, part, ctrl);
    }
    hipLaunchKernelGGL(k_lz_beta, dim3(1), dim3(NT), 0, st, part, nblk, j, ctrl);
    if (f64)
        hipLaunchKernelGGL(k_lz_scale<double>, dim3(nblk), dim3(NT), 0, st, n2, (double*)Q, j + 1, ctrl);
    else
        hipLaunchKernelGGL(k_lz_scale<float>, dim3(nblk), dim3(NT), 0, st, n2, (float*)Q, j + 1, ctrl);
    return hipGetLastError();
}

hipError_t launch_lz_rr_restart(bool f64, int n2, void* Q, int k, int keep, double tol_abs, int max_restarts,
                                int m_max, int nblk, LzCtrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL(k_lz_rr, dim3(1), dim3(WL), 0, st, k, keep, tol_abs, max_restarts, ctrl);
    auto go = [&](auto mmc) {
        constexpr int MM = decltype(mmc)::value;
        if (f64)
            hipLaunchKernelGGL((k_lz_restart<double, MM>), dim3(nblk), dim3(NT), 0, st, n2, (double*)Q, ctrl);
        else
            hipLaunchKernelGGL((k_lz_restart<float, MM>), dim3(nblk), dim3(NT), 0, st, n2, (float*)Q, ctrl);
    };
    if (m_max <= 32)
        go(std::integral_constant<int, 32>{});
    else
        go(std::integral_constant<int, LZ_MAXM>{});
    return hipGetLastError();
}

}  // namespace moto
