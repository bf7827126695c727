// explorer.hip -- per-candidate objectives of the multi-objective explorer
// (Methods, "Multi-objective initial-configuration explorer"; Algorithm 1,
// population loop) on a population of P candidates of one lattice:
//   * candidates x = x0 + P_Omega delta, each active spin projected back onto
//     the unit sphere (an active site whose sum vanishes keeps x0);
//   * l1 distances between every candidate and every member of S u A
//     (population, then archive), their sum over the population and their
//     minimum over S u A (the diversity objective);
//   * the per-candidate summary: spectral gap lambda_2 - lambda_1 from the
//     population eigen-solve, topological-charge violation, energy.
// The l1 kernel is HBM/L2-bound streaming: each workgroup keeps PT
// candidates' elements of one chunk in registers and streams the chunk of
// every member of S u A past them, so a chunk of the population is read
// ceil(P / PT) times instead of P times.
#include "kernels.hpp"

namespace moto {

constexpr int L1_EPT = 4;               // elements per thread in a chunk
constexpr int L1_CH = NT * L1_EPT;      // elements per chunk
constexpr int L1_PT = 4;                // candidates per workgroup
constexpr int L1_QB = 16;               // members reduced per LDS round

__global__ __launch_bounds__(NT) void k_candidates(int N, const double* __restrict__ x0,
                                                   const uint8_t* __restrict__ mask,
                                                   const double* __restrict__ delta, double* __restrict__ X,
                                                   uint8_t* __restrict__ mask_rep) {
    const int s = blockIdx.x * NT + threadIdx.x;
    const int p = blockIdx.y;
    if (s >= N) return;
    const size_t N3 = 3 * (size_t)N;
    const double a0 = x0[s], a1 = x0[N + s], a2 = x0[2 * (size_t)N + s];
    double o0 = a0, o1 = a1, o2 = a2;
    const bool on = mask == nullptr || mask[s] != 0;
    if (on) {
        const double* d = delta + (size_t)p * N3;
        const double v0 = a0 + d[s], v1 = a1 + d[N + s], v2 = a2 + d[2 * (size_t)N + s];
        const double n = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
        if (n > 0.0) {
            o0 = v0 / n;
            o1 = v1 / n;
            o2 = v2 / n;
        }
    }
    double* x = X + (size_t)p * N3;
    x[s] = o0;
    x[N + s] = o1;
    x[2 * (size_t)N + s] = o2;
    if (mask_rep) mask_rep[(size_t)p * N + s] = mask[s];
}

// part[(c * P + p) * Q + q] = sum over the elements of chunk c of
// |X_p - Y_q|, Y = [X (P members) | Arch (A members)], Q = P + A.
__global__ __launch_bounds__(NT) void k_l1_part(long long n3, int P, int A, const double* __restrict__ X,
                                                const double* __restrict__ Arch, double* __restrict__ part) {
    __shared__ double red[L1_QB][NT / 64][L1_PT];
    const int c = blockIdx.x;
    const int p0 = blockIdx.y * L1_PT;
    const int Q = P + A;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long long e0 = (long long)c * L1_CH + threadIdx.x;
    double xp[L1_PT][L1_EPT];
#pragma unroll
    for (int i = 0; i < L1_PT; ++i)
#pragma unroll
        for (int t = 0; t < L1_EPT; ++t) {
            const long long e = e0 + (long long)t * NT;
            xp[i][t] = (p0 + i < P && e < n3) ? X[(size_t)(p0 + i) * n3 + e] : 0.0;
        }
    for (int qb = 0; qb < Q; qb += L1_QB) {
        const int nq = min(L1_QB, Q - qb);
        for (int qq = 0; qq < nq; ++qq) {
            const int q = qb + qq;
            const double* y = q < P ? X + (size_t)q * n3 : Arch + (size_t)(q - P) * n3;
            double yv[L1_EPT];
#pragma unroll
            for (int t = 0; t < L1_EPT; ++t) {
                const long long e = e0 + (long long)t * NT;
                yv[t] = e < n3 ? y[e] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < L1_PT; ++i) {
                double s = 0.0;
#pragma unroll
                for (int t = 0; t < L1_EPT; ++t) {
                    const long long e = e0 + (long long)t * NT;
                    if (e < n3) s += fabs(xp[i][t] - yv[t]);
                }
                s = wave_sum(s);
                if (lane == 0) red[qq][wv][i] = s;
            }
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < nq * L1_PT; idx += NT) {
            const int qq = idx / L1_PT, i = idx % L1_PT;
            if (p0 + i < P) {
                double s = 0.0;
                for (int w = 0; w < NT / 64; ++w) s += red[qq][w][i];
                part[((size_t)c * P + p0 + i) * Q + qb + qq] = s;
            }
        }
        __syncthreads();
    }
}

// D[p * Q + q] = sum over chunks in chunk order (fixed order).
__global__ __launch_bounds__(NT) void k_l1_reduce(int P, int Q, int nchunk, const double* __restrict__ part,
                                                  double* __restrict__ D) {
    const int idx = blockIdx.x * NT + threadIdx.x;
    if (idx >= P * Q) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * P * Q + idx];
    D[idx] = s;
}

__global__ void k_explorer_finish(int P, int A, int k, const double* __restrict__ D,
                                  const double* __restrict__ E, const double* __restrict__ evals,
                                  const double* __restrict__ Qc, const double* __restrict__ Qx0, double Q_target,
                                  const EigCtrl* __restrict__ ctrl, moto_explorer_result* __restrict__ res) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int Q = P + A;
    const double* d = D + (size_t)p * Q;
    double sum = 0.0, mn = INFINITY;
    for (int q = 0; q < Q; ++q) {
        if (q == p) continue;
        if (q < P) sum += d[q];
        mn = fmin(mn, d[q]);
    }
    const double qt = isnan(Q_target) ? *Qx0 : Q_target;
    moto_explorer_result r{};
    r.E = E[p];
    r.lambda1 = evals[(size_t)p * k];
    r.lambda2 = evals[(size_t)p * k + 1];
    r.gap = r.lambda2 - r.lambda1;
    r.Q = Qc[p];
    r.violation = fabs(Qc[p] - qt);
    r.l1_sum = sum;
    r.l1_min = mn;
    r.status = ctrl[p].status;
    r.iters = ctrl[p].iters;
    r.n_hvp = ctrl[p].n_hvp;
    res[p] = r;
}

// --------------------------------------------------------------------------
int l1_chunks(long long n3) { return (int)((n3 + L1_CH - 1) / L1_CH); }

hipError_t launch_candidates(int N, int P, const double* x0, const uint8_t* mask, const double* delta, double* X,
                             uint8_t* mask_rep, hipStream_t st) {
    hipLaunchKernelGGL(k_candidates, dim3((N + NT - 1) / NT, P), dim3(NT), 0, st, N, x0, mask, delta, X,
                       mask ? mask_rep : nullptr);
    return hipGetLastError();
}

hipError_t launch_l1(long long n3, int P, int A, const double* X, const double* Arch, double* part, double* D,
                     hipStream_t st) {
    const int nchunk = l1_chunks(n3);
    hipLaunchKernelGGL(k_l1_part, dim3(nchunk, (P + L1_PT - 1) / L1_PT), dim3(NT), 0, st, n3, P, A, X, Arch, part);
    const int Q = P + A;
    hipLaunchKernelGGL(k_l1_reduce, dim3((P * Q + NT - 1) / NT), dim3(NT), 0, st, P, Q, nchunk, part, D);
    return hipGetLastError();
}

hipError_t launch_explorer_finish(int P, int A, int k, const double* D, const double* E, const double* evals,
                                  const double* Qc, const double* Qx0, double Q_target, const EigCtrl* ctrl,
                                  moto_explorer_result* res, hipStream_t st) {
    hipLaunchKernelGGL(k_explorer_finish, dim3((P + 63) / 64), dim3(64), 0, st, P, A, k, D, E, evals, Qc, Qx0,
                       Q_target, ctrl, res);
    return hipGetLastError();
}

}  // namespace moto
