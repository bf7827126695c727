// dense_wg.hpp -- small dense FP64 steps of the inner layer, each executed by
// one 256-thread workgroup: parallel cyclic Jacobi, the orthonormalising
// transform of a projected block, and the Rayleigh-Ritz step with the
// orthogonal complement for P.  LD is the largest basis size handled (the
// leading dimension of the LDS matrices); LD / 3 is the largest block width.
#pragma once

#include "kernels.hpp"

namespace moto {

// --------------------------------------------------------------------------
// Parallel cyclic Jacobi on an n x n symmetric matrix in LDS (leading
// dimension LD), round-robin ordering: the n/2 rotations of a round act on
// disjoint index pairs (Golub & Van Loan, parallel Jacobi).  On return diag(A)
// holds the eigenvalues and the columns of Z the eigenvectors.
// --------------------------------------------------------------------------
template <int LD>
__device__ void jacobi_wg(double* A, double* Z, int n, double tol, int max_sweeps) {
    __shared__ double red[8];
    __shared__ double cs[LD / 2 + 1], sn[LD / 2 + 1];
    __shared__ int pp[LD / 2 + 1], qq[LD / 2 + 1];
    const int tid = threadIdx.x;
    for (int i = tid; i < n * LD; i += NT) {
        const int r = i / LD, c = i % LD;
        Z[i] = (r == c) ? 1.0 : 0.0;
    }
    const int ne = n + (n & 1);
    const int half = ne / 2;
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double off = 0.0, fro = 0.0;
        for (int i = tid; i < n * n; i += NT) {
            const int r = i / n, c = i % n;
            const double v = A[r * LD + c];
            fro += v * v;
            if (r != c) off += v * v;
        }
        off = wave_sum(off);
        fro = wave_sum(fro);
        if ((tid & 63) == 0) {
            red[tid >> 6] = off;
            red[4 + (tid >> 6)] = fro;
        }
        __syncthreads();
        const double offt = red[0] + red[1] + red[2] + red[3];
        const double frot = red[4] + red[5] + red[6] + red[7];
        __syncthreads();
        if (!(offt > tol * tol * frot)) break;
        for (int round = 0; round < ne - 1; ++round) {
            if (tid < half) {
                const int pa = tid, pb = ne - 1 - tid;
                const int ia = pa == 0 ? 0 : 1 + (pa - 1 + round) % (ne - 1);
                const int ib = pb == 0 ? 0 : 1 + (pb - 1 + round) % (ne - 1);
                const int p = ia < ib ? ia : ib, q = ia < ib ? ib : ia;
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = A[p * LD + q];
                    if (apq != 0.0) {
                        const double tau = (A[q * LD + q] - A[p * LD + p]) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                cs[tid] = c;
                sn[tid] = s;
                pp[tid] = p;
                qq[tid] = q < n ? q : -1;
            }
            __syncthreads();
            for (int i = tid; i < half * n; i += NT) {  // rows: A <- J^T A
                const int kp = i / n, col = i % n;
                const int q = qq[kp];
                if (q < 0) continue;
                const int p = pp[kp];
                const double c = cs[kp], s = sn[kp];
                const double ap = A[p * LD + col], aq = A[q * LD + col];
                A[p * LD + col] = c * ap - s * aq;
                A[q * LD + col] = s * ap + c * aq;
            }
            __syncthreads();
            for (int i = tid; i < half * n; i += NT) {  // columns: A <- A J, Z <- Z J
                const int kp = i / n, row = i % n;
                const int q = qq[kp];
                if (q < 0) continue;
                const int p = pp[kp];
                const double c = cs[kp], s = sn[kp];
                const double ap = A[row * LD + p], aq = A[row * LD + q];
                A[row * LD + p] = c * ap - s * aq;
                A[row * LD + q] = s * ap + c * aq;
                const double zp = Z[row * LD + p], zq = Z[row * LD + q];
                Z[row * LD + p] = c * zp - s * zq;
                Z[row * LD + q] = s * zp + c * zq;
            }
            __syncthreads();
        }
    }
}

// --------------------------------------------------------------------------
// Orthonormalising transform of a target block Y against an orthonormal
// projection set Q (nq columns).  G holds the Gram entries
// G[j * (nq + mb) + i] = (Q|Y)_i . Y_j.  Writes
//   Bw[r + 2*MAXB*j] = Q_r . Y_j                 (projection coefficients)
//   Tw[row + mb*c]   = D Z_keep theta^-1/2       (orthonormaliser of Y - Q B)
// where M = Y^T Y - B^T B = Z diag(theta) Z^T after diagonal scaling D;
// columns whose projected norm is negligible get a zero transform.
// --------------------------------------------------------------------------
template <int LD>
__device__ void orth_small_body(int mb, int nq, double drop, const double* G, double* Bw, double* Tw) {
    constexpr int MBL = LD / 3;
    __shared__ double A[MBL * LD];
    __shared__ double Z[MBL * LD];
    __shared__ double dsc[MBL], th[MBL];
    __shared__ int keep[MBL];
    __shared__ int nkeep;
    const int tid = threadIdx.x;
    const int nrow = nq + mb;
    for (int i = tid; i < nq * mb; i += NT) {
        const int r = i % nq, j = i / nq;
        Bw[r + 2 * MAXB * j] = G[j * nrow + r];
    }
    for (int i = tid; i < mb * mb; i += NT) {
        const int r = i % mb, c = i / mb;
        double v = G[c * nrow + nq + r];
        for (int l = 0; l < nq; ++l) v -= G[r * nrow + l] * G[c * nrow + l];
        A[r * LD + c] = v;
    }
    __syncthreads();
    for (int j = tid; j < mb; j += NT) {
        const double full = G[j * nrow + nq + j];
        const double proj = A[j * LD + j];
        dsc[j] = (proj > drop * full && proj > 0.0) ? 1.0 / sqrt(proj) : 0.0;
    }
    __syncthreads();
    for (int i = tid; i < mb * mb; i += NT) {
        const int r = i % mb, c = i / mb;
        A[r * LD + c] *= dsc[r] * dsc[c];
    }
    __syncthreads();
    jacobi_wg<LD>(A, Z, mb, 1e-15, 40);
    if (tid == 0) {
        int r = 0;
        for (int i = 0; i < mb; ++i) {
            const double t = A[i * LD + i];
            if (t > drop) {
                keep[r] = i;
                th[r] = t;
                ++r;
            }
        }
        nkeep = r;
    }
    __syncthreads();
    for (int i = tid; i < mb * mb; i += NT) {
        const int row = i % mb, c = i / mb;
        Tw[row + mb * c] = c < nkeep ? dsc[row] * Z[row * LD + keep[c]] / sqrt(th[c]) : 0.0;
    }
    __syncthreads();
}

// --------------------------------------------------------------------------
// Rayleigh-Ritz on span(S), basis size ns (X = first mb columns):
//   G_B -> D G_B D = Z diag(theta) Z^T, keep theta > drop * max(theta),
//   T = D Z_keep theta^-1/2  (T^T G_B T = I);
//   T^T G_A T = Y diag(lam) Y^T;   C = T Y[:, lowest mb]   (X_new = S C);
//   C_wp = C with its X rows zeroed, made G_B-orthogonal to C (twice) and
//   G_B-orthonormalised with rank dropping -> Cp  (P_new = S Cp).
// Gtri: upper triangles (row-major) of S^T HS, then of S^T S.
// Writes C, Cp, lam, rank of the control block `out`.
// --------------------------------------------------------------------------
template <int LD>
__device__ void rr_body(int mb, int ns, double drop, const double* Gtri, EigCtrl* out) {
    constexpr int MBL = LD / 3;
    __shared__ double A[LD * LD];
    __shared__ double Z[LD * LD];
    __shared__ double Tm[LD * LD];
    __shared__ double dsc[LD], th[LD], ev[LD];
    __shared__ double h1[MBL * MBL];
    __shared__ int keep[LD], order[LD];
    __shared__ int rank_s;
    const int tid = threadIdx.x;
    const int Eh = ns * (ns + 1) / 2;
    auto GA = [&](int i, int j) {
        const int r = i < j ? i : j, c = i < j ? j : i;
        return Gtri[r * ns - r * (r - 1) / 2 + (c - r)];
    };
    auto GB = [&](int i, int j) {
        const int r = i < j ? i : j, c = i < j ? j : i;
        return Gtri[Eh + r * ns - r * (r - 1) / 2 + (c - r)];
    };
    double gbmax = 0.0;
    for (int i = 0; i < ns; ++i) gbmax = fmax(gbmax, GB(i, i));
    for (int i = tid; i < ns; i += NT) {
        const double gii = GB(i, i);
        dsc[i] = gii > 1e-24 * gbmax ? 1.0 / sqrt(gii) : 0.0;
    }
    __syncthreads();
    for (int i = tid; i < ns * ns; i += NT) {
        const int r = i / ns, c = i % ns;
        A[r * LD + c] = dsc[r] * GB(r, c) * dsc[c];
    }
    __syncthreads();
    jacobi_wg<LD>(A, Z, ns, 1e-15, 40);
    if (tid == 0) {
        double tmax = 0.0;
        for (int i = 0; i < ns; ++i) tmax = fmax(tmax, A[i * LD + i]);
        int r = 0;
        for (int i = 0; i < ns; ++i) {
            const double t = A[i * LD + i];
            if (t > drop * tmax) {
                keep[r] = i;
                th[r] = t;
                ++r;
            }
        }
        rank_s = r;
    }
    __syncthreads();
    const int r = rank_s;
    for (int i = tid; i < ns * r; i += NT) {  // T (ns x r)
        const int row = i / r, c = i % r;
        Tm[row * LD + c] = dsc[row] * Z[row * LD + keep[c]] / sqrt(th[c]);
    }
    __syncthreads();
    for (int i = tid; i < ns * r; i += NT) {  // Z <- G_A T
        const int row = i / r, c = i % r;
        double s = 0.0;
        for (int l = 0; l < ns; ++l) s += GA(row, l) * Tm[l * LD + c];
        Z[row * LD + c] = s;
    }
    __syncthreads();
    for (int i = tid; i < r * r; i += NT) {  // A <- T^T Z
        const int row = i / r, c = i % r;
        double s = 0.0;
        for (int l = 0; l < ns; ++l) s += Tm[l * LD + row] * Z[l * LD + c];
        A[row * LD + c] = s;
    }
    __syncthreads();
    for (int i = tid; i < r * r; i += NT) {
        const int row = i / r, c = i % r;
        if (row < c) {
            const double v = 0.5 * (A[row * LD + c] + A[c * LD + row]);
            A[row * LD + c] = v;
            A[c * LD + row] = v;
        }
    }
    __syncthreads();
    jacobi_wg<LD>(A, Z, r, 1e-15, 40);
    for (int i = tid; i < r; i += NT) ev[i] = A[i * LD + i];
    __syncthreads();
    for (int i = tid; i < r; i += NT) {
        const double li = ev[i];
        int rk = 0;
        for (int j = 0; j < r; ++j) rk += (ev[j] < li) || (ev[j] == li && j < i);
        order[rk] = i;
    }
    __syncthreads();
    const int mcol = r < mb ? r : mb;
    // C = T Y[:, order[0..mb)] -> A region (ld MBL) and out->C
    for (int i = tid; i < ns * mb; i += NT) {
        const int row = i % ns, j = i / ns;
        double s = 0.0;
        if (j < mcol) {
            const int yc = order[j];
            for (int l = 0; l < r; ++l) s += Tm[row * LD + l] * Z[l * LD + yc];
        }
        A[row * MBL + j] = s;
        out->C[row + ns * j] = s;
    }
    for (int j = tid; j < mb; j += NT) out->lam[j] = j < mcol ? ev[order[j]] : 0.0;
    if (tid == 0) out->rank = r;
    __syncthreads();
    // ---- P complement: Cwp in the Tm region (ld MBL) ----
    for (int i = tid; i < ns * mb; i += NT) {
        const int row = i % ns, j = i / ns;
        Tm[row * MBL + j] = row < mb ? 0.0 : A[row * MBL + j];
    }
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = tid; i < ns * mb; i += NT) {  // Z <- G_B Cwp
            const int row = i % ns, j = i / ns;
            double s = 0.0;
            for (int l = 0; l < ns; ++l) s += GB(row, l) * Tm[l * MBL + j];
            Z[row * MBL + j] = s;
        }
        __syncthreads();
        for (int i = tid; i < mb * mb; i += NT) {  // h1 <- C^T G_B Cwp
            const int p = i % mb, j = i / mb;
            double s = 0.0;
            for (int l = 0; l < ns; ++l) s += A[l * MBL + p] * Z[l * MBL + j];
            h1[p + MBL * j] = s;
        }
        __syncthreads();
        for (int i = tid; i < ns * mb; i += NT) {  // Cwp <- Cwp - C h1
            const int row = i % ns, j = i / ns;
            double s = Tm[row * MBL + j];
            for (int p = 0; p < mb; ++p) s -= A[row * MBL + p] * h1[p + MBL * j];
            Tm[row * MBL + j] = s;
        }
        __syncthreads();
    }
    // Mp = Cwp^T G_B Cwp
    for (int i = tid; i < ns * mb; i += NT) {
        const int row = i % ns, j = i / ns;
        double s = 0.0;
        for (int l = 0; l < ns; ++l) s += GB(row, l) * Tm[l * MBL + j];
        A[row * MBL + j] = s;
    }
    __syncthreads();
    for (int i = tid; i < mb * mb; i += NT) {
        const int p = i % mb, j = i / mb;
        double s = 0.0;
        for (int l = 0; l < ns; ++l) s += Tm[l * MBL + p] * A[l * MBL + j];
        h1[p + MBL * j] = s;
    }
    __syncthreads();
    for (int j = tid; j < mb; j += NT) {
        const double d = h1[j + MBL * j];
        dsc[j] = d > 1e-24 ? 1.0 / sqrt(d) : 0.0;
    }
    __syncthreads();
    for (int i = tid; i < mb * mb; i += NT) {
        const int p = i % mb, j = i / mb;
        Z[p * LD + j] = dsc[p] * h1[p + MBL * j] * dsc[j];
    }
    __syncthreads();
    jacobi_wg<LD>(Z, A, mb, 1e-15, 40);
    if (tid == 0) {
        int rr = 0;
        for (int i = 0; i < mb; ++i) {
            const double t = Z[i * LD + i];
            if (t > drop) {
                keep[rr] = i;
                th[rr] = t;
                ++rr;
            }
        }
        rank_s = rr;
    }
    __syncthreads();
    const int rp = rank_s;
    for (int i = tid; i < ns * mb; i += NT) {  // Cp = Cwp D Zp_keep theta^-1/2
        const int row = i % ns, j = i / ns;
        double s = 0.0;
        if (j < rp) {
            const int zc = keep[j];
            for (int l = 0; l < mb; ++l) s += Tm[row * MBL + l] * dsc[l] * A[l * LD + zc];
            s /= sqrt(th[j]);
        }
        out->Cp[row + ns * j] = s;
    }
    __syncthreads();
}

}  // namespace moto
