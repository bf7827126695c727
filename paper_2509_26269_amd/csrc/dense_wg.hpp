// dense_wg.hpp -- small dense FP64 steps of the inner layer, each executed by
// one wavefront: the symmetric eigen-solve (Householder tridiagonalisation
// and implicit QL), the orthonormalising transform of a projected block, and
// the Rayleigh-Ritz step with the orthogonal complement for P.  LD is the largest basis size handled (the
// leading dimension of the LDS matrices); LD / 3 is the largest block width.
#pragma once

#include "kernels.hpp"

namespace moto {

// --------------------------------------------------------------------------
// All bodies below run on ONE wavefront (the 64 lanes of the calling wave,
// lane = threadIdx.x & 63): the matrices are at most 48 x 48, and a single
// wave needs no workgroup barriers between the many short steps, only
// wave-level ordering of its LDS traffic.  Callers with larger workgroups
// let one wave call them and synchronise the workgroup afterwards.
// --------------------------------------------------------------------------
constexpr int WL = 64;  // lanes

// Order the LDS accesses of the wave: everything written before is visible
// to every lane after (LDS operations of one wave execute in order; the
// fences keep the compiler from moving accesses across).
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wlane() { return threadIdx.x & (WL - 1); }

// --------------------------------------------------------------------------
// Symmetric eigen-decomposition on one wavefront, the solver of every small
// dense step: Householder reduction to tridiagonal form with the reflections
// accumulated (lane r owns row r of the matrix and of Z), then the implicit
// QL iteration with Wilkinson shifts on the tridiagonal, its plane rotations
// applied to the columns of Z (Golub & Van Loan, Sections 8.3.1 and 8.3.5).
// The scalar recurrences of the QL sweep are computed by every lane alike,
// so control flow stays uniform.  On return
// diag(A) holds the eigenvalues (in no particular order) and column j of Z
// the eigenvector of A[j][j]; the off-diagonal part of A is left undefined.
// About n^2 short serial steps instead of a cyclic Jacobi's ~ 6 n rounds of
// n^2/2 rotations, which is what a single wavefront is limited by.
// --------------------------------------------------------------------------
// value of v held by lane i (i uniform across the wave)
__device__ __forceinline__ double rdlane(double v, int i) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), i);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), i);
    return __hiloint2double(hi, lo);
}

// 1/sqrt(t) for t > 0 to FP64 accuracy: the hardware estimate refined by two
// Newton steps (each doubles the correct bits), a short dependent chain in
// place of a correctly rounded square root followed by a division.
__device__ __forceinline__ double rsqrt_nr(double t) {
    double y = __builtin_amdgcn_rsq(t);
    y = y * (1.5 - 0.5 * t * y * y);
    y = y * (1.5 - 0.5 * t * y * y);
    return y;
}

template <int LD>
__device__ void symeig_wg(double* A, double* Z, int n) {
    __shared__ double hv[LD], hw[LD];
    const int lane = wlane();
    if (n <= 0) return;
    for (int r = lane; r < n; r += WL)
        for (int c = 0; c < n; ++c) Z[r * LD + c] = (r == c) ? 1.0 : 0.0;
    wsync();
    // ---- tridiagonalisation: A <- H A H, Z <- Z H, H = I - 2 v v^T ----
    for (int k = 0; k + 2 < n; ++k) {
        double x2 = 0.0;
        for (int i = k + 1 + lane; i < n; i += WL) {
            const double x = A[i * LD + k];
            x2 += x * x;
        }
        x2 = wave_sum(x2);
        if (x2 == 0.0) continue;
        const double x0 = A[(k + 1) * LD + k];
        const double nx = sqrt(x2);
        const double alpha = x0 >= 0.0 ? -nx : nx;
        // |v|^2 = |x|^2 - 2 alpha x0 + alpha^2 = 2 (|x|^2 - alpha x0) > 0
        const double inv = 1.0 / sqrt(2.0 * (x2 - alpha * x0));
        for (int i = k + 1 + lane; i < n; i += WL) hv[i] = (A[i * LD + k] - (i == k + 1 ? alpha : 0.0)) * inv;
        wsync();
        // p = A22 v, K = v^T p, w = p - K v
        double vp = 0.0;
        for (int i = k + 1 + lane; i < n; i += WL) {
            double pi = 0.0;
#pragma unroll 4
            for (int j = k + 1; j < n; ++j) pi += A[i * LD + j] * hv[j];
            hw[i] = pi;
            vp += pi * hv[i];
        }
        const double K = wave_sum(vp);
        wsync();
        for (int i = k + 1 + lane; i < n; i += WL) hw[i] -= K * hv[i];
        wsync();
        // A22 <- A22 - 2 (v w^T + w v^T); column k reduced to alpha e_(k+1)
        for (int i = k + 1 + lane; i < n; i += WL) {
            const double vi = hv[i], wi = hw[i];
#pragma unroll 4
            for (int j = k + 1; j < n; ++j) A[i * LD + j] -= 2.0 * (vi * hw[j] + wi * hv[j]);
            const double a = i == k + 1 ? alpha : 0.0;
            A[i * LD + k] = a;
            A[k * LD + i] = a;
        }
        // Z <- Z - 2 (Z v) v^T on columns k+1..n-1
        for (int r = lane; r < n; r += WL) {
            double t = 0.0;
#pragma unroll 4
            for (int j = k + 1; j < n; ++j) t += Z[r * LD + j] * hv[j];
            t *= 2.0;
#pragma unroll 4
            for (int j = k + 1; j < n; ++j) Z[r * LD + j] -= t * hv[j];
        }
        wsync();
    }
    // ---- implicit QL on the tridiagonal (d, e): lane i holds d_i and e_i
    // (= T[i+1][i]) in registers; the sweep's scalars are read with readlane
    // and computed by every lane alike, so control flow stays uniform ----
    double di = 0.0, ei = 0.0;
    if (lane < n) {
        di = A[lane * LD + lane];
        ei = lane + 1 < n ? A[(lane + 1) * LD + lane] : 0.0;
    }
    constexpr double eps = 2.220446049250313e-16;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 64; ++iter) {
            // m = first index >= l with a negligible e_m (or n - 1)
            const double dn = __shfl_down(di, 1, WL);
            const bool small = lane + 1 >= n || fabs(ei) <= eps * (fabs(di) + fabs(dn));
            const unsigned long long msk = __ballot(small && lane >= l);
            const int m = (int)__builtin_ctzll(msk);
            if (m == l) break;
            const double dl = rdlane(di, l), el = rdlane(ei, l);
            double g = (rdlane(di, l + 1) - dl) / (2.0 * el);
            double r = sqrt(g * g + 1.0);
            g = rdlane(di, m) - dl + el / (g + (g >= 0.0 ? r : -r));
            double sn = 1.0, cs = 1.0, p = 0.0;
            bool deflated = false;
            double dnext = rdlane(di, m);  // d_(i+1) before its update
            // column i + 1 of the lane's row of Z as updated by the previous
            // rotation of this sweep (carried in a register, stored once final)
            double zc = lane < n ? Z[lane * LD + m] : 0.0;
            int ilast = m;
            for (int i = m - 1; i >= l; --i) {
                const double e_i = rdlane(ei, i), d_i = rdlane(di, i);
                const double z0 = lane < n ? Z[lane * LD + i] : 0.0;
                const double f = sn * e_i, b = cs * e_i;
                const double t = f * f + g * g;
                if (t == 0.0) {
                    if (lane == i + 1) {
                        ei = 0.0;
                        di = dnext - p;
                    }
                    if (lane == m) ei = 0.0;
                    deflated = true;
                    break;
                }
                const double ri = rsqrt_nr(t);
                r = t * ri;
                if (lane == i + 1) ei = r;
                sn = f * ri;
                cs = g * ri;
                g = dnext - p;
                r = (d_i - g) * sn + 2.0 * cs * b;
                p = sn * r;
                if (lane == i + 1) di = g + p;
                g = cs * r - b;
                dnext = d_i;
                if (lane < n) Z[lane * LD + i + 1] = sn * z0 + cs * zc;
                zc = cs * z0 - sn * zc;
                ilast = i;
            }
            if (lane < n) Z[lane * LD + ilast] = zc;
            if (deflated) continue;
            if (lane == l) {
                di -= p;
                ei = g;
            }
            if (lane == m) ei = 0.0;
        }
    }
    wsync();
    if (lane < n) A[lane * LD + lane] = di;
    wsync();
}

// --------------------------------------------------------------------------
// Visit (a, b), a < na, b < nb, in lane-strided order of a * nb + b, with
// one integer division per call instead of one per element.
template <class F>
__device__ __forceinline__ void for2(int na, int nb, F&& f) {
    if (na <= 0 || nb <= 0) return;
    const int lane = wlane();
    int a = lane / nb, b = lane % nb;
    const int qa = WL / nb, qb = WL % nb;
    for (int i = lane; i < na * nb; i += WL) {
        f(a, b);
        a += qa;
        b += qb;
        if (b >= nb) {
            b -= nb;
            ++a;
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
    // G is read many times below: it is first copied to LDS
    constexpr int MBL = LD / 3;
    __shared__ double A[MBL * LD];
    __shared__ double Z[MBL * LD];
    __shared__ double dsc[MBL], th[MBL];
    __shared__ int keep[MBL];
    __shared__ int nkeep;
    __shared__ double Gl[LD * MBL];
    const int tid = wlane();
    const int nrow = nq + mb;
    for (int i = tid; i < nrow * mb; i += WL) Gl[i] = G[i];
    wsync();
    G = Gl;
    for2(mb, nq, [&](int j, int r) {
        Bw[r + 2 * MAXB * j] = G[j * nrow + r];
    });
    for2(mb, mb, [&](int c, int r) {
        double v = G[c * nrow + nq + r];
        for (int l = 0; l < nq; ++l) v -= G[r * nrow + l] * G[c * nrow + l];
        A[r * LD + c] = v;
    });
    wsync();
    for (int j = tid; j < mb; j += WL) {
        const double full = G[j * nrow + nq + j];
        const double proj = A[j * LD + j];
        dsc[j] = (proj > drop * full && proj > 0.0) ? 1.0 / sqrt(proj) : 0.0;
    }
    wsync();
    for2(mb, mb, [&](int c, int r) {
        A[r * LD + c] *= dsc[r] * dsc[c];
    });
    wsync();
    // a block that is already orthonormal (the second pass) has D M D = I + E
    // at rounding level: (I + E)^(-1/2) = I - E/2 + 3/8 E^2 replaces the
    // eigen-decomposition (Z holds that transform, th = 1)
    double emax = 0.0;
    for2(mb, mb, [&](int c, int r) {
        if (r != c) emax = fmax(emax, fabs(A[r * LD + c]));
    });
    emax = wave_max(emax);
    if (emax < 1e-5) {
        auto E = [&](int i, int j) { return i == j ? (dsc[i] > 0.0 ? A[i * LD + i] - 1.0 : 0.0) : A[i * LD + j]; };
        for2(mb, mb, [&](int i, int j) {
            double v = 0.0;
            for (int l = 0; l < mb; ++l) v += E(i, l) * E(l, j);
            Z[i * LD + j] = (i == j ? 1.0 : 0.0) - 0.5 * E(i, j) + 0.375 * v;
        });
        if (tid == 0) {
            int r = 0;
            for (int i = 0; i < mb; ++i)
                if (dsc[i] > 0.0) {
                    keep[r] = i;
                    th[r] = 1.0;
                    ++r;
                }
            nkeep = r;
        }
    } else {
        symeig_wg<LD>(A, Z, mb);
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
    }
    wsync();
    for2(mb, mb, [&](int c, int row) {
        Tw[row + mb * c] = c < nkeep ? dsc[row] * Z[row * LD + keep[c]] / sqrt(th[c]) : 0.0;
    });
    wsync();
}

// --------------------------------------------------------------------------
// Rayleigh-Ritz on span(S), basis size ns (X = first mb columns):
//   G_B -> D G_B D = Z diag(theta) Z^T, keep theta > drop * max(theta),
//   T = D Z_keep theta^-1/2  (T^T G_B T = I; when D G_B D is the identity up
//   to rounding, T = D (I + E)^(-1/2) by its series instead);
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
    __shared__ double GAf[LD * LD], GBf[LD * LD];
    const int tid = wlane();
    const int Eh = ns * (ns + 1) / 2;
    // both Grams as full symmetric matrices in LDS: the dense steps below
    // read them many times, and a global read costs far more than an LDS one
    for2(ns, ns, [&](int i, int j) {
        const int r = i < j ? i : j, c = i < j ? j : i;
        const int e = r * ns - r * (r - 1) / 2 + (c - r);
        GAf[i * LD + j] = Gtri[e];
        GBf[i * LD + j] = Gtri[Eh + e];
    });
    wsync();
    auto GA = [&](int i, int j) { return GAf[i * LD + j]; };
    auto GB = [&](int i, int j) { return GBf[i * LD + j]; };
    double gbmax = 0.0;
    for (int i = 0; i < ns; ++i) gbmax = fmax(gbmax, GB(i, i));
    for (int i = tid; i < ns; i += WL) {
        const double gii = GB(i, i);
        dsc[i] = gii > 1e-24 * gbmax ? 1.0 / sqrt(gii) : 0.0;
    }
    wsync();
    for2(ns, ns, [&](int r, int c) {
        A[r * LD + c] = dsc[r] * GB(r, c) * dsc[c];
    });
    wsync();
    // The basis is orthonormal by construction, so D G_B D = I + E with E
    // at the level of FP32 rounding: then T = D (I + E)^(-1/2) = D (I - E/2 +
    // 3/8 E^2) to FP64 accuracy, with the zero columns (dropped earlier) left
    // out.  Otherwise the general path: an eigen-decomposition with rank
    // dropping.
    double emax = 0.0;
    for2(ns, ns, [&](int r, int c) {
        if (r != c) emax = fmax(emax, fabs(A[r * LD + c]));
    });
    emax = wave_max(emax);
    const bool near_id = emax < 1e-5;
    if (near_id) {
        auto E = [&](int i, int j) { return i == j ? (dsc[i] > 0.0 ? A[i * LD + i] - 1.0 : 0.0) : A[i * LD + j]; };
        for2(ns, ns, [&](int i, int j) {  // Z <- E^2
            double v = 0.0;
            for (int l = 0; l < ns; ++l) v += E(i, l) * E(l, j);
            Z[i * LD + j] = v;
        });
        if (tid == 0) {
            int r = 0;
            for (int i = 0; i < ns; ++i)
                if (dsc[i] > 0.0) keep[r++] = i;
            rank_s = r;
        }
        wsync();
        const int r = rank_s;
        for2(ns, r, [&](int row, int c) {  // T (ns x r)
            const int k = keep[c];
            const double t0 = (row == k ? 1.0 : 0.0) - 0.5 * E(row, k) + 0.375 * Z[row * LD + k];
            Tm[row * LD + c] = dsc[row] * t0;
        });
        wsync();
    } else {
        symeig_wg<LD>(A, Z, ns);
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
        wsync();
        const int r = rank_s;
        for2(ns, r, [&](int row, int c) {  // T (ns x r)
            Tm[row * LD + c] = dsc[row] * Z[row * LD + keep[c]] / sqrt(th[c]);
        });
        wsync();
    }
    const int r = rank_s;
    for2(ns, r, [&](int row, int c) {  // Z <- G_A T
        double s = 0.0;
        for (int l = 0; l < ns; ++l) s += GA(row, l) * Tm[l * LD + c];
        Z[row * LD + c] = s;
    });
    wsync();
    for2(r, r, [&](int row, int c) {  // A <- T^T Z
        double s = 0.0;
        for (int l = 0; l < ns; ++l) s += Tm[l * LD + row] * Z[l * LD + c];
        A[row * LD + c] = s;
    });
    wsync();
    for2(r, r, [&](int row, int c) {
        if (row < c) {
            const double v = 0.5 * (A[row * LD + c] + A[c * LD + row]);
            A[row * LD + c] = v;
            A[c * LD + row] = v;
        }
    });
    wsync();
    symeig_wg<LD>(A, Z, r);
    // NaN ranks as +inf, so that the ranks below always form a permutation
    for (int i = tid; i < r; i += WL) ev[i] = A[i * LD + i] == A[i * LD + i] ? A[i * LD + i] : INFINITY;
    wsync();
    for (int i = tid; i < r; i += WL) {
        const double li = ev[i];
        int rk = 0;
        for (int j = 0; j < r; ++j) rk += (ev[j] < li) || (ev[j] == li && j < i);
        order[rk] = i;
    }
    wsync();
    const int mcol = r < mb ? r : mb;
    // C = T Y[:, order[0..mb)] -> A region (ld MBL) and out->C
    for2(mb, ns, [&](int j, int row) {
        double s = 0.0;
        if (j < mcol) {
            const int yc = order[j];
            for (int l = 0; l < r; ++l) s += Tm[row * LD + l] * Z[l * LD + yc];
        }
        A[row * MBL + j] = s;
        out->C[row + ns * j] = s;
    });
    for (int j = tid; j < mb; j += WL) out->lam[j] = j < mcol ? ev[order[j]] : 0.0;
    if (tid == 0) out->rank = r;
    wsync();
    // ---- P complement: Cwp in the Tm region (ld MBL) ----
    for2(mb, ns, [&](int j, int row) {
        Tm[row * MBL + j] = row < mb ? 0.0 : A[row * MBL + j];
    });
    wsync();
    for (int pass = 0; pass < 2; ++pass) {
        for2(mb, ns, [&](int j, int row) {  // Z <- G_B Cwp
            double s = 0.0;
            for (int l = 0; l < ns; ++l) s += GB(row, l) * Tm[l * MBL + j];
            Z[row * MBL + j] = s;
        });
        wsync();
        for2(mb, mb, [&](int j, int p) {  // h1 <- C^T G_B Cwp
            double s = 0.0;
            for (int l = 0; l < ns; ++l) s += A[l * MBL + p] * Z[l * MBL + j];
            h1[p + MBL * j] = s;
        });
        wsync();
        for2(mb, ns, [&](int j, int row) {  // Cwp <- Cwp - C h1
            double s = Tm[row * MBL + j];
            for (int p = 0; p < mb; ++p) s -= A[row * MBL + p] * h1[p + MBL * j];
            Tm[row * MBL + j] = s;
        });
        wsync();
    }
    // Mp = Cwp^T G_B Cwp
    for2(mb, ns, [&](int j, int row) {
        double s = 0.0;
        for (int l = 0; l < ns; ++l) s += GB(row, l) * Tm[l * MBL + j];
        A[row * MBL + j] = s;
    });
    wsync();
    for2(mb, mb, [&](int j, int p) {
        double s = 0.0;
        for (int l = 0; l < ns; ++l) s += Tm[l * MBL + p] * A[l * MBL + j];
        h1[p + MBL * j] = s;
    });
    wsync();
    for (int j = tid; j < mb; j += WL) {
        const double d = h1[j + MBL * j];
        dsc[j] = d > 1e-24 ? 1.0 / sqrt(d) : 0.0;
    }
    wsync();
    for2(mb, mb, [&](int j, int p) {
        Z[p * LD + j] = dsc[p] * h1[p + MBL * j] * dsc[j];
    });
    wsync();
    symeig_wg<LD>(Z, A, mb);
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
    wsync();
    const int rp = rank_s;
    for2(mb, ns, [&](int j, int row) {  // Cp = Cwp D Zp_keep theta^-1/2
        double s = 0.0;
        if (j < rp) {
            const int zc = keep[j];
            for (int l = 0; l < mb; ++l) s += Tm[row * MBL + l] * dsc[l] * A[l * LD + zc];
            s /= sqrt(th[j]);
        }
        out->Cp[row + ns * j] = s;
    });
    wsync();
}

}  // namespace moto
