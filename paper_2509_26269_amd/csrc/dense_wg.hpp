// dense_wg.hpp -- small dense FP64 steps of the inner layer, each executed by
// one wavefront (the multisection of the lowest-eigenpair solver optionally
// by all waves of the workgroup): the symmetric eigen-solves (the lowest eigenpairs by
// Householder reduction, multisection and inverse iteration; a complete
// decomposition by Householder reduction and implicit QL), the
// orthonormalising transform of a projected block, and the Rayleigh-Ritz step
// with the orthogonal complement for P.  LD is the largest basis size handled
// (the leading dimension of the LDS matrices); LD / 3 is the largest block
// width.
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
// Complete symmetric eigen-decomposition on one wavefront (the general
// Gram path of the Rayleigh-Ritz step, which needs every eigenpair; the
// other dense steps need only the lowest ones and use symeig_low below):
// Householder reduction to tridiagonal form with the reflections
// accumulated (lane r owns row r of the matrix and of Z), then the implicit
// QL iteration with Wilkinson shifts on the tridiagonal, its plane rotations
// applied to the columns of Z (Golub & Van Loan, Sections 8.3.1 and 8.3.5).
// The scalar recurrences of the QL sweep are computed by every lane alike,
// so control flow stays uniform.  On return
// diag(A) holds the eigenvalues (in no particular order) and column j of Z
// the eigenvector of A[j][j]; the off-diagonal part of A is left undefined.
// About n^2 short serial steps: one wavefront issues an instruction every
// ~4.6 cycles and waits ~7 for a dependent FP64 result, so the serial
// rotation chain, not arithmetic, sets its time.
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
// The lowest nw eigenpairs of a symmetric n x n matrix on one wavefront (the
// multisection optionally on NWV waves, see below), with every stage spread
// over the lanes instead of one serial sweep:
//  1. Householder reduction to tridiagonal T (lane r keeps row r of the
//     matrix in registers; the reflectors are stored, not accumulated);
//  2. eigenvalues by multisection of T's Sturm sequence: a group of lanes per
//     eigenvalue, each lane counting the eigenvalues below its own point with
//     the three-term recurrence of the leading minors det(T_i - x I), on T
//     scaled by a power of two to norm < 1 (so no overflow; rescaled against
//     underflow); the counts of the group pick the sub-interval;
//  3. eigenvectors of T by one step of inverse iteration (a lane per
//     eigenvalue, Gaussian elimination with partial pivoting, counter-based
//     start vectors), then modified Gram-Schmidt inside each cluster of
//     eigenvalues closer than 1e-3 ||T|| (the clustering rule of LAPACK's
//     stein);
//  4. back-transformation by the stored reflectors (a lane per vector).
// (Golub & Van Loan, Sections 8.3.1, 8.4.1 and 8.2.2.)  A (leading
// dimension lda) is destroyed: its storage holds the reflectors, which needs
// (n - 2) NM <= lda^2.  On return w[j] and column j of Z (leading dimension
// ldz) hold the j-th smallest eigenpair, j < min(nw, n), ascending.  A
// non-finite entry of A gives NaN eigenpairs.  sb: LDS scratch of
// symeig_low_doubles(NM, NWS) doubles; eigenvectors are solved NWS at a time.
// With NWV > 1 all NWV waves of the workgroup (threads 0 .. 64 NWV - 1) call
// it: the multisection then counts at 64 NWV points per round (fewer rounds),
// everything else runs on wave 0, and the waves meet at two workgroup
// barriers; on return only wave 0 has finished the eigenvectors (the others
// return after the multisection).
// --------------------------------------------------------------------------
constexpr int symeig_low_doubles(int nm, int nws) { return 3 * nm * nws + 5 * nm + WL + 2; }

// 1/x to FP64 accuracy: the hardware estimate refined by two Newton steps
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// a double moved across lanes by a DPP pattern (both 32-bit halves)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the wavefront, the same value on every lane, without an LDS round
// trip: partners at xor 1 and xor 2 inside quads, then mirrored lanes inside
// half-rows and rows (each row of 16 then holds its total on every lane),
// then the four row totals added in a fixed order.
__device__ __forceinline__ double wsum_dpp(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (rdlane(v, 0) + rdlane(v, 16)) + (rdlane(v, 32) + rdlane(v, 48));
}

__device__ __forceinline__ double wmax_dpp(double v) {
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    v = fmax(v, dpp_f64<0x140>(v));
    return fmax(fmax(rdlane(v, 0), rdlane(v, 16)), fmax(rdlane(v, 32), rdlane(v, 48)));
}

// number of eigenvalues of the scaled tridiagonal below x: sign changes of
// 1, p_0, ..., p_(n-1) with p_i = (dh_i - x) p_(i-1) - e2s_i p_(i-2)
// (e2s_i: squared off-diagonal between i - 1 and i, e2s_0 = 0); an exact zero
// takes the sign opposite to its predecessor (a tiny negative pivot).  The
// coefficients come from LDS sixteen at a time.  Entries n .. NM-1 are
// padding (dh = 4, e2s = 0: p_i = (4 - x) p_(i-1) keeps the sign for
// |x| <= 1), so the steps of a chunk need no per-step test of i < n.
template <int NM>
__device__ __forceinline__ int sturm_below(const double* dh, const double* e2s, int n, double x) {
    double pp = 0.0, p = 1.0;
    int cnt = 0;
#pragma unroll
    for (int c0 = 0; c0 < NM; c0 += 16) {
        if (c0 < n) {
            // the first 32 coefficients may stay in registers across calls;
            // later chunks are reloaded (bounds the register footprint)
            if (c0 >= 32) asm volatile("" ::: "memory");
            constexpr int QN = 16;
            double dc[QN], ec[QN];
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                dc[q] = c0 + q < NM ? dh[c0 + q] : 4.0;
                ec[q] = c0 + q < NM ? e2s[c0 + q] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                if (c0 + q < NM) {
                    double pn = fma(dc[q] - x, p, -(ec[q] * pp));
                    pn = pn == 0.0 ? -p * 0x1p-52 : pn;
                    cnt += (pn < 0.0) != (p < 0.0);
                    pp = p;
                    p = pn;
                    if ((q & 3) == 3) {
                        const double f = fmax(fabs(p), fabs(pp)) < 0x1p-600 ? 0x1p600 : 1.0;
                        p *= f;
                        pp *= f;
                    }
                }
            }
        }
    }
    return cnt;
}

// z = H_0 H_1 ... H_(n-3) y for the nw vectors in the columns of Z (leading
// dimension ldz), L lanes per vector (L * nw <= 64): lane t of the group of
// vector j holds rows t, t + L, ... in registers, and each reflection's dot
// product is summed over the group by DPP moves (quads, then half-rows).  The
// reflector rows V + k NM are zero outside k + 1 .. n - 1.
template <int NM, int L>
__device__ __forceinline__ void back_reflect_split(const double* V, double* Z, int ldz, int n, int nw) {
    static_assert(L == 4 || L == 8, "quad or half-row groups");
    constexpr int R = (NM + L - 1) / L;
    const int lane = wlane(), j = lane / L, t = lane - j * L;
    const bool act = j < nw;
    double y[R], vn[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int r = t + L * i;
        y[i] = (act && r < n) ? Z[r * ldz + j] : 0.0;
    }
    if (n >= 3) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = t + L * i;
            vn[i] = r < NM ? V[(n - 3) * NM + r] : 0.0;
        }
    }
    for (int k = n - 3; k >= 0; --k) {
        double vc[R];
#pragma unroll
        for (int i = 0; i < R; ++i) vc[i] = vn[i];
        if (k > 0) {  // the next reflector's rows load while this one is applied
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = t + L * i;
                vn[i] = r < NM ? V[(k - 1) * NM + r] : 0.0;
            }
        }
        double d = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i) d = fma(y[i], vc[i], d);
        d += dpp_f64<0xB1>(d);  // quad_perm [1, 0, 3, 2]
        d += dpp_f64<0x4E>(d);  // quad_perm [2, 3, 0, 1]
        if constexpr (L == 8) d += dpp_f64<0x141>(d);  // row_half_mirror: the other quad
        d *= 2.0;
#pragma unroll
        for (int i = 0; i < R; ++i) y[i] = fma(-d, vc[i], y[i]);
    }
    if (act) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = t + L * i;
            if (r < n) Z[r * ldz + j] = y[i];
        }
    }
}

// Multisection for the lowest nw eigenvalues of the scaled tridiagonal (dh,
// e2s as for sturm_below, spectrum inside (-1, 1)): g lanes per eigenvalue,
// a group inside one wave, each round cutting the bracket into g + 1 parts
// by the counts of the group; lamh[j] <- midpoint of the final bracket of the
// j-th smallest.  With NWV > 1 the NWV waves of the workgroup call it
// together and share the eigenvalues (more lanes per eigenvalue, fewer
// rounds).
template <int NM, int NWV>
__device__ __forceinline__ void multisect(const double* dh, const double* e2s, int n, int nw, double* lamh) {
    const int lane = wlane();
    const int gt = NWV > 1 ? (int)threadIdx.x : lane;
    int g = 1;
    while (2 * g * nw <= WL * NWV && g < (NWV > 1 ? 32 : 16)) g *= 2;
    // (g + 1)^-rounds < 2^-55
    const int rounds = g == 1 ? 56 : g == 2 ? 36 : g == 4 ? 25 : g == 8 ? 19 : (NWV == 1 || g == 16) ? 15 : 12;
    const int jg = gt / g, t = gt - jg * g;
    const int jw = jg < nw ? jg : nw - 1;
    const double ig1 = 1.0 / (double)(g + 1);
    const unsigned long long gm = (g == 64 ? ~0ull : ((1ull << g) - 1ull)) << (NWV > 1 ? lane - t : jg * g);
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < rounds; ++it) {
        const double wd = hi - lo;
        const int c = sturm_below<NM>(dh, e2s, n, lo + wd * ((double)(t + 1) * ig1));
        const int ts = __popcll(__ballot(c <= jw) & gm) - 1;  // last point with <= j eigenvalues below
        const double nlo = ts < 0 ? lo : lo + wd * ((double)(ts + 1) * ig1);
        const double nhi = ts + 1 >= g ? hi : lo + wd * ((double)(ts + 2) * ig1);
        lo = nlo;
        hi = nhi;
    }
    if (t == 0 && jg < nw) lamh[jg] = 0.5 * (lo + hi);
}

// all waves of a workgroup (NWV > 1), else the one calling wave
template <int NWV>
__device__ __forceinline__ void waves_sync() {
    if constexpr (NWV > 1)
        __syncthreads();
    else
        wsync();
}

template <int NM, int NWS, int NWV = 1>
__device__ __forceinline__ void symeig_low_nm(double* A, int lda, double* Z, int ldz, int n, int nw, double* w,
                                              double* sb) {
    static_assert(NWV == 1 || NWV == 2 || NWV == 4, "one, two or four waves");
    const int lane = wlane();
    double* U0 = sb;  // per eigenvector slot: inverse pivots, then the two superdiagonals of U
    double* U1 = U0 + NM * NWS;
    double* U2 = U1 + NM * NWS;
    double* dh = U2 + NM * NWS;
    double* eh = dh + NM;
    double* e2s = eh + NM;
    double* bc = e2s + NM;
    double* hw = bc + NM;
    double* lamh = hw + NM;
    if constexpr (NWV > 1) {
        // waves 1 .. NWV-1: only the multisection (after wave 0's reduction)
        if (threadIdx.x >= WL) {
            __syncthreads();
            if (lamh[WL] != 0.0) return;  // non-finite input
            multisect<NM, NWV>(dh, e2s, n, nw < n ? nw : n, lamh);
            __syncthreads();
            return;
        }
    }
    // ---- 1. tridiagonalisation, lane r holding row r ----
    double a[NM];
    bool fin = true;
#pragma unroll
    for (int c = 0; c < NM; ++c) {
        a[c] = (lane < n && c < n) ? A[lane * lda + c] : 0.0;
        fin = fin && (fabs(a[c]) <= 1.7976931348623157e308);
    }
    if (__ballot(!fin) != 0ull) {
        const int nv = nw < n ? nw : n;
        if (lane < nv) {
            w[lane] = NAN;
            for (int r = 0; r < n; ++r) Z[r * ldz + lane] = NAN;
        }
        wsync();
        if constexpr (NWV > 1) {
            if (lane == 0) lamh[WL] = 1.0;
            __syncthreads();
        }
        return;
    }
    wsync();  // A's storage takes the reflectors from here on: row k at V + k NM
    double* V = A;
    for (int k = 0; k + 2 < n; ++k) {
        if (lane == k) {
#pragma unroll
            for (int c = 0; c < NM; ++c) bc[c] = a[c];
        }
        wsync();
        const double x = (lane > k && lane < n) ? bc[lane] : 0.0;
        const double x0 = bc[k + 1];
        const double x2 = wsum_dpp(x * x);
        double v = 0.0, alpha = 0.0;
        if (x2 > 0.0) {
            const double nx = sqrt(x2);
            alpha = x0 >= 0.0 ? -nx : nx;
            // |x - alpha e|^2 = 2 (|x|^2 - alpha x0) > 0
            v = (x - (lane == k + 1 ? alpha : 0.0)) * rsqrt_nr(2.0 * (x2 - alpha * x0));
        }
        if (lane < NM) V[k * NM + lane] = v;
        if (lane == 0) eh[k] = alpha;
        wsync();
        if (x2 > 0.0) {
            // A <- H A H = A - 2 (v w^T + w v^T), p = A v, w = p - (v.p) v;
            // columns <= k (v is zero there) are never read again and skipped
            const double* vk = V + k * NM;
            double pa[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c0 = 0; c0 < NM; c0 += 8)
                if (c0 + 8 > k + 1) {
                    if constexpr (NM > 32) asm volatile("" ::: "memory");
#pragma unroll
                    for (int c = c0; c < c0 + 8; ++c) pa[c & 3] = fma(a[c], vk[c], pa[c & 3]);
                }
            const double p = (pa[0] + pa[1]) + (pa[2] + pa[3]);
            const double wv = p - wsum_dpp(p * v) * v;
            if (lane < NM) hw[lane] = wv;
            wsync();
#pragma unroll
            for (int c0 = 0; c0 < NM; c0 += 8)
                if (c0 + 8 > k + 1) {
                    // one chunk of broadcast operands live at a time (the
                    // scheduler would otherwise hoist all 2 NM of them)
                    if constexpr (NM > 32) asm volatile("" ::: "memory");
#pragma unroll
                    for (int c = c0; c < c0 + 8; ++c) a[c] -= 2.0 * (v * hw[c] + wv * vk[c]);
                }
        }
        wsync();
    }
    double dr = 0.0, sub = 0.0;
#pragma unroll
    for (int c = 0; c < NM; ++c) {
        dr = c == lane ? a[c] : dr;
        sub = c + 1 == lane ? a[c] : sub;
    }
    if (n >= 2 && lane == n - 1) eh[n - 2] = sub;  // the last subdiagonal entry
    wsync();
    const double er = lane + 1 < n ? eh[lane] : 0.0;
    const double el = (lane >= 1 && lane < n) ? eh[lane - 1] : 0.0;
    // power-of-two scale above the Gershgorin bound: ||T / s|| < 1
    const double gb = wmax_dpp(lane < n ? fabs(dr) + fabs(er) + fabs(el) : 0.0);
    int ex = 0;
    (void)frexp(gb, &ex);
    const double s = gb > 0.0 ? ldexp(1.0, ex) : 1.0, is = 1.0 / s;
    wsync();
    if (lane < NM) {
        dh[lane] = lane < n ? dr * is : 4.0;  // padding for sturm_below
        eh[lane] = er * is;
        e2s[lane] = (el * is) * (el * is);
    }
    wsync();
    if constexpr (NWV > 1) {
        if (lane == 0) lamh[WL] = 0.0;
        __syncthreads();
    }
    // ---- 2. multisection ----
    if (nw > n) nw = n;
    multisect<NM, NWV>(dh, e2s, n, nw, lamh);
    waves_sync<NWV>();
    // ---- 3. inverse iteration, NWS eigenvalues at a time; vector j in column j of Z ----
    constexpr double pmin = 0x1p-52;
    for (int j0 = 0; j0 < nw; j0 += NWS) {
        const int sl = lane - j0;
        if (sl >= 0 && sl < NWS && lane < nw) {
            const double lm = lamh[lane];
            const uint64_t seed = 0x5EED0000ull + (uint64_t)lane;
            double scale = 1.0;
            // one solve: lambda is exact to rounding, so the wanted component
            // grows by ~1 / (eps ||T||) and any other by 1 / gap; what is left
            // inside a cluster is removed below
            {
                auto rhs = [&](int i) { return 2.0 * splitmix_uniform(seed, (uint64_t)i) - 1.0; };
                // forward elimination with row interchanges; the current row
                // (r0, r1) sits at columns (i, i + 1), right-hand side cr
                double r0 = dh[0] - lm, r1 = eh[0], cr = rhs(0);
                for (int c0 = 0; c0 + 1 < n; c0 += 8) {
                    double sd[8], nd[8], ne[8], bn[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int i = c0 + q;
                        const bool ok = i + 1 < n;
                        sd[q] = ok ? eh[i] : 0.0;
                        nd[q] = ok ? dh[i + 1] : 0.0;
                        ne[q] = ok ? eh[i + 1] : 0.0;
                        bn[q] = ok ? rhs(i + 1) : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int i = c0 + q;
                        if (i + 1 < n) {
                            const double d1 = nd[q] - lm;
                            const bool sw = fabs(sd[q]) > fabs(r0) && fabs(sd[q]) > pmin;
                            const double iv = rcp_nr(sw ? sd[q] : (fabs(r0) > pmin ? r0 : pmin));
                            const double m = (sw ? r0 : sd[q]) * iv;
                            U0[i * NWS + sl] = iv;
                            U1[i * NWS + sl] = sw ? d1 : r1;
                            U2[i * NWS + sl] = sw ? ne[q] : 0.0;
                            Z[i * ldz + lane] = sw ? bn[q] : cr;
                            const double n0 = sw ? r1 - m * d1 : d1 - m * r1;
                            const double n1 = sw ? -m * ne[q] : ne[q];
                            cr = sw ? cr - m * bn[q] : bn[q] - m * cr;
                            r0 = n0;
                            r1 = n1;
                        }
                    }
                }
                U0[(n - 1) * NWS + sl] = rcp_nr(fabs(r0) > pmin ? r0 : pmin);
                U1[(n - 1) * NWS + sl] = 0.0;
                U2[(n - 1) * NWS + sl] = 0.0;
                Z[(n - 1) * ldz + lane] = cr;
                // back substitution, eight rows per LDS round trip
                double x1 = 0.0, x2 = 0.0, ss = 0.0;
                for (int c1 = n - 1; c1 >= 0; c1 -= 8) {
                    double u0[8], u1[8], u2[8], yy[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int i = c1 - q;
                        const bool ok = i >= 0;
                        u0[q] = ok ? U0[i * NWS + sl] : 0.0;
                        u1[q] = ok ? U1[i * NWS + sl] : 0.0;
                        u2[q] = ok ? U2[i * NWS + sl] : 0.0;
                        yy[q] = ok ? Z[i * ldz + lane] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int i = c1 - q;
                        if (i >= 0) {
                            const double xi = (yy[q] - u1[q] * x1 - u2[q] * x2) * u0[q];
                            Z[i * ldz + lane] = xi;
                            ss = fma(xi, xi, ss);
                            x2 = x1;
                            x1 = xi;
                        }
                    }
                }
                scale = rsqrt_nr(ss);
            }
            for (int i = 0; i < n; ++i) Z[i * ldz + lane] *= scale;
        }
        wsync();
    }
    // ---- modified Gram-Schmidt inside clusters (consecutive gaps <= 1e-3 of
    // the scaled norm), the own column in registers ----
    double y[NM];
#pragma unroll
    for (int c = 0; c < NM; ++c) y[c] = (lane < nw && c < n) ? Z[c * ldz + lane] : 0.0;
    const bool brk = lane < nw && (lane == 0 || lamh[lane] - lamh[lane - 1] > 1e-3);
    const unsigned long long bm = __ballot(brk) | (nw < WL ? (~0ull << nw) : 0ull);
    auto normalize = [&]() {
        double q4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < NM; ++c) q4[c & 3] = fma(y[c], y[c], q4[c & 3]);
        const double sc = rsqrt_nr((q4[0] + q4[1]) + (q4[2] + q4[3]));
#pragma unroll
        for (int c = 0; c < NM; ++c) y[c] *= sc;
    };
    for (int i = 0; i + 1 < nw; ++i) {
        if ((bm >> (i + 1)) & 1ull) continue;  // nothing after i in its cluster
        if (lane == i) {
            if (!brk) normalize();
#pragma unroll
            for (int c = 0; c < NM; ++c) bc[c] = y[c];
        }
        wsync();
        const unsigned long long between =
            lane > i ? ((~0ull << (i + 1)) & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull))) : 0ull;
        if (lane > i && lane < nw && (bm & between) == 0ull) {
            double q4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < NM; ++c) {
                if (NM > 32 && (c & 7) == 0) asm volatile("" ::: "memory");
                q4[c & 3] = fma(bc[c], y[c], q4[c & 3]);
            }
            const double cf = (q4[0] + q4[1]) + (q4[2] + q4[3]);
#pragma unroll
            for (int c = 0; c < NM; ++c) {
                if (NM > 32 && (c & 7) == 0) asm volatile("" ::: "memory");
                y[c] = fma(-cf, bc[c], y[c]);
            }
        }
        wsync();
    }
    if (lane > 0 && lane < nw && !brk) normalize();
    // ---- 4. back-transformation: z = H_0 H_1 ... H_(n-3) y ----
    if (nw <= 16) {
        // up to 16 vectors: through LDS to L lanes per vector
        if (lane < nw) {
#pragma unroll
            for (int c = 0; c < NM; ++c)
                if (c < n) Z[c * ldz + lane] = y[c];
        }
        wsync();
        if (nw <= 8)
            back_reflect_split<NM, 8>(V, Z, ldz, n, nw);
        else
            back_reflect_split<NM, 4>(V, Z, ldz, n, nw);
        if (lane < nw) w[lane] = lamh[lane] * s;
        wsync();
        return;
    }
    for (int k = n - 3; k >= 0; --k) {
        const double* vk = V + k * NM;
        double q4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c0 = 0; c0 < NM; c0 += 8)
            if (c0 + 8 > k + 1) {
                if constexpr (NM > 32) asm volatile("" ::: "memory");
#pragma unroll
                for (int c = c0; c < c0 + 8; ++c) q4[c & 3] = fma(y[c], vk[c], q4[c & 3]);
            }
        const double dt = 2.0 * ((q4[0] + q4[1]) + (q4[2] + q4[3]));
#pragma unroll
        for (int c0 = 0; c0 < NM; c0 += 8)
            if (c0 + 8 > k + 1) {
                if constexpr (NM > 32) asm volatile("" ::: "memory");
#pragma unroll
                for (int c = c0; c < c0 + 8; ++c) y[c] = fma(-dt, vk[c], y[c]);
            }
    }
    if (lane < nw) {
#pragma unroll
        for (int c = 0; c < NM; ++c)
            if (c < n) Z[c * ldz + lane] = y[c];
        w[lane] = lamh[lane] * s;
    }
    wsync();
}

// Dispatch on the register-array bound NM >= n, in buckets of 8 above 16 (16,
// 24, 32, 40, 48, 64) up to NMAX (default: the largest the leading dimension
// LD allows; callers whose n is known to be small pass a smaller NMAX and get
// fewer buckets).  The LDS scratch is shared by the buckets.  Same contract as
// symeig_low_nm with lda = ldz = LD.
template <int LD, int NWS, int NMAX = ((LD - 1 + 15) / 16) * 16, int NWV = 1>
__device__ __forceinline__ void symeig_low(double* A, double* Z, int n, int nw, double* w) {
    static_assert(NMAX % 16 == 0 && NMAX <= WL, "one lane per row, buckets of 16 at the top");
    __shared__ double sb[symeig_low_doubles(NMAX, NWS)];
    if (n <= 0 || nw <= 0) return;
    if (n <= 16 || NMAX == 16) {
        symeig_low_nm<16, NWS, NWV>(A, LD, Z, LD, n, nw, w, sb);
        return;
    }
    if constexpr (NMAX >= 32) {
        if (n <= 24) {
            symeig_low_nm<24, NWS, NWV>(A, LD, Z, LD, n, nw, w, sb);
            return;
        }
        if (n <= 32 || NMAX == 32) {
            symeig_low_nm<32, NWS, NWV>(A, LD, Z, LD, n, nw, w, sb);
            return;
        }
    }
    if constexpr (NMAX >= 48) {
        if (n <= 40) {
            symeig_low_nm<40, NWS, NWV>(A, LD, Z, LD, n, nw, w, sb);
            return;
        }
        if (n <= 48 || NMAX == 48) {
            symeig_low_nm<48, NWS, NWV>(A, LD, Z, LD, n, nw, w, sb);
            return;
        }
    }
    if constexpr (NMAX >= 64) symeig_low_nm<64, NWS, NWV>(A, LD, Z, LD, n, nw, w, sb);
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
__device__ bool orth_small_body(int mb, int nq, double drop, const double* G, double* Bw, double* Tw);

// --------------------------------------------------------------------------
// D = A B on one wavefront with FP64 16x16x4 matrix-core products.  Elements
// are read through fa(i, k) (i < M, k < K) and fb(k, j) (j < N) at clamped
// in-range indices (zero outside), so every lane issues the same loads, and
// handed to fd(i, j, value).  Lane l of one product supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] and receives D[l / 16 + 4 q][l % 16] in element q.
// Call with the whole wave.
//
// A dependent FP64 product waits ~190 cycles for its accumulator while the
// matrix pipe takes a new one every ~64, so the body keeps at least three
// accumulation chains in flight: every 16 x 16 tile of D at once (TM x TN
// chains, tile counts fixed at compile time so the accumulators stay in
// their registers) and, when there are fewer than three tiles, the K range
// split into interleaved phases summed at the end.
// --------------------------------------------------------------------------
typedef double wd4 __attribute__((ext_vector_type(4)));

template <int TM, int TN, class FA, class FB, class FD>
__device__ __forceinline__ void wave_gemm_tiles(int M, int N, int K, FA&& fa, FB&& fb, FD&& fd) {
    constexpr int T = TM * TN;
    constexpr int S = T >= 3 ? 1 : (T == 2 ? 2 : 3);
    const int lane = wlane(), lr = lane & 15, lk = lane >> 4;
    int arow[TM], bcol[TN];
    bool aok[TM], bok[TN];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
        const int r = 16 * t + lr;
        aok[t] = r < M;
        arow[t] = aok[t] ? r : M - 1;
    }
#pragma unroll
    for (int t = 0; t < TN; ++t) {
        const int c = 16 * t + lr;
        bok[t] = c < N;
        bcol[t] = bok[t] ? c : N - 1;
    }
    wd4 acc[S][TM][TN];
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[p][i][j] = wd4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4 * S) {
#pragma unroll
        for (int p = 0; p < S; ++p) {
            const int k = k0 + 4 * p + lk;
            const bool kok = k < K;
            const int kc = kok ? k : K - 1;
            double a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const double v = fa(arow[i], kc);
                a[i] = (aok[i] && kok) ? v : 0.0;
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const double v = fb(kc, bcol[j]);
                b[j] = (bok[j] && kok) ? v : 0.0;
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[p][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[p][i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            wd4 d = acc[0][i][j];
#pragma unroll
            for (int p = 1; p < S; ++p) d += acc[p][i][j];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 16 * i + lk + 4 * q, c = 16 * j + lr;
                if (r < M && c < N) fd(r, c, d[q]);
            }
        }
}

// Entry: TMX and TNX bound the tile counts of D (M <= 16 TMX, N <= 16 TNX).
// A product with TMX = TNX runs on a square tile grid of side
// max(ceil(M / 16), ceil(N / 16)), one with TNX = 1 (or TMX = 1) on a
// column (row) of tiles; only those shapes are compiled.
template <int TMX, int TNX, class FA, class FB, class FD>
__device__ __forceinline__ void wave_gemm(int M, int N, int K, FA&& fa, FB&& fb, FD&& fd) {
    static_assert(TMX >= 1 && TNX >= 1 && TMX <= 4 && TNX <= 4 && (TMX == TNX || TMX == 1 || TNX == 1),
                  "square, column or row tile grids");
    if (M > 0 && N > 0) {
        const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
        if constexpr (TMX == 1 && TNX == 1) {
            wave_gemm_tiles<1, 1>(M, N, K, fa, fb, fd);
        } else if constexpr (TNX == 1) {
            if (tm <= 1) wave_gemm_tiles<1, 1>(M, N, K, fa, fb, fd);
            else if (TMX == 2 || tm == 2) wave_gemm_tiles<(TMX < 2 ? TMX : 2), 1>(M, N, K, fa, fb, fd);
            else if (TMX == 3 || tm == 3) wave_gemm_tiles<(TMX < 3 ? TMX : 3), 1>(M, N, K, fa, fb, fd);
            else wave_gemm_tiles<TMX, 1>(M, N, K, fa, fb, fd);
        } else if constexpr (TMX == 1) {
            if (tn <= 1) wave_gemm_tiles<1, 1>(M, N, K, fa, fb, fd);
            else if (TNX == 2 || tn == 2) wave_gemm_tiles<1, (TNX < 2 ? TNX : 2)>(M, N, K, fa, fb, fd);
            else if (TNX == 3 || tn == 3) wave_gemm_tiles<1, (TNX < 3 ? TNX : 3)>(M, N, K, fa, fb, fd);
            else wave_gemm_tiles<1, TNX>(M, N, K, fa, fb, fd);
        } else {
            const int t = tm > tn ? tm : tn;
            if (t <= 1) wave_gemm_tiles<1, 1>(M, N, K, fa, fb, fd);
            else if (TMX == 2 || t == 2) wave_gemm_tiles<2, 2>(M, N, K, fa, fb, fd);
            else if (TMX == 3 || t == 3) wave_gemm_tiles<(TMX < 3 ? TMX : 3), (TMX < 3 ? TMX : 3)>(M, N, K, fa, fb, fd);
            else wave_gemm_tiles<TMX, TMX>(M, N, K, fa, fb, fd);
        }
    }
    wsync();
}

// Lanes i < n with pred(i) set, in increasing order, into list[]; returns
// their count (n <= 64).
template <class P>
__device__ __forceinline__ int wave_compact(int n, P&& pred, int* list) {
    const int lane = wlane();
    const bool on = lane < n && pred(lane);
    const unsigned long long m = __ballot(on);
    if (on) list[__popcll(m & ((1ull << lane) - 1ull))] = lane;
    wsync();
    return __popcll(m);
}

// --------------------------------------------------------------------------
// Inverse Cholesky factor on one wavefront, the fast path of the small
// orthonormalising transforms: for a symmetric positive definite n x n
// matrix M with unit diagonal (n <= 16, in A with leading dimension LD),
// M = R^T R and Z <- R^-1 (upper triangular), so that Y R^-1 has orthonormal
// columns when M = Y^T Y.  Returns false, leaving Z undefined, as soon as a
// pivot is not above tau (M is then too close to singular for this path and
// the caller falls back to the eigen-decomposition with rank dropping).  A is
// overwritten by the factor.  (Golub & Van Loan, Section 4.2.)
// --------------------------------------------------------------------------
template <int LD>
__device__ __forceinline__ bool chol_inv_wg(double* A, double* Z, int n, double tau, double* minpiv = nullptr) {
    const int lane = wlane();
    double dmin = INFINITY;
    for (int j = 0; j < n; ++j) {
        const double d = A[j * LD + j];
        if (!(d > tau)) return false;
        dmin = fmin(dmin, d);
        const double id = 1.0 / d;
        // trailing update with the unscaled column j, then its scaling
        for2(n - j - 1, n - j - 1, [&](int a, int b) {
            const int i = j + 1 + a, k = j + 1 + b;
            A[i * LD + k] -= A[i * LD + j] * A[k * LD + j] * id;
        });
        wsync();
        const double r = sqrt(d), ir = 1.0 / r;
        if (lane > j && lane < n) A[lane * LD + j] *= ir;
        if (lane == j) A[j * LD + j] = r;
        wsync();
    }
    // lane q: column q of L^-1 by forward substitution (L = R^T in the lower
    // triangle of A); R^-1 = (L^-1)^T, so that column is row q of R^-1
    if (lane < n) {
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i < n) {
                double v = i == lane ? 1.0 : 0.0;
#pragma unroll
                for (int k = 0; k < i; ++k) v -= A[i * LD + k] * x[k];
                x[i] = i < lane ? 0.0 : v / A[i * LD + i];
            }
        }
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (c < n) Z[lane * LD + c] = x[c];
    }
    wsync();
    if (minpiv) *minpiv = dmin;
    return true;
}

template <int LD>
__device__ bool orth_small_body(int mb, int nq, double drop, const double* G, double* Bw, double* Tw) {
    // G is read many times below: it is first copied to LDS
    constexpr int MBL = LD / 3;
    __shared__ double A[MBL * LD];
    __shared__ double Z[MBL * LD];
    __shared__ double dsc[MBL], th[MBL], thv[MBL];
    __shared__ int keep[MBL];
    __shared__ double Gl[LD * MBL];
    __shared__ double Mq[MBL * MBL];
    const int tid = wlane();
    const int nrow = nq + mb;
#pragma unroll 8  // several global loads in flight per lane
    for (int i = tid; i < nrow * mb; i += WL) Gl[i] = G[i];
    wsync();
    G = Gl;
    for2(mb, nq, [&](int j, int r) {
        Bw[r + 2 * MAXB * j] = G[j * nrow + r];
    });
    // M = Y^T Y - B^T B with B = Q^T Y (B[l][c] = G[c nrow + l]); B^T B kept
    wave_gemm<1, 1>(mb, mb, nq, [&](int r, int l) { return G[r * nrow + l]; }, [&](int l, int c) { return G[c * nrow + l]; },
              [&](int r, int c, double v) {
                  Mq[r * MBL + c] = v;
                  A[r * LD + c] = G[c * nrow + nq + r] - v;
              });
    double kept = 1.0;  // smallest fraction of a column's squared norm left by the projection
    if (tid < mb) {
        const double full = G[tid * nrow + nq + tid];
        const double proj = A[tid * LD + tid];
        dsc[tid] = (proj > drop * full && proj > 0.0) ? 1.0 / sqrt(proj) : 0.0;
        kept = proj > 0.0 && full > 0.0 ? proj / full : 0.0;
    }
    kept = -wmax_dpp(-kept);
    wsync();
    double emax = 0.0;
    for2(mb, mb, [&](int c, int r) {
        const double v = A[r * LD + c] * dsc[r] * dsc[c];
        A[r * LD + c] = v;
        if (r != c) emax = fmax(emax, fabs(v));
    });
    wsync();
    // a block that is already orthonormal (the second pass) has D M D = I + E
    // at rounding level: (I + E)^(-1/2) = I - E/2 + 3/8 E^2 replaces the
    // eigen-decomposition (Z holds that transform, th = 1)
    int nkeep;
    double minpiv = 0.0;
    bool settled = false;  // one pass suffices (see the Cholesky branch)
    if (wmax_dpp(emax) < 1e-5) {
        if (tid < mb) A[tid * LD + tid] = dsc[tid] > 0.0 ? A[tid * LD + tid] - 1.0 : 0.0;  // E in place
        nkeep = wave_compact(mb, [&](int i) { return dsc[i] > 0.0; }, keep);
        if (tid < nkeep) th[tid] = 1.0;
        wave_gemm<1, 1>(mb, mb, mb, [&](int i, int l) { return A[i * LD + l]; }, [&](int l, int j) { return A[l * LD + j]; },
                  [&](int i, int j, double v) {
                      Z[i * LD + j] = (i == j ? 1.0 : 0.0) - 0.5 * A[i * LD + j] + 0.375 * v;
                  });
    } else if (chol_inv_wg<LD>(A, Z, mb, 1e-6, &minpiv)) {
        // well conditioned: T = D R^-1 spans the same space (Rayleigh-Ritz
        // does not depend on which orthonormal basis of it is taken)
        nkeep = mb;
        settled = minpiv > 0.1 && kept > 0.25;
        if (tid < mb) {
            keep[tid] = tid;
            th[tid] = 1.0;
        }
        wsync();
    } else {
        // rebuild D M D (the factorisation overwrote it) and drop directions
        for2(mb, mb, [&](int c, int r) {
            A[r * LD + c] = (G[c * nrow + nq + r] - Mq[r * MBL + c]) * dsc[r] * dsc[c];
        });
        wsync();
        symeig_low<LD, MBL, 16>(A, Z, mb, mb, thv);
        nkeep = wave_compact(mb, [&](int i) { return thv[i] > drop; }, keep);
        if (tid < nkeep) th[tid] = thv[keep[tid]];
        wsync();
    }
    for2(mb, mb, [&](int c, int row) {
        Tw[row + mb * c] = c < nkeep ? dsc[row] * Z[row * LD + keep[c]] / sqrt(th[c]) : 0.0;
    });
    wsync();
    return settled;
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
// Writes C, Cp, lam, rank of the control block `out`.  The matrix products
// run on the matrix cores (wave_gemm), the eigenproblems in symeig_low.
// --------------------------------------------------------------------------
template <int LD, int NWV = 1>
__device__ __forceinline__ void rr_body(int mb, int ns, double drop, const double* Gtri, EigCtrl* out) {
    static_assert(LD - 1 <= WL, "one lane per basis column");
    constexpr int MBL = LD / 3;
    static_assert(MBL <= 16, "block width within one tile");
    constexpr int TX = (LD - 1 + 15) / 16;  // tiles along the basis
    __shared__ double A[LD * LD];
    __shared__ double Z[LD * LD];
    __shared__ double Tm[LD * LD];
    __shared__ double dsc[LD], th[LD], ev[LD];
    __shared__ double h1[MBL * MBL];
    __shared__ int keep[LD];
    __shared__ double GAf[LD * LD], GBf[LD * LD];
    __shared__ int shr[2];
    const int tid = wlane();
    const int wave = NWV > 1 ? (int)(threadIdx.x / WL) : 0;
    auto GA = [&](int i, int j) { return GAf[i * LD + j]; };
    auto GB = [&](int i, int j) { return GBf[i * LD + j]; };
    int r = 0, mcol = 0;
    {
        // both Grams as full symmetric matrices in LDS (every wave takes a
        // share): the dense steps below read them many times, and a global
        // read costs far more than an LDS one
        const int Eh = ns * (ns + 1) / 2;
        auto put = [&](int i, int j) {
            const int lo = i < j ? i : j, hi = i < j ? j : i;
            const int e = lo * ns - lo * (lo - 1) / 2 + (hi - lo);
            GAf[i * LD + j] = Gtri[e];
            GBf[i * LD + j] = Gtri[Eh + e];
        };
        if constexpr (NWV > 1) {
            for (int q = (int)threadIdx.x; q < ns * ns; q += NWV * WL) put(q / ns, q % ns);
        } else {
            for2(ns, ns, put);
        }
        waves_sync<NWV>();
    }
    if (wave == 0) {
        const double gbmax = wmax_dpp(tid < ns ? GB(tid, tid) : 0.0);
        if (tid < ns) {
            const double gii = GB(tid, tid);
            dsc[tid] = gii > 1e-24 * gbmax ? 1.0 / sqrt(gii) : 0.0;
        }
        wsync();
        double emax = 0.0;
        for2(ns, ns, [&](int r, int c) {
            const double v = dsc[r] * GB(r, c) * dsc[c];
            A[r * LD + c] = v;
            if (r != c) emax = fmax(emax, fabs(v));
        });
        wsync();
        // The basis is orthonormal by construction, so D G_B D = I + E with E
        // at the level of FP32 rounding: then T = D (I + E)^(-1/2) = D (I - E/2 +
        // 3/8 E^2) to FP64 accuracy, with the zero columns (dropped earlier) left
        // out.  Otherwise the general path: an eigen-decomposition with rank
        // dropping.
        const bool near_id = wmax_dpp(emax) < 1e-5;
        if (near_id) {
            // E in place of D G_B D (zero on the dropped columns)
            if (tid < ns) A[tid * LD + tid] = dsc[tid] > 0.0 ? A[tid * LD + tid] - 1.0 : 0.0;
            r = wave_compact(ns, [&](int i) { return dsc[i] > 0.0; }, keep);
            wave_gemm<TX, TX>(ns, ns, ns, [&](int i, int l) { return A[i * LD + l]; }, [&](int l, int j) { return A[l * LD + j]; },
                      [&](int i, int j, double v) { Z[i * LD + j] = v; });  // Z <- E^2
            for2(ns, r, [&](int row, int c) {  // T (ns x r)
                const int k = keep[c];
                const double t0 = (row == k ? 1.0 : 0.0) - 0.5 * A[row * LD + k] + 0.375 * Z[row * LD + k];
                Tm[row * LD + c] = dsc[row] * t0;
            });
            wsync();
        } else {
            symeig_wg<LD>(A, Z, ns);
            const double tmax = wmax_dpp(tid < ns ? A[tid * LD + tid] : -INFINITY);
            r = wave_compact(ns, [&](int i) { return A[i * LD + i] > drop * tmax; }, keep);
            if (tid < r) th[tid] = A[keep[tid] * LD + keep[tid]];
            wsync();
            for2(ns, r, [&](int row, int c) {  // T (ns x r)
                Tm[row * LD + c] = dsc[row] * Z[row * LD + keep[c]] / sqrt(th[c]);
            });
            wsync();
        }
        wave_gemm<TX, TX>(ns, r, ns, GA, [&](int l, int c) { return Tm[l * LD + c]; },
                  [&](int i, int c, double v) { Z[i * LD + c] = v; });  // Z <- G_A T
        // A <- T^T Z, made exactly symmetric: its upper triangle mirrored as
        // it is stored (the one-wave form keeps a separate averaging pass:
        // the persistent search kernel that inlines it sits at the register
        // limit, and the mirrored store moves part of it to scratch)
        auto TtZ = [&](auto&& store) {
            wave_gemm<TX, TX>(r, r, ns, [&](int i, int l) { return Tm[l * LD + i]; },
                              [&](int l, int c) { return Z[l * LD + c]; }, store);
        };
        if constexpr (NWV > 1) {
            TtZ([&](int i, int c, double v) {
                if (i <= c) {
                    A[i * LD + c] = v;
                    A[c * LD + i] = v;
                }
            });
        } else {
            TtZ([&](int i, int c, double v) { A[i * LD + c] = v; });
            for2(r, r, [&](int row, int c) {
                if (row < c) {
                    const double v = 0.5 * (A[row * LD + c] + A[c * LD + row]);
                    A[row * LD + c] = v;
                    A[c * LD + row] = v;
                }
            });
            wsync();
        }
        mcol = r < mb ? r : mb;
        if (NWV > 1 && tid == 0) {
            shr[0] = r;
            shr[1] = mcol;
        }
    }  // wave 0
    if constexpr (NWV > 1) {
        __syncthreads();
        r = shr[0];
        mcol = shr[1];
    }
    // the mb lowest eigenpairs, ascending (column j of Z); with NWV > 1 every
    // wave takes part in the multisection, the rest is wave 0's
    symeig_low<LD, MBL, ((LD - 1 + 15) / 16) * 16, NWV>(A, Z, r, mcol, ev);
    if (wave != 0) return;
    // C = T Y[:, 0..mb) -> A region (ld MBL) and out->C (zero beyond the rank)
    wave_gemm<TX, 1>(ns, mcol, r, [&](int row, int l) { return Tm[row * LD + l]; }, [&](int l, int j) { return Z[l * LD + j]; },
              [&](int row, int j, double v) {
                  A[row * MBL + j] = v;
                  out->C[row + ns * j] = v;
              });
    for2(mb - mcol, ns, [&](int j, int row) {
        A[row * MBL + mcol + j] = 0.0;
        out->C[row + ns * (mcol + j)] = 0.0;
    });
    if (tid < mb) out->lam[tid] = tid < mcol ? ev[tid] : 0.0;
    if (tid == 0) out->rank = r;
    wsync();
    // ---- P complement: Cwp in the Tm region (ld MBL) ----
    for2(mb, ns, [&](int j, int row) {
        Tm[row * MBL + j] = row < mb ? 0.0 : A[row * MBL + j];
    });
    wsync();
    auto Cw = [&](int l, int j) { return Tm[l * MBL + j]; };
    for (int pass = 0; pass < 2; ++pass) {
        wave_gemm<TX, 1>(ns, mb, ns, GB, Cw, [&](int row, int j, double v) { Z[row * MBL + j] = v; });  // Z <- G_B Cwp
        wave_gemm<1, 1>(mb, mb, ns, [&](int p, int l) { return A[l * MBL + p]; }, [&](int l, int j) { return Z[l * MBL + j]; },
                  [&](int p, int j, double v) { h1[p + MBL * j] = v; });  // h1 <- C^T G_B Cwp
        wave_gemm<TX, 1>(ns, mb, mb, [&](int row, int p) { return A[row * MBL + p]; },
                  [&](int p, int j) { return h1[p + MBL * j]; },
                  [&](int row, int j, double v) { Tm[row * MBL + j] -= v; });  // Cwp <- Cwp - C h1
    }
    // Mp = Cwp^T G_B Cwp
    wave_gemm<TX, 1>(ns, mb, ns, GB, Cw, [&](int row, int j, double v) { A[row * MBL + j] = v; });
    wave_gemm<1, 1>(mb, mb, ns, [&](int p, int l) { return Tm[l * MBL + p]; }, [&](int l, int j) { return A[l * MBL + j]; },
              [&](int p, int j, double v) { h1[p + MBL * j] = v; });
    if (tid < mb) {
        const double d = h1[tid + MBL * tid];
        dsc[tid] = d > 1e-24 ? 1.0 / sqrt(d) : 0.0;
    }
    wsync();
    for2(mb, mb, [&](int j, int p) {
        Z[p * LD + j] = dsc[p] * h1[p + MBL * j] * dsc[j];
    });
    wsync();
    int rp;
    if (chol_inv_wg<LD>(Z, A, mb, 1e-6)) {
        // well conditioned: Cp = Cwp D R^-1 (any orthonormal basis of the span)
        rp = mb;
        if (tid < mb) {
            keep[tid] = tid;
            th[tid] = 1.0;
        }
        wsync();
    } else {
        for2(mb, mb, [&](int j, int p) {
            Z[p * LD + j] = dsc[p] * h1[p + MBL * j] * dsc[j];
        });
        wsync();
        symeig_low<LD, MBL, 16>(Z, A, mb, mb, ev);
        rp = wave_compact(mb, [&](int i) { return ev[i] > drop; }, keep);
        if (tid < rp) th[tid] = 1.0 / sqrt(ev[keep[tid]]);
        wsync();
    }
    // Cp = Cwp D Zp_keep theta^-1/2 (zero beyond the kept rank)
    wave_gemm<TX, 1>(ns, rp, mb, [&](int row, int l) { return Tm[row * MBL + l] * dsc[l]; },
              [&](int l, int j) { return A[l * LD + keep[j]]; },
              [&](int row, int j, double v) { out->Cp[row + ns * j] = v * th[j]; });
    for2(mb - rp, ns, [&](int j, int row) { out->Cp[row + ns * (rp + j)] = 0.0; });
    wsync();
}

}  // namespace moto
