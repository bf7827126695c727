// batched.hip -- batching form: many saddle searches on lattices of uneven
// sizes in ONE persistent launch.  Each 256-thread workgroup runs complete
// searches (Algorithm 1, bilayer-kernel loop, then certification) for the
// lattices assigned to it, largest first, with every step of the path done
// by the workgroup itself:
//   energy/force (tile loop of the shared stencil body),
//   k smallest eigenpairs by the same orthonormal-basis LOBPCG as the
//   one-search path (tile-loop HVP in FP32, FP64 Grams by block reduction,
//   the shared one-workgroup Rayleigh-Ritz and orthonormalisation bodies),
//   the reflected force and the L-BFGS rotation step (two-loop recursion with
//   block reductions), the index-1 certification.
// Searches are independent, so there is no inter-workgroup communication and
// no host round trip until the whole batch is done.  Register arrays of the
// reductions are indexed with compile-time indices only (a runtime index
// would move the whole array to scratch memory).
#include "dense_wg.hpp"
#include "kernels.hpp"
#include "tile_ops.hpp"

namespace moto {

constexpr int BMB = 4;         // LOBPCG block width of the batched solver (k <= 2)
constexpr int BNS = 3 * BMB;   // Rayleigh-Ritz basis size
constexpr int BLD = BNS;       // LDS leading dimension of the dense steps
constexpr int BMEM = 16;       // max L-BFGS memory

using BArgs = BatchArgs;

// per-search workspace (offsets in bytes from the search's base)
struct BLayout {
    size_t F, c64, m32, c32, S, HS, Xs, V, Sm, Ym, G, Gp, dp, d, ctrl, Gsm, total;
};

__host__ __device__ inline size_t bal(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline BLayout batch_layout(int N, int mem) {
    BLayout o;
    size_t p = 0;
    const size_t v64 = bal(sizeof(double) * 3 * (size_t)N);
    o.F = p;
    p += v64;
    o.c64 = p;
    p += bal(sizeof(double) * (size_t)N);
    o.m32 = p;
    p += bal(sizeof(float) * 3 * (size_t)N);
    o.c32 = p;
    p += bal(sizeof(float) * (size_t)N);
    o.S = p;
    p += bal(sizeof(float) * 3 * BMB * 2 * (size_t)N);
    o.HS = p;
    p += bal(sizeof(float) * 3 * BMB * 2 * (size_t)N);
    o.Xs = p;
    p += bal(sizeof(float) * BMB * 3 * (size_t)N);
    o.V = p;
    p += 2 * v64;
    o.Sm = p;
    p += v64 * mem;
    o.Ym = p;
    p += v64 * mem;
    o.G = p;
    p += v64;
    o.Gp = p;
    p += v64;
    o.dp = p;
    p += v64;
    o.d = p;
    p += v64;
    o.ctrl = p;
    p += bal(sizeof(EigCtrl));
    o.Gsm = p;
    p += bal(sizeof(double) * 2 * BNS * (BNS + 1));
    o.total = p;
    return o;
}

size_t batch_search_bytes(int N, int mem) { return batch_layout(N, mem).total; }

// ---------------------------------------------------------------------------
// Block reductions of up to NV values (result broadcast to every thread).
// ---------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double* lds /* [NV][4] */) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) lds[q * 4 + w] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = lds[q * 4] + lds[q * 4 + 1] + lds[q * 4 + 2] + lds[q * 4 + 3];
    __syncthreads();
}

__device__ __forceinline__ double wg_max(double v, double* lds) {
    __syncthreads();
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Search state of one workgroup
// ---------------------------------------------------------------------------
struct BSearch {
    Geo g;
    int N, n2;
    double* m;
    double *F, *c64, *V, *Sm, *Ym, *G, *Gp, *dp, *d;
    float *m32, *c32, *S, *HS, *Xs;
    EigCtrl* ctrl;
    double* Gsm;
};

struct BShared {
    HvpLDS<float, true> hv;
    TileLDS<double> te;
    double red[4 * 160];
    double Cl[BNS * BMB], Cpl[BNS * BMB], lam[BMB], Bw[2 * BMB * BMB], Tw[BMB * BMB];
};

// energy/force at m (FP64): F and c; returns E
__device__ double b_energy(const BArgs& a, const BSearch& s, BShared& sh, bool want_F) {
    Coef<double> k;
    for (int q = 0; q < 3; ++q) k.cJ[q] = a.k.cJ[q];
    k.cD = a.k.cD;
    k.cK = a.k.cK;
    for (int q = 0; q < 3; ++q) k.B[q] = a.k.B[q];
    double v[NPART];
#pragma unroll
    for (int q = 0; q < NPART; ++q) v[q] = 0.0;
    for (int t = 0; t < s.g.tiles; ++t) {
        const int tx0 = (t % s.g.tiles_x) * TX, ty0 = (t / s.g.tiles_x) * TY;
        energy_tile<double>(sh.te, s.g, k, s.m, nullptr, nullptr, s.c64, want_F ? s.F : nullptr, tx0, ty0, v);
    }
    double e[1] = {v[0]};
    wg_sum<1>(e, sh.red);
    return e[0];
}

__device__ void b_hvp(const BArgs& a, const BSearch& s, BShared& sh, const float* W, float* HW) {
    Coef<float> k;
    for (int q = 0; q < 3; ++q) k.cJ[q] = (float)a.k.cJ[q];
    k.cD = (float)a.k.cD;
    k.cK = (float)a.k.cK;
    for (int q = 0; q < 3; ++q) k.B[q] = (float)a.k.B[q];
    for (int t = 0; t < s.g.tiles; ++t) {
        const int tx0 = (t % s.g.tiles_x) * TX, ty0 = (t / s.g.tiles_x) * TY;
        tangent_hvp_tile<float, true>(sh.hv, s.g, k, s.m32, s.c32, nullptr, BMB, W, HW, tx0, ty0);
    }
    __syncthreads();
}

// orthonormalise X (target 0) or W against [X P] (target 1), in place
__device__ void b_orth(const BArgs& a, const BSearch& s, BShared& sh, int target) {
    const int np = s.ctrl->np;
    const int nq = target == 1 ? BMB + np : 0;
    const int t0 = target == 1 ? BMB : 0;
    const int nrow = nq + BMB;
    constexpr int NE = (2 * BMB + BMB) * BMB;  // 48 max
    double acc[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) acc[q] = 0.0;
    for (int r = threadIdx.x; r < s.n2; r += NT) {
        float col[3 * BMB];
#pragma unroll
        for (int c = 0; c < 3 * BMB; ++c) {
            if (c < nq) {
                const int qc = c < BMB ? c : 2 * BMB + (c - BMB);
                col[c] = s.S[(size_t)qc * s.n2 + r];
            } else if (c < nrow) {
                col[c] = s.S[(size_t)(t0 + c - nq) * s.n2 + r];
            }
        }
#pragma unroll
        for (int j = 0; j < BMB; ++j)
#pragma unroll
            for (int i = 0; i < 3 * BMB; ++i)
                if (i < nrow) acc[j * 3 * BMB + i] += (double)col[i] * (double)col[nq + j];
    }
    wg_sum<NE>(acc, sh.red);
    if (threadIdx.x == 0) {
        // static indices only: a runtime index would move acc to scratch
#pragma unroll
        for (int j = 0; j < BMB; ++j)
#pragma unroll
            for (int i = 0; i < 3 * BMB; ++i)
                if (i < nrow) s.Gsm[j * nrow + i] = acc[j * 3 * BMB + i];
    }
    __syncthreads();
    if (threadIdx.x < WL) orth_small_body<BLD + 1>(BMB, nq, a.drop, s.Gsm, s.ctrl->Bw, s.ctrl->Tw);
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * MAXB * BMB; i += NT) {
        const int r = i % (2 * MAXB), j = i / (2 * MAXB);
        if (r < 2 * BMB) sh.Bw[r + 2 * BMB * j] = s.ctrl->Bw[i];
    }
    for (int i = threadIdx.x; i < BMB * BMB; i += NT) sh.Tw[i] = s.ctrl->Tw[i];
    __syncthreads();
    for (int r = threadIdx.x; r < s.n2; r += NT) {
        double q[2 * BMB], u[BMB];
#pragma unroll
        for (int i = 0; i < 2 * BMB; ++i)
            if (i < nq) q[i] = s.S[(size_t)(i < BMB ? i : 2 * BMB + (i - BMB)) * s.n2 + r];
#pragma unroll
        for (int j = 0; j < BMB; ++j) {
            double v = s.S[(size_t)(t0 + j) * s.n2 + r];
#pragma unroll
            for (int i = 0; i < 2 * BMB; ++i)
                if (i < nq) v -= sh.Bw[i + 2 * BMB * j] * q[i];
            u[j] = v;
        }
#pragma unroll
        for (int j = 0; j < BMB; ++j) {
            double v = 0.0;
#pragma unroll
            for (int l = 0; l < BMB; ++l) v += u[l] * sh.Tw[l + BMB * j];
            s.S[(size_t)(t0 + j) * s.n2 + r] = (float)v;
        }
    }
    __syncthreads();
}

// Rows [I0, I1) of the upper triangle of X^T Y (Y = HS for pass 0, S for
// pass 1) into Gsm, FP64 accumulation.  Row blocks keep the accumulators
// within registers.
template <int I0, int I1>
__device__ void b_gram_rows(const BSearch& s, BShared& sh, int ns, int pass) {
    constexpr int NE = (I1 - I0) * (2 * BNS - I0 - I1 + 1) / 2;
    const int Eh = ns * (ns + 1) / 2;
    double acc[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) acc[q] = 0.0;
    for (int r = threadIdx.x; r < s.n2; r += NT) {
        float x[BNS], y[BNS];
#pragma unroll
        for (int c = 0; c < BNS; ++c) {
            x[c] = 0.0f;
            y[c] = 0.0f;
            if (c < ns) {
                if (c >= I0 && c < I1) x[c] = s.S[(size_t)c * s.n2 + r];
                y[c] = pass == 0 ? s.HS[(size_t)c * s.n2 + r] : s.S[(size_t)c * s.n2 + r];
            }
        }
        int e = 0;
#pragma unroll
        for (int i = I0; i < I1; ++i)
#pragma unroll
            for (int j = i; j < BNS; ++j) acc[e++] += (double)x[i] * (double)y[j];
    }
    wg_sum<NE>(acc, sh.red);
    if (threadIdx.x == 0) {
        int e = 0;
#pragma unroll
        for (int i = I0; i < I1; ++i)
#pragma unroll
            for (int j = i; j < BNS; ++j) {
                if (i < ns && j < ns) s.Gsm[pass * Eh + i * ns - i * (i - 1) / 2 + (j - i)] = acc[e];
                ++e;
            }
    }
    __syncthreads();
}

// Rayleigh-Ritz Grams (upper triangles of S^T HS then S^T S) into Gsm
__device__ void b_gram(const BArgs& a, const BSearch& s, BShared& sh, int ns) {
    (void)a;
    for (int pass = 0; pass < 2; ++pass) {
        b_gram_rows<0, 4>(s, sh, ns, pass);
        if (ns > 4) b_gram_rows<4, BNS>(s, sh, ns, pass);
    }
}

// X <- S C, HX <- HS C, P <- S Cp, HP <- HS Cp, W <- HX - X Lam; residual norms
__device__ void b_update(const BArgs& a, const BSearch& s, BShared& sh, int ns, int kk, bool first) {
    for (int i = threadIdx.x; i < ns * BMB; i += NT) {
        sh.Cl[i] = s.ctrl->C[i];
        sh.Cpl[i] = s.ctrl->Cp[i];
    }
    for (int i = threadIdx.x; i < BMB; i += NT) sh.lam[i] = s.ctrl->lam[i];
    __syncthreads();
    const bool has_p = ns > BMB;
    double rs[BMB] = {0.0, 0.0, 0.0, 0.0};
    for (int r = threadIdx.x; r < s.n2; r += NT) {
        float sv[BNS];
#pragma unroll
        for (int i = 0; i < BNS; ++i)
            if (i < ns) sv[i] = s.S[(size_t)i * s.n2 + r];
        double xn[BMB];
#pragma unroll
        for (int j = 0; j < BMB; ++j) {
            double x = 0.0, p = 0.0;
#pragma unroll
            for (int i = 0; i < BNS; ++i)
                if (i < ns) {
                    x += sh.Cl[i + ns * j] * (double)sv[i];
                    p += sh.Cpl[i + ns * j] * (double)sv[i];
                }
            xn[j] = x;
            s.S[(size_t)j * s.n2 + r] = (float)x;
            if (has_p) s.S[(size_t)(2 * BMB + j) * s.n2 + r] = (float)p;
        }
#pragma unroll
        for (int i = 0; i < BNS; ++i)
            if (i < ns) sv[i] = s.HS[(size_t)i * s.n2 + r];
#pragma unroll
        for (int j = 0; j < BMB; ++j) {
            double hx = 0.0, hp = 0.0;
#pragma unroll
            for (int i = 0; i < BNS; ++i)
                if (i < ns) {
                    hx += sh.Cl[i + ns * j] * (double)sv[i];
                    hp += sh.Cpl[i + ns * j] * (double)sv[i];
                }
            s.HS[(size_t)j * s.n2 + r] = (float)hx;
            if (has_p) s.HS[(size_t)(2 * BMB + j) * s.n2 + r] = (float)hp;
            const float w = (float)(hx - sh.lam[j] * xn[j]);
            s.S[(size_t)(BMB + j) * s.n2 + r] = w;
            rs[j] += (double)w * (double)w;
        }
    }
    wg_sum<BMB>(rs, sh.red);
    if (threadIdx.x == 0) {
        EigCtrl* c = s.ctrl;
        bool conv = true, bad = false;
        for (int j = 0; j < BMB; ++j) {
            const double rj = sqrt(rs[j]);
            c->resid[j] = rj;
            if (!isfinite(rj) || !isfinite(c->lam[j])) bad = true;
            if (j < kk && !(rj <= a.eig_tol_abs)) conv = false;
        }
        c->n_hvp += BMB;
        if (!first) {
            c->iters += 1;
            c->np = BMB;
        }
        if (bad) {
            c->status = MOTO_NAN;
            c->done = 1;
        } else if (c->rank < kk) {
            c->status = MOTO_BREAKDOWN;
            c->done = 1;
        } else if (conv) {
            c->status = MOTO_CONVERGED;
            c->done = 1;
        } else if (c->iters >= a.eig_max_iter) {
            c->status = MOTO_NOT_CONVERGED;
            c->done = 1;
        }
    }
    __syncthreads();
}

// k smallest eigenpairs at m; warm: start from the saved block.  Leaves the
// first kk vectors (ambient FP64, unit) in s.V and the block in s.Xs.
__device__ void b_eig(const BArgs& a, const BSearch& s, BShared& sh, int kk, bool warm, unsigned long long seed) {
    const int N = s.N;
    if (threadIdx.x == 0) {
        s.ctrl->done = 0;
        s.ctrl->status = MOTO_NOT_CONVERGED;
        s.ctrl->iters = 0;
        s.ctrl->np = 0;
        s.ctrl->rank = BMB;
        s.ctrl->n_hvp = 0;
    }
    // FP32 spins and c for the HVP; start block in frame coordinates
    for (int i = threadIdx.x; i < N; i += NT) {
        const float mx = (float)s.m[i], my = (float)s.m[N + i], mz = (float)s.m[2 * N + i];
        s.m32[i] = mx;
        s.m32[N + i] = my;
        s.m32[2 * N + i] = mz;
        s.c32[i] = (float)s.c64[i];
        float e1[3], e2[3];
        onb(mx, my, mz, e1, e2);
        for (int j = 0; j < BMB; ++j) {
            float va, vb;
            if (warm) {
                const float x0 = s.Xs[(size_t)j * 3 * N + i], x1 = s.Xs[(size_t)j * 3 * N + N + i],
                            x2 = s.Xs[(size_t)j * 3 * N + 2 * N + i];
                va = e1[0] * x0 + e1[1] * x1 + e1[2] * x2;
                vb = e2[0] * x0 + e2[1] * x1 + e2[2] * x2;
            } else {
                va = (float)splitmix_uniform(seed, (uint64_t)j * 2 * N + i);
                vb = (float)splitmix_uniform(seed, (uint64_t)j * 2 * N + N + i);
            }
            s.S[(size_t)j * s.n2 + i] = va;
            s.S[(size_t)j * s.n2 + N + i] = vb;
        }
    }
    __syncthreads();
    b_orth(a, s, sh, 0);
    b_orth(a, s, sh, 0);
    b_hvp(a, s, sh, s.S, s.HS);
    b_gram(a, s, sh, BMB);
    if (threadIdx.x < WL) rr_body<BLD + 1>(BMB, BMB, a.drop, s.Gsm, s.ctrl);
    __syncthreads();
    b_update(a, s, sh, BMB, kk, true);
    for (int it = 0; it <= a.eig_max_iter + 1; ++it) {
        if (s.ctrl->done) break;
        b_orth(a, s, sh, 1);
        b_orth(a, s, sh, 1);
        b_hvp(a, s, sh, s.S + (size_t)BMB * s.n2, s.HS + (size_t)BMB * s.n2);
        const int ns = 2 * BMB + s.ctrl->np;
        b_gram(a, s, sh, ns);
        if (threadIdx.x < WL) rr_body<BLD + 1>(BMB, ns, a.drop, s.Gsm, s.ctrl);
        __syncthreads();
        b_update(a, s, sh, ns, kk, false);
    }
    // output: ambient block (saved) and the first kk unit vectors
    double nr[BMB] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < N; i += NT) {
        float e1[3], e2[3];
        onb(s.m32[i], s.m32[N + i], s.m32[2 * N + i], e1, e2);
        for (int j = 0; j < BMB; ++j) {
            const float va = s.S[(size_t)j * s.n2 + i], vb = s.S[(size_t)j * s.n2 + N + i];
            for (int c = 0; c < 3; ++c) {
                const float amb = va * e1[c] + vb * e2[c];
                s.Xs[(size_t)j * 3 * N + c * N + i] = amb;
                if (j < kk) {
                    s.V[(size_t)j * 3 * N + c * N + i] = (double)amb;
                    nr[j] += (double)amb * (double)amb;
                }
            }
        }
    }
    wg_sum<BMB>(nr, sh.red);
    for (int j = 0; j < kk; ++j) {
        const double sc = nr[j] > 0.0 ? 1.0 / sqrt(nr[j]) : 0.0;
        for (int i = threadIdx.x; i < 3 * N; i += NT) s.V[(size_t)j * 3 * N + i] *= sc;
    }
    __syncthreads();
}

// One outer step (reflected force, L-BFGS direction, cap, rotation).
// Returns ||F_mmf|| at m; *stopped set when it is <= tau_F (m unchanged).
struct LbfgsHdr {
    int count, head, have_prev;
};

__device__ double b_dot(const double* x, const double* y, int n3, double* red) {
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < n3; i += NT) v[0] += x[i] * y[i];
    wg_sum<1>(v, red);
    return v[0];
}

__device__ double b_step(const BArgs& a, const BSearch& s, BShared& sh, LbfgsHdr& h, int k_reflect, bool* stopped) {
    const int N = s.N, n3 = 3 * N;
    double fr[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < n3; i += NT)
        for (int r = 0; r < k_reflect; ++r) fr[r] += s.F[i] * s.V[(size_t)r * n3 + i];
    wg_sum<2>(fr, sh.red);
    double fn[1] = {0.0};
    for (int i = threadIdx.x; i < n3; i += NT) {
        double v = s.F[i];
        for (int r = 0; r < k_reflect; ++r) v -= 2.0 * fr[r] * s.V[(size_t)r * n3 + i];
        s.G[i] = -v;
        fn[0] += v * v;
    }
    wg_sum<1>(fn, sh.red);
    const double fnorm = sqrt(fn[0]);
    if (!(fnorm > a.tau_F)) {
        *stopped = true;
        return fnorm;
    }
    *stopped = false;
    // transport stored pairs, form the new one
    int slot = -1;
    int c_new = h.count, h_new = h.head;
    if (h.have_prev) {
        if (h.count < a.mem) {
            slot = (h.head + h.count) % a.mem;
            c_new = h.count + 1;
        } else {
            slot = h.head;
            h_new = (h.head + 1) % a.mem;
        }
    }
    for (int i = threadIdx.x; i < N; i += NT) {
        const double mi[3] = {s.m[i], s.m[N + i], s.m[2 * N + i]};
        for (int j = 0; j < c_new; ++j) {
            const int ph = (h_new + j) % a.mem;
            double* Sj = s.Sm + (size_t)ph * n3;
            double* Yj = s.Ym + (size_t)ph * n3;
            if (ph == slot) {
                const double md = mi[0] * s.dp[i] + mi[1] * s.dp[N + i] + mi[2] * s.dp[2 * N + i];
                const double mg = mi[0] * s.Gp[i] + mi[1] * s.Gp[N + i] + mi[2] * s.Gp[2 * N + i];
                for (int c = 0; c < 3; ++c) {
                    Sj[c * N + i] = s.dp[c * N + i] - md * mi[c];
                    Yj[c * N + i] = s.G[c * N + i] - (s.Gp[c * N + i] - mg * mi[c]);
                }
            } else {
                const double ms = mi[0] * Sj[i] + mi[1] * Sj[N + i] + mi[2] * Sj[2 * N + i];
                const double my = mi[0] * Yj[i] + mi[1] * Yj[N + i] + mi[2] * Yj[2 * N + i];
                for (int c = 0; c < 3; ++c) {
                    Sj[c * N + i] -= ms * mi[c];
                    Yj[c * N + i] -= my * mi[c];
                }
            }
        }
    }
    __syncthreads();
    h.count = c_new;
    h.head = h_new;
    // two-loop recursion on q = G (stored in d)
    double sy[BMEM], alph[BMEM];
    int newest = -1;
    for (int j = 0; j < h.count; ++j) {
        const int ph = (h.head + j) % a.mem;
        sy[j] = b_dot(s.Sm + (size_t)ph * n3, s.Ym + (size_t)ph * n3, n3, sh.red);
        if (sy[j] > a.sy_min) newest = j;
    }
    for (int i = threadIdx.x; i < n3; i += NT) s.d[i] = s.G[i];
    __syncthreads();
    for (int j = h.count - 1; j >= 0; --j) {
        if (!(sy[j] > a.sy_min)) continue;
        const int ph = (h.head + j) % a.mem;
        alph[j] = b_dot(s.Sm + (size_t)ph * n3, s.d, n3, sh.red) / sy[j];
        const double* Yj = s.Ym + (size_t)ph * n3;
        for (int i = threadIdx.x; i < n3; i += NT) s.d[i] -= alph[j] * Yj[i];
        __syncthreads();
    }
    double gamma = a.alpha0;
    if (newest >= 0) {
        const int ph = (h.head + newest) % a.mem;
        const double* Yn = s.Ym + (size_t)ph * n3;
        gamma = sy[newest] / b_dot(Yn, Yn, n3, sh.red);
    }
    for (int i = threadIdx.x; i < n3; i += NT) s.d[i] *= gamma;
    __syncthreads();
    for (int j = 0; j < h.count; ++j) {
        if (!(sy[j] > a.sy_min)) continue;
        const int ph = (h.head + j) % a.mem;
        const double beta = b_dot(s.Ym + (size_t)ph * n3, s.d, n3, sh.red) / sy[j];
        const double* Sj = s.Sm + (size_t)ph * n3;
        for (int i = threadIdx.x; i < n3; i += NT) s.d[i] += (alph[j] - beta) * Sj[i];
        __syncthreads();
    }
    // d = -r; reset if not a descent direction for G
    const double dG = -b_dot(s.d, s.G, n3, sh.red);
    const bool reset = !(dG < 0.0);
    if (reset) h.count = 0;
    // project, rotation cap
    double mx = 0.0;
    for (int i = threadIdx.x; i < N; i += NT) {
        double dd[3];
        for (int c = 0; c < 3; ++c) dd[c] = reset ? -a.alpha0 * s.G[c * N + i] : -s.d[c * N + i];
        const double md = s.m[i] * dd[0] + s.m[N + i] * dd[1] + s.m[2 * N + i] * dd[2];
        double n2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            dd[c] -= md * s.m[c * N + i];
            s.d[c * N + i] = dd[c];
            n2 += dd[c] * dd[c];
        }
        mx = fmax(mx, sqrt(n2));
    }
    mx = wg_max(mx, sh.red);
    const double sc = mx > a.theta_max ? a.theta_max / mx : 1.0;
    for (int i = threadIdx.x; i < N; i += NT) {
        double dd[3], mi[3], n2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            dd[c] = sc * s.d[c * N + i];
            mi[c] = s.m[c * N + i];
            n2 += dd[c] * dd[c];
            s.dp[c * N + i] = dd[c];
            s.Gp[c * N + i] = s.G[c * N + i];
        }
        const double th = sqrt(n2);
        if (th > 0.0) {
            const double ct = cos(th), st = sin(th) / th;
            double o[3], on = 0.0;
            for (int c = 0; c < 3; ++c) {
                o[c] = ct * mi[c] + st * dd[c];
                on += o[c] * o[c];
            }
            const double inv = 1.0 / sqrt(on);
            for (int c = 0; c < 3; ++c) s.m[c * N + i] = o[c] * inv;
        }
    }
    h.have_prev = 1;
    __syncthreads();
    return fnorm;
}

__global__ __launch_bounds__(NT) void k_batched_search(BArgs a, double* __restrict__ m_all,
                                                       const int* __restrict__ Ls, const int* __restrict__ order,
                                                       const long long* __restrict__ m_off,
                                                       const long long* __restrict__ ws_off, char* __restrict__ ws,
                                                       moto_search_result* __restrict__ res) {
    __shared__ BShared sh;
    for (int q = blockIdx.x; q < a.n; q += gridDim.x) {
        const int idx = order[q];
        BSearch s;
        const int L = Ls[idx];
        s.g = make_geo(L, L);
        s.N = L * L;
        s.n2 = 2 * s.N;
        s.m = m_all + m_off[idx];
        char* base = ws + ws_off[idx];
        const BLayout o = batch_layout(s.N, a.mem);
        s.F = (double*)(base + o.F);
        s.c64 = (double*)(base + o.c64);
        s.m32 = (float*)(base + o.m32);
        s.c32 = (float*)(base + o.c32);
        s.S = (float*)(base + o.S);
        s.HS = (float*)(base + o.HS);
        s.Xs = (float*)(base + o.Xs);
        s.V = (double*)(base + o.V);
        s.Sm = (double*)(base + o.Sm);
        s.Ym = (double*)(base + o.Ym);
        s.G = (double*)(base + o.G);
        s.Gp = (double*)(base + o.Gp);
        s.dp = (double*)(base + o.dp);
        s.d = (double*)(base + o.d);
        s.ctrl = (EigCtrl*)(base + o.ctrl);
        s.Gsm = (double*)(base + o.Gsm);
        LbfgsHdr h = {0, 0, 0};
        long long n_hvp = 0;
        bool stopped = false, nan = false;
        double fnorm = INFINITY;
        int it = 0;
        const unsigned long long seed = a.seed ^ (0x9E3779B97F4A7C15ull * (unsigned long long)(idx + 1));
        for (it = 0; it <= a.max_outer; ++it) {
            b_energy(a, s, sh, true);
            __syncthreads();
            b_eig(a, s, sh, a.kk, it > 0, seed);
            n_hvp += s.ctrl->n_hvp;
            if (s.ctrl->status == MOTO_NAN) {
                nan = true;
                break;
            }
            if (it == a.max_outer) {
                bool st2;
                BArgs a2 = a;
                a2.tau_F = INFINITY;
                fnorm = b_step(a2, s, sh, h, a.kk < 1 ? 0 : 1, &st2);
                break;
            }
            fnorm = b_step(a, s, sh, h, a.kk < 1 ? 0 : 1, &stopped);
            if (stopped || !isfinite(fnorm)) break;
        }
        // certification at the final point
        b_energy(a, s, sh, true);
        __syncthreads();
        b_eig(a, s, sh, 2, false, seed + 1);
        n_hvp += s.ctrl->n_hvp;
        const double E = b_energy(a, s, sh, false);
        if (threadIdx.x == 0) {
            const double l1 = s.ctrl->lam[0], l2 = s.ctrl->lam[1];
            int status;
            const bool conv = isfinite(fnorm) && fnorm <= a.tau_F;
            if (nan || !isfinite(fnorm) || !isfinite(l1) || !isfinite(l2) || s.ctrl->status == MOTO_NAN)
                status = MOTO_NAN;
            else if (!conv || s.ctrl->status != MOTO_CONVERGED)
                // an unconverged certifying solve only bounds the eigenvalues
                // from above: no SADDLE / HIGHER_INDEX verdict from it
                status = MOTO_NOT_CONVERGED;
            else if (l1 < -a.tau_lam && l2 > a.tau_lam)
                status = MOTO_SADDLE;
            else if (l2 < -a.tau_lam)
                status = MOTO_HIGHER_INDEX;
            else
                status = MOTO_DEGENERATE;
            moto_search_result r;
            r.status = status;
            r.iters = it;
            r.n_hvp = n_hvp;
            r.E = E;
            r.fnorm = fnorm;
            r.lambda1 = l1;
            r.lambda2 = l2;
            res[idx] = r;
        }
        __syncthreads();
    }
}

hipError_t launch_batched_search(const BatchArgs& a, double* m_all, const int* Ls, const int* order,
                                 const long long* m_off, const long long* ws_off, char* ws, moto_search_result* res,
                                 int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_batched_search, dim3(grid), dim3(NT), 0, st, a, m_all, Ls, order, m_off, ws_off, ws, res);
    return hipGetLastError();
}

}  // namespace moto
