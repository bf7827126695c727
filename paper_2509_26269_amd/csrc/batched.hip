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
    const uint8_t* mask;  // active sites of this lattice (null: all)
    int tile;             // tile shape of its lattice loops: BATCH_TILE_32x8 / 16x16 / 64x4
    double *F, *c64, *V, *Sm, *Ym, *G, *Gp, *dp, *d;
    float *m32, *c32, *S, *HS, *Xs;
    EigCtrl* ctrl;
    double* Gsm;
};

constexpr int BRCH = 64;  // rows per staged chunk of the Gram reductions

// LDS of the tile loops for one tile shape (TXV x 256 / TXV)
template <int TXV>
struct BTiles {
    HvpLDS<float, true, TXV> hv;
    TileLDS<double, TXV> te;
};

struct BShared {
    union {  // one search uses one tile shape at a time
        BTiles<32> t32;
        BTiles<16> t16;
        BTiles<64> t64;
    };
    double red[4 * 160];
    float st[2][BNS][BRCH];  // staged rows of two sets of basis columns
    double sy[BMEM], alph[BMEM];  // L-BFGS pair curvatures and two-loop coefficients
    double Cl[BNS * BMB], Cpl[BNS * BMB], lam[BMB], Bw[2 * BMB * BMB], Tw[BMB * BMB];
};

template <int TXV>
__device__ __forceinline__ BTiles<TXV>& b_tiles(BShared& sh) {
    if constexpr (TXV == 32)
        return sh.t32;
    else if constexpr (TXV == 16)
        return sh.t16;
    else
        return sh.t64;
}

// energy/force at m (FP64): F and c; returns E.  Tiles of TXV x 256 / TXV.
template <int TXV>
__device__ __forceinline__ double b_energy_t(const BArgs& a, const BSearch& s, BShared& sh, bool want_F) {
    using SHP = TileShape<TXV>;
    Coef<double> k;
    for (int q = 0; q < 3; ++q) k.cJ[q] = a.k.cJ[q];
    k.cD = a.k.cD;
    k.cK = a.k.cK;
    for (int q = 0; q < 3; ++q) k.B[q] = a.k.B[q];
    double v[NPART];
#pragma unroll
    for (int q = 0; q < NPART; ++q) v[q] = 0.0;
    const int ntx = (s.g.Lx + SHP::X - 1) / SHP::X, nty = (s.g.Ly + SHP::Y - 1) / SHP::Y;
    for (int t = 0; t < ntx * nty; ++t) {
        const int tx0 = (t % ntx) * SHP::X, ty0 = (t / ntx) * SHP::Y;
        energy_tile<double, TXV>(b_tiles<TXV>(sh).te, s.g, k, s.m, s.mask, nullptr, s.c64, want_F ? s.F : nullptr,
                                 tx0, ty0, v);
    }
    double e[1] = {v[0]};
    wg_sum<1>(e, sh.red);
    return e[0];
}

__device__ __forceinline__ double b_energy(const BArgs& a, const BSearch& s, BShared& sh, bool want_F) {
    if (s.tile == BATCH_TILE_16x16) return b_energy_t<16>(a, s, sh, want_F);
    if (s.tile == BATCH_TILE_64x4) return b_energy_t<64>(a, s, sh, want_F);
    return b_energy_t<32>(a, s, sh, want_F);
}

template <int TXV>
__device__ __forceinline__ void b_hvp_t(const BArgs& a, const BSearch& s, BShared& sh, const float* W, float* HW) {
    using SHP = TileShape<TXV>;
    Coef<float> k;
    for (int q = 0; q < 3; ++q) k.cJ[q] = (float)a.k.cJ[q];
    k.cD = (float)a.k.cD;
    k.cK = (float)a.k.cK;
    for (int q = 0; q < 3; ++q) k.B[q] = (float)a.k.B[q];
    const int ntx = (s.g.Lx + SHP::X - 1) / SHP::X, nty = (s.g.Ly + SHP::Y - 1) / SHP::Y;
    for (int t = 0; t < ntx * nty; ++t) {
        const int tx0 = (t % ntx) * SHP::X, ty0 = (t / ntx) * SHP::Y;
        tangent_hvp_tile<float, true, TXV>(b_tiles<TXV>(sh).hv, s.g, k, s.m32, s.c32, s.mask, BMB, W, HW, tx0,
                                           ty0);
    }
    __syncthreads();
}

__device__ __forceinline__ void b_hvp(const BArgs& a, const BSearch& s, BShared& sh, const float* W, float* HW) {
    if (s.tile == BATCH_TILE_16x16)
        b_hvp_t<16>(a, s, sh, W, HW);
    else if (s.tile == BATCH_TILE_64x4)
        b_hvp_t<64>(a, s, sh, W, HW);
    else
        b_hvp_t<32>(a, s, sh, W, HW);
}

// orthonormalise X (target 0) or W against [X P] (target 1), in place
__device__ __forceinline__ void b_orth(const BArgs& a, const BSearch& s, BShared& sh, int target) {
    const int np = s.ctrl->np;
    const int nq = target == 1 ? BMB + np : 0;
    const int t0 = target == 1 ? BMB : 0;
    const int nrow = nq + BMB;
    // Gram entries e = j * nrow + i (staged column i . target column j), one
    // per thread, summed over staged chunks of rows in a fixed order
    const int E = nrow * BMB;
    double acc = 0.0;
    int ei = 0, ej = 0;
    if (threadIdx.x < E) {
        ej = threadIdx.x / nrow;
        ei = threadIdx.x - ej * nrow;
    }
    for (int r0 = 0; r0 < s.n2; r0 += BRCH) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < nrow * BRCH; idx += NT) {
            const int c = idx / BRCH, rr = idx - c * BRCH, r = r0 + rr;
            const int col = c < nq ? (c < BMB ? c : 2 * BMB + (c - BMB)) : t0 + (c - nq);
            sh.st[0][c][rr] = r < s.n2 ? s.S[(size_t)col * s.n2 + r] : 0.0f;
        }
        __syncthreads();
        if (threadIdx.x < E) {
            const float* x = sh.st[0][ei];
            const float* y = sh.st[0][nq + ej];
            double d0 = 0.0, d1 = 0.0;
            for (int rr = 0; rr < BRCH; rr += 2) {
                d0 += (double)x[rr] * (double)y[rr];
                d1 += (double)x[rr + 1] * (double)y[rr + 1];
            }
            acc += d0 + d1;
        }
    }
    if (threadIdx.x < E) s.Gsm[threadIdx.x] = acc;
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

// Rayleigh-Ritz Grams (upper triangles of S^T HS then S^T S) into Gsm: one
// entry per thread, FP64 sums over staged chunks of rows in a fixed order
__device__ __forceinline__ void b_gram(const BArgs& a, const BSearch& s, BShared& sh, int ns) {
    (void)a;
    const int Eh = ns * (ns + 1) / 2, E = 2 * Eh;
    int ei = 0, ej = 0, ew = 0;
    if (threadIdx.x < E) {
        ew = threadIdx.x >= Eh;
        int p = threadIdx.x - ew * Eh, i = 0;
        while (p >= ns - i) {
            p -= ns - i;
            ++i;
        }
        ei = i;
        ej = i + p;
    }
    double acc = 0.0;
    for (int r0 = 0; r0 < s.n2; r0 += BRCH) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < ns * BRCH; idx += NT) {
            const int c = idx / BRCH, rr = idx - c * BRCH, r = r0 + rr;
            const bool in = r < s.n2;
            sh.st[0][c][rr] = in ? s.S[(size_t)c * s.n2 + r] : 0.0f;
            sh.st[1][c][rr] = in ? s.HS[(size_t)c * s.n2 + r] : 0.0f;
        }
        __syncthreads();
        if (threadIdx.x < E) {
            const float* x = sh.st[0][ei];
            const float* y = ew ? sh.st[0][ej] : sh.st[1][ej];
            double d0 = 0.0, d1 = 0.0;
            for (int rr = 0; rr < BRCH; rr += 2) {
                d0 += (double)x[rr] * (double)y[rr];
                d1 += (double)x[rr + 1] * (double)y[rr + 1];
            }
            acc += d0 + d1;
        }
    }
    if (threadIdx.x < E) s.Gsm[threadIdx.x] = acc;
    __syncthreads();
}

// X <- S C, HX <- HS C, P <- S Cp, HP <- HS Cp, W <- HX - X Lam; residual norms
__device__ __forceinline__ void b_update(const BArgs& a, const BSearch& s, BShared& sh, int ns, int kk, bool first) {
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
__device__ __forceinline__ void b_eig(const BArgs& a, const BSearch& s, BShared& sh, int kk, bool warm, unsigned long long seed) {
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
            const bool on = s.mask == nullptr || s.mask[i] != 0;
            s.S[(size_t)j * s.n2 + i] = on ? va : 0.0f;
            s.S[(size_t)j * s.n2 + N + i] = on ? vb : 0.0f;
        }
    }
    __syncthreads();
    // pass -1 orthonormalises and projects the start block alone; each later
    // pass the residual block W against [X P] (one copy of each step's code)
    for (int it = -1; it <= a.eig_max_iter + 1; ++it) {
        const bool first = it < 0;
        if (!first && s.ctrl->done) break;
        b_orth(a, s, sh, first ? 0 : 1);
        b_orth(a, s, sh, first ? 0 : 1);
        const size_t off = first ? 0 : (size_t)BMB * s.n2;
        b_hvp(a, s, sh, s.S + off, s.HS + off);
        const int ns = first ? BMB : 2 * BMB + s.ctrl->np;
        b_gram(a, s, sh, ns);
        if (threadIdx.x < WL) rr_body<BLD + 1>(BMB, ns, a.drop, s.Gsm, s.ctrl);
        __syncthreads();
        b_update(a, s, sh, ns, kk, first);
    }
    // output: ambient block (saved) and the first kk unit vectors
    double nr[BMB] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < N; i += NT) {
        float e1[3], e2[3];
        onb(s.m32[i], s.m32[N + i], s.m32[2 * N + i], e1, e2);
#pragma unroll
        for (int j = 0; j < BMB; ++j) {
            const float va = s.S[(size_t)j * s.n2 + i], vb = s.S[(size_t)j * s.n2 + N + i];
#pragma unroll
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
#pragma unroll
    for (int j = 0; j < BMB; ++j) {
        if (j >= kk) break;
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

__device__ __forceinline__ double b_dot(const double* x, const double* y, int n3, double* red) {
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < n3; i += NT) v[0] += x[i] * y[i];
    wg_sum<1>(v, red);
    return v[0];
}

__device__ __forceinline__ double b_step(const BArgs& a, const BSearch& s, BShared& sh, LbfgsHdr& h, int k_reflect, bool* stopped) {
    const int N = s.N, n3 = 3 * N;
    double fr[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < n3; i += NT)
#pragma unroll
        for (int r = 0; r < 2; ++r)
            if (r < k_reflect) fr[r] += s.F[i] * s.V[(size_t)r * n3 + i];
    wg_sum<2>(fr, sh.red);
    double fn[1] = {0.0};
    for (int i = threadIdx.x; i < n3; i += NT) {
        double v = s.F[i];
#pragma unroll
        for (int r = 0; r < 2; ++r)
            if (r < k_reflect) v -= 2.0 * fr[r] * s.V[(size_t)r * n3 + i];
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
    // (per-pair scalars in LDS: a register array indexed by the runtime pair
    // index would live in scratch memory)
    double* sy = sh.sy;
    double* alph = sh.alph;
    int newest = -1;
    for (int j = 0; j < h.count; ++j) {
        const int ph = (h.head + j) % a.mem;
        const double v = b_dot(s.Sm + (size_t)ph * n3, s.Ym + (size_t)ph * n3, n3, sh.red);
        if (threadIdx.x == 0) sy[j] = v;
        if (v > a.sy_min) newest = j;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n3; i += NT) s.d[i] = s.G[i];
    __syncthreads();
    for (int j = h.count - 1; j >= 0; --j) {
        if (!(sy[j] > a.sy_min)) continue;
        const int ph = (h.head + j) % a.mem;
        const double al = b_dot(s.Sm + (size_t)ph * n3, s.d, n3, sh.red) / sy[j];
        if (threadIdx.x == 0) alph[j] = al;
        const double* Yj = s.Ym + (size_t)ph * n3;
        for (int i = threadIdx.x; i < n3; i += NT) s.d[i] -= al * Yj[i];
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

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_batched_search(BArgs a, double* __restrict__ m_all,
                                                       const uint8_t* __restrict__ mask_all,
                                                       const int* __restrict__ Ls, const int* __restrict__ tiles,
                                                       const int* __restrict__ order,
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
        s.mask = mask_all ? mask_all + m_off[idx] / 3 : nullptr;
        s.tile = tiles[idx];
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

hipError_t launch_batched_search(const BatchArgs& a, double* m_all, const uint8_t* mask_all, const int* Ls,
                                 const int* tiles, const int* order, const long long* m_off,
                                 const long long* ws_off, char* ws, moto_search_result* res, int grid,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_batched_search, dim3(grid), dim3(NT), 0, st, a, m_all, mask_all, Ls, tiles, order, m_off,
                       ws_off, ws, res);
    return hipGetLastError();
}

}  // namespace moto
