// step.hip -- device kernels of the outer layer: reflected force and one
// L-BFGS / fixed / nonlinear-CG rotation step of every spin (Results,
// "Bilayer MMF": L-BFGS and CG are the paper's two outer optimisers;
// Supplementary Note 1, Algorithm 1, bilayer loop).
//
// The L-BFGS two-loop recursion is run in coefficient space: every vector it
// touches is a combination of the stored pairs S_j, Y_j and the current G, so
// one fused pass computes the Gram matrix of {S_0.., Y_0.., G} (after the
// projection transport of the stored pairs), a one-thread kernel runs the
// recursion on that small matrix, and one pass forms the direction.
#include "kernels.hpp"

namespace moto {

constexpr int SMEM = 16;                  // max L-BFGS memory
constexpr int SNV = 2 * SMEM + 1;         // max Gram basis size
constexpr int SNE = SNV * (SNV + 1) / 2;  // Gram entries (upper triangle)
constexpr int SPART = SNE + 1;            // + ||F_mmf||^2
constexpr int SCH = 64;                   // sites per staged chunk
constexpr int MAXR = 4;                   // max reflected modes

struct StepHdr {
    int count, head, have_prev, stopped;
    int iters;
    int cu;  // number of pairs the coefficients below refer to (G is coef[2*cu])
    int pad1, pad2;
    double fnorm;
    double cg_c;  // CG: the step taken last time = cg_c x its direction
    double coef[SNV];
};

constexpr int CG_RESTART = 50;  // CG restart period (steps)

struct StepPtrs {
    StepHdr* hdr;
    double *S, *Y, *G, *Gp, *dp, *d, *pgram, *pdot, *pmax;
    size_t vstride;  // doubles between stored vectors
    int nblk;
};

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

static int step_blocks(int N) {
    int nb = (N + SCH - 1) / SCH;
    return nb < 256 ? nb : 256;
}

static StepPtrs step_ptrs(void* state, int N, int mem, size_t* total) {
    StepPtrs P;
    char* base = (char*)state;
    const int nblk = step_blocks(N);
    const size_t v = al(sizeof(double) * 3 * (size_t)N);
    size_t o = 0;
    P.hdr = (StepHdr*)(base + o);
    o += al(sizeof(StepHdr));
    P.S = (double*)(base + o);
    o += v * mem;
    P.Y = (double*)(base + o);
    o += v * mem;
    P.G = (double*)(base + o);
    o += v;
    P.Gp = (double*)(base + o);
    o += v;
    P.dp = (double*)(base + o);
    o += v;
    P.d = (double*)(base + o);
    o += v;
    P.pgram = (double*)(base + o);
    o += al(sizeof(double) * SPART * nblk);
    P.pdot = (double*)(base + o);
    o += al(sizeof(double) * MAXR * nblk);
    P.pmax = (double*)(base + o);
    o += al(sizeof(double) * nblk);
    P.vstride = v / sizeof(double);
    P.nblk = nblk;
    if (total) *total = o;
    return P;
}

size_t step_state_bytes(int N, int mem) {
    size_t t = 0;
    step_ptrs(nullptr, N, mem, &t);
    return t;
}

// Ring bookkeeping shared by the Gram and control kernels: the pair formed
// at this step goes to `slot`; logical pair j (oldest first) lives in
// physical slot (h_new + j) % mem.
struct Ring {
    int c_new, h_new, slot;
};

__device__ __forceinline__ Ring ring_next(const StepHdr* h, int mem, int rule) {
    Ring r;
    r.slot = -1;
    r.c_new = h->count;
    r.h_new = h->head;
    if (h->have_prev && (rule == 0 || rule == 2)) {
        if (h->count < mem) {
            r.slot = (h->head + h->count) % mem;
            r.c_new = h->count + 1;
        } else {
            r.slot = h->head;
            r.h_new = (h->head + 1) % mem;
        }
    }
    return r;
}

// Members of a population stepped by one launch: member y = blockIdx.y owns
// the step state at + y sb bytes, spins and forces at + y m3 doubles and its
// modes at + y v3 doubles (all zero for a single search).
struct StepBatch {
    long long sb = 0, m3 = 0, v3 = 0;
};

__device__ __forceinline__ StepPtrs member_ptrs(StepPtrs P, const StepBatch& B) {
    const long long off = (long long)blockIdx.y * B.sb;
    auto sh = [&](auto* q) { return reinterpret_cast<decltype(q)>(reinterpret_cast<char*>(q) + off); };
    P.hdr = sh(P.hdr);
    P.S = sh(P.S);
    P.Y = sh(P.Y);
    P.G = sh(P.G);
    P.Gp = sh(P.Gp);
    P.dp = sh(P.dp);
    P.d = sh(P.d);
    P.pgram = sh(P.pgram);
    P.pdot = sh(P.pdot);
    P.pmax = sh(P.pmax);
    return P;
}

// (1) per-block partial dots F . v_r
__global__ __launch_bounds__(NT) void k_step_dots(StepArgs a, const double* __restrict__ F,
                                                  const double* __restrict__ V, StepPtrs P, StepBatch B) {
    P = member_ptrs(P, B);
    F += blockIdx.y * B.m3;
    V += blockIdx.y * B.v3;
    if (P.hdr->stopped) return;
    __shared__ double red[MAXR * (NT / 64)];
    double v[MAXR] = {0, 0, 0, 0};
    const size_t n3 = 3 * (size_t)a.N;
    const int per = (a.N + gridDim.x - 1) / gridDim.x;
    const int s0 = blockIdx.x * per, s1 = min(a.N, s0 + per);
    for (int s = s0 + threadIdx.x; s < s1; s += NT)
        for (int r = 0; r < a.k_reflect; ++r)
            for (int c = 0; c < 3; ++c) v[r] += F[c * a.N + s] * V[r * n3 + c * a.N + s];
    block_sum<MAXR>(v, red);
    if (threadIdx.x == 0)
        for (int r = 0; r < MAXR; ++r) P.pdot[(size_t)blockIdx.x * MAXR + r] = v[r];
}

// (2) G = -(F - 2 sum_r (F.v_r) v_r); projection transport of the stored
// pairs onto the tangent spaces at m; new pair s = P d_prev, y = G - P G_prev;
// Gram partials of {S_0..S_{c-1}, Y_0..Y_{c-1}, G} and ||F_mmf||^2.
__global__ __launch_bounds__(NT) void k_step_gram(StepArgs a, const double* __restrict__ m,
                                                  const double* __restrict__ F, const double* __restrict__ V,
                                                  StepPtrs P, StepBatch B) {
    P = member_ptrs(P, B);
    m += blockIdx.y * B.m3;
    F += blockIdx.y * B.m3;
    V += blockIdx.y * B.v3;
    const StepHdr* h = P.hdr;
    if (h->stopped) return;
    __shared__ double fr[MAXR];
    // rows padded by two doubles (16-byte aligned): the lanes of a wave read
    // different vectors at the same site, all on one LDS bank otherwise
    constexpr int SCHP = SCH + 2;
    __shared__ double stage[SNV][3][SCHP];
    const Ring rg = ring_next(h, a.mem, a.rule);
    const int c = rg.c_new;
    const int nv = 2 * c + 1;
    const int ne = nv * (nv + 1) / 2;
    // fr[r] = sum over the blocks' partials: wave r, lanes over the blocks
    static_assert(MAXR <= NT / 64, "a wave per reflected mode");
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        if (w < MAXR) {
            double s = 0.0;
            if (w < a.k_reflect)
                for (int b = lane; b < P.nblk; b += 64) s += P.pdot[(size_t)b * MAXR + w];
            s = wave_sum(s);
            if (lane == 0) fr[w] = s;
        }
    }
    // entries owned by this thread (upper triangle of the nv x nv Gram)
    constexpr int EQ = (SNE + NT - 1) / NT;
    int ei[EQ], ej[EQ];
#pragma unroll
    for (int q = 0; q < EQ; ++q) {
        ei[q] = ej[q] = 0;
        const int e = threadIdx.x + q * NT;
        if (e < ne) {
            int p = e, i = 0;
            while (p >= nv - i) {
                p -= nv - i;
                ++i;
            }
            ei[q] = i;
            ej[q] = i + p;
        }
    }
    double acc[EQ], fn2 = 0.0;
#pragma unroll
    for (int q = 0; q < EQ; ++q) acc[q] = 0.0;
    __syncthreads();
    const size_t n3 = 3 * (size_t)a.N;
    const int nchunks = (a.N + SCH - 1) / SCH;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        // the four waves stage the same SCH sites: each forms the site's
        // reflected force, gradient and new pair and transports every fourth
        // stored pair (wave 0 also writes G, the gradient column and |F|^2)
        static_assert(SCH == 64 && NT % SCH == 0, "one site per lane, whole waves");
        const int t = threadIdx.x % SCH, wv = threadIdx.x / SCH;
        {
            const int s = ch * SCH + t;
            if (s < a.N) {
                const double mi[3] = {m[s], m[a.N + s], m[2 * a.N + s]};
                double fm[3];
                for (int cc = 0; cc < 3; ++cc) {
                    double v = F[cc * a.N + s];
                    for (int r = 0; r < a.k_reflect; ++r) v -= 2.0 * fr[r] * V[r * n3 + cc * a.N + s];
                    fm[cc] = v;
                    if (wv == 0) fn2 += v * v;
                }
                double g[3] = {-fm[0], -fm[1], -fm[2]};
                if (wv == 0)
                    for (int cc = 0; cc < 3; ++cc) P.G[cc * a.N + s] = g[cc];
                // transport stored pairs / form the new one
                double sn[3] = {0, 0, 0}, yn[3] = {0, 0, 0};
                if (rg.slot >= 0) {
                    double dpv[3], gpv[3];
                    for (int cc = 0; cc < 3; ++cc) {
                        dpv[cc] = P.dp[cc * a.N + s];
                        gpv[cc] = P.Gp[cc * a.N + s];
                    }
                    const double md = mi[0] * dpv[0] + mi[1] * dpv[1] + mi[2] * dpv[2];
                    const double mg = mi[0] * gpv[0] + mi[1] * gpv[1] + mi[2] * gpv[2];
                    for (int cc = 0; cc < 3; ++cc) {
                        sn[cc] = dpv[cc] - md * mi[cc];
                        yn[cc] = g[cc] - (gpv[cc] - mg * mi[cc]);
                    }
                }
                for (int j = wv; j < c; j += NT / SCH) {
                    const int ph = (rg.h_new + j) % a.mem;
                    double* Sj = P.S + ph * P.vstride;
                    double* Yj = P.Y + ph * P.vstride;
                    double sv[3], yv[3];
                    if (ph == rg.slot) {
                        for (int cc = 0; cc < 3; ++cc) {
                            sv[cc] = sn[cc];
                            yv[cc] = yn[cc];
                        }
                    } else {
                        for (int cc = 0; cc < 3; ++cc) {
                            sv[cc] = Sj[cc * a.N + s];
                            yv[cc] = Yj[cc * a.N + s];
                        }
                        const double ms = mi[0] * sv[0] + mi[1] * sv[1] + mi[2] * sv[2];
                        const double my = mi[0] * yv[0] + mi[1] * yv[1] + mi[2] * yv[2];
                        for (int cc = 0; cc < 3; ++cc) {
                            sv[cc] -= ms * mi[cc];
                            yv[cc] -= my * mi[cc];
                        }
                    }
                    for (int cc = 0; cc < 3; ++cc) {
                        Sj[cc * a.N + s] = sv[cc];
                        Yj[cc * a.N + s] = yv[cc];
                        stage[j][cc][t] = sv[cc];
                        stage[c + j][cc][t] = yv[cc];
                    }
                }
                if (wv == 0)
                    for (int cc = 0; cc < 3; ++cc) stage[2 * c][cc][t] = g[cc];
            } else if (wv == 0) {
                for (int q = 0; q < nv; ++q)
                    for (int cc = 0; cc < 3; ++cc) stage[q][cc][t] = 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EQ; ++q) {
            if ((int)threadIdx.x + q * NT < ne) {
                double sacc = 0.0;
                for (int cc = 0; cc < 3; ++cc)
                    for (int tt = 0; tt < SCH; ++tt) sacc += stage[ei[q]][cc][tt] * stage[ej[q]][cc][tt];
                acc[q] += sacc;
            }
        }
        __syncthreads();
    }
    // ||F_mmf||^2 was accumulated by threads < SCH only
    __shared__ double red[NT / 64];
    double w = wave_sum(fn2);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    double* pg = P.pgram + (size_t)blockIdx.x * SPART;
#pragma unroll
    for (int q = 0; q < EQ; ++q)
        if ((int)threadIdx.x + q * NT < ne) pg[threadIdx.x + q * NT] = acc[q];
    if (threadIdx.x == 0) pg[SNE] = red[0] + red[1] + red[2] + red[3];
}

// (3) reduce the Gram (one wavefront per entry, fixed-order sums), then one
// thread: stop test, two-loop recursion in coefficient space, reset test;
// writes the direction coefficients.
__global__ __launch_bounds__(NT) void k_step_ctrl(StepArgs a, StepPtrs P, StepBatch B) {
    P = member_ptrs(P, B);
    StepHdr* h = P.hdr;
    if (h->stopped) return;
    __shared__ double gs[SNE + 1];
    const Ring rg = ring_next(h, a.mem, a.rule);
    const int c = rg.c_new;
    const int nv = 2 * c + 1;
    const int ne = nv * (nv + 1) / 2;
    const int lane = threadIdx.x & 63;
    for (int e = threadIdx.x >> 6; e <= ne; e += NT / 64) {
        const int ee = e < ne ? e : SNE;  // the last slot is |F_mmf|^2
        double s = 0.0;
        for (int b = lane; b < P.nblk; b += 64) s += P.pgram[(size_t)b * SPART + ee];
        s = wave_sum(s);
        if (lane == 0) gs[ee] = s;
    }
    // the serial control below runs on one thread; its arrays live in LDS
    // (as per-thread arrays indexed at run time they would sit in scratch,
    // a global-memory round trip per access)
    __shared__ double Gm[SNV][SNV];
    __shared__ double coef[SNV], q[SNV], alph[SMEM], rho[SMEM];
    __shared__ bool valid[SMEM];
    __syncthreads();
    // the Gram as a full matrix (every thread decodes its own entries)
    for (int e = threadIdx.x; e < ne; e += NT) {
        int p = e, i = 0;
        while (p >= nv - i) {
            p -= nv - i;
            ++i;
        }
        Gm[i][i + p] = gs[e];
        Gm[i + p][i] = gs[e];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double fn = sqrt(gs[SNE]);
    h->fnorm = fn;
    h->count = c;
    h->head = rg.h_new;
    if (!(fn > a.tau_F)) {  // converged (or NaN): do not move
        h->stopped = 1;
        return;
    }
    const int iG = 2 * c;
    for (int i = 0; i < nv; ++i) coef[i] = 0.0;
    bool reset = (a.rule == 1);
    if (a.rule == 2) {
        // nonlinear CG (Fletcher-Reeves) on G with one stored pair: S_0 is
        // the transported last step = cg_c x the transported last direction,
        // Y_0 = G - P G_prev, so |P G_prev|^2 = G.G - 2 G.Y_0 + Y_0.Y_0
        coef[iG] = -a.alpha0;
        if (c >= 1 && h->iters % CG_RESTART != 0) {
            const double GG = Gm[iG][iG], Gy = Gm[c][iG], yy = Gm[c][c];
            const double gpgp = GG - 2.0 * Gy + yy;
            const double beta = gpgp > 0.0 ? GG / gpgp : 0.0;
            const double bs = beta / h->cg_c;
            if (-GG + bs * Gm[0][iG] < 0.0) coef[0] = a.alpha0 * bs;
        }
    } else if (a.rule == 0) {
        for (int i = 0; i < nv; ++i) q[i] = 0.0;
        q[iG] = 1.0;
        int newest = -1;
        for (int j = 0; j < c; ++j) {
            const double sy = Gm[j][c + j];
            valid[j] = sy > a.sy_min;
            rho[j] = valid[j] ? 1.0 / sy : 0.0;
            if (valid[j]) newest = j;
        }
        for (int j = c - 1; j >= 0; --j) {
            if (!valid[j]) continue;
            double sq = 0.0;
            for (int i = 0; i < nv; ++i) sq += Gm[j][i] * q[i];
            alph[j] = rho[j] * sq;
            q[c + j] -= alph[j];
        }
        const double gamma = newest >= 0 ? Gm[newest][c + newest] / Gm[c + newest][c + newest] : a.alpha0;
        for (int i = 0; i < nv; ++i) q[i] *= gamma;
        for (int j = 0; j < c; ++j) {
            if (!valid[j]) continue;
            double yr = 0.0;
            for (int i = 0; i < nv; ++i) yr += Gm[c + j][i] * q[i];
            const double beta = rho[j] * yr;
            q[j] += alph[j] - beta;
        }
        double dG = 0.0;
        for (int i = 0; i < nv; ++i) {
            coef[i] = -q[i];
            dG += coef[i] * Gm[i][iG];
        }
        if (!(dG < 0.0)) reset = true;
    }
    if (reset) {
        for (int i = 0; i < nv; ++i) coef[i] = 0.0;
        coef[iG] = -a.alpha0;
        if (a.rule == 0) h->count = 0;
    }
    for (int i = 0; i < SNV; ++i) h->coef[i] = i < nv ? coef[i] : 0.0;
    h->cu = c;
}

// (4) direction d = P(sum coef . vectors) and per-block max |d_i|
__global__ __launch_bounds__(NT) void k_step_dir(StepArgs a, const double* __restrict__ m, StepPtrs P,
                                                 StepBatch B) {
    P = member_ptrs(P, B);
    m += blockIdx.y * B.m3;
    const StepHdr* h = P.hdr;
    if (h->stopped) return;
    __shared__ double red[NT / 64];
    const int cu = h->cu;
    double mx = 0.0;
    for (int s = blockIdx.x * NT + threadIdx.x; s < a.N; s += gridDim.x * NT) {
        double d[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < cu; ++j) {
            const int ph = (h->head + j) % a.mem;
            const double cs = h->coef[j], cy = h->coef[cu + j];
            if (cs == 0.0 && cy == 0.0) continue;
            const double* Sj = P.S + ph * P.vstride;
            const double* Yj = P.Y + ph * P.vstride;
            for (int cc = 0; cc < 3; ++cc) d[cc] += cs * Sj[cc * a.N + s] + cy * Yj[cc * a.N + s];
        }
        const double cg = h->coef[2 * cu];
        for (int cc = 0; cc < 3; ++cc) d[cc] += cg * P.G[cc * a.N + s];
        const double mi[3] = {m[s], m[a.N + s], m[2 * a.N + s]};
        const double md = mi[0] * d[0] + mi[1] * d[1] + mi[2] * d[2];
        double n2 = 0.0;
        for (int cc = 0; cc < 3; ++cc) {
            d[cc] -= md * mi[cc];
            P.d[cc * a.N + s] = d[cc];
            n2 += d[cc] * d[cc];
        }
        mx = fmax(mx, sqrt(n2));
    }
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) P.pmax[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// (5) rotation cap and exponential-map rotation of every spin; d -> d_prev,
// G -> G_prev.
__global__ __launch_bounds__(NT) void k_step_rot(StepArgs a, double* __restrict__ m, StepPtrs P, int nblk_dir,
                                                 StepBatch B) {
    P = member_ptrs(P, B);
    m += blockIdx.y * B.m3;
    const StepHdr* h = P.hdr;
    if (h->stopped) return;
    __shared__ double scale_s;
    if (threadIdx.x < 64) {  // largest per-site angle over the blocks' partials (wave 0)
        double mx = 0.0;
        for (int b = threadIdx.x; b < nblk_dir; b += 64) mx = fmax(mx, P.pmax[b]);
        mx = wave_max(mx);
        if (threadIdx.x == 0) scale_s = mx > a.theta_max ? a.theta_max / mx : 1.0;
    }
    __syncthreads();
    const double sc = scale_s;
    if (a.rule == 2 && blockIdx.x == 0 && threadIdx.x == 0) P.hdr->cg_c = a.alpha0 * sc;
    for (int s = blockIdx.x * NT + threadIdx.x; s < a.N; s += gridDim.x * NT) {
        double d[3], mi[3];
        double n2 = 0.0;
        for (int cc = 0; cc < 3; ++cc) {
            d[cc] = sc * P.d[cc * a.N + s];
            mi[cc] = m[cc * a.N + s];
            n2 += d[cc] * d[cc];
            P.dp[cc * a.N + s] = d[cc];
            P.Gp[cc * a.N + s] = P.G[cc * a.N + s];
        }
        const double th = sqrt(n2);
        if (th > 0.0) {
            const double ct = cos(th), st = sin(th) / th;
            double o[3], on = 0.0;
            for (int cc = 0; cc < 3; ++cc) {
                o[cc] = ct * mi[cc] + st * d[cc];
                on += o[cc] * o[cc];
            }
            const double inv = 1.0 / sqrt(on);
            for (int cc = 0; cc < 3; ++cc) m[cc * a.N + s] = o[cc] * inv;
        }
    }
}

__global__ void k_step_finish(StepPtrs P, double* __restrict__ out, StepBatch B) {
    if (threadIdx.x != 0) return;
    P = member_ptrs(P, B);
    out += 2 * blockIdx.y;
    StepHdr* h = P.hdr;
    out[0] = h->fnorm;
    out[1] = h->stopped ? 1.0 : 0.0;
    if (!h->stopped) {
        h->have_prev = 1;
        h->iters += 1;
    }
}

static hipError_t launch_step_members(const StepArgs& a, double* m, const double* F, const double* V, void* state,
                                      double* out, int members, const StepBatch& B, hipStream_t st) {
    StepPtrs P = step_ptrs(state, a.N, a.mem, nullptr);
    const int nb = P.nblk;
    if (a.k_reflect > 0) hipLaunchKernelGGL(k_step_dots, dim3(nb, members), dim3(NT), 0, st, a, F, V, P, B);
    hipLaunchKernelGGL(k_step_gram, dim3(nb, members), dim3(NT), 0, st, a, m, F, V, P, B);
    hipLaunchKernelGGL(k_step_ctrl, dim3(1, members), dim3(NT), 0, st, a, P, B);
    hipLaunchKernelGGL(k_step_dir, dim3(nb, members), dim3(NT), 0, st, a, m, P, B);
    hipLaunchKernelGGL(k_step_rot, dim3(nb, members), dim3(NT), 0, st, a, m, P, nb, B);
    hipLaunchKernelGGL(k_step_finish, dim3(1, members), dim3(64), 0, st, P, out, B);
    return hipGetLastError();
}

hipError_t launch_step(const StepArgs& a, double* m, const double* F, const double* V, void* state, double* out,
                       hipStream_t st) {
    return launch_step_members(a, m, F, V, state, out, 1, StepBatch{}, st);
}

// One step of P members in one set of launches (member y: spins and forces at
// + y 3N, modes at + y k 3N, step state at + y state_bytes, output at + 2y);
// members whose state says stopped are left alone.
hipError_t launch_step_population(const StepArgs& a, int P, int k, double* m, const double* F, const double* V,
                                  void* state, size_t state_bytes, double* out, hipStream_t st) {
    StepBatch B;
    B.sb = (long long)state_bytes;
    B.m3 = 3LL * a.N;
    B.v3 = (long long)k * 3LL * a.N;
    return launch_step_members(a, m, F, V, state, out, P, B, st);
}

__global__ void k_step_stop(StepHdr* h) {
    if (threadIdx.x == 0) h->stopped = 1;
}

// Marks member y's step state stopped (a member whose eigen-solve failed).
hipError_t launch_step_stop(void* state, int N, int mem, size_t state_bytes, int y, hipStream_t st) {
    StepPtrs P = step_ptrs((char*)state + state_bytes * (size_t)y, N, mem, nullptr);
    hipLaunchKernelGGL(k_step_stop, dim3(1), dim3(64), 0, st, P.hdr);
    return hipGetLastError();
}

// ---- descent seed: m <- R(m, scale * v1 / max_i |v1_i|) ----
__global__ __launch_bounds__(NT) void k_maxnorm(int N, const double* __restrict__ v, double* __restrict__ part) {
    __shared__ double red[NT / 64];
    double mx = 0.0;
    for (int s = blockIdx.x * NT + threadIdx.x; s < N; s += gridDim.x * NT)
        mx = fmax(mx, sqrt(v[s] * v[s] + v[N + s] * v[N + s] + v[2 * N + s] * v[2 * N + s]));
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(NT) void k_seed_rot(int N, double* __restrict__ m, const double* __restrict__ v,
                                                 double sse, const double* __restrict__ part, int nblk) {
    __shared__ double sc;
    if (threadIdx.x < 64) {  // largest partial (wave 0)
        double mx = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 64) mx = fmax(mx, part[b]);
        mx = wave_max(mx);
        if (threadIdx.x == 0) sc = mx > 0.0 ? sse / mx : 0.0;
    }
    __syncthreads();
    for (int s = blockIdx.x * NT + threadIdx.x; s < N; s += gridDim.x * NT) {
        double d[3], mi[3], n2 = 0.0;
        for (int cc = 0; cc < 3; ++cc) {
            d[cc] = sc * v[cc * N + s];
            mi[cc] = m[cc * N + s];
            n2 += d[cc] * d[cc];
        }
        const double th = sqrt(n2);
        if (th > 0.0) {
            const double ct = cos(th), st = sin(th) / th;
            double o[3], on = 0.0;
            for (int cc = 0; cc < 3; ++cc) {
                o[cc] = ct * mi[cc] + st * d[cc];
                on += o[cc] * o[cc];
            }
            const double inv = 1.0 / sqrt(on);
            for (int cc = 0; cc < 3; ++cc) m[cc * N + s] = o[cc] * inv;
        }
    }
}

hipError_t launch_seed_rotate(int N, double* m, const double* v1, double scale_sign_eta, double* part,
                              hipStream_t st) {
    int nb = (N + NT - 1) / NT;
    nb = nb < 256 ? nb : 256;
    hipLaunchKernelGGL(k_maxnorm, dim3(nb), dim3(NT), 0, st, N, v1, part);
    hipLaunchKernelGGL(k_seed_rot, dim3(nb), dim3(NT), 0, st, N, m, v1, scale_sign_eta, part, nb);
    return hipGetLastError();
}

__global__ void k_f64_to_f32(const double* __restrict__ s, float* __restrict__ d, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (float)s[i];
}

hipError_t launch_f64_to_f32(const double* src, float* dst, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, src, dst, n);
    return hipGetLastError();
}

__global__ void k_mask_zero(double* __restrict__ v, const uint8_t* __restrict__ mask, int N, int ncomp) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N || mask[s]) return;
    for (int c = 0; c < ncomp; ++c) v[(size_t)c * N + s] = 0.0;
}

// zero fill of a byte range in 16-byte words (buffers are 256-byte aligned);
// a kernel rather than a memset so that the drivers stay graph-capturable
__global__ __launch_bounds__(NT) void k_zero(uint4* __restrict__ p, size_t n16) {
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n16; i += (size_t)gridDim.x * NT) p[i] = z;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
    if (bytes % 16 != 0 || ((uintptr_t)p & 15) != 0) return hipErrorInvalidValue;
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const size_t nb = (n16 + NT - 1) / NT;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)(nb < 1024 ? nb : 1024)), dim3(NT), 0, st, (uint4*)p, n16);
    return hipGetLastError();
}

// The descent's outcome assembled on the device (MOTO_ASYNC): stop flag and
// ||F|| from the step output, steps taken from the step state, energy and
// lambda_1 (Eo[0], Eo[1]) and the charge Q.
__global__ void k_descend_result(StepPtrs P, const double* __restrict__ out, const double* __restrict__ Eo,
                                 const double* __restrict__ Q, moto_descend_result* __restrict__ res) {
    if (threadIdx.x != 0) return;
    moto_descend_result r;
    r.converged = out[1] != 0.0 ? 1 : 0;
    r.iters = P.hdr->iters;
    r.E = Eo[0];
    r.Q = Q[0];
    r.fnorm = out[0];
    r.lambda1 = Eo[1];
    *res = r;
}

hipError_t launch_descend_result(void* state, int N, int mem, const double* out, const double* Eo, const double* Q,
                                 moto_descend_result* res, hipStream_t st) {
    StepPtrs P = step_ptrs(state, N, mem, nullptr);
    hipLaunchKernelGGL(k_descend_result, dim3(1), dim3(64), 0, st, P, out, Eo, Q, res);
    return hipGetLastError();
}

hipError_t launch_mask_zero(double* v, const uint8_t* mask, int N, int ncomp, hipStream_t st) {
    hipLaunchKernelGGL(k_mask_zero, dim3((N + NT - 1) / NT), dim3(NT), 0, st, v, mask, N, ncomp);
    return hipGetLastError();
}

}  // namespace moto
