// shells.hip -- lattice kernels for Hamiltonians with more than three
// exchange shells (the paper's Pd/Fe/Ir(111) parameter set has 35 shells,
// 360 bonds per site; Supplementary Note 4, Table S1).
//
// With hundreds of offsets per site the stencil is bound by LDS reads and
// VALU adds, not by HBM: a workgroup stages a TX x TY tile with a halo of R
// rows and columns (R = the largest |dx|, |dy| of the table, at most 12) in
// LDS and each thread sums the shells of its site from there, shell by shell
// (one multiply by cJ[s] per shell).  The spin Hamiltonian is the one of the
// three-shell kernels (Methods, Eq. param-hamiltonian): exchange on every
// shell, interfacial DMI on the nearest-neighbour shell, uniaxial anisotropy,
// Zeeman field.
#include <utility>

#include "kernels.hpp"

namespace moto {

constexpr int LXG = TX + 2 * GEN_RMAX;
constexpr int LYG = TY + 2 * GEN_RMAX;

template <class T>
struct GenLDS {
    T u[3][LYG][LXG];
    uint8_t act[LYG][LXG];
};

struct GenTile {
    int b, tx0, ty0;
};

__device__ __forceinline__ GenTile gen_tile(const Geo& g) {
    GenTile t;
    const int bid = blockIdx.x;
    t.b = bid / g.tiles;
    const int r = bid - t.b * g.tiles;
    t.tx0 = (r % g.tiles_x) * TX;
    t.ty0 = (r / g.tiles_x) * TY;
    return t;
}

// (A u) at LDS position (cx, cy): sum_s cJ[s] sum_{delta in s} u(. + delta)
// + cD sum_{delta in NN} [dhat u_z - z (dhat . u)] + cK u_z z.
template <class T>
__device__ __forceinline__ void apply_A_gen(const GenLDS<T>& L, const GenShells& gs, const Coef<T>& k, int cx, int cy,
                                            T (&a)[3]) {
    a[0] = a[1] = a[2] = T(0);
    for (int s = 0; s < gs.ns; ++s) {
        T S0 = T(0), S1 = T(0), S2 = T(0);
        const int o1 = gs.start[s + 1];
        for (int o = gs.start[s]; o < o1; ++o) {
            const int yy = cy + gs.dy[o], xx = cx + gs.dx[o];
            S0 += L.u[0][yy][xx];
            S1 += L.u[1][yy][xx];
            S2 += L.u[2][yy][xx];
        }
        const T cj = (T)gs.cJ[s];
        a[0] += cj * S0;
        a[1] += cj * S1;
        a[2] += cj * S2;
    }
    if (k.cD != T(0)) {
        for (int o = gs.start[0]; o < gs.start[1]; ++o) {
            const int ddx = gs.dx[o], ddy = gs.dy[o];
            const int yy = cy + ddy, xx = cx + ddx;
            const T u0 = L.u[0][yy][xx], u1 = L.u[1][yy][xx], u2 = L.u[2][yy][xx];
            const T hx = k.cD * (T(ddx) + T(0.5) * T(ddy));
            const T hy = k.cD * (T(0.86602540378443864676) * T(ddy));
            a[0] += hx * u2;
            a[1] += hy * u2;
            a[2] -= hx * u0 + hy * u1;
        }
    }
    a[2] += k.cK * L.u[2][cy][cx];
}

// Energy, gradient, c, F of the general-shell Hamiltonian; partial slot 0 of
// each tile holds sum_i (1/2 m_i.(A m)_i - B.m_i), the others are zero.
template <class T>
__global__ __launch_bounds__(NT) void k_energy_grad_gen(Geo g, GenShells gs, Coef<T> k, const T* __restrict__ m,
                                                        const uint8_t* __restrict__ mask, T* __restrict__ grad,
                                                        T* __restrict__ cout, T* __restrict__ F,
                                                        double* __restrict__ part) {
    __shared__ GenLDS<T> L;
    __shared__ double red[NPART * (NT / 64)];
    const GenTile t = gen_tile(g);
    const int R = gs.R, W = TX + 2 * R, H = TY + 2 * R;
    const size_t N = g.N;
    const T* mb = m + (size_t)t.b * 3 * N;
    for (int i = threadIdx.x; i < W * H; i += NT) {
        const int lx = i % W, ly = i / W;
        const int x = wrapi(t.tx0 + lx - R, g.Lx), y = wrapi(t.ty0 + ly - R, g.Ly);
        const int s = x + g.Lx * y;
        L.u[0][ly][lx] = mb[s];
        L.u[1][ly][lx] = mb[N + s];
        L.u[2][ly][lx] = mb[2 * N + s];
    }
    __syncthreads();
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = t.tx0 + lx, y = t.ty0 + ly;
    double v[NPART];
#pragma unroll
    for (int q = 0; q < NPART; ++q) v[q] = 0.0;
    if (x < g.Lx && y < g.Ly) {
        const int cx = lx + R, cy = ly + R;
        const size_t s = (size_t)t.b * N + x + (size_t)g.Lx * y;
        const size_t s3 = (size_t)t.b * 3 * N + x + (size_t)g.Lx * y;
        T a[3];
        apply_A_gen(L, gs, k, cx, cy, a);
        const T mi[3] = {L.u[0][cy][cx], L.u[1][cy][cx], L.u[2][cy][cx]};
        const T gi[3] = {a[0] - k.B[0], a[1] - k.B[1], a[2] - k.B[2]};
        const T ci = mi[0] * gi[0] + mi[1] * gi[1] + mi[2] * gi[2];
        if (grad) {
            grad[s3] = gi[0];
            grad[s3 + N] = gi[1];
            grad[s3 + 2 * N] = gi[2];
        }
        if (cout) cout[s] = ci;
        if (F) {
            const bool act = mask == nullptr || mask[s] != 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) F[s3 + c * N] = act ? -(gi[c] - ci * mi[c]) : T(0);
        }
        const double mam = (double)mi[0] * a[0] + (double)mi[1] * a[1] + (double)mi[2] * a[2];
        const double bm = (double)k.B[0] * mi[0] + (double)k.B[1] * mi[1] + (double)k.B[2] * mi[2];
        v[0] = 0.5 * mam - bm;
    }
    block_sum<NPART>(v, red);
    if (threadIdx.x == 0)
        for (int q = 0; q < NPART; ++q) part[(size_t)blockIdx.x * NPART + q] = v[q];
}

// Tangent HVP (frame or ambient layout, as the three-shell tile kernel):
// W_j = M H(m) M V_j with (H v)_i = P_i (A v)_i - c_i v_i, one vector at a
// time through an HX x HY tile with the full GEN_RMAX halo.  Each thread owns
// HN sites HS apart in x, so the address arithmetic and the offset-table
// reads of every bond are shared by HN sites; the rest is one LDS read and
// one add per bond and component.
constexpr int HX = 64, HY = 16, HN = 4, HS = HX / HN;
constexpr int HLX = HX + 2 * GEN_RMAX, HLY = HY + 2 * GEN_RMAX;
static_assert((HX / HN) * HY == NT, "one thread per HN sites");

template <class T>
struct HvpGenLDS {
    T u[3][HLY][HLX];
};

// (A u) at the HN sites of a thread (LDS row cy, columns cx + k HS,
// k < HN): shell by shell over the plan's offsets; one address per offset
// serves the HN sites (immediate offsets k HS from it).  Sites HS apart keep
// the lanes of a wave on consecutive words (no LDS bank conflicts).
template <class T>
__device__ __forceinline__ void apply_A_blk(const HvpGenLDS<T>& L, const int* __restrict__ rel, const GenShells& gs,
                                            T cD, int cy, int cx, T (&acc)[HN][3]) {
    constexpr int PL = HLY * HLX;  // plane stride
    const T* base = &L.u[0][0][0] + cy * HLX + cx;
    for (int s = 0; s < gs.ns; ++s) {
        T sm[HN][3];
#pragma unroll
        for (int k = 0; k < HN; ++k) sm[k][0] = sm[k][1] = sm[k][2] = T(0);
        const int o1 = gs.start[s + 1];
#pragma unroll 6
        for (int o = gs.start[s]; o < o1; ++o) {
            const T* p = base + rel[o];
#pragma unroll
            for (int k = 0; k < HN; ++k) {
                sm[k][0] += p[k * HS];
                sm[k][1] += p[PL + k * HS];
                sm[k][2] += p[2 * PL + k * HS];
            }
        }
        const T cj = (T)gs.cJ[s];
#pragma unroll
        for (int k = 0; k < HN; ++k) {
            acc[k][0] += cj * sm[k][0];
            acc[k][1] += cj * sm[k][1];
            acc[k][2] += cj * sm[k][2];
        }
    }
    if (cD != T(0)) {
        for (int o = gs.start[0]; o < gs.start[1]; ++o) {
            const int ddx = gs.dx[o], ddy = gs.dy[o];
            const T* p = base + ddy * HLX + ddx;
            const T hx = cD * (T(ddx) + T(0.5) * T(ddy));
            const T hy = cD * (T(0.86602540378443864676) * T(ddy));
#pragma unroll
            for (int k = 0; k < HN; ++k) {
                const T u0 = p[k * HS], u1 = p[PL + k * HS], u2 = p[2 * PL + k * HS];
                acc[k][0] += hx * u2;
                acc[k][1] += hy * u2;
                acc[k][2] -= hx * u0 + hy * u1;
            }
        }
    }
}

template <class T, bool FRAME>
__global__ __launch_bounds__(NT) void k_tangent_hvp_gen(Geo g, GenShells gs, Coef<T> k, const T* __restrict__ m,
                                                        const T* __restrict__ c, const uint8_t* __restrict__ mask,
                                                        int nvec, long long vbs, const T* __restrict__ V,
                                                        T* __restrict__ W, const int* __restrict__ done) {
    if (done != nullptr && *done) return;
    constexpr int DV = FRAME ? 2 : 3;
    __shared__ HvpGenLDS<T> L;
    __shared__ uint8_t act[HLY][HLX];
    __shared__ int rel[GEN_MAX_OFF];  // LDS offset of every bond, dy HLX + dx
    for (int o = threadIdx.x; o < gs.n_off; o += NT) rel[o] = gs.dy[o] * HLX + gs.dx[o];
    const int ntx = (g.Lx + HX - 1) / HX, nty = (g.Ly + HY - 1) / HY;
    const int bid = blockIdx.x;
    const int b = bid / (ntx * nty);
    const int r = bid - b * ntx * nty;
    const int tx0 = (r % ntx) * HX, ty0 = (r / ntx) * HY;
    const size_t N = g.N;
    const T* mb = m + (size_t)b * 3 * N;
    const uint8_t* mk = mask ? mask + (size_t)b * N : nullptr;
    const T* Vb = V + (size_t)b * vbs;
    T* Wb = W + (size_t)b * vbs;
    for (int i = threadIdx.x; i < HLX * HLY; i += NT) {
        const int lx = i % HLX, ly = i / HLX;
        const int s = wrapi(tx0 + lx - GEN_RMAX, g.Lx) + g.Lx * wrapi(ty0 + ly - GEN_RMAX, g.Ly);
        act[ly][lx] = mk ? (mk[s] != 0) : 1;
    }
    const int lxo = threadIdx.x % HS, lyo = threadIdx.x / HS;
    const int y = ty0 + lyo;
    const int cy = lyo + GEN_RMAX, cx = lxo + GEN_RMAX;
    // own sites: frames (or spins) and c
    T f[HN][6], cc[HN];
    int so[HN];
    bool val[HN];
#pragma unroll
    for (int q = 0; q < HN; ++q) {
        const int x = tx0 + lxo + q * HS;
        val[q] = x < g.Lx && y < g.Ly;
        so[q] = val[q] ? x + g.Lx * y : 0;
        const T m0 = val[q] ? mb[so[q]] : T(0), m1 = val[q] ? mb[N + so[q]] : T(0),
                m2 = val[q] ? mb[2 * N + so[q]] : T(1);
        cc[q] = val[q] ? c[(size_t)b * N + so[q]] : T(0);
        if constexpr (FRAME) {
            T e1[3], e2[3];
            onb(m0, m1, m2, e1, e2);
            f[q][0] = e1[0];
            f[q][1] = e1[1];
            f[q][2] = e1[2];
            f[q][3] = e2[0];
            f[q][4] = e2[1];
            f[q][5] = e2[2];
        } else {
            f[q][0] = m0;
            f[q][1] = m1;
            f[q][2] = m2;
            f[q][3] = f[q][4] = f[q][5] = T(0);
        }
    }
    for (int j = 0; j < nvec; ++j) {
        const T* vj = Vb + (size_t)j * DV * N;
        __syncthreads();
        for (int i = threadIdx.x; i < HLX * HLY; i += NT) {
            const int lx = i % HLX, ly = i / HLX;
            const int s = wrapi(tx0 + lx - GEN_RMAX, g.Lx) + g.Lx * wrapi(ty0 + ly - GEN_RMAX, g.Ly);
            const bool on = act[ly][lx];
            if constexpr (FRAME) {
                T f1[3], f2[3];
                onb(mb[s], mb[N + s], mb[2 * N + s], f1, f2);
                const T a = on ? vj[s] : T(0);
                const T bb = on ? vj[N + s] : T(0);
                L.u[0][ly][lx] = a * f1[0] + bb * f2[0];
                L.u[1][ly][lx] = a * f1[1] + bb * f2[1];
                L.u[2][ly][lx] = a * f1[2] + bb * f2[2];
            } else {
                L.u[0][ly][lx] = on ? vj[s] : T(0);
                L.u[1][ly][lx] = on ? vj[N + s] : T(0);
                L.u[2][ly][lx] = on ? vj[2 * N + s] : T(0);
            }
        }
        __syncthreads();
        T acc[HN][3];
#pragma unroll
        for (int q = 0; q < HN; ++q) acc[q][0] = acc[q][1] = acc[q][2] = T(0);
        apply_A_blk<T>(L, rel, gs, k.cD, cy, cx, acc);
        T* wj = Wb + (size_t)j * DV * N;
#pragma unroll
        for (int q = 0; q < HN; ++q) {
            if (!val[q]) continue;
            const bool on = act[cy][cx + q * HS];
            const T u0 = L.u[0][cy][cx + q * HS], u1 = L.u[1][cy][cx + q * HS], u2 = L.u[2][cy][cx + q * HS];
            const T a0 = acc[q][0], a1 = acc[q][1], a2 = acc[q][2] + k.cK * u2;
            if constexpr (FRAME) {
                const T av = f[q][0] * u0 + f[q][1] * u1 + f[q][2] * u2;
                const T bv = f[q][3] * u0 + f[q][4] * u1 + f[q][5] * u2;
                const T wa = f[q][0] * a0 + f[q][1] * a1 + f[q][2] * a2 - cc[q] * av;
                const T wb = f[q][3] * a0 + f[q][4] * a1 + f[q][5] * a2 - cc[q] * bv;
                wj[so[q]] = on ? wa : T(0);
                wj[N + so[q]] = on ? wb : T(0);
            } else {
                const T ma = f[q][0] * a0 + f[q][1] * a1 + f[q][2] * a2;
                wj[so[q]] = on ? a0 - ma * f[q][0] - cc[q] * u0 : T(0);
                wj[N + so[q]] = on ? a1 - ma * f[q][1] - cc[q] * u1 : T(0);
                wj[2 * N + so[q]] = on ? a2 - ma * f[q][2] - cc[q] * u2 : T(0);
            }
        }
    }
}

// --------------------------------------------------------------------------
hipError_t launch_energy_grad_gen(const Geo& g, const CoefD& kd, bool f64, int batch, const void* m,
                                  const uint8_t* mask, void* grad, void* c, void* F, double* part, hipStream_t st) {
    if (!kd.gen || kd.gen->R > GEN_RMAX) return hipErrorInvalidValue;
    const dim3 grid(batch * g.tiles);
    if (f64)
        hipLaunchKernelGGL(k_energy_grad_gen<double>, grid, dim3(NT), 0, st, g, *kd.gen, coef_cast<double>(kd),
                           (const double*)m, mask, (double*)grad, (double*)c, (double*)F, part);
    else
        hipLaunchKernelGGL(k_energy_grad_gen<float>, grid, dim3(NT), 0, st, g, *kd.gen, coef_cast<float>(kd),
                           (const float*)m, mask, (float*)grad, (float*)c, (float*)F, part);
    return hipGetLastError();
}

hipError_t launch_tangent_hvp_gen(const Geo& g, const CoefD& kd, bool f64, bool frame, int batch, const void* m,
                                  const void* c, const uint8_t* mask, int nvec, long long vbs, const void* V, void* W,
                                  const int* done, hipStream_t st) {
    if (!kd.gen || kd.gen->R > GEN_RMAX) return hipErrorInvalidValue;
    if (vbs <= 0) vbs = (long long)nvec * (frame ? 2 : 3) * g.N;
    const dim3 grid(batch * ((g.Lx + HX - 1) / HX) * ((g.Ly + HY - 1) / HY));
    auto go = [&](auto tc, auto fc) {
        using T = decltype(tc);
        constexpr bool FR = decltype(fc)::value;
        hipLaunchKernelGGL((k_tangent_hvp_gen<T, FR>), grid, dim3(NT), 0, st, g, *kd.gen, coef_cast<T>(kd),
                           (const T*)m, (const T*)c, mask, nvec, vbs, (const T*)V, (T*)W, done);
    };
    if (f64) {
        if (frame)
            go(double(0), std::true_type{});
        else
            go(double(0), std::false_type{});
    } else {
        if (frame)
            go(float(0), std::true_type{});
        else
            go(float(0), std::false_type{});
    }
    return hipGetLastError();
}

}  // namespace moto
