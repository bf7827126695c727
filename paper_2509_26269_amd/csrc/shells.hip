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
// time through an HX x HY tile staged with the full GEN_RMAX halo.
//
// The exchange sum over the disc of bonds is evaluated row by row as a 1-D
// convolution: a thread owns HSP consecutive sites of one row and, for each
// row offset dy, reads the HSP + 2 GEN_RMAX values of that input row once
// (16-byte LDS reads) into registers and applies the row's 2 GEN_RMAX + 1
// couplings (a per-block LDS table, zero off the disc and beyond the plan's
// shells) to all HSP sites from there: about 2 LDS values per site, row and
// component instead of one per bond, at the price of multiply-adds over the
// full square of offsets (the disc fills 58 % of it).  DMI (nearest
// neighbours) and anisotropy are added per site afterwards.
constexpr int HX = 64, HY = 16, HSP = 8, HNT = (HX / HSP) * HY;
constexpr int HLX = HX + 2 * GEN_RMAX, HLY = HY + 2 * GEN_RMAX;
constexpr int HW = 2 * GEN_RMAX + 1;   // couplings per row
constexpr int HWIN = HSP + 2 * GEN_RMAX;  // window values per row
static_assert(HLX % 4 == 0 && HSP % 4 == 0, "16-byte aligned row windows");

template <class T>
struct HvpGenLDS {
    T u[3][HLY][HLX];
    T wt[HW][HW];  // wt[dy + R][dx + R] = cJ of the shell of (dx, dy)
};

template <class T, bool FRAME>
__global__ __launch_bounds__(HNT) void k_tangent_hvp_gen(Geo g, GenShells gs, Coef<T> k, const T* __restrict__ m,
                                                         const T* __restrict__ c, const uint8_t* __restrict__ mask,
                                                         int nvec, long long vbs, const T* __restrict__ V,
                                                         T* __restrict__ W, const int* __restrict__ done) {
    if (done != nullptr && *done) return;
    constexpr int DV = FRAME ? 2 : 3;
    __shared__ __align__(16) HvpGenLDS<T> L;
    __shared__ uint8_t act[HLY][HLX];
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
    // couplings of the disc, activity of the staged sites
    for (int i = threadIdx.x; i < HW * HW; i += HNT) (&L.wt[0][0])[i] = T(0);
    for (int i = threadIdx.x; i < HLX * HLY; i += HNT) {
        const int lx = i % HLX, ly = i / HLX;
        const int s = wrapi(tx0 + lx - GEN_RMAX, g.Lx) + g.Lx * wrapi(ty0 + ly - GEN_RMAX, g.Ly);
        act[ly][lx] = mk ? (mk[s] != 0) : 1;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < gs.n_off; o += HNT) {
        int sh = 0;
        while (o >= gs.start[sh + 1]) ++sh;
        L.wt[gs.dy[o] + GEN_RMAX][gs.dx[o] + GEN_RMAX] = (T)gs.cJ[sh];
    }
    const int lx0 = (threadIdx.x % (HX / HSP)) * HSP, ly0 = threadIdx.x / (HX / HSP);
    const int y = ty0 + ly0;
    const int cy = ly0 + GEN_RMAX, cx = lx0 + GEN_RMAX;
    const int R = gs.R;
    for (int j = 0; j < nvec; ++j) {
        const T* vj = Vb + (size_t)j * DV * N;
        __syncthreads();
        for (int i = threadIdx.x; i < HLX * HLY; i += HNT) {
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
        // exchange: row-by-row convolution of each component
        T a[HSP][3];
        for (int cc = 0; cc < 3; ++cc) {
            T acc[HSP];
#pragma unroll
            for (int q = 0; q < HSP; ++q) acc[q] = T(0);
            for (int dy = -R; dy <= R; ++dy) {
                const T* rp = &L.u[cc][cy + dy][lx0];
                T win[HWIN];
#pragma unroll
                for (int i = 0; i < HWIN; ++i) win[i] = rp[i];
                const T* wr = &L.wt[dy + GEN_RMAX][0];
#pragma unroll
                for (int d = 0; d < HW; ++d) {
                    const T w = wr[d];
#pragma unroll
                    for (int q = 0; q < HSP; ++q) acc[q] += w * win[q + d];
                }
            }
#pragma unroll
            for (int q = 0; q < HSP; ++q) a[q][cc] = acc[q];
        }
        // nearest-neighbour DMI and anisotropy, per site
        if (k.cD != T(0)) {
#pragma unroll
            for (int o = 0; o < 6; ++o) {
                constexpr int NDX[6] = {1, 0, -1, -1, 0, 1}, NDY[6] = {0, 1, 1, 0, -1, -1};
                const int ddx = NDX[o], ddy = NDY[o];
                const T hx = k.cD * (T(ddx) + T(0.5) * T(ddy));
                const T hy = k.cD * (T(0.86602540378443864676) * T(ddy));
#pragma unroll
                for (int q = 0; q < HSP; ++q) {
                    const T u0 = L.u[0][cy + ddy][cx + q + ddx], u1 = L.u[1][cy + ddy][cx + q + ddx],
                            u2 = L.u[2][cy + ddy][cx + q + ddx];
                    a[q][0] += hx * u2;
                    a[q][1] += hy * u2;
                    a[q][2] -= hx * u0 + hy * u1;
                }
            }
        }
        T* wj = Wb + (size_t)j * DV * N;
#pragma unroll
        for (int q = 0; q < HSP; ++q) {
            const int x = tx0 + lx0 + q;
            if (x >= g.Lx || y >= g.Ly) continue;
            const int so = x + g.Lx * y;
            const bool on = act[cy][cx + q];
            const T u0 = L.u[0][cy][cx + q], u1 = L.u[1][cy][cx + q], u2 = L.u[2][cy][cx + q];
            const T ci = c[(size_t)b * N + so];
            const T m0 = mb[so], m1 = mb[N + so], m2 = mb[2 * N + so];
            const T a0 = a[q][0], a1 = a[q][1], a2 = a[q][2] + k.cK * u2;
            if constexpr (FRAME) {
                T e1[3], e2[3];
                onb(m0, m1, m2, e1, e2);
                const T av = e1[0] * u0 + e1[1] * u1 + e1[2] * u2;
                const T bv = e2[0] * u0 + e2[1] * u1 + e2[2] * u2;
                const T wa = e1[0] * a0 + e1[1] * a1 + e1[2] * a2 - ci * av;
                const T wb = e2[0] * a0 + e2[1] * a1 + e2[2] * a2 - ci * bv;
                wj[so] = on ? wa : T(0);
                wj[N + so] = on ? wb : T(0);
            } else {
                const T ma = m0 * a0 + m1 * a1 + m2 * a2;
                wj[so] = on ? a0 - ma * m0 - ci * u0 : T(0);
                wj[N + so] = on ? a1 - ma * m1 - ci * u1 : T(0);
                wj[2 * N + so] = on ? a2 - ma * m2 - ci * u2 : T(0);
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
        hipLaunchKernelGGL((k_tangent_hvp_gen<T, FR>), grid, dim3(HNT), 0, st, g, *kd.gen, coef_cast<T>(kd),
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
