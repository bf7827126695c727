// tile_ops.hpp -- per-tile bodies of the lattice kernels, shared by the
// one-launch-per-step kernels (one tile per workgroup) and the persistent
// batched search (one workgroup looping over the tiles of its lattice).
//
// A tile is TX x TY output sites (TileShape; 32 x 8 unless a caller picks
// another shape); the workgroup stages the (TX+4) x (TY+4)
// neighbourhood in LDS with periodic wrap and evaluates the three-shell
// stencil of the spin Hamiltonian (Methods, Eq. param-hamiltonian) at one
// site per thread.
#pragma once

#include "kernels.hpp"

namespace moto {

template <class T, int TXV>
__device__ __forceinline__ void stage_tile(TileLDS<T, TXV>& t, const Geo& g, const T* __restrict__ mb, int tx0,
                                           int ty0) {
    using SH = TileShape<TXV>;
    for (int i = threadIdx.x; i < SH::SITES; i += NT) {
        const int lx = i % SH::LX, ly = i / SH::LX;
        const int x = wrapi(tx0 + lx - HALO, g.Lx), y = wrapi(ty0 + ly - HALO, g.Ly);
        const int s = x + g.Lx * y;
        t.u[0][ly][lx] = mb[s];
        t.u[1][ly][lx] = mb[g.N + s];
        t.u[2][ly][lx] = mb[2 * g.N + s];
    }
}

// Energy, gradient, c, F of one tile; per-thread partial slots (not reduced):
//   [e_i, -m.S_0, -m.S_1, -m.S_2, m.Q_0, m.Q_1, m.Q_2, -m_z^2, -m_x, -m_y, -m_z]
// with e_i = 1/2 m_i.(A m)_i - B.m_i.  Pointers are of the lattice (batch
// offset applied); grad, c, F, mask may be null.  Ends with a barrier.
template <class T, int TXV>
__device__ __forceinline__ void energy_tile(TileLDS<T, TXV>& t, const Geo& g, const Coef<T>& k, const T* __restrict__ mb,
                                            const uint8_t* __restrict__ mk, T* __restrict__ gb,
                                            T* __restrict__ cb, T* __restrict__ fb, int tx0, int ty0,
                                            double (&v)[NPART]) {
    __syncthreads();
    stage_tile(t, g, mb, tx0, ty0);
    __syncthreads();
    const int lx = threadIdx.x % TXV, ly = threadIdx.x / TXV;
    const int x = tx0 + lx, y = ty0 + ly;
    if (x < g.Lx && y < g.Ly) {
        const int cx = lx + HALO, cy = ly + HALO;
        const int s = x + g.Lx * y;
        T a[3];
        apply_A_tile(t, cx, cy, k, a);
        const T mi[3] = {t.u[0][cy][cx], t.u[1][cy][cx], t.u[2][cy][cx]};
        const T gi[3] = {a[0] - k.B[0], a[1] - k.B[1], a[2] - k.B[2]};
        const T ci = mi[0] * gi[0] + mi[1] * gi[1] + mi[2] * gi[2];
        if (gb) {
            gb[s] = gi[0];
            gb[g.N + s] = gi[1];
            gb[2 * g.N + s] = gi[2];
        }
        if (cb) cb[s] = ci;
        if (fb) {
            const bool act = mk == nullptr || mk[s] != 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) fb[c * g.N + s] = act ? -(gi[c] - ci * mi[c]) : T(0);
        }
        const double mam = (double)mi[0] * a[0] + (double)mi[1] * a[1] + (double)mi[2] * a[2];
        const double bm = (double)k.B[0] * mi[0] + (double)k.B[1] * mi[1] + (double)k.B[2] * mi[2];
        v[0] += 0.5 * mam - bm;
        T S[3][3], Q[3][3];
        shell_sums(t, cx, cy, S, Q);
#pragma unroll
        for (int sh = 0; sh < 3; ++sh) {
            v[1 + sh] += -((double)mi[0] * S[sh][0] + (double)mi[1] * S[sh][1] + (double)mi[2] * S[sh][2]);
            v[4 + sh] += (double)mi[0] * Q[sh][0] + (double)mi[1] * Q[sh][1] + (double)mi[2] * Q[sh][2];
        }
        v[7] += -(double)mi[2] * mi[2];
        v[8] += -(double)mi[0];
        v[9] += -(double)mi[1];
        v[10] += -(double)mi[2];
    }
}

// LDS of the tangent HVP: staged vector planes, frames (or spins), activity.
template <class T, bool FRAME, int TXV = TX>
struct HvpLDS {
    TileLDS<T, TXV> t;
    T fr[FRAME ? 6 : 3][TileShape<TXV>::LY][TileShape<TXV>::LX];
    uint8_t act[TileShape<TXV>::LY][TileShape<TXV>::LX];
};

// Tangent Hessian-vector product on one tile (Methods, HVP operator mode):
// W_j = M H(m) M V_j, (H v)_i = P_i (A v)_i - c_i v_i.
//   FRAME: V, W in frame coordinates [nvec][2][N]; the ambient vector of a
//   staged site is a e1 + b e2, and the output is (e1.(A u) - c a,
//   e2.(A u) - c b) (P_i drops out against the tangent basis).
//   AMBIENT: V, W = [nvec][3][N]; output P_i (A u)_i - c_i u_i.
// Pointers are of the lattice (batch offset applied).
template <class T, bool FRAME, int TXV>
__device__ __forceinline__ void tangent_hvp_tile(HvpLDS<T, FRAME, TXV>& sh, const Geo& g, const Coef<T>& k,
                                                 const T* __restrict__ mb, const T* __restrict__ cb,
                                                 const uint8_t* __restrict__ mk, int nvec, const T* __restrict__ Vb,
                                                 T* __restrict__ Wb, int tx0, int ty0) {
    constexpr int DV = FRAME ? 2 : 3;
    using SH = TileShape<TXV>;
    __syncthreads();
    for (int i = threadIdx.x; i < SH::SITES; i += NT) {
        const int lx = i % SH::LX, ly = i / SH::LX;
        const int x = wrapi(tx0 + lx - HALO, g.Lx), y = wrapi(ty0 + ly - HALO, g.Ly);
        const int s = x + g.Lx * y;
        const T mx = mb[s], my = mb[g.N + s], mz = mb[2 * g.N + s];
        if constexpr (FRAME) {
            T e1[3], e2[3];
            onb(mx, my, mz, e1, e2);
            sh.fr[0][ly][lx] = e1[0];
            sh.fr[1][ly][lx] = e1[1];
            sh.fr[2][ly][lx] = e1[2];
            sh.fr[3][ly][lx] = e2[0];
            sh.fr[4][ly][lx] = e2[1];
            sh.fr[5][ly][lx] = e2[2];
        } else {
            sh.fr[0][ly][lx] = mx;
            sh.fr[1][ly][lx] = my;
            sh.fr[2][ly][lx] = mz;
        }
        sh.act[ly][lx] = mk ? (mk[s] != 0) : 1;
    }
    const int lx = threadIdx.x % TXV, ly = threadIdx.x / TXV;
    const int x = tx0 + lx, y = ty0 + ly;
    const bool valid = x < g.Lx && y < g.Ly;
    const int cx = lx + HALO, cy = ly + HALO;
    const int sc = x + g.Lx * y;
    const T ci = valid ? cb[sc] : T(0);
    const size_t vstride = (size_t)DV * g.N;
    for (int j = 0; j < nvec; ++j) {
        __syncthreads();
        const T* vj = Vb + j * vstride;
        for (int i = threadIdx.x; i < SH::SITES; i += NT) {
            const int lx2 = i % SH::LX, ly2 = i / SH::LX;
            const int x2 = wrapi(tx0 + lx2 - HALO, g.Lx), y2 = wrapi(ty0 + ly2 - HALO, g.Ly);
            const int s = x2 + g.Lx * y2;
            const bool on = sh.act[ly2][lx2];
            if constexpr (FRAME) {
                const T a = on ? vj[s] : T(0);
                const T b = on ? vj[g.N + s] : T(0);
                sh.t.u[0][ly2][lx2] = a * sh.fr[0][ly2][lx2] + b * sh.fr[3][ly2][lx2];
                sh.t.u[1][ly2][lx2] = a * sh.fr[1][ly2][lx2] + b * sh.fr[4][ly2][lx2];
                sh.t.u[2][ly2][lx2] = a * sh.fr[2][ly2][lx2] + b * sh.fr[5][ly2][lx2];
            } else {
                sh.t.u[0][ly2][lx2] = on ? vj[s] : T(0);
                sh.t.u[1][ly2][lx2] = on ? vj[g.N + s] : T(0);
                sh.t.u[2][ly2][lx2] = on ? vj[2 * g.N + s] : T(0);
            }
        }
        __syncthreads();
        if (valid) {
            T a[3];
            apply_A_tile(sh.t, cx, cy, k, a);
            T* wj = Wb + j * vstride;
            const bool on = sh.act[cy][cx];
            const T u0 = sh.t.u[0][cy][cx], u1 = sh.t.u[1][cy][cx], u2 = sh.t.u[2][cy][cx];
            if constexpr (FRAME) {
                const T e10 = sh.fr[0][cy][cx], e11 = sh.fr[1][cy][cx], e12 = sh.fr[2][cy][cx];
                const T e20 = sh.fr[3][cy][cx], e21 = sh.fr[4][cy][cx], e22 = sh.fr[5][cy][cx];
                const T av = e10 * u0 + e11 * u1 + e12 * u2;
                const T bv = e20 * u0 + e21 * u1 + e22 * u2;
                const T wa = e10 * a[0] + e11 * a[1] + e12 * a[2] - ci * av;
                const T wb = e20 * a[0] + e21 * a[1] + e22 * a[2] - ci * bv;
                wj[sc] = on ? wa : T(0);
                wj[g.N + sc] = on ? wb : T(0);
            } else {
                const T m0 = sh.fr[0][cy][cx], m1 = sh.fr[1][cy][cx], m2 = sh.fr[2][cy][cx];
                const T ma = m0 * a[0] + m1 * a[1] + m2 * a[2];
                wj[sc] = on ? a[0] - ma * m0 - ci * u0 : T(0);
                wj[g.N + sc] = on ? a[1] - ma * m1 - ci * u1 : T(0);
                wj[2 * g.N + sc] = on ? a[2] - ma * m2 - ci * u2 : T(0);
            }
        }
    }
}

}  // namespace moto
