// common.hpp -- shared device helpers of the MI355X bilayer minimum-mode kernel.
//
// Lattice stencil of the spin Hamiltonian (Methods, Eq. param-hamiltonian) on
// the periodic rhombic triangular lattice, tangent frames, reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "moto.h"

namespace moto {

// --------------------------------------------------------------------------
// Tiling of one lattice: TX x TY output sites per 256-thread workgroup, one
// site per thread; the stencil reaches 2 sites in x and y (third shell), so
// the staged tile is (TX + 4) x (TY + 4).
// --------------------------------------------------------------------------
constexpr int TX = 32;
constexpr int TY = 8;
constexpr int HALO = 2;
constexpr int LXH = TX + 2 * HALO;  // 36
constexpr int LYH = TY + 2 * HALO;  // 12
constexpr int NT = 256;
constexpr int TILE_SITES = LXH * LYH;  // 432

struct Geo {
    int Lx, Ly, N;
    int tiles_x, tiles_y, tiles;  // tiles per lattice
};

__host__ __device__ inline Geo make_geo(int Lx, int Ly) {
    Geo g;
    g.Lx = Lx;
    g.Ly = Ly;
    g.N = Lx * Ly;
    g.tiles_x = (Lx + TX - 1) / TX;
    g.tiles_y = (Ly + TY - 1) / TY;
    g.tiles = g.tiles_x * g.tiles_y;
    return g;
}

// Stencil coefficients with the factors of the ordered-pair sums folded in:
//   (A v)_i = sum_s cJ[s] * (sum_{delta in shell s} v_{i+delta})
//           + cD * sum_{delta in NN} (z x dhat) x v_{i+delta}
//           + cK * v_iz z
// with cJ = -2 J, cD = 2 D_1, cK = -2 K.  The gradient is g = A m - B.
template <class T>
struct Coef {
    T cJ[3];
    T cD;
    T cK;
    T B[3];
};

__device__ __forceinline__ int wrapi(int x, int L) {
    int r = x % L;
    return r < 0 ? r + L : r;
}

// Orthonormal tangent basis of Duff et al. (JCGT 2017) for a unit vector n.
template <class T>
__device__ __forceinline__ void onb(T nx, T ny, T nz, T e1[3], T e2[3]) {
    const T sgn = copysign(T(1), nz);
    const T a = T(-1) / (sgn + nz);
    const T b = nx * ny * a;
    e1[0] = T(1) + sgn * nx * nx * a;
    e1[1] = sgn * b;
    e1[2] = -sgn * nx;
    e2[0] = b;
    e2[1] = sgn + ny * ny * a;
    e2[2] = -ny;
}

// Tile shapes: TXV x (NT / TXV) output sites, one per thread of a 256-thread
// workgroup (32 x 8 by default; the batched searches also use 16 x 16 and
// 64 x 4).
template <int TXV>
struct TileShape {
    static constexpr int X = TXV, Y = NT / TXV;
    static constexpr int LX = X + 2 * HALO, LY = Y + 2 * HALO, SITES = LX * LY;
};

// Staged tile: three component planes of (TY+4) x (TX+4) values.
template <class T, int TXV = TX>
struct TileLDS {
    T u[3][TileShape<TXV>::LY][TileShape<TXV>::LX];
};

// (A u) at tile-local centre (cx, cy) of the staged planes.  Offsets of the
// first three shells of the triangular lattice (dx, dy):
//   shell 1: (1,0) (0,1) (-1,1) (-1,0) (0,-1) (1,-1)
//   shell 2: (1,1) (-1,2) (-2,1) (-1,-1) (1,-2) (2,-1)
//   shell 3: (2,0) (0,2) (-2,2) (-2,0) (0,-2) (2,-2)
// Interfacial DMI through the pair differences of the three NN directions
// dhat = (1,0), (1/2, sqrt3/2), (-1/2, sqrt3/2):
//   (z x dhat) x v = dhat v_z - z (dhat . v).
template <class T, int TXV>
__device__ __forceinline__ void apply_A_tile(const TileLDS<T, TXV>& t, int cx, int cy, const Coef<T>& k,
                                             T out[3]) {
    const T h = T(0.5);
    const T r3 = T(0.86602540378443864676);
#define U(c, dx, dy) t.u[c][cy + (dy)][cx + (dx)]
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T s1 = U(c, 1, 0) + U(c, 0, 1) + U(c, -1, 1) + U(c, -1, 0) + U(c, 0, -1) + U(c, 1, -1);
        const T s2 = U(c, 1, 1) + U(c, -1, 2) + U(c, -2, 1) + U(c, -1, -1) + U(c, 1, -2) + U(c, 2, -1);
        const T s3 = U(c, 2, 0) + U(c, 0, 2) + U(c, -2, 2) + U(c, -2, 0) + U(c, 0, -2) + U(c, 2, -2);
        out[c] = k.cJ[0] * s1 + k.cJ[1] * s2 + k.cJ[2] * s3;
    }
    const T d1x = U(0, 1, 0) - U(0, -1, 0), d1z = U(2, 1, 0) - U(2, -1, 0);
    const T d2x = U(0, 0, 1) - U(0, 0, -1), d2y = U(1, 0, 1) - U(1, 0, -1), d2z = U(2, 0, 1) - U(2, 0, -1);
    const T d3x = U(0, -1, 1) - U(0, 1, -1), d3y = U(1, -1, 1) - U(1, 1, -1), d3z = U(2, -1, 1) - U(2, 1, -1);
    out[0] += k.cD * (d1z + h * d2z - h * d3z);
    out[1] += k.cD * (r3 * (d2z + d3z));
    out[2] -= k.cD * (d1x + h * d2x + r3 * d2y - h * d3x + r3 * d3y);
    out[2] += k.cK * U(2, 0, 0);
#undef U
}

// Unit-strength sums for the parameter partials at the centre:
//   S_s = sum_{delta in shell s} u_{i+delta}            (s = 0, 1, 2)
//   Q_s = sum_{delta in shell s} (z x dhat) x u_{i+delta}
// Shell 2 pairs: (1,1) dhat (sqrt3/2, 1/2); (-1,2) (0, 1); (-2,1) (-sqrt3/2, 1/2).
// Shell 3 pairs: (2,0) (1, 0); (0,2) (1/2, sqrt3/2); (-2,2) (-1/2, sqrt3/2).
template <class T, int TXV>
__device__ __forceinline__ void pair_dmi(const TileLDS<T, TXV>& t, int cx, int cy, int ax, int ay, T dhx,
                                         T dhy, T q[3]) {
    const T dx = t.u[0][cy + ay][cx + ax] - t.u[0][cy - ay][cx - ax];
    const T dy = t.u[1][cy + ay][cx + ax] - t.u[1][cy - ay][cx - ax];
    const T dz = t.u[2][cy + ay][cx + ax] - t.u[2][cy - ay][cx - ax];
    q[0] += dhx * dz;
    q[1] += dhy * dz;
    q[2] -= dhx * dx + dhy * dy;
}

template <class T, int TXV>
__device__ __forceinline__ void shell_sums(const TileLDS<T, TXV>& t, int cx, int cy, T S[3][3], T Q[3][3]) {
#define U(c, dx, dy) t.u[c][cy + (dy)][cx + (dx)]
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        S[0][c] = U(c, 1, 0) + U(c, 0, 1) + U(c, -1, 1) + U(c, -1, 0) + U(c, 0, -1) + U(c, 1, -1);
        S[1][c] = U(c, 1, 1) + U(c, -1, 2) + U(c, -2, 1) + U(c, -1, -1) + U(c, 1, -2) + U(c, 2, -1);
        S[2][c] = U(c, 2, 0) + U(c, 0, 2) + U(c, -2, 2) + U(c, -2, 0) + U(c, 0, -2) + U(c, 2, -2);
        Q[0][c] = Q[1][c] = Q[2][c] = T(0);
    }
#undef U
    const T h = T(0.5);
    const T r3 = T(0.86602540378443864676);
    pair_dmi(t, cx, cy, 1, 0, T(1), T(0), Q[0]);
    pair_dmi(t, cx, cy, 0, 1, h, r3, Q[0]);
    pair_dmi(t, cx, cy, -1, 1, -h, r3, Q[0]);
    pair_dmi(t, cx, cy, 1, 1, r3, h, Q[1]);
    pair_dmi(t, cx, cy, -1, 2, T(0), T(1), Q[1]);
    pair_dmi(t, cx, cy, -2, 1, -r3, h, Q[1]);
    pair_dmi(t, cx, cy, 2, 0, T(1), T(0), Q[2]);
    pair_dmi(t, cx, cy, 0, 2, h, r3, Q[2]);
    pair_dmi(t, cx, cy, -2, 2, -h, r3, Q[2]);
}

// --------------------------------------------------------------------------
// Deterministic reductions (fixed order, no atomics).
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block sum over NT threads of NV values; result valid in thread 0 (out[]).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /* [NV][NT/64] */) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) lds[q * (NT / 64) + w] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int i = 0; i < NT / 64; ++i) s += lds[q * (NT / 64) + i];
            v[q] = s;
        }
    }
    __syncthreads();
}

// SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014): counter-based
// uniform numbers for start blocks.
__device__ __forceinline__ double splitmix_uniform(uint64_t seed, uint64_t idx) {
    uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

}  // namespace moto
