// stencil.hip -- lattice kernels: energy/gradient, tangent HVP, Euclidean
// Hessian apply, mixed parameter derivatives, topological charge.
//
// Every kernel stages a (TX+4) x (TY+4) tile of 3-vectors in LDS (periodic
// wrap at the halo) and evaluates the three-shell stencil of the spin
// Hamiltonian (Methods, Eq. param-hamiltonian) at one site per thread.
#include <mutex>

#include "kernels.hpp"
#include "tile_ops.hpp"

namespace moto {

// Map a block to (lattice b, tile origin).
struct TileIdx {
    int b, tx0, ty0;
};

__device__ __forceinline__ TileIdx tile_of(const Geo& g) {
    TileIdx r;
    r.b = blockIdx.x / g.tiles;
    const int t = blockIdx.x - r.b * g.tiles;
    r.tx0 = (t % g.tiles_x) * TX;
    r.ty0 = (t / g.tiles_x) * TY;
    return r;
}

// --------------------------------------------------------------------------
// Energy, gradient, c, F and parameter partials.
// Per-block partial sums (FP64) of
//   [e_i, -m.S_0, -m.S_1, -m.S_2, m.Q_0, m.Q_1, m.Q_2, -m_z^2, -m_x, -m_y, -m_z]
// with e_i = 1/2 m_i.(A m)_i - B.m_i, so that E = sum_i e_i and
// dE/dJ_s = -sum_i m_i.S_s, dE/dD_s = sum_i m_i.Q_s, dE/dK = -sum m_z^2,
// dE/dB = -sum m.
// --------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(NT) void k_energy_grad(Geo g, Coef<T> k, const T* __restrict__ m,
                                                    const uint8_t* __restrict__ mask, T* __restrict__ grad,
                                                    T* __restrict__ cout, T* __restrict__ F,
                                                    double* __restrict__ part) {
    __shared__ TileLDS<T> t;
    __shared__ double red[NPART * (NT / 64)];
    const TileIdx ti = tile_of(g);
    const size_t off3 = (size_t)ti.b * 3 * g.N, off1 = (size_t)ti.b * g.N;
    double v[NPART];
#pragma unroll
    for (int q = 0; q < NPART; ++q) v[q] = 0.0;
    energy_tile(t, g, k, m + off3, mask ? mask + off1 : nullptr, grad ? grad + off3 : nullptr,
                cout ? cout + off1 : nullptr, F ? F + off3 : nullptr, ti.tx0, ti.ty0, v);
    block_sum<NPART>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NPART; ++q) part[(size_t)blockIdx.x * NPART + q] = v[q];
    }
}

// Mixed derivatives d(g.U)/dtheta as per-block partials in the same slots:
//   [0, -2 U.S_0, -2 U.S_1, -2 U.S_2, 2 U.Q_0, 2 U.Q_1, 2 U.Q_2, -2 U_z m_z, -U_x, -U_y, -U_z]
template <class T>
__global__ __launch_bounds__(NT) void k_param_mixed(Geo g, const T* __restrict__ m, const T* __restrict__ U,
                                                    double* __restrict__ part) {
    __shared__ TileLDS<T> t;
    __shared__ double red[NPART * (NT / 64)];
    const TileIdx ti = tile_of(g);
    const size_t off3 = (size_t)ti.b * 3 * g.N;
    const T* mb = m + off3;
    for (int i = threadIdx.x; i < TILE_SITES; i += NT) {
        const int lx = i % LXH, ly = i / LXH;
        const int x = wrapi(ti.tx0 + lx - HALO, g.Lx), y = wrapi(ti.ty0 + ly - HALO, g.Ly);
        const int s = x + g.Lx * y;
        t.u[0][ly][lx] = mb[s];
        t.u[1][ly][lx] = mb[g.N + s];
        t.u[2][ly][lx] = mb[2 * g.N + s];
    }
    __syncthreads();
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = ti.tx0 + lx, y = ti.ty0 + ly;
    double v[NPART];
#pragma unroll
    for (int q = 0; q < NPART; ++q) v[q] = 0.0;
    if (x < g.Lx && y < g.Ly) {
        const int cx = lx + HALO, cy = ly + HALO;
        const int s = x + g.Lx * y;
        const T* ub = U + off3;
        const T ui[3] = {ub[s], ub[g.N + s], ub[2 * g.N + s]};
        T S[3][3], Q[3][3];
        shell_sums(t, cx, cy, S, Q);
#pragma unroll
        for (int sh = 0; sh < 3; ++sh) {
            v[1 + sh] = -2.0 * ((double)ui[0] * S[sh][0] + (double)ui[1] * S[sh][1] + (double)ui[2] * S[sh][2]);
            v[4 + sh] = 2.0 * ((double)ui[0] * Q[sh][0] + (double)ui[1] * Q[sh][1] + (double)ui[2] * Q[sh][2]);
        }
        v[7] = -2.0 * (double)ui[2] * t.u[2][cy][cx];
        v[8] = -(double)ui[0];
        v[9] = -(double)ui[1];
        v[10] = -(double)ui[2];
    }
    block_sum<NPART>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NPART; ++q) part[(size_t)blockIdx.x * NPART + q] = v[q];
    }
}

// Parameter-weighted gradient sum  out_i = sum_q w_q dg_i/dtheta_q  (the
// adjoint of the parameter partials; g is linear in theta):
//   J_s: -2 S_s,  D_s: 2 Q_s,  K: -2 m_z z,  B_a: -e_a.
// w = [batch][2 ns + 4] (FP64), theta order (J_0.., D_0.., K, Bx, By, Bz).
template <class T>
__global__ __launch_bounds__(NT) void k_param_grad_apply(Geo g, int ns, const T* __restrict__ m,
                                                         const double* __restrict__ w, T* __restrict__ out) {
    __shared__ TileLDS<T> t;
    const TileIdx ti = tile_of(g);
    const size_t off3 = (size_t)ti.b * 3 * g.N;
    const T* mb = m + off3;
    for (int i = threadIdx.x; i < TILE_SITES; i += NT) {
        const int lx = i % LXH, ly = i / LXH;
        const int x = wrapi(ti.tx0 + lx - HALO, g.Lx), y = wrapi(ti.ty0 + ly - HALO, g.Ly);
        const int s = x + g.Lx * y;
        t.u[0][ly][lx] = mb[s];
        t.u[1][ly][lx] = mb[g.N + s];
        t.u[2][ly][lx] = mb[2 * g.N + s];
    }
    __syncthreads();
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = ti.tx0 + lx, y = ti.ty0 + ly;
    if (x >= g.Lx || y >= g.Ly) return;
    const int cx = lx + HALO, cy = ly + HALO;
    const int s = x + g.Lx * y;
    const double* wb = w + (size_t)ti.b * (2 * ns + 4);
    T S[3][3], Q[3][3];
    shell_sums(t, cx, cy, S, Q);
    double o[3];
    for (int c = 0; c < 3; ++c) {
        double v = -wb[2 * ns + 1 + c];
        for (int sh = 0; sh < ns; ++sh) v += -2.0 * wb[sh] * S[sh][c] + 2.0 * wb[ns + sh] * Q[sh][c];
        o[c] = v;
    }
    o[2] += -2.0 * wb[2 * ns] * (double)t.u[2][cy][cx];
    T* ob = out + off3;
    ob[s] = (T)o[0];
    ob[g.N + s] = (T)o[1];
    ob[2 * g.N + s] = (T)o[2];
}

// Fixed-order reduction of the per-block partials of each lattice; maps the
// slots to E[b] and dtheta[b][.] = (J_0..J_{ns-1}, D_0..D_{ns-1}, K, Bx, By, Bz).
__global__ __launch_bounds__(NT) void k_reduce_partials(const double* __restrict__ part, int tiles, int ns,
                                                        double* __restrict__ E, double* __restrict__ dth) {
    __shared__ double red[NPART * (NT / 64)];
    const int b = blockIdx.x;
    double v[NPART];
#pragma unroll
    for (int q = 0; q < NPART; ++q) v[q] = 0.0;
    for (int i = threadIdx.x; i < tiles; i += NT) {
        const double* p = part + ((size_t)b * tiles + i) * NPART;
#pragma unroll
        for (int q = 0; q < NPART; ++q) v[q] += p[q];
    }
    block_sum<NPART>(v, red);
    if (threadIdx.x == 0) {
        if (E) E[b] = v[0];
        if (dth) {
            const int np = 2 * ns + 4;
            double* o = dth + (size_t)b * np;
            for (int s = 0; s < ns; ++s) {
                o[s] = v[1 + s];
                o[ns + s] = v[4 + s];
            }
            o[2 * ns] = v[7];
            o[2 * ns + 1] = v[8];
            o[2 * ns + 2] = v[9];
            o[2 * ns + 3] = v[10];
        }
    }
}

// --------------------------------------------------------------------------
// Tangent Hessian-vector product  W_j = M H(m) M V_j  (Methods, HVP operator
// mode): (H v)_i = P_i (A v)_i - c_i v_i.
//   FRAME: V, W in frame coordinates [nvec][2][N]; the ambient vector of a
//   staged site is a e1 + b e2, and the output is (e1.(A u) - c a,
//   e2.(A u) - c b) (P_i drops out against the tangent basis).
//   AMBIENT: V, W = [nvec][3][N]; output P_i (A u)_i - c_i u_i.
// An optional device flag `done` turns the launch into a no-op (used by the
// eigen-solver once converged).
// --------------------------------------------------------------------------
template <class T, bool FRAME>
__global__ __launch_bounds__(NT) void k_tangent_hvp(Geo g, Coef<T> k, const T* __restrict__ m,
                                                    const T* __restrict__ c, const uint8_t* __restrict__ mask,
                                                    int nvec, const T* __restrict__ V, T* __restrict__ W,
                                                    const int* __restrict__ done) {
    if (done != nullptr && *done) return;
    constexpr int DV = FRAME ? 2 : 3;
    __shared__ HvpLDS<T, FRAME> sh;
    const TileIdx ti = tile_of(g);
    const size_t vb = (size_t)ti.b * nvec * DV * g.N;
    tangent_hvp_tile<T, FRAME>(sh, g, k, m + (size_t)ti.b * 3 * g.N, c + (size_t)ti.b * g.N,
                               mask ? mask + (size_t)ti.b * g.N : nullptr, nvec, V + vb, W + vb, ti.tx0, ti.ty0);
}

// Euclidean Hessian apply W_j = A V_j (ambient, unmasked).
template <class T>
__global__ __launch_bounds__(NT) void k_hessian_apply(Geo g, Coef<T> k, int nvec, const T* __restrict__ V,
                                                      T* __restrict__ W) {
    __shared__ TileLDS<T> t;
    const TileIdx ti = tile_of(g);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = ti.tx0 + lx, y = ti.ty0 + ly;
    const int sc = x + g.Lx * y;
    const size_t vstride = (size_t)3 * g.N;
    for (int j = 0; j < nvec; ++j) {
        const T* vj = V + ((size_t)ti.b * nvec + j) * vstride;
        __syncthreads();
        for (int i = threadIdx.x; i < TILE_SITES; i += NT) {
            const int lx2 = i % LXH, ly2 = i / LXH;
            const int x2 = wrapi(ti.tx0 + lx2 - HALO, g.Lx), y2 = wrapi(ti.ty0 + ly2 - HALO, g.Ly);
            const int s = x2 + g.Lx * y2;
            t.u[0][ly2][lx2] = vj[s];
            t.u[1][ly2][lx2] = vj[g.N + s];
            t.u[2][ly2][lx2] = vj[2 * g.N + s];
        }
        __syncthreads();
        if (x < g.Lx && y < g.Ly) {
            T a[3];
            apply_A_tile(t, lx + HALO, ly + HALO, k, a);
            T* wj = W + ((size_t)ti.b * nvec + j) * vstride;
            wj[sc] = a[0];
            wj[g.N + sc] = a[1];
            wj[2 * g.N + sc] = a[2];
        }
    }
}

// Berg-Luescher charge: per-block partials of -(1/4pi) * sum of the signed
// solid angles of the two triangles (x,y),(x+1,y),(x,y+1) and
// (x+1,y),(x+1,y+1),(x,y+1) of every cell (slot 0).
__global__ __launch_bounds__(NT) void k_topo_charge(Geo g, const double* __restrict__ m,
                                                    double* __restrict__ part) {
    __shared__ double red[NPART * (NT / 64)];
    const TileIdx ti = tile_of(g);
    const double* mb = m + (size_t)ti.b * 3 * g.N;
    const int x = ti.tx0 + threadIdx.x % TX, y = ti.ty0 + threadIdx.x / TX;
    double v[NPART];
#pragma unroll
    for (int q = 0; q < NPART; ++q) v[q] = 0.0;
    if (x < g.Lx && y < g.Ly) {
        const int x1 = (x + 1) % g.Lx, y1 = (y + 1) % g.Ly;
        const int s00 = x + g.Lx * y, s10 = x1 + g.Lx * y, s01 = x + g.Lx * y1, s11 = x1 + g.Lx * y1;
        const int tri[2][3] = {{s00, s10, s01}, {s10, s11, s01}};
        double q = 0.0;
        for (int t2 = 0; t2 < 2; ++t2) {
            double a[3], b[3], c[3];
            for (int cc = 0; cc < 3; ++cc) {
                a[cc] = mb[cc * g.N + tri[t2][0]];
                b[cc] = mb[cc * g.N + tri[t2][1]];
                c[cc] = mb[cc * g.N + tri[t2][2]];
            }
            const double bc0 = b[1] * c[2] - b[2] * c[1], bc1 = b[2] * c[0] - b[0] * c[2],
                         bc2 = b[0] * c[1] - b[1] * c[0];
            const double num = a[0] * bc0 + a[1] * bc1 + a[2] * bc2;
            const double den = 1.0 + (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) +
                               (b[0] * c[0] + b[1] * c[1] + b[2] * c[2]) + (c[0] * a[0] + c[1] * a[1] + c[2] * a[2]);
            q += 2.0 * atan2(num, den);
        }
        v[0] = -q / (4.0 * M_PI);
    }
    block_sum<NPART>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NPART; ++q) part[(size_t)blockIdx.x * NPART + q] = v[q];
    }
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------

hipError_t launch_energy_grad(const Geo& g, const CoefD& kd, bool f64, int batch, const void* m,
                              const uint8_t* mask, void* grad, void* c, void* F, double* part,
                              hipStream_t st) {
    if (kd.gen) return launch_energy_grad_gen(g, kd, f64, batch, m, mask, grad, c, F, part, st);
    dim3 grid(batch * g.tiles);
    if (f64)
        hipLaunchKernelGGL(k_energy_grad<double>, grid, dim3(NT), 0, st, g, coef_cast<double>(kd),
                           (const double*)m, mask, (double*)grad, (double*)c, (double*)F, part);
    else
        hipLaunchKernelGGL(k_energy_grad<float>, grid, dim3(NT), 0, st, g, coef_cast<float>(kd),
                           (const float*)m, mask, (float*)grad, (float*)c, (float*)F, part);
    return hipGetLastError();
}

hipError_t launch_param_mixed(const Geo& g, bool f64, int batch, const void* m, const void* U, double* part,
                              hipStream_t st) {
    dim3 grid(batch * g.tiles);
    if (f64)
        hipLaunchKernelGGL(k_param_mixed<double>, grid, dim3(NT), 0, st, g, (const double*)m, (const double*)U,
                           part);
    else
        hipLaunchKernelGGL(k_param_mixed<float>, grid, dim3(NT), 0, st, g, (const float*)m, (const float*)U,
                           part);
    return hipGetLastError();
}

hipError_t launch_param_grad_apply(const Geo& g, int ns, bool f64, int batch, const void* m, const double* w,
                                  void* out, hipStream_t st) {
    dim3 grid(batch * g.tiles);
    if (f64)
        hipLaunchKernelGGL(k_param_grad_apply<double>, grid, dim3(NT), 0, st, g, ns, (const double*)m, w,
                           (double*)out);
    else
        hipLaunchKernelGGL(k_param_grad_apply<float>, grid, dim3(NT), 0, st, g, ns, (const float*)m, w,
                           (float*)out);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* part, int batch, int tiles, int ns, double* E, double* dth,
                                  hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(batch), dim3(NT), 0, st, part, tiles, ns, E, dth);
    return hipGetLastError();
}

hipError_t launch_tangent_hvp(const Geo& g, const CoefD& kd, bool f64, bool frame, int batch, const void* m,
                              const void* c, const uint8_t* mask, int nvec, const void* V, void* W,
                              const int* done, hipStream_t st, int variant, long long vbs) {
    if (kd.gen) return launch_tangent_hvp_gen(g, kd, f64, frame, batch, m, c, mask, nvec, vbs, V, W, done, st);
    if (frame) return launch_hvp_frame(variant, g, kd, f64, batch, m, c, mask, nvec, V, W, done, st, vbs);
    if (vbs > 0 && vbs != (long long)nvec * 3 * g.N) return hipErrorInvalidValue;
    dim3 grid(batch * g.tiles);
    if (f64)
        hipLaunchKernelGGL((k_tangent_hvp<double, false>), grid, dim3(NT), 0, st, g, coef_cast<double>(kd),
                           (const double*)m, (const double*)c, mask, nvec, (const double*)V, (double*)W, done);
    else
        hipLaunchKernelGGL((k_tangent_hvp<float, false>), grid, dim3(NT), 0, st, g, coef_cast<float>(kd),
                           (const float*)m, (const float*)c, mask, nvec, (const float*)V, (float*)W, done);
    return hipGetLastError();
}

hipError_t launch_hessian_apply(const Geo& g, const CoefD& kd, bool f64, int batch, int nvec, const void* V,
                                void* W, hipStream_t st) {
    dim3 grid(batch * g.tiles);
    if (f64)
        hipLaunchKernelGGL(k_hessian_apply<double>, grid, dim3(NT), 0, st, g, coef_cast<double>(kd), nvec,
                           (const double*)V, (double*)W);
    else
        hipLaunchKernelGGL(k_hessian_apply<float>, grid, dim3(NT), 0, st, g, coef_cast<float>(kd), nvec,
                           (const float*)V, (float*)W);
    return hipGetLastError();
}

hipError_t launch_topo_charge(const Geo& g, int batch, const double* m, double* part, hipStream_t st) {
    hipLaunchKernelGGL(k_topo_charge, dim3(batch * g.tiles), dim3(NT), 0, st, g, m, part);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Scratch of the allocation-free energy/gradient entry point: the per-tile
// partial sums live in this file-scope array, one copy per GPU for the life
// of the process.  Host code must not use the array's name as an address (on
// the host it is only a stand-in); energy_scratch() looks up each device's
// copy once, with that device current, and hands out that pointer.
// --------------------------------------------------------------------------
static __device__ __align__(256) double scratch[ENERGY_SCRATCH_BYTES / sizeof(double)];

hipError_t energy_scratch(double** out) {
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static double* ptr[MAXDEV] = {};
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        ptr[dev] = (double*)p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

}  // namespace moto
