// hvp.hip -- frame-layout tangent Hessian-vector product (Methods, HVP
// operator mode): W_j = M H(m) M V_j with (H v)_i = P_i (A v)_i - c_i v_i and
// tangent vectors stored as two coordinates in the per-site frame (e1, e2).
// This is the memory-bound kernel of the inner layer: 12 bytes of spins plus
// 16 bytes per vector and site (FP32).
//
// Several variants compute the same values and differ only in tiling:
//   tiled<TX,TY>:  one output site per thread on a TX x TY tile; the
//                  (TX+4) x (TY+4) neighbourhood of every vector is staged in
//                  LDS one vector at a time (frames staged once per tile);
//   band<NVP>:     tiles up to 128 sites wide (a full row band for lattices up
//                  to 128 wide, so the periodic x-halo stays in the same cache
//                  lines); NVP vectors staged per pass with one frame build per
//                  site; each thread owns one column and 4 rows and sweeps the
//                  input rows once (register sliding window);
//   march<NVP>:    one workgroup per full-width strip of rows, marching down
//                  the strip one input row at a time with the accumulators of
//                  five output rows in registers (each input element is read
//                  and converted once; see the kernel).
// All but the first order the blocks so that consecutive tiles of a lattice
// run on the same XCD: workgroups are dealt round-robin to the 8 XCDs, each
// with its own L2, and halo rows re-read by the next tile then hit that L2
// instead of HBM.  The autotuner in the host API times the variants on the
// caller's shape and keeps the fastest.
#include <type_traits>

#include "kernels.hpp"

namespace moto {

__device__ __forceinline__ int xcd_order(bool remap) {
    const int G = gridDim.x;
    return (remap && G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
}

// (A u) at flat LDS index ci of three planes with row stride SX; offsets of
// the first three shells and the NN interfacial DMI as in apply_A_tile.
template <class T, int SX>
__device__ __forceinline__ void apply_A_flat(const T* __restrict__ p0, const T* __restrict__ p1,
                                             const T* __restrict__ p2, int ci, const Coef<T>& k, T out[3]) {
    const T h = T(0.5);
    const T r3 = T(0.86602540378443864676);
    const T* pc[3] = {p0, p1, p2};
#define U(c, dx, dy) pc[c][ci + (dy) * SX + (dx)]
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

// --------------------------------------------------------------------------
// tiled<TX, TY>
// --------------------------------------------------------------------------
template <class T, int TXT, int TYT, bool REMAP>
__global__ __launch_bounds__(NT) void k_hvp_tiled(Geo g, Coef<T> k, const T* __restrict__ m,
                                                  const T* __restrict__ c, const uint8_t* __restrict__ mask, int nvec, long long vbs,
                                                  const T* __restrict__ V, T* __restrict__ W,
                                                  const int* __restrict__ done, int tiles_x, int tiles_y) {
    static_assert(TXT * TYT == NT, "one site per thread");
    if (done != nullptr && *done) return;
    constexpr int SX = TXT + 2 * HALO, SY = TYT + 2 * HALO, SS = SX * SY;
    __shared__ T u[3][SS];
    __shared__ T fr[6][SS];
    __shared__ uint8_t act[SS];
    const int bid = xcd_order(REMAP);
    const int tiles = tiles_x * tiles_y;
    const int b = bid / tiles, t = bid - b * tiles;
    const int tx0 = (t % tiles_x) * TXT, ty0 = (t / tiles_x) * TYT;
    const size_t off1 = (size_t)b * g.N;
    const T* mb = m + 3 * off1;
    const uint8_t* mk = mask ? mask + off1 : nullptr;
    const size_t vstride = (size_t)2 * g.N;
    const T* Vb = V + (size_t)b * vbs;
    T* Wb = W + (size_t)b * vbs;
    int sidx[(SS + NT - 1) / NT];
#pragma unroll
    for (int q = 0; q < (SS + NT - 1) / NT; ++q) {
        const int i = threadIdx.x + q * NT;
        sidx[q] = 0;
        if (i < SS) {
            const int ly = i / SX, lx = i - ly * SX;
            const int xs = wrapi(tx0 + lx - HALO, g.Lx), ys = wrapi(ty0 + ly - HALO, g.Ly);
            const int s = xs + g.Lx * ys;
            sidx[q] = s;
            T e1[3], e2[3];
            onb(mb[s], mb[g.N + s], mb[2 * g.N + s], e1, e2);
            fr[0][i] = e1[0];
            fr[1][i] = e1[1];
            fr[2][i] = e1[2];
            fr[3][i] = e2[0];
            fr[4][i] = e2[1];
            fr[5][i] = e2[2];
            act[i] = mk ? (mk[s] != 0) : 1;
        }
    }
    const int lx = threadIdx.x % TXT, ly = threadIdx.x / TXT;
    const int x = tx0 + lx, y = ty0 + ly;
    const bool valid = x < g.Lx && y < g.Ly;
    const int ci = (ly + HALO) * SX + lx + HALO;
    const int sc = valid ? x + g.Lx * y : 0;
    const T cc = c[off1 + sc];
    for (int j = 0; j < nvec; ++j) {
        const T* vj = Vb + j * vstride;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < (SS + NT - 1) / NT; ++q) {
            const int i = threadIdx.x + q * NT;
            if (i < SS) {
                const int s = sidx[q];
                const bool on = act[i];
                const T a = on ? vj[s] : T(0);
                const T bb = on ? vj[g.N + s] : T(0);
                u[0][i] = a * fr[0][i] + bb * fr[3][i];
                u[1][i] = a * fr[1][i] + bb * fr[4][i];
                u[2][i] = a * fr[2][i] + bb * fr[5][i];
            }
        }
        __syncthreads();
        if (valid) {
            T Au[3];
            apply_A_flat<T, SX>(u[0], u[1], u[2], ci, k, Au);
            const T e10 = fr[0][ci], e11 = fr[1][ci], e12 = fr[2][ci];
            const T e20 = fr[3][ci], e21 = fr[4][ci], e22 = fr[5][ci];
            const T u0 = u[0][ci], u1 = u[1][ci], u2 = u[2][ci];
            const T av = e10 * u0 + e11 * u1 + e12 * u2;
            const T bv = e20 * u0 + e21 * u1 + e22 * u2;
            const T wa = e10 * Au[0] + e11 * Au[1] + e12 * Au[2] - cc * av;
            const T wb = e20 * Au[0] + e21 * Au[1] + e22 * Au[2] - cc * bv;
            const bool on = act[ci];
            T* wj = Wb + j * vstride;
            wj[sc] = on ? wa : T(0);
            wj[g.N + sc] = on ? wb : T(0);
        }
    }
}

// --------------------------------------------------------------------------
// band<NVP>
// --------------------------------------------------------------------------
constexpr int BD_TX = 128;                // max tile width
constexpr int BD_TY = 8;                  // tile height
constexpr int BD_NG = NT / BD_TX;         // row groups per tile (2)
constexpr int BD_R = BD_TY / BD_NG;       // rows per thread (4)
constexpr int BD_SX = BD_TX + 2 * HALO;   // staged width (132)
constexpr int BD_SY = BD_TY + 2 * HALO;   // staged height (12)

// shell of a lattice offset (dx, dy) of the three-shell stencil, -1 if none
__device__ constexpr int bd_shell(int dx, int dy) {
    return (dx * dx + dx * dy + dy * dy) == 1 ? 0
           : (dx * dx + dx * dy + dy * dy) == 3 ? 1
           : (dx * dx + dx * dy + dy * dy) == 4 ? 2
                                                 : -1;
}

template <class T, int NVP>
__global__ __launch_bounds__(NT) void k_hvp_band(Geo g, Coef<T> k, const T* __restrict__ m,
                                                 const T* __restrict__ c, const uint8_t* __restrict__ mask, int nvec, long long vbs,
                                                 const T* __restrict__ V, T* __restrict__ W,
                                                 const int* __restrict__ done, int tiles_x, int tiles_y) {
    if (done != nullptr && *done) return;
    __shared__ T su[NVP][3][BD_SY][BD_SX];
    const int bid = xcd_order(true);
    const int tiles = tiles_x * tiles_y;
    const int b = bid / tiles;
    const int t = bid - b * tiles;
    const int tx0 = (t % tiles_x) * BD_TX, ty0 = (t / tiles_x) * BD_TY;
    const int txw = min(BD_TX, g.Lx - tx0);
    const int sxw = txw + 2 * HALO;
    const size_t off3 = (size_t)b * 3 * g.N, off1 = (size_t)b * g.N;
    const T* mb = m + off3;
    const uint8_t* mk = mask ? mask + off1 : nullptr;
    const size_t vstride = (size_t)2 * g.N;
    const T* Vb = V + (size_t)b * vbs;
    T* Wb = W + (size_t)b * vbs;
    const int lx = threadIdx.x % BD_TX, rg = threadIdx.x / BD_TX;
    const int x = tx0 + lx;
    const bool colok = lx < txw;
    T e1[BD_R][3], e2[BD_R][3], cc[BD_R];
    bool act[BD_R], rok[BD_R];
    int sc[BD_R];
#pragma unroll
    for (int o = 0; o < BD_R; ++o) {
        const int y = ty0 + rg * BD_R + o;
        rok[o] = colok && y < g.Ly;
        sc[o] = rok[o] ? x + g.Lx * y : 0;
        onb(mb[sc[o]], mb[g.N + sc[o]], mb[2 * g.N + sc[o]], e1[o], e2[o]);
        cc[o] = c[off1 + sc[o]];
        act[o] = mk == nullptr || mk[sc[o]] != 0;
    }
    const T h = T(0.5), r3 = T(0.86602540378443864676);
    for (int j0 = 0; j0 < nvec; j0 += NVP) {
        const int nv = min(NVP, nvec - j0);
        __syncthreads();
        for (int i = threadIdx.x; i < BD_SY * sxw; i += NT) {
            const int ly = i / sxw, lxs = i - ly * sxw;
            const int xs = wrapi(tx0 + lxs - HALO, g.Lx), ys = wrapi(ty0 + ly - HALO, g.Ly);
            const int s = xs + g.Lx * ys;
            T f1[3], f2[3];
            onb(mb[s], mb[g.N + s], mb[2 * g.N + s], f1, f2);
            const bool on = mk == nullptr || mk[s] != 0;
#pragma unroll
            for (int j = 0; j < NVP; ++j) {
                if (j < nv) {
                    const T a = on ? Vb[(j0 + j) * vstride + s] : T(0);
                    const T bb = on ? Vb[(j0 + j) * vstride + g.N + s] : T(0);
                    su[j][0][ly][lxs] = a * f1[0] + bb * f2[0];
                    su[j][1][ly][lxs] = a * f1[1] + bb * f2[1];
                    su[j][2][ly][lxs] = a * f1[2] + bb * f2[2];
                }
            }
        }
        __syncthreads();
        if (!colok) continue;
        for (int j = 0; j < nv; ++j) {
            T acc[BD_R][3];
#pragma unroll
            for (int o = 0; o < BD_R; ++o) acc[o][0] = acc[o][1] = acc[o][2] = T(0);
            T uc[BD_R][3];
#pragma unroll
            for (int q = 0; q < BD_R + 2 * HALO; ++q) {
                const int ly = rg * BD_R + q;
                T uu[5][3];
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx)
#pragma unroll
                    for (int cpt = 0; cpt < 3; ++cpt) uu[dx + 2][cpt] = su[j][cpt][ly][lx + HALO + dx];
#pragma unroll
                for (int o = 0; o < BD_R; ++o) {
                    const int dy = q - (o + HALO);
                    if (dy < -2 || dy > 2) continue;
                    if (dy == 0) {
                        uc[o][0] = uu[2][0];
                        uc[o][1] = uu[2][1];
                        uc[o][2] = uu[2][2];
                        acc[o][2] += k.cK * uu[2][2];
                    }
#pragma unroll
                    for (int dx = -2; dx <= 2; ++dx) {
                        const int sh = bd_shell(dx, dy);
                        if (sh < 0) continue;
                        const T cj = k.cJ[sh];
                        acc[o][0] += cj * uu[dx + 2][0];
                        acc[o][1] += cj * uu[dx + 2][1];
                        acc[o][2] += cj * uu[dx + 2][2];
                        if (sh == 0) {  // interfacial DMI: cD [dhat u_z - z (dhat . u)]
                            const T dhx = T(dx) + h * T(dy), dhy = r3 * T(dy);
                            acc[o][0] += k.cD * dhx * uu[dx + 2][2];
                            acc[o][1] += k.cD * dhy * uu[dx + 2][2];
                            acc[o][2] -= k.cD * (dhx * uu[dx + 2][0] + dhy * uu[dx + 2][1]);
                        }
                    }
                }
            }
            T* wj = Wb + (j0 + j) * vstride;
#pragma unroll
            for (int o = 0; o < BD_R; ++o) {
                if (!rok[o]) continue;
                const T av = e1[o][0] * uc[o][0] + e1[o][1] * uc[o][1] + e1[o][2] * uc[o][2];
                const T bv = e2[o][0] * uc[o][0] + e2[o][1] * uc[o][1] + e2[o][2] * uc[o][2];
                const T wa = e1[o][0] * acc[o][0] + e1[o][1] * acc[o][1] + e1[o][2] * acc[o][2] - cc[o] * av;
                const T wb = e2[o][0] * acc[o][0] + e2[o][1] * acc[o][1] + e2[o][2] * acc[o][2] - cc[o] * bv;
                wj[sc[o]] = act[o] ? wa : T(0);
                wj[g.N + sc[o]] = act[o] ? wb : T(0);
            }
        }
    }
}


// --------------------------------------------------------------------------
// march<NVP, XW>
// --------------------------------------------------------------------------
// One workgroup of XW threads owns a strip of rows [y0, y1) of one lattice
// (full width, Lx <= XW, thread x = column x) and a group of NVP vectors, and
// marches down the strip one input row R at a time, R = y0-2 .. y1+1:
//   * the thread of column x turns its raw row data (spin, c, mask, frame
//     coordinates) into ambient vectors u = a e1 + b e2 and publishes them in
//     a double-buffered LDS row (with the periodic x-halo duplicated);
//   * every offset (dx, dy) of the stencil sends row R's value at x + dx into
//     the accumulator of output row R - dy at column x.  The accumulators of
//     the five rows R-2 .. R+2 live in registers (a ring rotated at compile
//     time by unrolling the march five times), so only the four x-neighbours
//     are read from LDS and each input element is converted exactly once;
//   * row R - 2 is then complete and is projected onto its frame and stored.
// The centre term -c u and the anisotropy enter the accumulator of row R
// when R is converted; the frames of the last three rows are kept in a
// per-thread LDS ring.  Strip halos cost 4 extra input rows per strip.
// The products are written with raw buffer stores and no branch: a row
// outside the strip, a lane past the row's end or a slot past the vector
// group gets an offset beyond the buffer's range, and the hardware drops
// that store.  With the stores unconditional the compiler counts the ones
// issued after a prefetch, so the wait for a prefetched row no longer
// waits for the previous row's stores to complete.
template <int DX, int DY>
__device__ constexpr int m_shell() {
    return (DX * DX + DX * DY + DY * DY) == 1 ? 0 : (DX * DX + DX * DY + DY * DY) == 3 ? 1 : 2;
}

// acc (+)= M(dx, dy) u for one stencil offset: exchange of the offset's shell
// plus, on the first shell, the interfacial DMI term cD [dhat u_z - z (dhat . u)]
// with dhat = (dx + dy/2, sqrt(3)/2 dy) (lattice coordinates -> Cartesian).
template <int DX, int DY, bool ASSIGN, class T>
__device__ __forceinline__ void m_offset(T (&a)[3], const T (&u)[3], const T (&cJ)[3], T cD, T cDh, T cDr) {
    constexpr int sh = m_shell<DX, DY>();
    const T cj = cJ[sh];
    if (ASSIGN) {
        a[0] = cj * u[0];
        a[1] = cj * u[1];
        a[2] = cj * u[2];
    } else {
        a[0] += cj * u[0];
        a[1] += cj * u[1];
        a[2] += cj * u[2];
    }
    if constexpr (sh == 0) {
        constexpr int px = 2 * DX + DY;  // 2 dhat_x in units of 1/2
        const T dx = px == 2 ? cD : px == -2 ? -cD : px == 1 ? cDh : -cDh;
        a[0] += dx * u[2];
        a[2] -= dx * u[0];
        if constexpr (DY != 0) {
            const T dy = DY > 0 ? cDr : -cDr;
            a[1] += dy * u[2];
            a[2] -= dy * u[1];
        }
    }
}

// Frame of a unit spin for the march kernel: the Duff et al. basis, with the
// FP32 reciprocal taken by the hardware (|s + n_z| is in [1, 2], so the
// one-ulp rcp is well conditioned); FP64 keeps the exact division.
template <class T>
__device__ __forceinline__ void onb_march(T nx, T ny, T nz, T e1[3], T e2[3]) {
    const T sgn = copysign(T(1), nz);
    T a;
    if constexpr (sizeof(T) == 4)
        a = -__builtin_amdgcn_rcpf(sgn + nz);
    else
        a = T(-1) / (sgn + nz);
    const T b = nx * ny * a;
    e1[0] = T(1) + sgn * nx * nx * a;
    e1[1] = sgn * b;
    e1[2] = -sgn * nx;
    e2[0] = b;
    e2[1] = sgn + ny * ny * a;
    e2[2] = -ny;
}

// element at a 32-bit byte offset from a uniform base (selects the
// scalar-base + 32-bit vector-offset addressing form)
template <class T>
__device__ __forceinline__ T ld_off(const T* __restrict__ base, unsigned byte_off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ void st_off(T* __restrict__ base, unsigned byte_off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
// non-temporal forms for the data a launch touches once (vectors in,
// products out)
template <class T>
__device__ __forceinline__ T ld_off_nt(const T* __restrict__ base, unsigned byte_off) {
    return __builtin_nontemporal_load(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off));
}
template <class T>
__device__ __forceinline__ void st_off_nt(T* __restrict__ base, unsigned byte_off, T v) {
    __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off));
}

// raw buffer stores (stride 0: the range is num_records bytes; a store at
// or past it is dropped)
constexpr unsigned BUF_OOB = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// non-temporal (AUX 2): the products are not read again by this launch
template <class T>
__device__ __forceinline__ void buf_st_nt(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff, T v) {
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 2);
    else
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, voff, soff, 2);
}

template <class T, int NVP, int XW, bool MASKED>
__global__ __launch_bounds__(XW) void k_hvp_march(Geo g, Coef<T> k, const T* __restrict__ m,
                                                  const T* __restrict__ c, const uint8_t* __restrict__ mask, int nvec, long long vbs,
                                                  const T* __restrict__ V, T* __restrict__ W,
                                                  const int* __restrict__ done, int nstrip, int ngroups) {
    if (done != nullptr && *done) return;
    constexpr int RS = XW + 4;  // halo 2 | XW columns | halo 2
    __shared__ T rb[2][3 * NVP][RS];
    __shared__ T cen[3][MASKED ? 7 : 6][XW];
    const int lid = xcd_order(true);
    const int grp = lid % ngroups;
    const int rest = lid / ngroups;
    const int strip = rest % nstrip;
    const int b = rest / nstrip;
    const int SH = (g.Ly + nstrip - 1) / nstrip;
    const int y0 = strip * SH;
    const int y1 = min(g.Ly, y0 + SH);
    if (y0 >= y1) return;
    const int j0 = grp * NVP;
    const int nv = min(NVP, nvec - j0);
    const int x = threadIdx.x;
    const bool lane = x < g.Lx;
    // second LDS slot of this column in the periodic x-halo (needs Lx >= 4)
    const int sec = !lane ? -1 : x >= g.Lx - 2 ? x - g.Lx + 2 : x < 2 ? x + g.Lx + 2 : -1;
    // uniform plane pointers; per-lane offsets are 32-bit site indices
    const size_t N = g.N;
    const T* __restrict__ mx = m + (size_t)b * 3 * N;
    const T* __restrict__ my = mx + N;
    const T* __restrict__ mz = my + N;
    const T* __restrict__ cb = c + (size_t)b * N;
    const uint8_t* __restrict__ mk = MASKED ? mask + (size_t)b * N : nullptr;
    const T* __restrict__ Vb = V + (size_t)b * vbs + (size_t)j0 * 2 * N;
    const int PB = (int)(N * sizeof(T));  // bytes of one coordinate plane
    const __amdgpu_buffer_rsrc_t rwb = buf_rsrc(W + (size_t)b * vbs + (size_t)j0 * 2 * N, 2LL * nv * PB);
    const T cJ[3] = {k.cJ[0], k.cJ[1], k.cJ[2]};
    const T cD = k.cD, cDh = T(0.5) * k.cD, cDr = T(0.86602540378443864676) * k.cD, cK = k.cK;

    // raw data of the next input row (prefetched one step ahead); lanes past
    // the row keep a zero vector, so they contribute nothing
    T rm0 = 0, rm1 = 0, rm2 = 1, rc = 0, ra[NVP], rv[NVP];
    bool ract = true;
#pragma unroll
    for (int j = 0; j < NVP; ++j) ra[j] = rv[j] = T(0);
    int yin = wrapi(y0 - 2, g.Ly);
    auto load_raw = [&](int yy) {
        if (lane) {
            const unsigned s = (unsigned)(x + g.Lx * yy);
            const unsigned o = s * (unsigned)sizeof(T);
            rm0 = ld_off(mx, o);
            rm1 = ld_off(my, o);
            rm2 = ld_off(mz, o);
            rc = ld_off(cb, o);
            if constexpr (MASKED) ract = ld_off(mk, s) != 0;
#pragma unroll
            for (int j = 0; j < NVP; ++j) {
                // slots past the group's end re-read vector 0; their
                // accumulators are never stored
                const size_t pj = j < nv ? (size_t)(2 * j) * N : 0;
                ra[j] = ld_off_nt(Vb + pj, o);
                rv[j] = ld_off_nt(Vb + pj + N, o);
            }
        }
    };
    load_raw(yin);
    // every later prefetch is followed by its step's stores; dropped stores
    // here give the loop's entry the same pattern, so the first wait of the
    // loop also counts them instead of draining the queue
#pragma unroll
    for (int j = 0; j < 2 * NVP; ++j) buf_st_nt<T>(rwb, BUF_OOB, j * PB, T(0));

    T acc[5][NVP][3];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int j = 0; j < NVP; ++j) acc[q][j][0] = acc[q][j][1] = acc[q][j][2] = T(0);

    const int nsteps = y1 - y0 + 4;
    int cw = 0;  // centre-ring slot of the row being converted

    auto step = [&](auto qc, int R, int it) {
        constexpr int q = decltype(qc)::value;
        // ring slot of the accumulator of row R + d
#define SL(d) ((q + (d) + 10) % 5)
        const int buf = it & 1;
        // 1. convert row R
        T e1[3], e2[3];
        onb_march(rm0, rm1, rm2, e1, e2);
        const T nc = -rc;
        T u[NVP][3];
#pragma unroll
        for (int j = 0; j < NVP; ++j) {
            T a = ra[j], bb = rv[j];
            if constexpr (MASKED) {
                a = ract ? a : T(0);
                bb = ract ? bb : T(0);
            }
            u[j][0] = a * e1[0] + bb * e2[0];
            u[j][1] = a * e1[1] + bb * e2[1];
            u[j][2] = a * e1[2] + bb * e2[2];
            if (lane) {
                rb[buf][3 * j + 0][x + 2] = u[j][0];
                rb[buf][3 * j + 1][x + 2] = u[j][1];
                rb[buf][3 * j + 2][x + 2] = u[j][2];
            }
            if (sec >= 0) {
                rb[buf][3 * j + 0][sec] = u[j][0];
                rb[buf][3 * j + 1][sec] = u[j][1];
                rb[buf][3 * j + 2][sec] = u[j][2];
            }
        }
        if (R >= y0 && R < y1) {
            cen[cw][0][x] = e1[0];
            cen[cw][1][x] = e1[1];
            cen[cw][2][x] = e1[2];
            cen[cw][3][x] = e2[0];
            cen[cw][4][x] = e2[1];
            cen[cw][5][x] = e2[2];
            if constexpr (MASKED) cen[cw][MASKED ? 6 : 0][x] = ract ? T(1) : T(0);
        }
        // own-column offsets (dx = 0) and the centre term
#pragma unroll
        for (int j = 0; j < NVP; ++j) {
            m_offset<0, -2, true>(acc[SL(2)][j], u[j], cJ, cD, cDh, cDr);
            m_offset<0, -1, false>(acc[SL(1)][j], u[j], cJ, cD, cDh, cDr);
            m_offset<0, 1, false>(acc[SL(-1)][j], u[j], cJ, cD, cDh, cDr);
            m_offset<0, 2, false>(acc[SL(-2)][j], u[j], cJ, cD, cDh, cDr);
            acc[SL(0)][j][0] += nc * u[j][0];
            acc[SL(0)][j][1] += nc * u[j][1];
            acc[SL(0)][j][2] += nc * u[j][2] + cK * u[j][2];
        }
        // 2. prefetch row R + 1
        if (it + 1 < nsteps) {
            yin = yin + 1 == g.Ly ? 0 : yin + 1;
            load_raw(yin);
        }
        __syncthreads();
        // 3. x-neighbours of row R from LDS
#pragma unroll
        for (int j = 0; j < NVP; ++j) {
            T um2[3], um1[3], up1[3], up2[3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                um2[cc] = rb[buf][3 * j + cc][x];
                um1[cc] = rb[buf][3 * j + cc][x + 1];
                up1[cc] = rb[buf][3 * j + cc][x + 3];
                up2[cc] = rb[buf][3 * j + cc][x + 4];
            }
            // output row R - dy receives offset (dx, dy)
            m_offset<1, -2, false>(acc[SL(2)][j], up1, cJ, cD, cDh, cDr);
            m_offset<2, -2, false>(acc[SL(2)][j], up2, cJ, cD, cDh, cDr);
            m_offset<1, -1, false>(acc[SL(1)][j], up1, cJ, cD, cDh, cDr);
            m_offset<2, -1, false>(acc[SL(1)][j], up2, cJ, cD, cDh, cDr);
            m_offset<-1, -1, false>(acc[SL(1)][j], um1, cJ, cD, cDh, cDr);
            m_offset<1, 0, false>(acc[SL(0)][j], up1, cJ, cD, cDh, cDr);
            m_offset<-1, 0, false>(acc[SL(0)][j], um1, cJ, cD, cDh, cDr);
            m_offset<2, 0, false>(acc[SL(0)][j], up2, cJ, cD, cDh, cDr);
            m_offset<-2, 0, false>(acc[SL(0)][j], um2, cJ, cD, cDh, cDr);
            m_offset<1, 1, false>(acc[SL(-1)][j], up1, cJ, cD, cDh, cDr);
            m_offset<-1, 1, false>(acc[SL(-1)][j], um1, cJ, cD, cDh, cDr);
            m_offset<-2, 1, false>(acc[SL(-1)][j], um2, cJ, cD, cDh, cDr);
            m_offset<-1, 2, false>(acc[SL(-2)][j], um1, cJ, cD, cDh, cDr);
            m_offset<-2, 2, false>(acc[SL(-2)][j], um2, cJ, cD, cDh, cDr);
        }
        // 4. row R - 2 is complete
        const int yo = R - 2;
        const int cr = cw == 2 ? 0 : cw + 1;  // slot of row R - 2
        {
            // before the strip's first row the slot holds stale frames:
            // those stores are out of range and dropped
            const T f10 = cen[cr][0][x], f11 = cen[cr][1][x], f12 = cen[cr][2][x];
            const T f20 = cen[cr][3][x], f21 = cen[cr][4][x], f22 = cen[cr][5][x];
            bool on = true;
            if constexpr (MASKED) on = cen[cr][MASKED ? 6 : 0][x] != T(0);
            const bool row_ok = lane && yo >= y0 && yo < y1;
            const unsigned so = row_ok ? (unsigned)(x + g.Lx * yo) * (unsigned)sizeof(T) : BUF_OOB;
#pragma unroll
            for (int j = 0; j < NVP; ++j) {
                const T wa = f10 * acc[SL(-2)][j][0] + f11 * acc[SL(-2)][j][1] + f12 * acc[SL(-2)][j][2];
                const T wb = f20 * acc[SL(-2)][j][0] + f21 * acc[SL(-2)][j][1] + f22 * acc[SL(-2)][j][2];
                const unsigned sj = j < nv ? so : BUF_OOB;
                buf_st_nt<T>(rwb, sj, 2 * j * PB, on ? wa : T(0));
                buf_st_nt<T>(rwb, sj, (2 * j + 1) * PB, on ? wb : T(0));
            }
        }
        cw = cw == 2 ? 0 : cw + 1;
#undef SL
    };

    for (int it = 0; it < nsteps; it += 5) {
        const int R = y0 - 2 + it;
        step(std::integral_constant<int, 0>{}, R, it);
        if (it + 1 < nsteps) step(std::integral_constant<int, 1>{}, R + 1, it + 1);
        if (it + 2 < nsteps) step(std::integral_constant<int, 2>{}, R + 2, it + 2);
        if (it + 3 < nsteps) step(std::integral_constant<int, 3>{}, R + 3, it + 3);
        if (it + 4 < nsteps) step(std::integral_constant<int, 4>{}, R + 4, it + 4);
    }
}

// --------------------------------------------------------------------------
// march2<NVP, NT2>: the row march with two adjacent columns per thread
// --------------------------------------------------------------------------
// Same algorithm as k_hvp_march, for even Lx: thread t owns columns 2t and
// 2t + 1, so every global access is an aligned 8-byte pair (half the memory
// instructions, twice the bytes per request), the LDS row is written and
// read in pairs, and the two own columns are each other's dx = +-1
// neighbours straight from registers.  NT2 threads cover up to 2 NT2
// columns.
template <class T>
__device__ __forceinline__ void ld2(const T* __restrict__ base, unsigned byte_off, T& a, T& b) {
    typedef T V2 __attribute__((ext_vector_type(2)));
    const V2 v = *reinterpret_cast<const V2*>(reinterpret_cast<const char*>(base) + byte_off);
    a = v.x;
    b = v.y;
}
template <class T>
__device__ __forceinline__ void st2(T* __restrict__ base, unsigned byte_off, T a, T b) {
    typedef T V2 __attribute__((ext_vector_type(2)));
    V2 v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<V2*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
// streaming form for the vectors, read once per launch: non-temporal, so
// they do not displace the reused rows
template <class T>
__device__ __forceinline__ void ld2_nt(const T* __restrict__ base, unsigned byte_off, T& a, T& b) {
    typedef T V2 __attribute__((ext_vector_type(2)));
    const V2 v = __builtin_nontemporal_load(reinterpret_cast<const V2*>(reinterpret_cast<const char*>(base) + byte_off));
    a = v.x;
    b = v.y;
}
// an aligned pair of products as one raw buffer store (non-temporal)
template <class T>
__device__ __forceinline__ void buf_st2_nt(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff, T a, T b) {
    if constexpr (sizeof(T) == 4) {
        typedef unsigned U2 __attribute__((ext_vector_type(2)));
        U2 v;
        v.x = __builtin_bit_cast(unsigned, a);
        v.y = __builtin_bit_cast(unsigned, b);
        __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 2);
    } else {
        typedef unsigned U4 __attribute__((ext_vector_type(4)));
        const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
        const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
        U4 v;
        v.x = (unsigned)ua;
        v.y = (unsigned)(ua >> 32);
        v.z = (unsigned)ub;
        v.w = (unsigned)(ub >> 32);
        __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, 2);
    }
}

template <class T, int NVP, int NT2, bool MASKED>
__global__ __launch_bounds__(NT2) void k_hvp_march2(Geo g, Coef<T> k, const T* __restrict__ m,
                                                   const T* __restrict__ c, const uint8_t* __restrict__ mask,
                                                   int nvec, long long vbs, const T* __restrict__ V, T* __restrict__ W,
                                                   const int* __restrict__ done, int nstrip, int ngroups) {
    if (done != nullptr && *done) return;
    constexpr int XW = 2 * NT2;
    constexpr int RS = XW + 4;  // halo 2 | XW columns | halo 2
    __shared__ __align__(16) T rb[2][3 * NVP][RS];
    __shared__ T cen[3][MASKED ? 7 : 6][XW];
    const int lid = xcd_order(true);
    const int grp = lid % ngroups;
    const int rest = lid / ngroups;
    const int strip = rest % nstrip;
    const int b = rest / nstrip;
    const int SH = (g.Ly + nstrip - 1) / nstrip;
    const int y0 = strip * SH;
    const int y1 = min(g.Ly, y0 + SH);
    if (y0 >= y1) return;
    const int j0 = grp * NVP;
    const int nv = min(NVP, nvec - j0);
    const int x = 2 * threadIdx.x;  // first of the two columns
    const bool lane = x < g.Lx;      // Lx is even: both columns or neither
    // halo: the last pair also fills slots 0,1; the first pair slots Lx+2, Lx+3
    const int sec = !lane ? -1 : x == g.Lx - 2 ? 0 : x == 0 ? g.Lx + 2 : -1;
    const size_t N = g.N;
    const T* __restrict__ mx = m + (size_t)b * 3 * N;
    const T* __restrict__ my = mx + N;
    const T* __restrict__ mz = my + N;
    const T* __restrict__ cb = c + (size_t)b * N;
    const uint8_t* __restrict__ mk = MASKED ? mask + (size_t)b * N : nullptr;
    const T* __restrict__ Vb = V + (size_t)b * vbs + (size_t)j0 * 2 * N;
    const int PB = (int)(N * sizeof(T));  // bytes of one coordinate plane
    const __amdgpu_buffer_rsrc_t rwb = buf_rsrc(W + (size_t)b * vbs + (size_t)j0 * 2 * N, 2LL * nv * PB);
    const T cJ[3] = {k.cJ[0], k.cJ[1], k.cJ[2]};
    const T cD = k.cD, cDh = T(0.5) * k.cD, cDr = T(0.86602540378443864676) * k.cD, cK = k.cK;

    // raw data of the next input row, two columns (index 0: x, 1: x + 1)
    T rm0[2] = {0, 0}, rm1[2] = {0, 0}, rm2[2] = {1, 1}, rc[2] = {0, 0}, ra[NVP][2], rv[NVP][2];
    bool ract[2] = {true, true};
#pragma unroll
    for (int j = 0; j < NVP; ++j) ra[j][0] = ra[j][1] = rv[j][0] = rv[j][1] = T(0);
    int yin = wrapi(y0 - 2, g.Ly);
    auto load_raw = [&](int yy) {
        if (lane) {
            const unsigned s = (unsigned)(x + g.Lx * yy);
            const unsigned o = s * (unsigned)sizeof(T);
            ld2(mx, o, rm0[0], rm0[1]);
            ld2(my, o, rm1[0], rm1[1]);
            ld2(mz, o, rm2[0], rm2[1]);
            ld2(cb, o, rc[0], rc[1]);
            if constexpr (MASKED) {
                const unsigned short mm = *reinterpret_cast<const unsigned short*>(mk + s);
                ract[0] = (mm & 0xff) != 0;
                ract[1] = (mm >> 8) != 0;
            }
#pragma unroll
            for (int j = 0; j < NVP; ++j) {
                // slots past the group's end re-read vector 0; never stored
                const size_t pj = j < nv ? (size_t)(2 * j) * N : 0;
                ld2_nt(Vb + pj, o, ra[j][0], ra[j][1]);
                ld2_nt(Vb + pj + N, o, rv[j][0], rv[j][1]);
            }
        }
    };
    load_raw(yin);
    // dropped stores: the loop's entry sees the same prefetch-then-stores
    // pattern as every later step (see k_hvp_march)
#pragma unroll
    for (int j = 0; j < 2 * NVP; ++j) buf_st2_nt<T>(rwb, BUF_OOB, j * PB, T(0), T(0));

    T acc[5][NVP][2][3];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int j = 0; j < NVP; ++j)
#pragma unroll
            for (int h = 0; h < 2; ++h) acc[q][j][h][0] = acc[q][j][h][1] = acc[q][j][h][2] = T(0);

    const int nsteps = y1 - y0 + 4;
    int cw = 0;

    auto step = [&](auto qc, int R, int it) {
        constexpr int q = decltype(qc)::value;
#define SL(d) ((q + (d) + 10) % 5)
        const int buf = it & 1;
        T e1[2][3], e2[2][3];
        onb_march(rm0[0], rm1[0], rm2[0], e1[0], e2[0]);
        onb_march(rm0[1], rm1[1], rm2[1], e1[1], e2[1]);
        T u[NVP][2][3];
#pragma unroll
        for (int j = 0; j < NVP; ++j) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                T a = ra[j][h], bb = rv[j][h];
                if constexpr (MASKED) {
                    a = ract[h] ? a : T(0);
                    bb = ract[h] ? bb : T(0);
                }
                u[j][h][0] = a * e1[h][0] + bb * e2[h][0];
                u[j][h][1] = a * e1[h][1] + bb * e2[h][1];
                u[j][h][2] = a * e1[h][2] + bb * e2[h][2];
            }
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                if (lane) st2(&rb[buf][3 * j + cc][0], (unsigned)((x + 2) * sizeof(T)), u[j][0][cc], u[j][1][cc]);
                if (sec >= 0) st2(&rb[buf][3 * j + cc][0], (unsigned)(sec * sizeof(T)), u[j][0][cc], u[j][1][cc]);
            }
        }
        if (R >= y0 && R < y1) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                cen[cw][0][x + h] = e1[h][0];
                cen[cw][1][x + h] = e1[h][1];
                cen[cw][2][x + h] = e1[h][2];
                cen[cw][3][x + h] = e2[h][0];
                cen[cw][4][x + h] = e2[h][1];
                cen[cw][5][x + h] = e2[h][2];
                if constexpr (MASKED) cen[cw][MASKED ? 6 : 0][x + h] = ract[h] ? T(1) : T(0);
            }
        }
        // own-column offsets, the centre term, and the partner column (dx = +-1)
#pragma unroll
        for (int j = 0; j < NVP; ++j) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const T nc = -rc[h];
                m_offset<0, -2, true>(acc[SL(2)][j][h], u[j][h], cJ, cD, cDh, cDr);
                m_offset<0, -1, false>(acc[SL(1)][j][h], u[j][h], cJ, cD, cDh, cDr);
                m_offset<0, 1, false>(acc[SL(-1)][j][h], u[j][h], cJ, cD, cDh, cDr);
                m_offset<0, 2, false>(acc[SL(-2)][j][h], u[j][h], cJ, cD, cDh, cDr);
                acc[SL(0)][j][h][0] += nc * u[j][h][0];
                acc[SL(0)][j][h][1] += nc * u[j][h][1];
                acc[SL(0)][j][h][2] += nc * u[j][h][2] + cK * u[j][h][2];
            }
            // column x + 1 is the dx = +1 neighbour of column x, and x the
            // dx = -1 neighbour of x + 1
            m_offset<1, -2, false>(acc[SL(2)][j][0], u[j][1], cJ, cD, cDh, cDr);
            m_offset<1, -1, false>(acc[SL(1)][j][0], u[j][1], cJ, cD, cDh, cDr);
            m_offset<1, 0, false>(acc[SL(0)][j][0], u[j][1], cJ, cD, cDh, cDr);
            m_offset<1, 1, false>(acc[SL(-1)][j][0], u[j][1], cJ, cD, cDh, cDr);
            m_offset<-1, -1, false>(acc[SL(1)][j][1], u[j][0], cJ, cD, cDh, cDr);
            m_offset<-1, 0, false>(acc[SL(0)][j][1], u[j][0], cJ, cD, cDh, cDr);
            m_offset<-1, 1, false>(acc[SL(-1)][j][1], u[j][0], cJ, cD, cDh, cDr);
            m_offset<-1, 2, false>(acc[SL(-2)][j][1], u[j][0], cJ, cD, cDh, cDr);
        }
        if (it + 1 < nsteps) {
            yin = yin + 1 == g.Ly ? 0 : yin + 1;
            load_raw(yin);
        }
        __syncthreads();
        // columns x - 2, x - 1 (pair L) and x + 2, x + 3 (pair R) from LDS
#pragma unroll
        for (int j = 0; j < NVP; ++j) {
            T L0[3], L1[3], R0[3], R1[3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                ld2(&rb[buf][3 * j + cc][0], (unsigned)(x * sizeof(T)), L0[cc], L1[cc]);
                ld2(&rb[buf][3 * j + cc][0], (unsigned)((x + 4) * sizeof(T)), R0[cc], R1[cc]);
            }
            // column x: dx = -2 -> L0, -1 -> L1, +2 -> R0
            m_offset<2, -2, false>(acc[SL(2)][j][0], R0, cJ, cD, cDh, cDr);
            m_offset<2, -1, false>(acc[SL(1)][j][0], R0, cJ, cD, cDh, cDr);
            m_offset<-1, -1, false>(acc[SL(1)][j][0], L1, cJ, cD, cDh, cDr);
            m_offset<-1, 0, false>(acc[SL(0)][j][0], L1, cJ, cD, cDh, cDr);
            m_offset<2, 0, false>(acc[SL(0)][j][0], R0, cJ, cD, cDh, cDr);
            m_offset<-2, 0, false>(acc[SL(0)][j][0], L0, cJ, cD, cDh, cDr);
            m_offset<-1, 1, false>(acc[SL(-1)][j][0], L1, cJ, cD, cDh, cDr);
            m_offset<-2, 1, false>(acc[SL(-1)][j][0], L0, cJ, cD, cDh, cDr);
            m_offset<-1, 2, false>(acc[SL(-2)][j][0], L1, cJ, cD, cDh, cDr);
            m_offset<-2, 2, false>(acc[SL(-2)][j][0], L0, cJ, cD, cDh, cDr);
            // column x + 1: dx = -2 -> L1, +1 -> R0, +2 -> R1
            m_offset<1, -2, false>(acc[SL(2)][j][1], R0, cJ, cD, cDh, cDr);
            m_offset<2, -2, false>(acc[SL(2)][j][1], R1, cJ, cD, cDh, cDr);
            m_offset<1, -1, false>(acc[SL(1)][j][1], R0, cJ, cD, cDh, cDr);
            m_offset<2, -1, false>(acc[SL(1)][j][1], R1, cJ, cD, cDh, cDr);
            m_offset<1, 0, false>(acc[SL(0)][j][1], R0, cJ, cD, cDh, cDr);
            m_offset<2, 0, false>(acc[SL(0)][j][1], R1, cJ, cD, cDh, cDr);
            m_offset<-2, 0, false>(acc[SL(0)][j][1], L1, cJ, cD, cDh, cDr);
            m_offset<1, 1, false>(acc[SL(-1)][j][1], R0, cJ, cD, cDh, cDr);
            m_offset<-2, 1, false>(acc[SL(-1)][j][1], L1, cJ, cD, cDh, cDr);
            m_offset<-2, 2, false>(acc[SL(-2)][j][1], L1, cJ, cD, cDh, cDr);
        }
        const int yo = R - 2;
        const int cr = cw == 2 ? 0 : cw + 1;
        {
            // unconditional stores; rows outside the strip (stale frames)
            // and lanes past the row go out of range and are dropped
            const bool row_ok = lane && yo >= y0 && yo < y1;
            const unsigned so = row_ok ? (unsigned)(x + g.Lx * yo) * (unsigned)sizeof(T) : BUF_OOB;
            T wa[NVP][2], wb[NVP][2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const T f10 = cen[cr][0][x + h], f11 = cen[cr][1][x + h], f12 = cen[cr][2][x + h];
                const T f20 = cen[cr][3][x + h], f21 = cen[cr][4][x + h], f22 = cen[cr][5][x + h];
                bool on = true;
                if constexpr (MASKED) on = cen[cr][MASKED ? 6 : 0][x + h] != T(0);
#pragma unroll
                for (int j = 0; j < NVP; ++j) {
                    const T va = f10 * acc[SL(-2)][j][h][0] + f11 * acc[SL(-2)][j][h][1] + f12 * acc[SL(-2)][j][h][2];
                    const T vb = f20 * acc[SL(-2)][j][h][0] + f21 * acc[SL(-2)][j][h][1] + f22 * acc[SL(-2)][j][h][2];
                    wa[j][h] = on ? va : T(0);
                    wb[j][h] = on ? vb : T(0);
                }
            }
#pragma unroll
            for (int j = 0; j < NVP; ++j) {
                const unsigned sj = j < nv ? so : BUF_OOB;
                buf_st2_nt<T>(rwb, sj, 2 * j * PB, wa[j][0], wa[j][1]);
                buf_st2_nt<T>(rwb, sj, (2 * j + 1) * PB, wb[j][0], wb[j][1]);
            }
        }
        cw = cw == 2 ? 0 : cw + 1;
#undef SL
    };

    for (int it = 0; it < nsteps; it += 5) {
        const int R = y0 - 2 + it;
        step(std::integral_constant<int, 0>{}, R, it);
        if (it + 1 < nsteps) step(std::integral_constant<int, 1>{}, R + 1, it + 1);
        if (it + 2 < nsteps) step(std::integral_constant<int, 2>{}, R + 2, it + 2);
        if (it + 3 < nsteps) step(std::integral_constant<int, 3>{}, R + 3, it + 3);
        if (it + 4 < nsteps) step(std::integral_constant<int, 4>{}, R + 4, it + 4);
    }
}

// --------------------------------------------------------------------------
// variant table
// --------------------------------------------------------------------------
static const char* kNames[HVP_NVARIANTS] = {"tiled32x8",          "tiled32x8+xcd",      "tiled64x4+xcd",
                                            "tiled128x2+xcd",     "band128x8/4vec+xcd", "band128x8/2vec+xcd",
                                            "band128x8/1vec+xcd", "march/4vec",         "march/2vec",
                                            "march/1vec",         "march2/2vec",        "march2/1vec"};

const char* hvp_variant_name(int v) { return (v >= 0 && v < HVP_NVARIANTS) ? kNames[v] : "?"; }

// the row march needs the whole row in one workgroup and a two-column halo
// that does not overlap itself
// the march's store range is 32-bit: a vector group's slice (at most 4
// FP64 vectors x 2 coordinates) must stay below 2^31 bytes
static bool march_fits(const Geo& g) { return g.Lx >= 4 && g.Lx <= 512 && (long long)g.N * 64 < (1LL << 31); }

// the paired march also needs an even width (aligned column pairs)
static bool march2_fits(const Geo& g) { return march_fits(g) && (g.Lx % 2) == 0; }

bool hvp_variant_ok(int v, const Geo& g, bool f64) {
    if (v < 0 || v >= HVP_NVARIANTS) return false;
    if (f64 && (v == 4 || v == 7)) return false;
    if (v >= 7 && v <= 9 && !march_fits(g)) return false;
    if (v >= 10 && !march2_fits(g)) return false;
    return true;
}

int hvp_default_variant(const Geo& g, bool f64) { return march_fits(g) ? (f64 ? 8 : 7) : 2; }

template <class T, int TXT, int TYT, bool REMAP>
static void go_tiled(const Geo& g, const CoefD& kd, int batch, const void* m, const void* c, const uint8_t* mask,
                     int nvec, long long vbs, const void* V, void* W, const int* done, hipStream_t st) {
    const int tx = (g.Lx + TXT - 1) / TXT, ty = (g.Ly + TYT - 1) / TYT;
    hipLaunchKernelGGL((k_hvp_tiled<T, TXT, TYT, REMAP>), dim3(batch * tx * ty), dim3(NT), 0, st, g, coef_cast<T>(kd),
                       (const T*)m, (const T*)c, mask, nvec, vbs, (const T*)V, (T*)W, done, tx, ty);
}

template <class T, int NVP>
static void go_band(const Geo& g, const CoefD& kd, int batch, const void* m, const void* c, const uint8_t* mask,
                    int nvec, long long vbs, const void* V, void* W, const int* done, hipStream_t st) {
    const int tx = (g.Lx + BD_TX - 1) / BD_TX, ty = (g.Ly + BD_TY - 1) / BD_TY;
    hipLaunchKernelGGL((k_hvp_band<T, NVP>), dim3(batch * tx * ty), dim3(NT), 0, st, g, coef_cast<T>(kd),
                       (const T*)m, (const T*)c, mask, nvec, vbs, (const T*)V, (T*)W, done, tx, ty);
}

// strips per lattice: about `target` workgroups in all (one resident round
// at the march kernels' occupancy: 1024 of up to 256 threads, 256 of the
// 512-thread rows), strips of at least 8 rows (the 4 halo rows of a strip
// are read twice)
static int march_strips(const Geo& g, int batch, int ngroups, int target) {
    const long long have = (long long)batch * ngroups;
    const int want = (int)((target + have - 1) / have);
    return max(1, min(want, max(1, g.Ly / 8)));
}

template <class T, int NVP, int XW>
static void go_march_xw(const Geo& g, const CoefD& kd, int batch, const void* m, const void* c,
                        const uint8_t* mask, int nvec, long long vbs, const void* V, void* W, const int* done, hipStream_t st) {
    const int ngroups = (nvec + NVP - 1) / NVP;
    const int nstrip = march_strips(g, batch, ngroups, XW > 256 ? 256 : 1024);
    if (mask)
        hipLaunchKernelGGL((k_hvp_march<T, NVP, XW, true>), dim3(batch * nstrip * ngroups), dim3(XW), 0, st, g,
                           coef_cast<T>(kd), (const T*)m, (const T*)c, mask, nvec, vbs, (const T*)V, (T*)W, done,
                           nstrip, ngroups);
    else
        hipLaunchKernelGGL((k_hvp_march<T, NVP, XW, false>), dim3(batch * nstrip * ngroups), dim3(XW), 0, st, g,
                           coef_cast<T>(kd), (const T*)m, (const T*)c, mask, nvec, vbs, (const T*)V, (T*)W, done,
                           nstrip, ngroups);
}

template <class T, int NVP>
static void go_march(const Geo& g, const CoefD& kd, int batch, const void* m, const void* c, const uint8_t* mask,
                     int nvec, long long vbs, const void* V, void* W, const int* done, hipStream_t st) {
    if (g.Lx <= 64)
        go_march_xw<T, NVP, 64>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st);
    else if (g.Lx <= 128)
        go_march_xw<T, NVP, 128>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st);
    else if (g.Lx <= 256)
        go_march_xw<T, NVP, 256>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st);
    else
        go_march_xw<T, NVP, 512>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st);
}

template <class T, int NVP>
static void go_march2(const Geo& g, const CoefD& kd, int batch, const void* m, const void* c, const uint8_t* mask,
                      int nvec, long long vbs, const void* V, void* W, const int* done, hipStream_t st) {
    const int ngroups = (nvec + NVP - 1) / NVP;
    const int nstrip = march_strips(g, batch, ngroups, g.Lx > 256 ? 256 : 1024);
    const dim3 grid(batch * nstrip * ngroups);
    auto launch = [&](auto ntc) {
        constexpr int NT2 = decltype(ntc)::value;
        if (mask)
            hipLaunchKernelGGL((k_hvp_march2<T, NVP, NT2, true>), grid, dim3(NT2), 0, st, g, coef_cast<T>(kd),
                               (const T*)m, (const T*)c, mask, nvec, vbs, (const T*)V, (T*)W, done, nstrip, ngroups);
        else
            hipLaunchKernelGGL((k_hvp_march2<T, NVP, NT2, false>), grid, dim3(NT2), 0, st, g, coef_cast<T>(kd),
                               (const T*)m, (const T*)c, mask, nvec, vbs, (const T*)V, (T*)W, done, nstrip, ngroups);
    };
    if (g.Lx <= 128)
        launch(std::integral_constant<int, 64>{});
    else if (g.Lx <= 256)
        launch(std::integral_constant<int, 128>{});
    else
        launch(std::integral_constant<int, 256>{});
}

template <class T>
static void go(int v, const Geo& g, const CoefD& kd, int batch, const void* m, const void* c, const uint8_t* mask,
               int nvec, long long vbs, const void* V, void* W, const int* done, hipStream_t st) {
    switch (v) {
        case 0: go_tiled<T, 32, 8, false>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st); break;
        case 1: go_tiled<T, 32, 8, true>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st); break;
        case 3: go_tiled<T, 128, 2, true>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st); break;
        case 4:
            if constexpr (sizeof(T) == 4) go_band<T, 4>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st);
            break;
        case 5: go_band<T, 2>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st); break;
        case 6: go_band<T, 1>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st); break;
        case 7:
            if constexpr (sizeof(T) == 4) go_march<T, 4>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st);
            break;
        case 8: go_march<T, 2>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st); break;
        case 9: go_march<T, 1>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st); break;
        case 10: go_march2<T, 2>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st); break;
        case 11: go_march2<T, 1>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st); break;
        default: go_tiled<T, 64, 4, true>(g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st); break;
    }
}

hipError_t launch_hvp_frame(int variant, const Geo& g, const CoefD& kd, bool f64, int batch, const void* m,
                            const void* c, const uint8_t* mask, int nvec, const void* V, void* W, const int* done,
                            hipStream_t st, long long vbs) {
    const int v = hvp_variant_ok(variant, g, f64) ? variant : hvp_default_variant(g, f64);
    if (vbs <= 0) vbs = (long long)nvec * 2 * g.N;
    if (f64)
        go<double>(v, g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st);
    else
        go<float>(v, g, kd, batch, m, c, mask, nvec, vbs, V, W, done, st);
    return hipGetLastError();
}

}  // namespace moto
