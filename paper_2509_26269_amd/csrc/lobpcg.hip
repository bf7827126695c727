// lobpcg.hip -- device kernels of the inner layer: block LOBPCG (Knyazev
// 2001) on the tangent Hessian in frame coordinates, with every small dense
// step solved on the device in FP64 by one workgroup.
//
// Block storage (precision T, frame coordinates, rows n2 = 2N):
//   S  = [X | W | P]  = 3*mb column vectors, column-major
//   HS = [HX | HW | HP]
// The basis is kept orthonormal so that no large coefficient ever multiplies
// FP32 data (the recurrences HX <- HS C stay consistent with H X):
//   * W (the residual block) is orthonormalised against [X P] and itself,
//     twice, BEFORE its HVP (so HW is exact for the basis actually used);
//   * the new P is an orthonormal basis of the complement of the new X in
//     span(X_new, W/P part of the Ritz vectors), built in coefficient space
//     (the orthogonal-P construction of Duersch, Shao, Yang & Gu, SISC 2018);
//   * Rayleigh-Ritz still orthonormalises the Gram (SVQB, Stathopoulos & Wu
//     2002) and drops dependent directions before the eigen-solve.
// One iteration: orth(W) x2 -> HW = H W -> Grams S^T HS, S^T S (FP64,
// fixed-order reduction) -> Rayleigh-Ritz (tridiagonal QL) -> block update
// X, P, HX, HP, W = HX - X Lam -> convergence control.  Every kernel returns
// at once when the control block says the solve is done, so chunks of
// iterations can be queued without host round trips.
//
// Populations: every kernel takes blockIdx.y as the member of a population
// of independent solves on lattices of one geometry (EigArgs::P, strides
// s_ms, part_ms, g_ms); the dense per-member steps then run as P
// workgroups side by side, so a population costs about one solve's latency.
#include <algorithm>
#include <type_traits>

#include "dense_wg.hpp"
#include "kernels.hpp"

namespace moto {

constexpr int RCH = 64;                              // rows per staged chunk
static_assert(RCH % 4 == 0, "dot_chunk takes four rows per step");
constexpr int GENT = 2 * MAXS * (MAXS + 1) / 2;      // Gram entries (upper triangles of 2 matrices)
constexpr int GQ = (GENT + NT - 1) / NT;             // entries per thread
constexpr int OENT = MAXS * MAXB;                    // orthonormalisation Gram entries
constexpr int OQ = (OENT + NT - 1) / NT;
constexpr int PSTRIDE = GENT;                        // doubles per block partial row
constexpr int RED_BLOCKS = 64;                       // workgroups of the partial-row reduction
typedef double mf_d4 __attribute__((ext_vector_type(4)));  // accumulator of a 16x16x4 FP64 product
constexpr int UKS = MAXS / 4;                        // k-steps of 4 basis columns
constexpr int UPDATE_MFMA_MIN_MB = 5;                // block widths whose FP32 row kernels run on the matrix cores

// FP64 dot product of two staged chunks (RCH rows) with four interleaved
// partial sums, so the chain of dependent adds is RCH / 4 long; the order is
// fixed, so the result is reproducible
template <class T>
__device__ __forceinline__ double dot_chunk(const T* __restrict__ x, const T* __restrict__ y) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 4
    for (int rr = 0; rr < RCH; rr += 4) {
        s0 += (double)x[rr] * (double)y[rr];
        s1 += (double)x[rr + 1] * (double)y[rr + 1];
        s2 += (double)x[rr + 2] * (double)y[rr + 2];
        s3 += (double)x[rr + 3] * (double)y[rr + 3];
    }
    return (s0 + s1) + (s2 + s3);
}

__device__ __forceinline__ int sol_ns(const EigArgs& a, const EigCtrl* ctrl, int ns_fixed) {
    return ns_fixed >= 0 ? ns_fixed : 2 * a.mb + ctrl->np;
}

// --------------------------------------------------------------------------
// Start block: warm vectors (ambient FP64 or the saved ambient block)
// converted to frame coordinates at m, SplitMix64 columns for the rest;
// masked rows zero.  Resets the control block.
// --------------------------------------------------------------------------
template <class T>
__global__ void k_eig_init(EigArgs a, T* __restrict__ S, const double* __restrict__ m,
                           const double* __restrict__ Vwarm, int nwarm, const T* __restrict__ Xsave, int use_save,
                           const uint8_t* __restrict__ mask, int N, uint64_t seed, EigCtrl* ctrl) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    S += y * a.s_ms;
    m += (size_t)y * 3 * N;
    if (Vwarm) Vwarm += (size_t)y * nwarm * 3 * N;
    if (Xsave) Xsave += (size_t)y * a.mb * 3 * N;
    if (mask) mask += (size_t)y * N;
    ctrl += y;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->done = 0;
        ctrl->status = MOTO_NOT_CONVERGED;
        ctrl->iters = 0;
        ctrl->np = 0;
        ctrl->n_hvp = 0;
        ctrl->rank = a.mb;
    }
    if (s >= N) return;
    T e1[3], e2[3];
    onb((T)m[s], (T)m[N + s], (T)m[2 * N + s], e1, e2);
    const bool on = mask == nullptr || mask[s] != 0;
    for (int j = 0; j < a.mb; ++j) {
        T va, vb;
        if (use_save) {
            const T x0 = Xsave[(size_t)j * 3 * N + s], x1 = Xsave[(size_t)j * 3 * N + N + s],
                    x2 = Xsave[(size_t)j * 3 * N + 2 * N + s];
            va = e1[0] * x0 + e1[1] * x1 + e1[2] * x2;
            vb = e2[0] * x0 + e2[1] * x1 + e2[2] * x2;
        } else if (j < nwarm) {
            const double* v = Vwarm + (size_t)j * 3 * N;
            va = (T)(e1[0] * v[s] + e1[1] * v[N + s] + e1[2] * v[2 * N + s]);
            vb = (T)(e2[0] * v[s] + e2[1] * v[N + s] + e2[2] * v[2 * N + s]);
        } else {
            va = (T)splitmix_uniform(seed, (uint64_t)j * 2 * N + s);
            vb = (T)splitmix_uniform(seed, (uint64_t)j * 2 * N + N + s);
        }
        S[(size_t)j * a.n2 + s] = on ? va : T(0);
        S[(size_t)j * a.n2 + N + s] = on ? vb : T(0);
    }
}

// --------------------------------------------------------------------------
// Non-finite input (a NaN or infinite spin component or Weingarten scalar)
// ends the solve before its first step: status MOTO_NAN, eigenvalues and
// residuals NaN.  Launched after the control block is reset; every wave that
// finds such a site writes the same values.
// --------------------------------------------------------------------------
__device__ __forceinline__ void mark_nan(EigCtrl* c) {
    c->status = MOTO_NAN;
    c->done = 1;
    for (int j = 0; j < MAXB; ++j) {
        c->lam[j] = __builtin_nan("");
        c->resid[j] = __builtin_nan("");
    }
}
__device__ __forceinline__ void mark_nan(LzCtrl* c) {
    c->status = MOTO_NAN;
    c->done = 1;
    mark_nan(&c->out);
}

template <class C>
__global__ __launch_bounds__(NT) void k_check_finite(const double* __restrict__ m, const double* __restrict__ c,
                                                     int N, C* __restrict__ ctrl) {
    const int y = blockIdx.y;
    m += (size_t)y * 3 * N;
    c += (size_t)y * N;
    bool bad = false;
    for (int s = blockIdx.x * NT + threadIdx.x; s < N; s += gridDim.x * NT)
        bad = bad || !(isfinite(m[s]) && isfinite(m[N + s]) && isfinite(m[2 * N + s]) && isfinite(c[s]));
    if (__any(bad) && (threadIdx.x & 63) == 0) mark_nan(ctrl + y);
}

// --------------------------------------------------------------------------
// Orthonormalisation of a target block Y (X at the start, W afterwards)
// against the projection set Q = [X P] (empty at the start):
//   B = Q^T Y,  M = Y^T Y - B^T B  (= (Y - Q B)^T (Y - Q B) for orthonormal Q),
//   M -> D M D = Z diag(theta) Z^T,  Tw = D Z_keep theta^-1/2 (zero-padded),
//   Y <- (Y - Q B) Tw.
// Columns whose projected norm is negligible are zeroed (and so dropped by
// the Rayleigh-Ritz rank test).
// --------------------------------------------------------------------------
// Masked solves: the rows of inactive sites are zero in every column that
// is ever read (the start block is masked and the HVP is M H M), so the
// vector row kernels skip them: a Gram gains nothing from them, and an
// update or transform leaves them as they are (a column slot written only by
// those kernels may then hold stale values there, which no kernel reads: the
// Gram kernels stage such rows as zeros, the HVP masks its input).  The
// matrix-core row kernels, used from block width 5, process every row.
__device__ __forceinline__ const uint8_t* member_mask(const EigArgs& a) {
    return a.mask ? a.mask + blockIdx.y * a.mask_ms : nullptr;
}
__device__ __forceinline__ bool row_active(const uint8_t* mk, int nsite, int r) {
    return mk == nullptr || mk[r < nsite ? r : r - nsite] != 0;
}
// whole-workgroup test: does the RCH-row chunk at r0 hold an active row
// (also the barrier before the chunk is staged)
__device__ __forceinline__ bool chunk_active(const uint8_t* mk, int nsite, int n2, int r0, int rch) {
    bool any = false;
    for (int rr = threadIdx.x; rr < rch; rr += NT) any = any || (r0 + rr < n2 && row_active(mk, nsite, r0 + rr));
    return __syncthreads_or(any) != 0;
}

struct OrthCols {
    int nq;       // projection columns
    int qcol[MAXS];
    int t0;       // first target column
};

__device__ __forceinline__ void orth_cols(const EigArgs& a, int target, const EigCtrl* ctrl, OrthCols& oc) {
    oc.nq = 0;
    oc.t0 = target == 0 ? 0 : a.mb;
    if (target >= 1) {
        for (int i = 0; i < a.mb; ++i) oc.qcol[oc.nq++] = i;                    // X
        for (int i = 0; i < ctrl->np; ++i) oc.qcol[oc.nq++] = 2 * a.mb + i;     // P
    }
}

template <class T, bool MSK>
__global__ __launch_bounds__(NT) void k_orth_gram(EigArgs a, int target, const T* __restrict__ S,
                                                  double* __restrict__ part, const EigCtrl* __restrict__ ctrl) {
    S += blockIdx.y * a.s_ms;
    part += blockIdx.y * a.part_ms;
    ctrl += blockIdx.y;
    if (ctrl->done || (target == 2 && ctrl->orth_skip)) return;
    __shared__ OrthCols oc;
    __shared__ T ts[MAXS][RCH];
    if (threadIdx.x == 0) orth_cols(a, target, ctrl, oc);
    __syncthreads();
    const int nrow = oc.nq + a.mb;  // staged columns: Q then Y
    const int E = nrow * a.mb;      // entry e = j * nrow + i : (stage col i) . (Y col j)
    double acc[OQ];
#pragma unroll
    for (int q = 0; q < OQ; ++q) acc[q] = 0.0;
    const uint8_t* mk = MSK ? member_mask(a) : nullptr;
    const int nchunks = (a.n2 + RCH - 1) / RCH;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int r0 = ch * RCH;
        if constexpr (MSK) {
            if (!chunk_active(mk, a.Nsite, a.n2, r0, RCH)) continue;
        } else {
            __syncthreads();
        }
        for (int idx = threadIdx.x; idx < nrow * RCH; idx += NT) {
            const int c = idx / RCH, rr = idx % RCH, r = r0 + rr;
            const int col = c < oc.nq ? oc.qcol[c] : oc.t0 + (c - oc.nq);
            const bool in = r < a.n2 && (!MSK || row_active(mk, a.Nsite, r));
            ts[c][rr] = in ? S[(size_t)col * a.n2 + r] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < OQ; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < E) {
                const int j = e / nrow, i = e % nrow;
                const T* x = ts[i];
                const T* y = ts[oc.nq + j];
                acc[q] += dot_chunk(x, y);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < OQ; ++q) {
        const int e = threadIdx.x + q * NT;
        if (e < E) part[(size_t)blockIdx.x * PSTRIDE + e] = acc[q];
    }
}

// The orthonormalisation Gram and transform on the matrix cores (FP32 blocks,
// the same lane layout as the Rayleigh-Ritz products below).  Gram: staged
// columns [Q Y] (nrow = nq + mb, up to three 16-column tiles) against the
// target block Y (one tile), 16-row slices per wave, four products per tile
// and slice; partial rows in k_orth_gram's layout (entry j * nrow + i).
__global__ __launch_bounds__(NT) void k_orth_gram_mfma(EigArgs a, int target, const float* __restrict__ S,
                                                       double* __restrict__ part,
                                                       const EigCtrl* __restrict__ ctrl) {
    S += blockIdx.y * a.s_ms;
    part += blockIdx.y * a.part_ms;
    ctrl += blockIdx.y;
    if (ctrl->done || (target == 2 && ctrl->orth_skip)) return;
    constexpr int TT = (MAXS + 15) / 16;
    __shared__ OrthCols oc;
    __shared__ double acc_l[TT][256];
    if (threadIdx.x == 0) orth_cols(a, target, ctrl, oc);
    __syncthreads();
    const int mb = a.mb, nq = oc.nq, nrow = nq + mb, n2 = a.n2;
    const int nt = (nrow + 15) >> 4;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ln = lane & 15, lg = lane >> 4;
    // physical column of staged column 16 I + ln, and of target column ln
    int pc[TT];
#pragma unroll
    for (int I = 0; I < TT; ++I) {
        const int c = 16 * I + ln;
        pc[I] = c >= nrow ? -1 : c < nq ? oc.qcol[c] : oc.t0 + (c - nq);
    }
    const int tc = ln < mb ? oc.t0 + ln : -1;
    mf_d4 g[TT];
#pragma unroll
    for (int I = 0; I < TT; ++I) g[I] = mf_d4{0.0, 0.0, 0.0, 0.0};
    const int nslices = (n2 + 15) >> 4;
    const int nw = gridDim.x * (NT / 64);
    for (int sl = blockIdx.x * (NT / 64) + wv; sl < nslices; sl += nw) {
        const int rb = sl * 16 + 4 * lg;
        float sv[TT][4], tv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) tv[q] = (tc >= 0 && rb + q < n2) ? S[(size_t)tc * n2 + rb + q] : 0.0f;
#pragma unroll
        for (int I = 0; I < TT; ++I)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                sv[I][q] = (I < nt && pc[I] >= 0 && rb + q < n2) ? S[(size_t)pc[I] * n2 + rb + q] : 0.0f;
#pragma unroll
        for (int I = 0; I < TT; ++I) {
            if (I < nt) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    g[I] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)sv[I][q], (double)tv[q], g[I], 0, 0, 0);
            }
        }
    }
    for (int w = 0; w < NT / 64; ++w) {
        if (wv == w) {
#pragma unroll
            for (int I = 0; I < TT; ++I)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = (lg + 4 * q) * 16 + ln;  // tile row lg + 4 q, column ln
                    acc_l[I][e] = w == 0 ? g[I][q] : acc_l[I][e] + g[I][q];
                }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < nrow * mb; e += NT) {
        const int j = e / nrow, i = e - j * nrow;
        part[(size_t)blockIdx.x * PSTRIDE + e] = acc_l[i >> 4][(i & 15) * 16 + j];
    }
}

// Y <- (Y - Q B) Tw = [Q Y] [-B Tw; Tw] as 16-row tiles times that
// nrow x mb coefficient matrix (formed in LDS), in place: each wave reads
// all staged columns of its rows before it writes the new Y.
__global__ __launch_bounds__(NT) void k_orth_apply_mfma(EigArgs a, int target, float* __restrict__ S,
                                                        const EigCtrl* __restrict__ ctrl) {
    S += blockIdx.y * a.s_ms;
    ctrl += blockIdx.y;
    if (ctrl->done || (target == 2 && ctrl->orth_skip)) return;
    __shared__ OrthCols oc;
    __shared__ double cc[MAXS][16];
    if (threadIdx.x == 0) orth_cols(a, target, ctrl, oc);
    __syncthreads();
    const int mb = a.mb, nq = oc.nq, nrow = nq + mb, n2 = a.n2;
    for (int e = threadIdx.x; e < MAXS * 16; e += NT) {
        const int i = e >> 4, j = e & 15;
        double v = 0.0;
        if (i < nrow && j < mb) {
            if (i < nq) {
                for (int l = 0; l < mb; ++l) v -= ctrl->Bw[i + 2 * MAXB * l] * ctrl->Tw[l + mb * j];
            } else {
                v = ctrl->Tw[(i - nq) + mb * j];
            }
        }
        cc[i][j] = v;
    }
    __syncthreads();
    const int ks = (nrow + 3) >> 2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ln = lane & 15, lg = lane >> 4;
    const int ntiles = (n2 + 15) >> 4;
    const int nw = gridDim.x * (NT / 64);
    for (int tile = blockIdx.x * (NT / 64) + wv; tile < ntiles; tile += nw) {
        const int r0 = tile * 16, ra = r0 + ln;
        mf_d4 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < UKS; ++t) {
            if (t < ks) {
                const int i = 4 * t + lg;
                const int col = i >= nrow ? -1 : i < nq ? oc.qcol[i] : oc.t0 + (i - nq);
                const double av = (col >= 0 && ra < n2) ? (double)S[(size_t)col * n2 + ra] : 0.0;
                y = __builtin_amdgcn_mfma_f64_16x16x4f64(cc[i][ln], av, y, 0, 0, 0);
            }
        }
        // transposed product: lane (ln, lg) holds row r0 + ln of target
        // columns lg + 4 q (16 consecutive rows per store)
        if (ra < n2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int col = lg + 4 * q;
                if (col < mb) S[(size_t)(oc.t0 + col) * n2 + ra] = (float)y[q];
            }
        }
    }
}

// Multi-block fixed-order reduction of per-block partial rows:
// G[e] = sum_b part[b][e] over the entries in use (kind 0: orthonormalisation
// Gram of `arg` = target, kind 1: Rayleigh-Ritz Grams of `arg` = ns_fixed).
// One wavefront per entry: lane l sums blocks l, l + 64, ..., then a fixed
// butterfly across the lanes.
__global__ __launch_bounds__(NT) void k_reduce_rows(EigArgs a, const double* __restrict__ part, int nblk, int kind,
                                                    int arg, double* __restrict__ G,
                                                    const EigCtrl* __restrict__ ctrl) {
    part += blockIdx.y * a.part_ms;
    G += blockIdx.y * a.g_ms;
    ctrl += blockIdx.y;
    if (ctrl->done || (kind == 0 && arg == 2 && ctrl->orth_skip)) return;
    int E;
    if (kind == 0) {
        const int nq = arg >= 1 ? a.mb + ctrl->np : 0;
        E = (nq + a.mb) * a.mb;
    } else {
        const int ns = sol_ns(a, ctrl, arg);
        E = ns * (ns + 1);
    }
    const int lane = threadIdx.x & 63;
    const int nw = gridDim.x * (NT / 64);
    for (int e = blockIdx.x * (NT / 64) + (threadIdx.x >> 6); e < E; e += nw) {
        double s = 0.0;
#pragma unroll 4  // several loads in flight per lane
        for (int b = lane; b < nblk; b += 64) s += part[(size_t)b * PSTRIDE + e];
        s = wave_sum(s);
        if (lane == 0) G[e] = s;
    }
}

__global__ __launch_bounds__(WL) void k_orth_small(EigArgs a, int target, const double* __restrict__ G,
                                                   EigCtrl* __restrict__ ctrl) {
    G += blockIdx.y * a.g_ms;
    ctrl += blockIdx.y;
    if (ctrl->done || (target == 2 && ctrl->orth_skip)) return;
    const int nq = target >= 1 ? a.mb + ctrl->np : 0;
    const bool settled = orth_small_body<MAXS + 1>(a.mb, nq, a.drop, G, ctrl->Bw, ctrl->Tw);
    // after a first pass that kept every column, lost at most half of each
    // column's norm to the projection and met an inverse Cholesky factor with
    // pivots above 0.1, the block is orthonormal and orthogonal to [X P] to a
    // few FP32 roundings, which the Rayleigh-Ritz step's near-identity series
    // absorbs: the second pass is not needed
    if (target == 1 && wlane() == 0) ctrl->orth_skip = settled ? 1 : 0;
}

// MB: compile-time bound on the block width (mb <= MB), so that the per-row
// register arrays are sized for the actual block and never spill.
template <class T, int MB, bool MSK>
__global__ __launch_bounds__(NT) void k_orth_apply(EigArgs a, int target, T* __restrict__ S,
                                                   const EigCtrl* __restrict__ ctrl) {
    S += blockIdx.y * a.s_ms;
    ctrl += blockIdx.y;
    if (ctrl->done || (target == 2 && ctrl->orth_skip)) return;
    __shared__ OrthCols oc;
    __shared__ double B[2 * MAXB * MAXB];
    __shared__ double Tw[MAXB * MAXB];
    if (threadIdx.x == 0) orth_cols(a, target, ctrl, oc);
    for (int i = threadIdx.x; i < 2 * MAXB * MAXB; i += NT) B[i] = ctrl->Bw[i];
    for (int i = threadIdx.x; i < MAXB * MAXB; i += NT) Tw[i] = ctrl->Tw[i];
    __syncthreads();
    const int mb = a.mb, nq = oc.nq;
    const uint8_t* mk = MSK ? member_mask(a) : nullptr;
    for (int r = blockIdx.x * NT + threadIdx.x; r < a.n2; r += gridDim.x * NT) {
        if constexpr (MSK) {
            if (!row_active(mk, a.Nsite, r)) continue;
        }
        // at the widest bucket, keep the compiler from hoisting the LDS
        // coefficients (B: 2 MB x MB, Tw: MB x MB doubles) out of the row
        // loop into registers: that runs at the register limit and spills
        // to scratch; re-reading them from LDS per row does not
        if constexpr (MB > 8) asm volatile("" ::: "memory");
        double q[2 * MB], u[MB];
#pragma unroll
        for (int i = 0; i < 2 * MB; ++i)
            if (i < nq) q[i] = (double)S[(size_t)oc.qcol[i] * a.n2 + r];
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            if (j < mb) {
                double v = (double)S[(size_t)(oc.t0 + j) * a.n2 + r];
#pragma unroll
                for (int i = 0; i < 2 * MB; ++i)
                    if (i < nq) v -= B[i + 2 * MAXB * j] * q[i];
                u[j] = v;
            }
        }
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            if (j < mb) {
                double v = 0.0;
#pragma unroll
                for (int l = 0; l < MB; ++l)
                    if (l < mb) v += u[l] * Tw[l + mb * j];
                S[(size_t)(oc.t0 + j) * a.n2 + r] = (T)v;
            }
        }
    }
}

// --------------------------------------------------------------------------
// Rayleigh-Ritz Grams: entries e < ns(ns+1)/2 are S_i.HS_j (i <= j), the next
// ns(ns+1)/2 are S_i.S_j.  Per-block FP64 partial rows, then k_reduce_rows.
// --------------------------------------------------------------------------
__device__ __forceinline__ void tri_index(int p, int ns, int& i, int& j) {
    int ii = 0;
    while (p >= ns - ii) {
        p -= ns - ii;
        ++ii;
    }
    i = ii;
    j = ii + p;
}

template <class T, bool MSK>
__global__ __launch_bounds__(NT) void k_gram(EigArgs a, int ns_fixed, const T* __restrict__ S,
                                             const T* __restrict__ HS, double* __restrict__ part,
                                             const EigCtrl* __restrict__ ctrl) {
    S += blockIdx.y * a.s_ms;
    HS += blockIdx.y * a.s_ms;
    part += blockIdx.y * a.part_ms;
    ctrl += blockIdx.y;
    if (ctrl->done) return;
    const int ns = sol_ns(a, ctrl, ns_fixed);
    const int Eh = ns * (ns + 1) / 2, E = 2 * Eh;
    __shared__ T ts[MAXS][RCH];
    __shared__ T th[MAXS][RCH];
    int ei[GQ], ej[GQ], ew[GQ];
#pragma unroll
    for (int q = 0; q < GQ; ++q) {
        const int e = threadIdx.x + q * NT;
        ei[q] = ej[q] = ew[q] = 0;
        if (e < E) {
            ew[q] = e >= Eh;
            tri_index(e - ew[q] * Eh, ns, ei[q], ej[q]);
        }
    }
    double acc[GQ];
#pragma unroll
    for (int q = 0; q < GQ; ++q) acc[q] = 0.0;
    const uint8_t* mk = MSK ? member_mask(a) : nullptr;
    const int nchunks = (a.n2 + RCH - 1) / RCH;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int r0 = ch * RCH;
        if constexpr (MSK) {
            if (!chunk_active(mk, a.Nsite, a.n2, r0, RCH)) continue;
        } else {
            __syncthreads();
        }
        for (int idx = threadIdx.x; idx < ns * RCH; idx += NT) {
            const int col = idx / RCH, rr = idx % RCH;
            const int r = r0 + rr;
            const bool in = r < a.n2 && (!MSK || row_active(mk, a.Nsite, r));
            ts[col][rr] = in ? S[(size_t)col * a.n2 + r] : T(0);
            th[col][rr] = in ? HS[(size_t)col * a.n2 + r] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < GQ; ++q) {
            if (threadIdx.x + q * NT < E) {
                const T* x = ts[ei[q]];
                const T* y = ew[q] ? ts[ej[q]] : th[ej[q]];
                acc[q] += dot_chunk(x, y);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < GQ; ++q) {
        const int e = threadIdx.x + q * NT;
        if (e < E) part[(size_t)blockIdx.x * PSTRIDE + e] = acc[q];
    }
}

// The Rayleigh-Ritz Grams on the matrix cores (FP32 blocks): a wave takes
// 16-row slices of the basis; lane l = n + 16 g loads rows r0 + 4 g .. + 3 of
// column 16 I + n of S and of HS (one 16-byte run per column and lane group)
// and feeds element q of them to the q-th of four v_mfma_f64_16x16x4f64
// products per column-tile pair (I <= J): as A (= S^T, 16 x 4) and as B
// (= HS or S, 4 x 16) the rows of one slice then pair up the same way, so
// each product adds rows r0 + 4 g + q, g = 0..3, to the 16 x 16 tile
// (I, J).  FP32 values widened to FP64, FP64 products and sums.  The four
// waves of a workgroup add their tiles in LDS in a fixed order and the
// workgroup writes the upper triangles in k_gram's partial-row layout.
// --------------------------------------------------------------------------
constexpr int GT = (MAXS + 15) / 16;  // 16-column tiles of the basis

__global__ __launch_bounds__(NT) void k_gram_mfma(EigArgs a, int ns_fixed, const float* __restrict__ S,
                                                  const float* __restrict__ HS, double* __restrict__ part,
                                                  const EigCtrl* __restrict__ ctrl) {
    S += blockIdx.y * a.s_ms;
    HS += blockIdx.y * a.s_ms;
    part += blockIdx.y * a.part_ms;
    ctrl += blockIdx.y;
    if (ctrl->done) return;
    // tile pairs (I, J), I <= J < GT, in the order (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)
    constexpr int NPR = GT * (GT + 1) / 2;
    __shared__ double acc_l[2][NPR][256];
    const int ns = sol_ns(a, ctrl, ns_fixed);
    const int nt = (ns + 15) >> 4;
    const int n2 = a.n2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ln = lane & 15, lg = lane >> 4;
    mf_d4 ga[NPR], gb[NPR];
#pragma unroll
    for (int q = 0; q < NPR; ++q) {
        ga[q] = mf_d4{0.0, 0.0, 0.0, 0.0};
        gb[q] = ga[q];
    }
    const int nslices = (n2 + 15) >> 4;
    const int nw = gridDim.x * (NT / 64);
    for (int sl = blockIdx.x * (NT / 64) + wv; sl < nslices; sl += nw) {
        const int rb = sl * 16 + 4 * lg;  // first of this lane group's four rows
        float sv[GT][4], hv[GT][4];
#pragma unroll
        for (int I = 0; I < GT; ++I) {
            const int col = 16 * I + ln;
            const bool cin = I < nt && col < ns;
            if (cin && rb + 4 <= n2) {
                const float2 s01 = *(const float2*)(S + (size_t)col * n2 + rb);
                const float2 s23 = *(const float2*)(S + (size_t)col * n2 + rb + 2);
                const float2 h01 = *(const float2*)(HS + (size_t)col * n2 + rb);
                const float2 h23 = *(const float2*)(HS + (size_t)col * n2 + rb + 2);
                sv[I][0] = s01.x, sv[I][1] = s01.y, sv[I][2] = s23.x, sv[I][3] = s23.y;
                hv[I][0] = h01.x, hv[I][1] = h01.y, hv[I][2] = h23.x, hv[I][3] = h23.y;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool in = cin && rb + q < n2;
                    sv[I][q] = in ? S[(size_t)col * n2 + rb + q] : 0.0f;
                    hv[I][q] = in ? HS[(size_t)col * n2 + rb + q] : 0.0f;
                }
            }
        }
        int pr = 0;
#pragma unroll
        for (int I = 0; I < GT; ++I)
#pragma unroll
            for (int J = I; J < GT; ++J, ++pr) {
                if (J < nt) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double a = sv[I][q];
                        ga[pr] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, (double)hv[J][q], ga[pr], 0, 0, 0);
                        gb[pr] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, (double)sv[J][q], gb[pr], 0, 0, 0);
                    }
                }
            }
    }
    // waves 0..3 add their tiles into LDS one after another (fixed order)
    for (int w = 0; w < NT / 64; ++w) {
        if (wv == w) {
#pragma unroll
            for (int pr = 0; pr < NPR; ++pr)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = (lg + 4 * q) * 16 + ln;  // tile row lg + 4 q, column ln
                    acc_l[0][pr][e] = w == 0 ? ga[pr][q] : acc_l[0][pr][e] + ga[pr][q];
                    acc_l[1][pr][e] = w == 0 ? gb[pr][q] : acc_l[1][pr][e] + gb[pr][q];
                }
        }
        __syncthreads();
    }
    // upper triangles: entry (i, j), i <= j < ns, from tile (i / 16, j / 16)
    const int Eh = ns * (ns + 1) / 2;
    for (int e = threadIdx.x; e < Eh; e += NT) {
        int i, j;
        tri_index(e, ns, i, j);
        const int I = i >> 4, J = j >> 4;
        const int pr = I * GT - I * (I - 1) / 2 + (J - I);
        const int t = (i & 15) * 16 + (j & 15);
        part[(size_t)blockIdx.x * PSTRIDE + e] = acc_l[0][pr][t];
        part[(size_t)blockIdx.x * PSTRIDE + Eh + e] = acc_l[1][pr][t];
    }
}

// Rayleigh-Ritz step (FP64): see rr_body.  Wave 0 does the dense steps; the
// RR_WAVES waves together do the multisection of the eigen-solve.
constexpr int RR_WAVES = 4;
__global__ __launch_bounds__(RR_WAVES * WL) void k_rr(EigArgs a, int ns_fixed, const double* __restrict__ Gtri,
                                                      EigCtrl* __restrict__ ctrl) {
    Gtri += blockIdx.y * a.g_ms;
    ctrl += blockIdx.y;
    if (ctrl->done) return;
    rr_body<MAXS + 1, RR_WAVES>(a.mb, sol_ns(a, ctrl, ns_fixed), a.drop, Gtri, ctrl);
}

// --------------------------------------------------------------------------
// Block update from the Ritz coefficients (in place, row by row):
//   X <- S C,  HX <- HS C,  P <- S Cp,  HP <- HS Cp,  W <- HX - X Lam,
// and per-block partial sums of |W_j|^2.  At the start (ns == mb) P is left
// alone.
// --------------------------------------------------------------------------
template <class T, int MB, bool MSK>
__global__ __launch_bounds__(NT) void k_update(EigArgs a, int ns_fixed, T* __restrict__ S, T* __restrict__ HS,
                                               double* __restrict__ part, const EigCtrl* __restrict__ ctrl) {
    S += blockIdx.y * a.s_ms;
    HS += blockIdx.y * a.s_ms;
    part += blockIdx.y * a.part_ms;
    ctrl += blockIdx.y;
    if (ctrl->done) return;
    const int ns = sol_ns(a, ctrl, ns_fixed);
    const int mb = a.mb;
    __shared__ double C[MAXS * MAXB];
    __shared__ double Cp[MAXS * MAXB];
    __shared__ double lam[MAXB];
    __shared__ double red[MAXB * (NT / 64)];
    for (int i = threadIdx.x; i < ns * mb; i += NT) {
        C[i] = ctrl->C[i];
        Cp[i] = ctrl->Cp[i];
    }
    for (int i = threadIdx.x; i < mb; i += NT) lam[i] = ctrl->lam[i];
    __syncthreads();
    double rs[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) rs[j] = 0.0;
    const bool has_p = ns > mb;
    const uint8_t* mk = MSK ? member_mask(a) : nullptr;
    for (int r = blockIdx.x * NT + threadIdx.x; r < a.n2; r += gridDim.x * NT) {
        if constexpr (MSK) {
            if (!row_active(mk, a.Nsite, r)) continue;
        }
        T sv[3 * MB];
#pragma unroll
        for (int i = 0; i < 3 * MB; ++i)
            if (i < ns) sv[i] = S[(size_t)i * a.n2 + r];
        double xn[MB];
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            if (j < mb) {
                double x = 0.0, p = 0.0;
#pragma unroll
                for (int i = 0; i < 3 * MB; ++i) {
                    if (i < ns) {
                        x += C[i + ns * j] * (double)sv[i];
                        p += Cp[i + ns * j] * (double)sv[i];
                    }
                }
                xn[j] = x;
                S[(size_t)j * a.n2 + r] = (T)x;
                if (has_p) S[(size_t)(2 * mb + j) * a.n2 + r] = (T)p;
            }
        }
#pragma unroll
        for (int i = 0; i < 3 * MB; ++i)
            if (i < ns) sv[i] = HS[(size_t)i * a.n2 + r];
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            if (j < mb) {
                double hx = 0.0, hp = 0.0;
#pragma unroll
                for (int i = 0; i < 3 * MB; ++i) {
                    if (i < ns) {
                        hx += C[i + ns * j] * (double)sv[i];
                        hp += Cp[i + ns * j] * (double)sv[i];
                    }
                }
                HS[(size_t)j * a.n2 + r] = (T)hx;
                if (has_p) HS[(size_t)(2 * mb + j) * a.n2 + r] = (T)hp;
                const T w = (T)(hx - lam[j] * xn[j]);
                S[(size_t)(mb + j) * a.n2 + r] = w;
                rs[j] += (double)w * (double)w;
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        if (j < mb) {
            const double s = wave_sum(rs[j]);
            if (lane == 0) red[j * (NT / 64) + wv] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x < mb) {
        const int j = threadIdx.x;
        part[(size_t)blockIdx.x * MAXB + j] = red[j * 4] + red[j * 4 + 1] + red[j * 4 + 2] + red[j * 4 + 3];
    }
}

// --------------------------------------------------------------------------
// The same block update on the matrix cores (FP32 blocks, wider blocks):
// 16-row tiles of S and HS times the ns x ncol coefficient matrix [C | Cp]
// (ncol = 2 mb, or mb at the start), as v_mfma_f64_16x16x4f64 products: the
// FP32 block values are widened to FP64, products and sums are FP64, so the
// arithmetic is that of k_update in another summation order.  Each wave owns
// whole 16-row tiles (it reads every input column of its rows before it
// writes any output); one LDS load of a coefficient fragment serves a whole
// 16 x 16 x 4 product instead of one multiply-add.
// Lane layout of the 16x16x4 FP64 product (A 16 x 4, B 4 x 16, D 16 x 16):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[l / 16 + 4 i][l % 16] in accumulator element i.  Here A = a 16 x 4
// slice of the block (rows r0.., columns 4t..), B = rows 4t.. of [C | Cp].
// Residual partials |W_j|^2 per workgroup, as k_update writes them.
// --------------------------------------------------------------------------

__global__ __launch_bounds__(NT) void k_update_mfma(EigArgs a, int ns_fixed, float* __restrict__ S,
                                                    float* __restrict__ HS, double* __restrict__ part,
                                                    const EigCtrl* __restrict__ ctrl) {
    S += blockIdx.y * a.s_ms;
    HS += blockIdx.y * a.s_ms;
    part += blockIdx.y * a.part_ms;
    ctrl += blockIdx.y;
    if (ctrl->done) return;
    __shared__ double red[MAXB][NT / 64];
    const int ns = sol_ns(a, ctrl, ns_fixed);
    const int mb = a.mb, n2 = a.n2;
    const bool has_p = ns > mb;
    const int ncol = has_p ? 2 * mb : mb;
    const bool two = ncol > 16;  // a second 16-column tile of outputs
    const int ks = (ns + 3) >> 2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ln = lane & 15, lg = lane >> 4;
    // [C | Cp] in LDS, zero-padded to UKS * 4 rows and 32 columns: each
    // product reads its B fragment with one LDS load (keeping the fragments
    // in registers would cost 48 VGPRs and half the occupancy)
    __shared__ double cc[UKS * 4][32];
    for (int e = threadIdx.x; e < UKS * 4 * 32; e += NT) {
        const int i = e >> 5, j = e & 31;
        double v = 0.0;
        if (i < ns && j < ncol) v = j < mb ? ctrl->C[i + ns * j] : ctrl->Cp[i + ns * (j - mb)];
        cc[i][j] = v;
    }
    double lamj[2], rs[2] = {0.0, 0.0};
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const int j = 16 * nt + ln;
        lamj[nt] = j < mb ? ctrl->lam[j] : 0.0;
    }
    __syncthreads();
    const int ntiles = (n2 + 15) >> 4;
    const int nw = gridDim.x * (NT / 64);
    for (int tile = blockIdx.x * (NT / 64) + wv; tile < ntiles; tile += nw) {
        const int r0 = tile * 16;
        const int ra = r0 + ln;
        mf_d4 xs0 = {0.0, 0.0, 0.0, 0.0}, xs1 = xs0, xh0 = xs0, xh1 = xs0;
#pragma unroll
        for (int t = 0; t < UKS; ++t) {
            if (t < ks) {
                const int i = 4 * t + lg;
                const bool in = i < ns && ra < n2;
                const double as = in ? (double)S[(size_t)i * n2 + ra] : 0.0;
                const double ah = in ? (double)HS[(size_t)i * n2 + ra] : 0.0;
                const double b0 = cc[i][ln];
                xs0 = __builtin_amdgcn_mfma_f64_16x16x4f64(as, b0, xs0, 0, 0, 0);
                xh0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ah, b0, xh0, 0, 0, 0);
                if (two) {
                    const double b1 = cc[i][16 + ln];
                    xs1 = __builtin_amdgcn_mfma_f64_16x16x4f64(as, b1, xs1, 0, 0, 0);
                    xh1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ah, b1, xh1, 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int j = 16 * nt + ln;
            if (nt == 1 && !two) break;
            const mf_d4 xs = nt == 0 ? xs0 : xs1;
            const mf_d4 xh = nt == 0 ? xh0 : xh1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = r0 + lg + 4 * q;
                if (row >= n2) continue;
                if (j < mb) {
                    S[(size_t)j * n2 + row] = (float)xs[q];
                    HS[(size_t)j * n2 + row] = (float)xh[q];
                    const float w = (float)(xh[q] - lamj[nt] * xs[q]);
                    S[(size_t)(mb + j) * n2 + row] = w;
                    rs[nt] += (double)w * (double)w;
                } else if (j < ncol) {
                    S[(size_t)(mb + j) * n2 + row] = (float)xs[q];  // P column j - mb
                    HS[(size_t)(mb + j) * n2 + row] = (float)xh[q];
                }
            }
        }
    }
    // |W_j|^2: the four lane groups of column j, then the waves (fixed order)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        double v = rs[nt];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        const int j = 16 * nt + ln;
        if (lg == 0 && j < mb) red[j][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < mb) {
        const int j = threadIdx.x;
        part[(size_t)blockIdx.x * MAXB + j] = (red[j][0] + red[j][1]) + (red[j][2] + red[j][3]);
    }
}

// Convergence control: residual norms (one wavefront per column, fixed-order
// sums), then one thread checks NaN, rank, convergence and the cap.
__global__ __launch_bounds__(NT) void k_eig_control(EigArgs a, const double* __restrict__ part, int nblk,
                                                    EigCtrl* __restrict__ ctrl, int first) {
    part += blockIdx.y * a.part_ms;
    ctrl += blockIdx.y;
    if (ctrl->done) return;
    __shared__ double rsq[MAXB];
    const int lane = threadIdx.x & 63;
    for (int j = threadIdx.x >> 6; j < a.mb; j += NT / 64) {
        double s = 0.0;
#pragma unroll 8  // several loads in flight per lane
        for (int b = lane; b < nblk; b += 64) s += part[(size_t)b * MAXB + j];
        s = wave_sum(s);
        if (lane == 0) rsq[j] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    bool conv = true, bad = false;
    for (int j = 0; j < a.mb; ++j) {
        const double rj = sqrt(rsq[j]);
        ctrl->resid[j] = rj;
        if (!isfinite(rj) || !isfinite(ctrl->lam[j])) bad = true;
        if (j < a.k && !(rj <= a.tol_abs)) conv = false;
    }
    ctrl->n_hvp += a.mb;
    if (!first) {
        ctrl->iters += 1;
        ctrl->np = a.mb;
    }
    if (bad) {
        ctrl->status = MOTO_NAN;
        ctrl->done = 1;
    } else if (ctrl->rank < a.k) {
        ctrl->status = MOTO_BREAKDOWN;
        ctrl->done = 1;
    } else if (conv) {
        ctrl->status = MOTO_CONVERGED;
        ctrl->done = 1;
    } else if (ctrl->iters >= a.max_iter) {
        ctrl->status = MOTO_NOT_CONVERGED;
        ctrl->done = 1;
    }
}

// all_done = AND of the members' done flags (one wavefront, fixed order)
__global__ __launch_bounds__(WL) void k_eig_all_done(int P, const EigCtrl* __restrict__ ctrl,
                                                     int* __restrict__ all_done) {
    int d = 1;
    for (int y = threadIdx.x; y < P; y += WL) d &= ctrl[y].done != 0;
    d = __all(d);
    if (threadIdx.x == 0) *all_done = d;
}

// --------------------------------------------------------------------------
// Output: the first k block columns to ambient FP64 unit vectors with the
// sign rule (entry of largest magnitude, first in [3][N] order, positive);
// the whole block saved ambient for a warm restart.
// Partials per block and column: [|v|^2, max|v_c,s|, first flat index of it].
// --------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(NT) void k_eig_out1(EigArgs a, const T* __restrict__ S, const double* __restrict__ m,
                                                 int N, double* __restrict__ V, double* __restrict__ part,
                                                 T* __restrict__ Xsave) {
    __shared__ double rn[MAXB][NT / 64], rm[MAXB][NT / 64], ri[MAXB][NT / 64];
    const int s = blockIdx.x * NT + threadIdx.x;
    const int y = blockIdx.y;
    S += y * a.s_ms;
    m += (size_t)y * 3 * N;
    V += (size_t)y * a.k * 3 * N;
    part += y * a.part_ms;
    if (Xsave) Xsave += (size_t)y * a.mb * 3 * N;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    T e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
    if (s < N) onb((T)m[s], (T)m[N + s], (T)m[2 * N + s], e1, e2);
    for (int j = 0; j < a.mb; ++j) {
        double nrm = 0.0, mx = -1.0, mi = 1e300;
        if (s < N) {
            const T va = S[(size_t)j * a.n2 + s], vb = S[(size_t)j * a.n2 + N + s];
            for (int c = 0; c < 3; ++c) {
                const T amb = va * e1[c] + vb * e2[c];
                if (Xsave) Xsave[(size_t)j * 3 * N + c * N + s] = amb;
                if (j < a.k) {
                    const double v = (double)amb;
                    V[(size_t)j * 3 * N + c * N + s] = v;
                    nrm += v * v;
                    const double av = fabs(v);
                    const double idx = (double)(c * N + s);
                    if (av > mx || (av == mx && idx < mi)) {
                        mx = av;
                        mi = idx;
                    }
                }
            }
        }
        if (j < a.k) {
            nrm = wave_sum(nrm);
            for (int o = 32; o > 0; o >>= 1) {
                const double omx = __shfl_xor(mx, o, 64), omi = __shfl_xor(mi, o, 64);
                if (omx > mx || (omx == mx && omi < mi)) {
                    mx = omx;
                    mi = omi;
                }
            }
            if (lane == 0) {
                rn[j][wv] = nrm;
                rm[j][wv] = mx;
                ri[j][wv] = mi;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < a.k) {
        const int j = threadIdx.x;
        double n = 0.0, mx = -1.0, mi = 1e300;
        for (int w = 0; w < NT / 64; ++w) {
            n += rn[j][w];
            if (rm[j][w] > mx || (rm[j][w] == mx && ri[j][w] < mi)) {
                mx = rm[j][w];
                mi = ri[j][w];
            }
        }
        double* p = part + ((size_t)blockIdx.x * MAXB + j) * 3;
        p[0] = n;
        p[1] = mx;
        p[2] = mi;
    }
}

__global__ void k_eig_out2(EigArgs a, const double* __restrict__ part, int nblk, const double* __restrict__ V,
                           int N, double* __restrict__ scale, const EigCtrl* __restrict__ ctrl,
                           double* __restrict__ evals, double* __restrict__ resid) {
    const int y = blockIdx.y;
    part += y * a.part_ms;
    V += (size_t)y * a.k * 3 * N;
    scale += y * a.part_ms;
    ctrl += y;
    if (evals) evals += y * a.k;
    if (resid) resid += y * a.k;
    const int j = threadIdx.x;
    if (j >= a.k) return;
    double n = 0.0, mx = -1.0, mi = 1e300;
#pragma unroll 8  // several loads in flight
    for (int b = 0; b < nblk; ++b) {
        const double* p = part + ((size_t)b * MAXB + j) * 3;
        n += p[0];
        if (p[1] > mx || (p[1] == mx && p[2] < mi)) {
            mx = p[1];
            mi = p[2];
        }
    }
    const long long idx = (long long)mi;
    const double sgn = (idx >= 0 && idx < 3LL * N && V[(size_t)j * 3 * N + idx] < 0.0) ? -1.0 : 1.0;
    scale[j] = n > 0.0 ? sgn / sqrt(n) : 0.0;
    if (evals) evals[j] = ctrl->lam[j];
    if (resid) resid[j] = ctrl->resid[j];
}

// scale of member y, column j at scale[y * part_ms + j]
__global__ void k_eig_out3(int k, int N, int P, long long part_ms, double* __restrict__ V,
                           const double* __restrict__ scale) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t tot = (size_t)P * k * 3 * N;
    if (i >= tot) return;
    const size_t col = i / (3 * (size_t)N);
    const size_t y = col / k, j = col - y * k;
    V[i] *= scale[y * part_ms + j];
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
// workgroups of the Gram kernels: up to 256, and up to 1024 for bases of
// more than 2^18 rows, where each of 256 workgroups would walk 16 or more
// RCH-row chunks one after another (128 on a 1024x1024 lattice); the
// partial-row workspace is sized from this count
int gram_blocks(int n2) {
    const int nch = (n2 + RCH - 1) / RCH;
    const int cap = n2 > (1 << 18) ? 1024 : 256;
    return nch < cap ? nch : cap;
}

// workgroups of the row-update kernels: one row per thread for the vector
// kernels; for the matrix-core kernels one 16-row tile per wave (64 rows per
// workgroup), so that a small lattice still keeps every compute unit busy
// (each wave would otherwise wait out the load latency of several tiles in
// turn); at most 1024, with grid-stride loops beyond
bool rows_on_matrix_cores(bool f64, int mb) { return !f64 && mb >= UPDATE_MFMA_MIN_MB; }

int update_blocks(int n2, bool f64, int mb) {
    const bool mfma = rows_on_matrix_cores(f64, mb);
    const int rows = mfma ? (NT / 64) * 16 : NT;
    const int nb = (n2 + rows - 1) / rows;
    return nb < 1024 ? nb : 1024;
}

// dispatch on the block-width bucket (4, 8 or 16 columns)
template <class F>
static void go_mb(int mb, F&& f) {
    if (mb <= 4)
        f(std::integral_constant<int, 4>{});
    else if (mb <= 8)
        f(std::integral_constant<int, 8>{});
    else
        f(std::integral_constant<int, MAXB>{});
}

hipError_t launch_eig_init(bool f64, const EigArgs& a, void* S, const double* m, const double* Vwarm, int nwarm,
                           const void* Xsave, int use_save, const uint8_t* mask, int N, uint64_t seed,
                           EigCtrl* ctrl, hipStream_t st) {
    dim3 grid((N + NT - 1) / NT, a.P);
    if (f64)
        hipLaunchKernelGGL(k_eig_init<double>, grid, dim3(NT), 0, st, a, (double*)S, m, Vwarm, nwarm,
                           (const double*)Xsave, use_save, mask, N, seed, ctrl);
    else
        hipLaunchKernelGGL(k_eig_init<float>, grid, dim3(NT), 0, st, a, (float*)S, m, Vwarm, nwarm,
                           (const float*)Xsave, use_save, mask, N, seed, ctrl);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double* m, const double* c, int N, int P, EigCtrl* ctrl, hipStream_t st) {
    const int nb = std::min((N + NT - 1) / NT, 1024);
    hipLaunchKernelGGL(k_check_finite<EigCtrl>, dim3(nb, P), dim3(NT), 0, st, m, c, N, ctrl);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double* m, const double* c, int N, LzCtrl* ctrl, hipStream_t st) {
    const int nb = std::min((N + NT - 1) / NT, 1024);
    hipLaunchKernelGGL(k_check_finite<LzCtrl>, dim3(nb, 1), dim3(NT), 0, st, m, c, N, ctrl);
    return hipGetLastError();
}

// dispatch on masking (the vector row kernels skip inactive rows only in
// their masked instantiation)
template <class F>
static void go_mask(const EigArgs& a, F&& f) {
    if (a.mask)
        f(std::true_type{});
    else
        f(std::false_type{});
}

hipError_t launch_orth(bool f64, const EigArgs& a, int target, void* S, double* part, int nblk, double* G,
                       EigCtrl* ctrl, hipStream_t st) {
    const bool mf = rows_on_matrix_cores(f64, a.mb);
    if (mf)
        hipLaunchKernelGGL(k_orth_gram_mfma, dim3(nblk, a.P), dim3(NT), 0, st, a, target, (const float*)S, part,
                           ctrl);
    else
        go_mask(a, [&](auto mk) {
            constexpr bool M = decltype(mk)::value;
            if (f64)
                hipLaunchKernelGGL((k_orth_gram<double, M>), dim3(nblk, a.P), dim3(NT), 0, st, a, target,
                                   (const double*)S, part, ctrl);
            else
                hipLaunchKernelGGL((k_orth_gram<float, M>), dim3(nblk, a.P), dim3(NT), 0, st, a, target,
                                   (const float*)S, part, ctrl);
        });
    hipLaunchKernelGGL(k_reduce_rows, dim3(RED_BLOCKS, a.P), dim3(NT), 0, st, a, part, nblk, 0, target, G, ctrl);
    hipLaunchKernelGGL(k_orth_small, dim3(1, a.P), dim3(WL), 0, st, a, target, G, ctrl);
    const int nb = update_blocks(a.n2, f64, a.mb);
    if (mf) {
        hipLaunchKernelGGL(k_orth_apply_mfma, dim3(nb, a.P), dim3(NT), 0, st, a, target, (float*)S, ctrl);
        return hipGetLastError();
    }
    go_mask(a, [&](auto mk) {
        constexpr bool M = decltype(mk)::value;
        go_mb(a.mb, [&](auto mbc) {
            constexpr int W = decltype(mbc)::value;
            if (f64)
                hipLaunchKernelGGL((k_orth_apply<double, W, M>), dim3(nb, a.P), dim3(NT), 0, st, a, target,
                                   (double*)S, ctrl);
            else
                hipLaunchKernelGGL((k_orth_apply<float, W, M>), dim3(nb, a.P), dim3(NT), 0, st, a, target,
                                   (float*)S, ctrl);
        });
    });
    return hipGetLastError();
}

hipError_t launch_gram(bool f64, const EigArgs& a, int ns, const void* S, const void* HS, double* part, int nblk,
                       double* G, const EigCtrl* ctrl, hipStream_t st) {
    if (rows_on_matrix_cores(f64, a.mb))
        hipLaunchKernelGGL(k_gram_mfma, dim3(nblk, a.P), dim3(NT), 0, st, a, ns, (const float*)S, (const float*)HS,
                           part, ctrl);
    else
        go_mask(a, [&](auto mk) {
            constexpr bool M = decltype(mk)::value;
            if (f64)
                hipLaunchKernelGGL((k_gram<double, M>), dim3(nblk, a.P), dim3(NT), 0, st, a, ns, (const double*)S,
                                   (const double*)HS, part, ctrl);
            else
                hipLaunchKernelGGL((k_gram<float, M>), dim3(nblk, a.P), dim3(NT), 0, st, a, ns, (const float*)S,
                                   (const float*)HS, part, ctrl);
        });
    hipLaunchKernelGGL(k_reduce_rows, dim3(RED_BLOCKS, a.P), dim3(NT), 0, st, a, part, nblk, 1, ns, G, ctrl);
    return hipGetLastError();
}

hipError_t launch_rr(const EigArgs& a, int ns, const double* G, EigCtrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL(k_rr, dim3(1, a.P), dim3(RR_WAVES * WL), 0, st, a, ns, G, ctrl);
    return hipGetLastError();
}

hipError_t launch_update(bool f64, const EigArgs& a, int ns, void* S, void* HS, double* part, int nblk,
                         EigCtrl* ctrl, hipStream_t st) {
    if (rows_on_matrix_cores(f64, a.mb)) {
        hipLaunchKernelGGL(k_update_mfma, dim3(nblk, a.P), dim3(NT), 0, st, a, ns, (float*)S, (float*)HS, part, ctrl);
        return hipGetLastError();
    }
    go_mask(a, [&](auto mk) {
        constexpr bool M = decltype(mk)::value;
        go_mb(a.mb, [&](auto mbc) {
            constexpr int W = decltype(mbc)::value;
            if (f64)
                hipLaunchKernelGGL((k_update<double, W, M>), dim3(nblk, a.P), dim3(NT), 0, st, a, ns, (double*)S,
                                   (double*)HS, part, ctrl);
            else
                hipLaunchKernelGGL((k_update<float, W, M>), dim3(nblk, a.P), dim3(NT), 0, st, a, ns, (float*)S,
                                   (float*)HS, part, ctrl);
        });
    });
    return hipGetLastError();
}

hipError_t launch_eig_control(const EigArgs& a, const double* part, int nblk, EigCtrl* ctrl, int first,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_eig_control, dim3(1, a.P), dim3(NT), 0, st, a, part, nblk, ctrl, first);
    return hipGetLastError();
}

// outcome of every member in one array (status, iterations, HVP columns)
__global__ void k_eig_gather_info(int P, const EigCtrl* __restrict__ ctrl, moto_info* __restrict__ out) {
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= P) return;
    moto_info r;
    r.status = ctrl[y].status;
    r.iters = ctrl[y].iters;
    r.n_hvp = ctrl[y].n_hvp;
    out[y] = r;
}

hipError_t launch_eig_gather_info(int P, const EigCtrl* ctrl, moto_info* out, hipStream_t st) {
    hipLaunchKernelGGL(k_eig_gather_info, dim3((P + 63) / 64), dim3(64), 0, st, P, ctrl, out);
    return hipGetLastError();
}

hipError_t launch_eig_all_done(const EigArgs& a, const EigCtrl* ctrl, int* all_done, hipStream_t st) {
    hipLaunchKernelGGL(k_eig_all_done, dim3(1), dim3(WL), 0, st, a.P, ctrl, all_done);
    return hipGetLastError();
}

hipError_t launch_eig_output(bool f64, const EigArgs& a, const void* S, const double* m, int N, double* V,
                             double* part, const EigCtrl* ctrl, double* evals, double* resid, void* Xsave,
                             hipStream_t st) {
    const int nb = (N + NT - 1) / NT;
    if (f64)
        hipLaunchKernelGGL(k_eig_out1<double>, dim3(nb, a.P), dim3(NT), 0, st, a, (const double*)S, m, N, V, part,
                           (double*)Xsave);
    else
        hipLaunchKernelGGL(k_eig_out1<float>, dim3(nb, a.P), dim3(NT), 0, st, a, (const float*)S, m, N, V, part,
                           (float*)Xsave);
    double* scale = part + (size_t)nb * MAXB * 3;
    hipLaunchKernelGGL(k_eig_out2, dim3(1, a.P), dim3(64), 0, st, a, part, nb, V, N, scale, ctrl, evals, resid);
    const size_t tot = (size_t)a.P * a.k * 3 * N;
    hipLaunchKernelGGL(k_eig_out3, dim3((unsigned)((tot + NT - 1) / NT)), dim3(NT), 0, st, a.k, N, a.P, a.part_ms,
                       V, scale);
    return hipGetLastError();
}

}  // namespace moto
