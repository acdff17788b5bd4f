// kernels.hip -- gfx950 kernels of the supernodal Cholesky numeric phase and
// of the triangular solves.
//
// Storage: supernode s is an m_s x w_s column-major panel at Lx + lptr[s]
// (leading dimension m_s); row k of the panel is global row rows[rptr[s]+k]
// of the permuted matrix, the first w_s rows are the columns of s.  Each
// supernode is cut into column blocks of kNB; the inverse of every block's
// diagonal triangle is kept (column-major nb x nb) at Linv + inv_off[blk].
//
// Kernels (paper Sec. 3, Listing 1 names the dense operations):
//   k_assemble     scatter A into the zeroed panels
//   k_potrf        POTRF of one diagonal block in LDS, plus its inverse
//   k_tiles        MFMA tiles: TRSM (rows times the transposed block
//                  inverse), trailing SYRK/GEMM inside a supernode, and the
//                  SYRK/GEMM update scatter-added through relative indices
//                  into ancestor panels
//   k_solve_fwd / k_solve_bwd   block-level forward / backward substitution
#include <hip/hip_runtime.h>

#include <climits>

#include "kernels.h"

namespace spc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    using acc = d4;
    // D(16x16) += A(16x4) B(4x16): lane l supplies A[l%16][l/16] and
    // B[l/16][l%16]; element v of lane l is D[l/16 + 4v][l%16] (measured on
    // gfx950: the four rows of a lane are interleaved by 4).
    static __device__ __forceinline__ acc run(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
    using acc = f4;
    // same operand layout; element v of lane l is D[4*(l/16) + v][l%16]
    static __device__ __forceinline__ acc run(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

__device__ __forceinline__ bool finite_pos(double d) { return d > 0.0 && d <= 1.7976931348623157e308; }
__device__ __forceinline__ bool finite_pos(float d) { return d > 0.0f && d <= 3.402823466e38f; }

template <typename T>
__global__ void k_zero(T *x, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) x[i] = T(0);
}

__global__ void k_status_reset(unsigned long long *status, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) status[i] = ~0ull;
}

template <typename T>
__global__ void k_assemble(const int64_t *amap, int64_t nnz, const double *values, T *Lx) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) Lx[amap[k]] = (T)values[k];
}

// ---------------------------------------------------------------------------
// k_potrf: one workgroup (4 waves) per diagonal block (nb <= kNB = 64), held
// in LDS.  Blocked column Cholesky with 16-column panels:
//   - wave 0 factors the panel (rows >= its first column) with lane = row and
//     the panel's 16 columns in registers, wave-synchronously: for column j,
//     d = a_jj (read from lane j), l_jj = sqrt(d), l_ij = a_ij / l_jj, and the
//     panel columns right of j lose l_ij l_kj (l_kj read from lane k);
//   - all waves subtract the panel's product from the trailing lower part.
// Then the inverse, blockwise: each wave inverts one 16x16 diagonal block by
// forward substitution (lane = column), and for block rows I = 1..3
//   Linv[I][J] = -inv(L_II) sum_{J <= K < I} L[I][K] Linv[K][J].
// L stays in the lower triangle of A; the strict lower part of L^{-1} is
// kept transposed in the strict upper triangle (A[c][a] = Linv[a][c]) and
// its diagonal in rdg.  A pivot that is not positive and finite lowers the
// status word to its column.  L^{-1} is stored column-major:
// Linv[blk][k * nb + i] = (L^{-1})_ik.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T lane_read(T v, int src);
template <>
__device__ __forceinline__ double lane_read<double>(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <>
__device__ __forceinline__ float lane_read<float>(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// 1/sqrt(d): hardware estimate refined by Newton steps (two in double),
// so the pivot chain has no division.
__device__ __forceinline__ double rsqrt_nr(double d) {
    double y = __builtin_amdgcn_rsq(d);
    y = y * (1.5 - 0.5 * d * y * y);
    return y * (1.5 - 0.5 * d * y * y);
}
__device__ __forceinline__ float rsqrt_nr(float d) {
    float y = __builtin_amdgcn_rsqf(d);
    return y * (1.5f - 0.5f * d * y * y);
}

template <typename T>
__global__ __launch_bounds__(256) void k_potrf(const PanelTask *tasks, const int32_t *super_ptr,
                                               const int64_t *rptr, const int64_t *lptr,
                                               const int64_t *inv_off, T *Lx, T *Linv,
                                               unsigned long long *status, const int32_t *status_slot) {
    constexpr int NB = kNB, PW = 16;
    __shared__ T A[NB][NB + 1];
    __shared__ T rdg[NB];
    __shared__ T Tb[PW][NB + 1];
    __shared__ int badcol;
    const PanelTask tk = tasks[blockIdx.x];
    const int s = tk.s;
    const int64_t m = rptr[s + 1] - rptr[s];
    const int c0 = tk.c0, nb = tk.c1 - tk.c0;
    T *P = Lx + lptr[s];
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    {
        // issue every load before the first use (HBM latency is ~1-2 us)
        T ld[NB * NB / 256];
#pragma unroll
        for (int q = 0; q < NB * NB / 256; ++q) {
            const int e = t + 256 * q, i = e % NB, k = e / NB;
            ld[q] = (i < nb && k <= i) ? P[(int64_t)(c0 + k) * m + c0 + i] : (i == k ? T(1) : T(0));
        }
#pragma unroll
        for (int q = 0; q < NB * NB / 256; ++q) {
            const int e = t + 256 * q;
            A[e % NB][e / NB] = ld[q];
        }
    }
    if (t == 0) badcol = -1;
    __syncthreads();
    const int npan = (nb + PW - 1) / PW;
    for (int pb = 0; pb < npan; ++pb) {
        const int p0 = PW * pb;
        if (wv == 0) {
            const int i = lane;
            T r[PW];
#pragma unroll
            for (int c = 0; c < PW; ++c) r[c] = A[i][p0 + c];
#pragma unroll
            for (int c = 0; c < PW; ++c) {
                const int j = p0 + c;
                const T d = lane_read(r[c], j);
                if (i == 0 && j < nb && !finite_pos(d) && badcol < 0) badcol = j;
                const T rs = rsqrt_nr(d);  // 1/sqrt(d)
                const T lij = (i == j) ? d * rs : r[c] * rs;
                r[c] = lij;
#pragma unroll
                for (int c2 = c + 1; c2 < PW; ++c2) r[c2] -= lij * lane_read(lij, p0 + c2);
            }
            if (i >= p0)
#pragma unroll
                for (int c = 0; c < PW; ++c)
                    if (c <= i - p0) A[i][p0 + c] = r[c];
        }
        __syncthreads();
        // trailing lower part: rows and columns >= p0 + PW
        const int q0 = p0 + PW, rem = NB - q0;
        for (int e = t; e < rem * rem; e += 256) {
            const int i = q0 + e % rem, k = q0 + e / rem;
            if (k > i) continue;
            T acc = T(0);
#pragma unroll
            for (int c = 0; c < PW; ++c) acc += A[i][p0 + c] * A[k][p0 + c];
            A[i][k] -= acc;
        }
        __syncthreads();
    }
    if (t == 0 && badcol >= 0)
        atomicMin(status + (status_slot ? status_slot[s] : 0), (unsigned long long)(super_ptr[s] + c0 + badcol));
    // inverses of the 16x16 diagonal blocks: wave w, lane c -> column c
    {
        const int b0 = PW * wv;
        const int c = lane;
        if (c < PW) {
            T y[PW];
#pragma unroll
            for (int a = 0; a < PW; ++a) {
                T v = (a == c) ? T(1) : T(0);
#pragma unroll
                for (int k = 0; k < a; ++k) v -= A[b0 + a][b0 + k] * y[k];
                y[a] = v / A[b0 + a][b0 + a];
            }
#pragma unroll
            for (int a = 0; a < PW; ++a) {
                if (a > c) A[b0 + c][b0 + a] = y[a];
                else if (a == c) rdg[b0 + a] = y[a];
            }
        }
    }
    __syncthreads();
    // off-diagonal blocks by the 2x2 block formula for a lower triangle,
    // inv [L11 0; L21 L22] = [X11 0; -X22 L21 X11  X22]: first inside each
    // 32-block (16-blocks), then for the 64-block (32-blocks).  INV(a, c)
    // reads the inverse built so far from its transposed storage.
#define SPC_INV(a, c) ((c) < (a) ? A[c][a] : ((c) == (a) ? rdg[a] : T(0)))
    T *Tf = &Tb[0][0];  // flat scratch, >= 1024 entries
#pragma unroll
    for (int lvl = 0; lvl < 2; ++lvl) {
        const int h = lvl == 0 ? 16 : 32;
        constexpr int NOUT = 4;                       // outputs per thread, at most
        const int nout = lvl == 0 ? 2 : 4;            // 2 blocks x 16^2 or 1 x 32^2, over 256 threads
        // Tf = L21 X11, h x h per block (row a, column b)
#pragma unroll
        for (int q = 0; q < NOUT; ++q) {
            if (q >= nout) break;
            const int e = t + 256 * q;
            const int o = (e / (h * h)) * 2 * h, rem = e % (h * h), a = rem % h, b = rem / h;
            T acc = T(0);
            for (int c = b; c < h; ++c) acc += A[o + h + a][o + c] * SPC_INV(o + c, o + b);
            Tf[e] = acc;
        }
        __syncthreads();
        // X21 = -X22 Tf, written transposed into the upper triangle
        T out[NOUT];
#pragma unroll
        for (int q = 0; q < NOUT; ++q) {
            out[q] = T(0);
            if (q >= nout) break;
            const int e = t + 256 * q;
            const int base = (e / (h * h)) * h * h;
            const int o = (e / (h * h)) * 2 * h, rem = e % (h * h), a = rem % h, b = rem / h;
            T acc = T(0);
            for (int c = 0; c <= a; ++c) acc += SPC_INV(o + h + a, o + h + c) * Tf[base + b * h + c];
            out[q] = -acc;
        }
#pragma unroll
        for (int q = 0; q < NOUT; ++q) {
            if (q >= nout) break;
            const int e = t + 256 * q;
            const int o = (e / (h * h)) * 2 * h, rem = e % (h * h), a = rem % h, b = rem / h;
            A[o + b][o + h + a] = out[q];
        }
        __syncthreads();
    }
#undef SPC_INV
    T *Vi = Linv + inv_off[tk.blk];
#pragma unroll
    for (int q = 0; q < NB * NB / 256; ++q) {
        const int e = t + 256 * q, i = e % NB, k = e / NB;
        if (i < nb && k < nb) {
            if (k <= i) P[(int64_t)(c0 + k) * m + c0 + i] = A[i][k];
            Vi[k * nb + i] = (k < i) ? A[k][i] : (k == i ? rdg[i] : T(0));
        }
    }
}

// ---------------------------------------------------------------------------
// k_small: one workgroup per small supernode (w <= kSmallW, m <= kSmallM),
// the whole m x w panel in LDS:
//   1. column Cholesky of the panel, right-looking: l_jj = sqrt(d_j),
//      l_ij = a_ij / l_jj, then a_ik -= l_ij l_kj for the columns right of j
//      (POTRF of the diagonal block and TRSM of the rows below at once);
//   2. the inverse of the diagonal triangle, one column per thread by
//      forward substitution (kept for the solves);
//   3. the Schur update C = P P^T of the rows below the block, scatter-added
//      into the ancestors through the relative indices, as in k_tiles.
// Pivots that are not positive and finite lower the status word.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_small(const int32_t *snodes, const int32_t *super_ptr,
                                               const int64_t *rptr, const int64_t *lptr, const int32_t *rows,
                                               const int32_t *colpair, const UpdatePair *pairs,
                                               const int32_t *rel, const int32_t *first_blk,
                                               const int64_t *inv_off, T *Lx, T *Linv,
                                               unsigned long long *status, const int32_t *status_slot) {
    constexpr int MS = kSmallM, WS = kSmallW;
    __shared__ T A[WS][MS + 1];   // A[c][i] = panel entry (row i, column c)
    __shared__ T Vt[WS][WS + 1];  // inverse, Vt[c][a] = (L^{-1})_ac
    const int s = snodes[blockIdx.x];
    const int64_t m = rptr[s + 1] - rptr[s];
    const int w = super_ptr[s + 1] - super_ptr[s];
    T *P = Lx + lptr[s];
    const int tid = threadIdx.x;
    for (int e = tid; e < w * MS; e += 256) {
        const int i = e % MS, c = e / MS;
        A[c][i] = (i < m) ? P[(int64_t)c * m + i] : T(0);
    }
    __syncthreads();
    int bad = -1;
    for (int j = 0; j < w; ++j) {
        const T d = A[j][j];
        if (bad < 0 && !finite_pos(d)) bad = j;
        const T ljj = sqrt(d);
        __syncthreads();  // every thread has read d
        for (int i = j + tid; i < m; i += 256) A[j][i] = (i == j) ? ljj : A[j][i] / ljj;
        __syncthreads();
        const int rem = w - j - 1;
        for (int e = tid; e < rem * m; e += 256) {
            const int k = j + 1 + e / m, i = e % m;
            if (i >= k) A[k][i] -= A[j][i] * A[j][k];
        }
        __syncthreads();
    }
    if (tid == 0 && bad >= 0)
        atomicMin(status + (status_slot ? status_slot[s] : 0), (unsigned long long)(super_ptr[s] + bad));
    // write the panel back (lower part of the diagonal block, all rows below)
    for (int e = tid; e < w * MS; e += 256) {
        const int i = e % MS, c = e / MS;
        if (i < m && i >= c) P[(int64_t)c * m + i] = A[c][i];
    }
    // inverse of the diagonal triangle: thread c owns column c
    if (tid < w) {
        const int c = tid;
        for (int a = 0; a < w; ++a) {
            T v = (a == c) ? T(1) : T(0);
            for (int k = c; k < a; ++k) v -= A[k][a] * Vt[c][k];
            Vt[c][a] = (a < c) ? T(0) : v / A[a][a];
        }
    }
    __syncthreads();
    T *Vi = Linv + inv_off[first_blk[s]];
    for (int e = tid; e < w * w; e += 256) Vi[e] = Vt[e / w][e % w];
    // Schur update of the rows below, scatter-added into the ancestors
    const int mb = (int)m - w;
    for (int e = tid; e < mb * mb; e += 256) {
        const int r = w + e % mb, cc = w + e / mb;  // row r, column cc (positions in R_s)
        if (cc > r) continue;
        T acc = T(0);
        for (int k = 0; k < w; ++k) acc += A[k][r] * A[k][cc];
        const UpdatePair pr = pairs[colpair[rptr[s] + cc]];
        const int t = pr.target;
        const int64_t mt = rptr[t + 1] - rptr[t];
        const int64_t colt = rows[rptr[s] + cc] - super_ptr[t];
        const int64_t rowt = rel[pr.rel_off + (r - pr.i0)];
        atomicAdd(&Lx[lptr[t] + colt * mt + rowt], -acc);
    }
}

// ---------------------------------------------------------------------------
// MFMA tiles.  Task (s, i0, j0, k0, k1, jmax, blk):
//   C[r][c] = sum_{k0 <= k < k1} P[i0 + r][k] * Q[c][k]
// over a 64x64 tile, 256 threads = 4 waves in a 2x2 grid of 32x32, each a
// 2x2 set of 16x16x4 MFMA blocks; K staged through LDS 16 at a time.
//   MODE_TRAILING: Q = P rows j0.. ; P[i][j] -= C for i >= j, j < jmax.
//   MODE_SCATTER:  Q = P rows j0.. ; C (i >= j) scatter-added atomically into
//                  the ancestors: column rows[j] of target t (pair of j), row
//                  position rel[...] of R_t.
//   MODE_TRSM:     Q = inverse of block blk, Q[c][k'] stored at k' * nb + c;
//                  P[i][k0 + c] = C
//                  (rows times the transposed inverse: X = B L^{-T}).
// ---------------------------------------------------------------------------
enum { MODE_TRAILING = 0, MODE_SCATTER = 1, MODE_TRSM = 2 };

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_tiles(const TileTask *tasks, const int32_t *super_ptr,
                                               const int64_t *rptr, const int64_t *lptr,
                                               const int32_t *rows, const int32_t *colpair,
                                               const UpdatePair *pairs, const int32_t *rel,
                                               const T *Linv, const int64_t *inv_off, T *Lx) {
    constexpr int TM = kTile, KB = 16;
    using acc_t = typename Mfma<T>::acc;
    __shared__ T As[KB][TM + 4];
    __shared__ T Bs[KB][TM + 4];
    __shared__ T Cs[TM][TM + 1];
    const TileTask tk = tasks[blockIdx.x];
    const int s = tk.s;
    const int64_t m = rptr[s + 1] - rptr[s];
    T *P = Lx + lptr[s];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    const int lr = tid & 63, lk = tid >> 6;
    const bool row_ok = tk.i0 + lr < m;
    const bool col_ok = tk.j0 + lr < tk.jmax;
    const int kw = tk.k1 - tk.k0;
    const T *Q = (MODE == MODE_TRSM) ? Linv + inv_off[tk.blk] : nullptr;
    for (int kb = tk.k0; kb < tk.k1; kb += KB) {
#pragma unroll
        for (int e = 0; e < KB / 4; ++e) {
            const int kk = lk + 4 * e;
            const int k = kb + kk;
            const bool kin = k < tk.k1;
            As[kk][lr] = (kin && row_ok) ? P[(int64_t)k * m + tk.i0 + lr] : T(0);
            if (MODE == MODE_TRSM)
                Bs[kk][lr] = (kin && col_ok) ? Q[(k - tk.k0) * kw + lr] : T(0);
            else
                Bs[kk][lr] = (kin && col_ok) ? P[(int64_t)k * m + tk.j0 + lr] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KB; kk += 4) {
            T af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) af[a] = As[kk + (lane >> 4)][wr + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bf[b] = Bs[kk + (lane >> 4)][wc + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::run(af[a], bf[b], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wr + a * 16 + Mfma<T>::row(lane, v);
                const int c = wc + b * 16 + (lane & 15);
                Cs[c][r] = acc[a][b][v];
            }
    __syncthreads();
    const int r = tid & 63, cg = tid >> 6;
    const int gi = tk.i0 + r;
    if (gi >= m) return;
    for (int cc = 0; cc < 16; ++cc) {
        const int c = cg * 16 + cc;
        const int gj = tk.j0 + c;
        if (gj >= tk.jmax) continue;
        const T v = Cs[c][r];
        if (MODE == MODE_TRSM) {
            P[(int64_t)gj * m + gi] = v;
        } else if (MODE == MODE_TRAILING) {
            if (gj <= gi) P[(int64_t)gj * m + gi] -= v;
        } else {
            if (gj > gi) continue;
            const UpdatePair pr = pairs[colpair[rptr[s] + gj]];
            const int t = pr.target;
            const int64_t mt = rptr[t + 1] - rptr[t];
            const int64_t colt = rows[rptr[s] + gj] - super_ptr[t];
            const int64_t rowt = rel[pr.rel_off + (gi - pr.i0)];
            atomicAdd(&Lx[lptr[t] + colt * mt + rowt], -v);
        }
    }
}

// ---------------------------------------------------------------------------
// k_tiles128: the trailing and scatter updates on 128x128 tiles for the
// large supernodes.  4 waves in a 2x2 grid of 64x64 quadrants, each a 4x4
// set of 16x16x4 MFMA blocks; K staged through LDS 16 at a time with the
// next chunk prefetched into registers while the current one is consumed.
// The epilogue goes through LDS in four passes of 32 columns.
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_tiles128(const TileTask *tasks, const int32_t *super_ptr,
                                                  const int64_t *rptr, const int64_t *lptr,
                                                  const int32_t *rows, const int32_t *colpair,
                                                  const UpdatePair *pairs, const int32_t *rel, T *Lx) {
    constexpr int TM = 128, KB = 16, PADA = 4;
    using acc_t = typename Mfma<T>::acc;
    __shared__ T smem[2 * KB * (TM + PADA)];
    T(*As)[TM + PADA] = reinterpret_cast<T(*)[TM + PADA]>(smem);
    T(*Bs)[TM + PADA] = reinterpret_cast<T(*)[TM + PADA]>(smem + KB * (TM + PADA));
    const TileTask tk = tasks[blockIdx.x];
    const int s = tk.s;
    const int64_t m = rptr[s + 1] - rptr[s];
    T *P = Lx + lptr[s];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    // loader: thread covers row lr (0..127) and k-rows lk, lk+2, ..., lk+14
    const int lr = tid & 127, lk = tid >> 7;
    const bool row_ok = tk.i0 + lr < m;
    const bool col_ok = tk.j0 + lr < tk.jmax;
    const T *pa = P + tk.i0 + lr;
    const T *pb = P + tk.j0 + lr;
    T ra[KB / 2], rb[KB / 2];
    auto load = [&](int kb) {
#pragma unroll
        for (int e = 0; e < KB / 2; ++e) {
            const int k = kb + lk + 2 * e;
            const bool kin = k < tk.k1;
            ra[e] = (kin && row_ok) ? pa[(int64_t)k * m] : T(0);
            rb[e] = (kin && col_ok) ? pb[(int64_t)k * m] : T(0);
        }
    };
    load(tk.k0);
    for (int kb = tk.k0; kb < tk.k1; kb += KB) {
#pragma unroll
        for (int e = 0; e < KB / 2; ++e) {
            As[lk + 2 * e][lr] = ra[e];
            Bs[lk + 2 * e][lr] = rb[e];
        }
        __syncthreads();
        if (kb + KB < tk.k1) load(kb + KB);
#pragma unroll
        for (int kk = 0; kk < KB; kk += 4) {
            T af[4], bf[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) af[a] = As[kk + (lane >> 4)][wr + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 4; ++b) bf[b] = Bs[kk + (lane >> 4)][wc + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<T>::run(af[a], bf[b], acc[a][b]);
        }
        __syncthreads();
    }
    // epilogue: 4 passes of 32 columns staged as Cs[32][128 + 1]
    T(*Cs)[TM + 1] = reinterpret_cast<T(*)[TM + 1]>(smem);
    const int r = tid & 127, ch = tid >> 7;  // row, column half of the pass
    const int gi = tk.i0 + r;
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        // the waves holding columns [32 pass, 32 pass + 32) stage them
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = wc + b * 16 + (lane & 15);
                if ((c >> 5) != pass) continue;
#pragma unroll
                for (int v = 0; v < 4; ++v) Cs[c & 31][wr + a * 16 + Mfma<T>::row(lane, v)] = acc[a][b][v];
            }
        __syncthreads();
        if (gi < m) {
            for (int cc = 0; cc < 16; ++cc) {
                const int c = 32 * pass + ch * 16 + cc;
                const int gj = tk.j0 + c;
                if (gj >= tk.jmax || gj > gi) continue;
                const T v = Cs[c & 31][r];
                if (MODE == MODE_TRAILING) {
                    P[(int64_t)gj * m + gi] -= v;
                } else {
                    const UpdatePair pr = pairs[colpair[rptr[s] + gj]];
                    const int t = pr.target;
                    const int64_t mt = rptr[t + 1] - rptr[t];
                    const int64_t colt = rows[rptr[s] + gj] - super_ptr[t];
                    const int64_t rowt = rel[pr.rel_off + (gi - pr.i0)];
                    atomicAdd(&Lx[lptr[t] + colt * mt + rowt], -v);
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Triangular solves on permuted work vectors (n x nrhs, column-major,
// leading dimension n), one launch per level of the block tree.
// Forward, block q (rows g0.., width nb), tasks = chunks of rows below it:
//   x_q = Linv_q y_q;  the first task stores x_q in X;  every task does
//   Y[rows[r]] -= sum_k P[r][c0+k] x_q[k] for its rows (atomic).
// Backward: each task adds sum_r P[r][c0+k] X[rows[r]] over its rows into
//   Acc; the last task of the block (counter) forms t = X_q - Acc_q and
//   stores x_q = Linv_q^T t.  Rows below belong to ancestors, whose x is
//   final when the block's level runs.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_perm_in(const int32_t *perm, int64_t n, int nrhs, const double *B, int64_t ldb, T *W) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    int64_t k = i % n, r = i / n;
    W[i] = (T)B[perm[k] + r * ldb];
}

template <typename T>
__global__ void k_perm_out(const int32_t *perm, int64_t n, int nrhs, const T *W, double *B, int64_t ldb) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    int64_t k = i % n, r = i / n;
    B[perm[k] + r * ldb] = (double)W[i];
}

constexpr int kMaxRhs = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_solve_fwd(const SolveTask *tasks, const SolveBlock *blocks,
                                                   const int32_t *super_ptr, const int64_t *rptr,
                                                   const int64_t *lptr, const int32_t *rows, const T *Lx,
                                                   const T *Linv, const int64_t *inv_off, T *Y, T *X,
                                                   int64_t n, int nrhs) {
    constexpr int NB = kNB;
    __shared__ T Vi[NB][NB + 1];
    __shared__ T yq[NB][kMaxRhs];
    __shared__ T xq[NB][kMaxRhs];
    const SolveTask tk = tasks[blockIdx.x];
    const SolveBlock B = blocks[tk.blk];
    const int64_t m = rptr[B.s + 1] - rptr[B.s];
    const int nb = B.c1 - B.c0;
    const T *P = Lx + lptr[B.s];
    const int32_t *R = rows + rptr[B.s];
    const int64_t g0 = super_ptr[B.s] + B.c0;
    const T *Q = Linv + inv_off[tk.blk];
    const int tid = threadIdx.x;
    // inverse (column-major nb x nb) and the block's right-hand sides
    for (int e = tid; e < nb * nb; e += 256) {
        const int i = e % nb, c = e / nb;
        Vi[i][c] = Q[e];
    }
    for (int e = tid; e < NB * kMaxRhs; e += 256) {
        const int i = e % NB, q = e / NB;
        yq[i][q] = (i < nb && q < nrhs) ? Y[g0 + i + (int64_t)q * n] : T(0);
    }
    __syncthreads();
    for (int e = tid; e < NB * kMaxRhs; e += 256) {
        const int i = e % NB, q = e / NB;
        T a = T(0);
        if (i < nb)
            for (int c = 0; c <= i; ++c) a += Vi[i][c] * yq[c][q];
        xq[i][q] = a;
    }
    __syncthreads();
    if (tk.r0 == B.c1)
        for (int e = tid; e < nb * nrhs; e += 256) {
            const int i = e % nb, q = e / nb;
            X[g0 + i + (int64_t)q * n] = xq[i][q];
        }
    for (int r = tk.r0 + tid; r < tk.r1; r += 256) {
        T acc[kMaxRhs];
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q) acc[q] = T(0);
        for (int k = 0; k < nb; ++k) {
            const T l = P[(int64_t)(B.c0 + k) * m + r];
#pragma unroll
            for (int q = 0; q < kMaxRhs; ++q) acc[q] += l * xq[k][q];
        }
        const int64_t gr = R[r];
        for (int q = 0; q < nrhs; ++q) atomicAdd(&Y[gr + (int64_t)q * n], -acc[q]);
    }
}

// Backward.  A block with one task sums its rows locally and finishes the
// block itself; a block split over several tasks adds the partial sums into
// Acc, and the last task to arrive (block counter) finishes it.
template <typename T>
__global__ __launch_bounds__(256) void k_solve_bwd(const SolveTask *tasks, const SolveBlock *blocks,
                                                   const int32_t *super_ptr, const int64_t *rptr,
                                                   const int64_t *lptr, const int32_t *rows, const T *Lx,
                                                   const T *Linv, const int64_t *inv_off, T *X, T *Acc,
                                                   int32_t *counters, int64_t n, int nrhs) {
    constexpr int NB = kNB;
    __shared__ T Pt[64][NB + 1];  // row tile of P, later the block inverse
    __shared__ T Yr[64][kMaxRhs + 1];
    __shared__ T Sm[4][NB][kMaxRhs / 4 + 1];  // partial sums of the 4 row groups
    __shared__ int last;
    const SolveTask tk = tasks[blockIdx.x];
    const SolveBlock B = blocks[tk.blk];
    const int64_t m = rptr[B.s + 1] - rptr[B.s];
    const int nb = B.c1 - B.c0;
    const T *P = Lx + lptr[B.s];
    const int32_t *R = rows + rptr[B.s];
    const int64_t g0 = super_ptr[B.s] + B.c0;
    const int tid = threadIdx.x;
    const int k = tid & 63, qg = tid >> 6;
    T acc[kMaxRhs / 4];
#pragma unroll
    for (int q = 0; q < kMaxRhs / 4; ++q) acc[q] = T(0);
    for (int rb = tk.r0; rb < tk.r1; rb += 64) {
        const int nr = min(64, tk.r1 - rb);
        for (int e = tid; e < nr * nb; e += 256) {
            const int r = e % nr, c = e / nr;
            Pt[r][c] = P[(int64_t)(B.c0 + c) * m + rb + r];
        }
        for (int e = tid; e < nr * nrhs; e += 256) {
            const int r = e % nr, q = e / nr;
            Yr[r][q] = X[(int64_t)R[rb + r] + (int64_t)q * n];
        }
        __syncthreads();
        if (k < nb)
            for (int r = 0; r < nr; ++r) {
                const T l = Pt[r][k];
#pragma unroll
                for (int q = 0; q < kMaxRhs / 4; ++q)
                    if (qg + 4 * q < nrhs) acc[q] += l * Yr[r][qg + 4 * q];
            }
        __syncthreads();
    }
    // Yr[i][q] <- t = X_q - (sum over rows below), for the block's columns
    if (B.ntasks == 1) {
#pragma unroll
        for (int q = 0; q < kMaxRhs / 4; ++q) Sm[qg][k][q] = acc[q];
        __syncthreads();
        for (int e = tid; e < nb * nrhs; e += 256) {
            const int i = e % nb, q = e / nb;
            Yr[i][q] = X[g0 + i + (int64_t)q * n] - Sm[q % 4][i][q / 4];
        }
    } else {
        if (tk.r1 > tk.r0 && k < nb)
#pragma unroll
            for (int q = 0; q < kMaxRhs / 4; ++q) {
                const int qq = qg + 4 * q;
                if (qq < nrhs) atomicAdd(&Acc[g0 + k + (int64_t)qq * n], acc[q]);
            }
        __threadfence();
        __syncthreads();
        if (tid == 0) last = (atomicAdd(&counters[tk.blk], 1) == B.ntasks - 1);
        __syncthreads();
        if (!last) return;
        __threadfence();
        for (int e = tid; e < nb * nrhs; e += 256) {
            const int i = e % nb, q = e / nb;
            const int64_t idx = g0 + i + (int64_t)q * n;
            const T a = __hip_atomic_exchange(&Acc[idx], T(0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            Yr[i][q] = X[idx] - a;
        }
        if (tid == 0) counters[tk.blk] = 0;
    }
    // x_q = Linv^T t
    const T *Q = Linv + inv_off[tk.blk];
    for (int e = tid; e < nb * nb; e += 256) {
        const int i = e % nb, c = e / nb;
        Pt[i][c] = Q[e];
    }
    __syncthreads();
    for (int e = tid; e < nb * nrhs; e += 256) {
        const int c = e % nb, q = e / nb;
        T a = T(0);
        for (int i = c; i < nb; ++i) a += Pt[i][c] * Yr[i][q];
        X[g0 + c + (int64_t)q * n] = a;
    }
}

// ---------------------------------------------------------------------------
// FP64 kernels of iterative refinement.  A is applied in full through a CSR
// of the symmetric pattern whose entries point into the caller's lower-CSC
// values (valmap), so refinement always uses the values given.  Vectors are
// n x nrhs column-major with leading dimension ld.
// ---------------------------------------------------------------------------
// Y = B - A X (beta = -1, with B) or Y = A X (B == nullptr)
__global__ void k_spmv(const int64_t *rowptr, const int32_t *colidx, const int64_t *valmap,
                       const double *values, const double *X, const double *B, double *Y, int64_t n,
                       int nrhs, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc[kMaxRhs];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) acc[q] = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const double a = values[valmap[e]];
        const int64_t c = colidx[e];
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q)
            if (q < nrhs) acc[q] += a * X[c + q * ld];
    }
    for (int q = 0; q < nrhs; ++q) Y[i + q * ld] = B ? B[i + q * ld] - acc[q] : acc[q];
}

// out = max_i sum_j |a_ij| (as the bit pattern of a non-negative double)
__global__ void k_norm_inf_A(const int64_t *rowptr, const int64_t *valmap, const double *values, int64_t n,
                             unsigned long long *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double sum = 0.0;
    if (i < n)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) sum += fabs(values[valmap[e]]);
    for (int off = 32; off > 0; off >>= 1) sum = fmax(sum, __shfl_xor(sum, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(sum));
}

// out[q] = max_i |V[i, q]| (bit patterns), grid.y = q
__global__ void k_colmax(const double *V, int64_t n, int64_t ld, unsigned long long *out) {
    const int q = blockIdx.y;
    double mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        mx = fmax(mx, fabs(V[i + q * ld]));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) atomicMax(&out[q], (unsigned long long)__double_as_longlong(mx));
}

// out[q] += sum_i U[i, q] V[i, q], grid.y = q
__global__ void k_coldot(const double *U, const double *V, int64_t n, int64_t ld, double *out) {
    const int q = blockIdx.y;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += U[i + q * ld] * V[i + q * ld];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(&out[q], acc);
}

// Y[:, q] = a_q X[:, q] + b_q Y[:, q]; a_q = a[q] (device) or a0 when a is
// null, likewise b_q; b_q = 0 does not read Y.
__global__ void k_axpby(const double *a, double a0, const double *X, const double *b, double b0, double *Y,
                        int64_t n, int64_t ld) {
    const int q = blockIdx.y;
    const double aq = a ? a[q] : a0, bq = b ? b[q] : b0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        Y[i + q * ld] = (bq == 0.0) ? aq * X[i + q * ld] : aq * X[i + q * ld] + bq * Y[i + q * ld];
}

// copy n x q between leading dimensions
__global__ void k_copy_cols(const double *X, int64_t ldx, double *Y, int64_t ldy, int64_t n) {
    const int q = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        Y[i + q * ldy] = X[i + q * ldx];
}

// Batched right-hand sides: system i's n_i x nrhs block (leading dimension
// ld[i]) <-> rows off[i].. of the merged n x nrhs array (leading dimension
// n).  grid.x = systems, grid.y = right-hand sides.
__global__ void k_batch_move(double *const *ptrs, const int64_t *lds, const int64_t *offs, double *M, int64_t n,
                             int to_merged) {
    const int i = blockIdx.x, q = blockIdx.y;
    const int64_t o = offs[i], ni = offs[i + 1] - o, ld = lds[i];
    double *X = ptrs[i];
    for (int64_t r = threadIdx.x; r < ni; r += blockDim.x) {
        if (to_merged) M[o + r + q * n] = X[r + q * ld];
        else X[r + q * ld] = M[o + r + q * n];
    }
}

inline unsigned grid1(int64_t count, int block) {
    int64_t g = (count + block - 1) / block;
    return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

void launch_status_reset(unsigned long long *status, int count, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_status_reset, dim3((count + 255) / 256), dim3(256), 0, st, status, count);
}

template <typename T>
void launch_zero(T *x, int64_t count, hipStream_t st) {
    if (count <= 0) return;
    int64_t g = (count + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)g), dim3(256), 0, st, x, count);
}

template <typename T>
void launch_assemble(const DevPlan &P, int64_t nnz, const double *values, T *Lx, hipStream_t st) {
    if (nnz <= 0) return;
    hipLaunchKernelGGL(k_assemble<T>, dim3(grid1(nnz, 256)), dim3(256), 0, st, P.amap, nnz, values, Lx);
}

template <typename T>
void launch_potrf(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, T *Linv, unsigned long long *status,
                  hipStream_t st) {
    if (t1 <= t0) return;
    hipLaunchKernelGGL(k_potrf<T>, dim3((unsigned)(t1 - t0)), dim3(256), 0, st, P.potrf_tasks + t0,
                       P.super_ptr, P.rptr, P.lptr, P.inv_off, Lx, Linv, status, P.status_slot);
}

template <typename T>
void launch_small(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, T *Linv, unsigned long long *status,
                  hipStream_t st) {
    if (t1 <= t0) return;
    hipLaunchKernelGGL(k_small<T>, dim3((unsigned)(t1 - t0)), dim3(256), 0, st, P.small_snodes + t0, P.super_ptr,
                       P.rptr, P.lptr, P.rows, P.colpair, P.pairs, P.rel, P.first_blk, P.inv_off, Lx, Linv, status,
                       P.status_slot);
}

template <typename T>
void launch_tiles(const DevPlan &P, int mode, int64_t t0, int64_t t1, T *Lx, const T *Linv, hipStream_t st) {
    if (t1 <= t0) return;
    const dim3 g((unsigned)(t1 - t0)), b(256);
    if (mode == kTilesTrailing)
        hipLaunchKernelGGL((k_tiles<T, MODE_TRAILING>), g, b, 0, st, P.int_tiles + t0, P.super_ptr, P.rptr,
                           P.lptr, P.rows, P.colpair, P.pairs, P.rel, Linv, P.inv_off, Lx);
    else if (mode == kTilesScatter)
        hipLaunchKernelGGL((k_tiles<T, MODE_SCATTER>), g, b, 0, st, P.ext_tiles + t0, P.super_ptr, P.rptr,
                           P.lptr, P.rows, P.colpair, P.pairs, P.rel, Linv, P.inv_off, Lx);
    else
        hipLaunchKernelGGL((k_tiles<T, MODE_TRSM>), g, b, 0, st, P.trsm_tiles + t0, P.super_ptr, P.rptr,
                           P.lptr, P.rows, P.colpair, P.pairs, P.rel, Linv, P.inv_off, Lx);
}

template <typename T>
void launch_tiles128(const DevPlan &P, int mode, int64_t t0, int64_t t1, T *Lx, hipStream_t st) {
    if (t1 <= t0) return;
    const dim3 g((unsigned)(t1 - t0)), b(256);
    if (mode == kTilesTrailing)
        hipLaunchKernelGGL((k_tiles128<T, MODE_TRAILING>), g, b, 0, st, P.int_tiles_big + t0, P.super_ptr,
                           P.rptr, P.lptr, P.rows, P.colpair, P.pairs, P.rel, Lx);
    else
        hipLaunchKernelGGL((k_tiles128<T, MODE_SCATTER>), g, b, 0, st, P.ext_tiles_big + t0, P.super_ptr,
                           P.rptr, P.lptr, P.rows, P.colpair, P.pairs, P.rel, Lx);
}

template <typename T>
void launch_perm_in(const DevPlan &P, int64_t n, int nrhs, const double *B, int64_t ldb, T *W,
                    hipStream_t st) {
    if (n * nrhs <= 0) return;
    hipLaunchKernelGGL(k_perm_in<T>, dim3(grid1(n * nrhs, 256)), dim3(256), 0, st, P.perm, n, nrhs, B,
                       ldb, W);
}

template <typename T>
void launch_perm_out(const DevPlan &P, int64_t n, int nrhs, const T *W, double *B, int64_t ldb,
                     hipStream_t st) {
    if (n * nrhs <= 0) return;
    hipLaunchKernelGGL(k_perm_out<T>, dim3(grid1(n * nrhs, 256)), dim3(256), 0, st, P.perm, n, nrhs, W,
                       B, ldb);
}

template <typename T>
void launch_solve_fwd(const DevPlan &P, int64_t t0, int64_t t1, const T *Lx, const T *Linv, T *Y, T *X,
                      int64_t n, int nrhs, hipStream_t st) {
    if (t1 <= t0) return;
    hipLaunchKernelGGL(k_solve_fwd<T>, dim3((unsigned)(t1 - t0)), dim3(256), 0, st, P.stasks + t0, P.sblocks,
                       P.super_ptr, P.rptr, P.lptr, P.rows, Lx, Linv, P.inv_off, Y, X, n, nrhs);
}

template <typename T>
void launch_solve_bwd(const DevPlan &P, int64_t t0, int64_t t1, const T *Lx, const T *Linv, T *X, T *Acc,
                      int32_t *counters, int64_t n, int nrhs, hipStream_t st) {
    if (t1 <= t0) return;
    hipLaunchKernelGGL(k_solve_bwd<T>, dim3((unsigned)(t1 - t0)), dim3(256), 0, st, P.stasks + t0, P.sblocks,
                       P.super_ptr, P.rptr, P.lptr, P.rows, Lx, Linv, P.inv_off, X, Acc, counters, n, nrhs);
}


void launch_spmv(const int64_t *rowptr, const int32_t *colidx, const int64_t *valmap, const double *values,
                 const double *X, const double *B, double *Y, int64_t n, int nrhs, int64_t ld, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_spmv, dim3(grid1(n, 256)), dim3(256), 0, st, rowptr, colidx, valmap, values, X, B, Y, n,
                       nrhs, ld);
}
void launch_norm_inf_A(const int64_t *rowptr, const int64_t *valmap, const double *values, int64_t n,
                       unsigned long long *out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_norm_inf_A, dim3(grid1(n, 256)), dim3(256), 0, st, rowptr, valmap, values, n, out);
}
static unsigned red_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}
void launch_colmax(const double *V, int64_t n, int nrhs, int64_t ld, unsigned long long *out, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_colmax, dim3(red_grid(n), nrhs), dim3(256), 0, st, V, n, ld, out);
}
void launch_coldot(const double *U, const double *V, int64_t n, int nrhs, int64_t ld, double *out, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_coldot, dim3(red_grid(n), nrhs), dim3(256), 0, st, U, V, n, ld, out);
}
void launch_axpby(const double *a, double a0, const double *X, const double *b, double b0, double *Y, int64_t n,
                  int nrhs, int64_t ld, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_axpby, dim3(red_grid(n), nrhs), dim3(256), 0, st, a, a0, X, b, b0, Y, n, ld);
}
void launch_batch_move(double *const *ptrs, const int64_t *lds, const int64_t *offs, double *M, int64_t n,
                       int count, int nrhs, bool to_merged, hipStream_t st) {
    if (count <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_batch_move, dim3(count, nrhs), dim3(256), 0, st, ptrs, lds, offs, M, n, to_merged ? 1 : 0);
}
void launch_copy_cols(const double *X, int64_t ldx, double *Y, int64_t ldy, int64_t n, int nrhs, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_copy_cols, dim3(red_grid(n), nrhs), dim3(256), 0, st, X, ldx, Y, ldy, n);
}
template void launch_zero<int32_t>(int32_t *, int64_t, hipStream_t);
template void launch_zero<unsigned long long>(unsigned long long *, int64_t, hipStream_t);

#define SPC_INSTANTIATE(T)                                                                                  \
    template void launch_zero<T>(T *, int64_t, hipStream_t);                                                \
    template void launch_assemble<T>(const DevPlan &, int64_t, const double *, T *, hipStream_t);           \
    template void launch_potrf<T>(const DevPlan &, int64_t, int64_t, T *, T *, unsigned long long *,         \
                                  hipStream_t);                                                             \
    template void launch_tiles<T>(const DevPlan &, int, int64_t, int64_t, T *, const T *, hipStream_t);     \
    template void launch_small<T>(const DevPlan &, int64_t, int64_t, T *, T *, unsigned long long *,         \
                                  hipStream_t);                                                             \
    template void launch_tiles128<T>(const DevPlan &, int, int64_t, int64_t, T *, hipStream_t);             \
    template void launch_perm_in<T>(const DevPlan &, int64_t, int, const double *, int64_t, T *,            \
                                    hipStream_t);                                                           \
    template void launch_perm_out<T>(const DevPlan &, int64_t, int, const T *, double *, int64_t,           \
                                     hipStream_t);                                                          \
    template void launch_solve_fwd<T>(const DevPlan &, int64_t, int64_t, const T *, const T *, T *, T *,     \
                                      int64_t, int, hipStream_t);                                           \
    template void launch_solve_bwd<T>(const DevPlan &, int64_t, int64_t, const T *, const T *, T *, T *,     \
                                      int32_t *, int64_t, int, hipStream_t);
SPC_INSTANTIATE(double)
SPC_INSTANTIATE(float)

}  // namespace spc
