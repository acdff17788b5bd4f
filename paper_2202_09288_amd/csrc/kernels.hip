// kernels.hip -- gfx950 kernels of the supernodal Cholesky numeric phase and
// of the triangular solves.
//
// Storage: supernode s is an m_s x w_s column-major panel at Lx + lptr[s]
// (leading dimension m_s); row k of the panel is global row rows[rptr[s]+k]
// of the permuted matrix, the first w_s rows are the columns of s.
//
// Kernels (paper Sec. 3, Listing 1 names the dense operations):
//   k_assemble     scatter A into the zeroed panels
//   k_potrf        POTRF of one diagonal block in LDS
//   k_trsm         TRSM of a chunk of rows below a factored diagonal block
//   k_tiles        SYRK/GEMM update tiles on MFMA, subtracted in place
//                  (inside a panel) or scatter-added through relative
//                  indices into ancestor panels
//   k_solve_*      supernodal forward / backward substitution
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

__global__ void k_status_reset(unsigned long long *status) { *status = ~0ull; }

template <typename T>
__global__ void k_assemble(const int64_t *amap, int64_t nnz, const double *values, T *Lx) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) Lx[amap[k]] = (T)values[k];
}

// ---------------------------------------------------------------------------
// Panel factorization of block columns of width nb <= kPanelNB.
// k_potrf: one workgroup per diagonal block, factored in LDS by the column
//   Cholesky l_jj = sqrt(a_jj - sum l_jk^2), l_ij = (a_ij - sum l_ik l_jk)/l_jj
//   (right-looking order inside the block) and written back.  A pivot that
//   is not positive and finite lowers the status word to its column.
// k_trsm: one workgroup per chunk of rows below the block: X D^T = B by
//   forward substitution against the factored block.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_potrf(const PanelTask *tasks, const int32_t *super_ptr,
                                               const int64_t *rptr, const int64_t *lptr, T *Lx,
                                               unsigned long long *status) {
    constexpr int NB = kPanelNB;
    __shared__ T D[NB][NB + 1];
    const PanelTask tk = tasks[blockIdx.x];
    const int s = tk.s;
    const int64_t m = rptr[s + 1] - rptr[s];
    const int c0 = tk.r0, nb = tk.r1 - tk.r0;
    T *P = Lx + lptr[s];
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += 256) {
        int i = e % NB, j = e / NB;
        D[i][j] = (i < nb && j < nb && i >= j) ? P[(int64_t)(c0 + j) * m + c0 + i] : T(0);
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (tid == 0) {
            T d = D[j][j];
            if (!finite_pos(d)) atomicMin(status, (unsigned long long)(super_ptr[s] + c0 + j));
            D[j][j] = sqrt(d);
        }
        __syncthreads();
        T djj = D[j][j];
        for (int i = j + 1 + tid; i < nb; i += 256) D[i][j] /= djj;
        __syncthreads();
        for (int e = tid; e < NB * NB; e += 256) {
            int i = e % NB, k = e / NB;
            if (k > j && i >= k && i < nb) D[i][k] -= D[i][j] * D[k][j];
        }
        __syncthreads();
    }
    for (int e = tid; e < NB * NB; e += 256) {
        int i = e % NB, j = e / NB;
        if (i < nb && j < nb && i >= j) P[(int64_t)(c0 + j) * m + c0 + i] = D[i][j];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_trsm(const PanelTask *tasks, const int32_t *super_ptr,
                                              const int64_t *rptr, const int64_t *lptr, T *Lx) {
    constexpr int NB = kPanelNB, RCH = kPanelRows;
    __shared__ T D[NB][NB + 1];
    __shared__ T X[NB][RCH + 1];
    const PanelTask tk = tasks[blockIdx.x];
    const int s = tk.s;
    const int64_t m = rptr[s + 1] - rptr[s];
    const int w = super_ptr[s + 1] - super_ptr[s];
    const int c0 = tk.b * NB;
    const int nb = min(NB, w - c0);
    const int nr = tk.r1 - tk.r0;
    T *P = Lx + lptr[s];
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += 256) {
        int i = e % NB, j = e / NB;
        D[i][j] = (i < nb && j < nb && i >= j) ? P[(int64_t)(c0 + j) * m + c0 + i] : T(0);
    }
    for (int e = tid; e < NB * RCH; e += 256) {
        int r = e % RCH, j = e / RCH;
        X[j][r] = (r < nr && j < nb) ? P[(int64_t)(c0 + j) * m + tk.r0 + r] : T(0);
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        T djj = D[j][j];
        for (int r = tid; r < nr; r += 256) X[j][r] /= djj;
        __syncthreads();
        for (int e = tid; e < NB * RCH; e += 256) {
            int r = e % RCH, k = e / RCH;
            if (k > j && k < nb && r < nr) X[k][r] -= X[j][r] * D[k][j];
        }
        __syncthreads();
    }
    for (int e = tid; e < NB * RCH; e += 256) {
        int r = e % RCH, j = e / RCH;
        if (r < nr && j < nb) P[(int64_t)(c0 + j) * m + tk.r0 + r] = X[j][r];
    }
}

// ---------------------------------------------------------------------------
// Update tiles on MFMA.  Task (s, i0, j0, k0, k1, jmax): C = P[i0:i0+64, k0:k1]
// P[j0:j0+64, k0:k1]^T for the lower part (row >= column), columns < jmax.
// 256 threads = 4 waves in a 2x2 grid of 32x32 sub-tiles, each a 2x2 set of
// 16x16x4 MFMA blocks.  K is staged through LDS 16 at a time.
//   EXTERNAL = false: P -= C inside the same panel (trailing update).
//   EXTERNAL = true:  C is scatter-added (atomic) into the ancestors: entry
//                     (r, c) goes to column rows[c] of target t = pair of c,
//                     at row position rel[...] of R_t.
// ---------------------------------------------------------------------------
template <typename T, bool EXTERNAL>
__global__ __launch_bounds__(256) void k_tiles(const TileTask *tasks, const int32_t *super_ptr,
                                               const int64_t *rptr, const int64_t *lptr,
                                               const int32_t *rows, const int32_t *colpair,
                                               const UpdatePair *pairs, const int32_t *rel, T *Lx) {
    constexpr int TM = kTile, KB = 16;
    using acc_t = typename Mfma<T>::acc;
    __shared__ T As[KB][TM + 4];
    __shared__ T Bs[KB][TM + 4];
    __shared__ T Cs[TM][TM + 1];
    const TileTask tk = tasks[blockIdx.x];
    const int s = tk.s;
    const int64_t m = rptr[s + 1] - rptr[s];
    const T *P = Lx + lptr[s];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    acc_t acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    const int lr = tid & 63, lk = tid >> 6;
    const bool row_ok = tk.i0 + lr < m;
    const bool col_ok = tk.j0 + lr < tk.jmax;
    for (int kb = tk.k0; kb < tk.k1; kb += KB) {
#pragma unroll
        for (int e = 0; e < KB / 4; ++e) {
            int kk = lk + 4 * e;
            int k = kb + kk;
            bool kin = k < tk.k1;
            As[kk][lr] = (kin && row_ok) ? P[(int64_t)k * m + tk.i0 + lr] : T(0);
            Bs[kk][lr] = (kin && col_ok) ? P[(int64_t)k * m + tk.j0 + lr] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KB; kk += 4) {
            T af[2], bf[2];
            for (int a = 0; a < 2; ++a) af[a] = As[kk + (lane >> 4)][wr + a * 16 + (lane & 15)];
            for (int b = 0; b < 2; ++b) bf[b] = Bs[kk + (lane >> 4)][wc + b * 16 + (lane & 15)];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::run(af[a], bf[b], acc[a][b]);
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int v = 0; v < 4; ++v) {
                int r = wr + a * 16 + Mfma<T>::row(lane, v);
                int c = wc + b * 16 + (lane & 15);
                Cs[c][r] = acc[a][b][v];
            }
    __syncthreads();
    const int r = tid & 63, cg = tid >> 6;
    const int gi = tk.i0 + r;
    if (gi >= m) return;
    for (int cc = 0; cc < 16; ++cc) {
        const int c = cg * 16 + cc;
        const int gj = tk.j0 + c;
        if (gj >= tk.jmax || gj > gi) continue;
        const T v = Cs[c][r];
        if (!EXTERNAL) {
            Lx[lptr[s] + (int64_t)gj * m + gi] -= v;
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

// ---------------------------------------------------------------------------
// Triangular solves on the permuted work vectors W (n x nrhs, column-major,
// leading dimension n).  A solve block is columns c0..c1-1 of supernode s.
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

// One workgroup per block: x_blk = D^{-1} x_blk (forward) or D^{-T} x_blk.
template <typename T, bool FORWARD>
__global__ __launch_bounds__(256) void k_solve_diag(const int32_t *order, const SolveBlock *blocks,
                                                    const int32_t *super_ptr, const int64_t *rptr,
                                                    const int64_t *lptr, const T *Lx, T *W, int64_t n,
                                                    int nrhs) {
    constexpr int NB = kSolveNB;
    __shared__ T D[NB][NB + 1];
    __shared__ T X[NB][kMaxRhs + 1];
    const SolveBlock B = blocks[order[blockIdx.x]];
    const int64_t m = rptr[B.s + 1] - rptr[B.s];
    const int nb = B.c1 - B.c0;
    const T *P = Lx + lptr[B.s];
    const int64_t g0 = super_ptr[B.s] + B.c0;
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += 256) {
        int i = e % NB, j = e / NB;
        D[i][j] = (i < nb && j < nb && i >= j) ? P[(int64_t)(B.c0 + j) * m + B.c0 + i] : T(0);
    }
    for (int e = tid; e < NB * kMaxRhs; e += 256) {
        int i = e % NB, q = e / NB;
        X[i][q] = (i < nb && q < nrhs) ? W[g0 + i + (int64_t)q * n] : T(0);
    }
    __syncthreads();
    if (FORWARD) {
        for (int j = 0; j < nb; ++j) {
            if (tid < nrhs) X[j][tid] /= D[j][j];
            __syncthreads();
            for (int e = tid; e < NB * kMaxRhs; e += 256) {
                int i = e % NB, q = e / NB;
                if (i > j && i < nb && q < nrhs) X[i][q] -= D[i][j] * X[j][q];
            }
            __syncthreads();
        }
    } else {
        for (int j = nb - 1; j >= 0; --j) {
            if (tid < nrhs) X[j][tid] /= D[j][j];
            __syncthreads();
            for (int e = tid; e < NB * kMaxRhs; e += 256) {
                int i = e % NB, q = e / NB;
                if (i < j && q < nrhs) X[i][q] -= D[j][i] * X[j][q];
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < NB * kMaxRhs; e += 256) {
        int i = e % NB, q = e / NB;
        if (i < nb && q < nrhs) W[g0 + i + (int64_t)q * n] = X[i][q];
    }
}

// Forward: W[rows[r]] -= sum_k P[r, c0+k] x[k] for rows r0..r1-1 of the task
// (one thread per row, all right-hand sides).
// Backward: x[k] -= sum_r P[r, c0+k] W[rows[r]] (rows staged in LDS by 64).
template <typename T, bool FORWARD>
__global__ __launch_bounds__(256) void k_solve_update(const SolveTask *tasks, const SolveBlock *blocks,
                                                      const int32_t *super_ptr, const int64_t *rptr,
                                                      const int64_t *lptr, const int32_t *rows,
                                                      const T *Lx, T *W, int64_t n, int nrhs) {
    constexpr int NB = kSolveNB;
    const SolveTask tk = tasks[blockIdx.x];
    const SolveBlock B = blocks[tk.blk];
    const int64_t m = rptr[B.s + 1] - rptr[B.s];
    const int nb = B.c1 - B.c0;
    const T *P = Lx + lptr[B.s];
    const int32_t *R = rows + rptr[B.s];
    const int64_t g0 = super_ptr[B.s] + B.c0;
    const int tid = threadIdx.x;
    if (FORWARD) {
        __shared__ T X[NB][kMaxRhs];
        for (int e = tid; e < NB * kMaxRhs; e += 256) {
            int i = e % NB, q = e / NB;
            X[i][q] = (i < nb && q < nrhs) ? W[g0 + i + (int64_t)q * n] : T(0);
        }
        __syncthreads();
        for (int r = tk.r0 + tid; r < tk.r1; r += 256) {
            T acc[kMaxRhs];
            for (int q = 0; q < kMaxRhs; ++q) acc[q] = T(0);
            for (int k = 0; k < nb; ++k) {
                T l = P[(int64_t)(B.c0 + k) * m + r];
#pragma unroll
                for (int q = 0; q < kMaxRhs; ++q) acc[q] += l * X[k][q];
            }
            const int64_t gr = R[r];
            for (int q = 0; q < nrhs; ++q) atomicAdd(&W[gr + (int64_t)q * n], -acc[q]);
        }
    } else {
        __shared__ T Pt[64][NB + 1];
        __shared__ T Y[64][kMaxRhs + 1];
        const int k = tid & 63, qg = tid >> 6;
        T acc[kMaxRhs / 4];
        for (int q = 0; q < kMaxRhs / 4; ++q) acc[q] = T(0);
        for (int rb = tk.r0; rb < tk.r1; rb += 64) {
            const int nr = min(64, tk.r1 - rb);
            for (int e = tid; e < 64 * NB; e += 256) {
                int r = e % 64, c = e / 64;
                Pt[r][c] = (r < nr && c < nb) ? P[(int64_t)(B.c0 + c) * m + rb + r] : T(0);
            }
            for (int e = tid; e < 64 * kMaxRhs; e += 256) {
                int r = e % 64, q = e / 64;
                Y[r][q] = (r < nr && q < nrhs) ? W[(int64_t)R[rb + r] + (int64_t)q * n] : T(0);
            }
            __syncthreads();
            for (int r = 0; r < nr; ++r) {
                T l = Pt[r][k];
#pragma unroll
                for (int q = 0; q < kMaxRhs / 4; ++q) acc[q] += l * Y[r][qg + 4 * q];
            }
            __syncthreads();
        }
        if (k < nb)
            for (int q = 0; q < kMaxRhs / 4; ++q) {
                int qq = qg + 4 * q;
                if (qq < nrhs) atomicAdd(&W[g0 + k + (int64_t)qq * n], -acc[q]);
            }
    }
}

inline unsigned grid1(int64_t count, int block) {
    int64_t g = (count + block - 1) / block;
    return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

template <typename T>
void launch_zero(T *x, int64_t count, hipStream_t st) {
    if (count <= 0) return;
    int64_t g = (count + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)g), dim3(256), 0, st, x, count);
}

void launch_status_reset(unsigned long long *status, hipStream_t st) {
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(1), 0, st, status);
}

template <typename T>
void launch_assemble(const DevPlan &P, int64_t nnz, const double *values, T *Lx, hipStream_t st) {
    if (nnz <= 0) return;
    hipLaunchKernelGGL(k_assemble<T>, dim3(grid1(nnz, 256)), dim3(256), 0, st, P.amap, nnz, values, Lx);
}

template <typename T>
void launch_potrf(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, unsigned long long *status,
                  hipStream_t st) {
    if (t1 <= t0) return;
    hipLaunchKernelGGL(k_potrf<T>, dim3((unsigned)(t1 - t0)), dim3(256), 0, st, P.potrf_tasks + t0,
                       P.super_ptr, P.rptr, P.lptr, Lx, status);
}

template <typename T>
void launch_trsm(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, hipStream_t st) {
    if (t1 <= t0) return;
    hipLaunchKernelGGL(k_trsm<T>, dim3((unsigned)(t1 - t0)), dim3(256), 0, st, P.panel_tasks + t0,
                       P.super_ptr, P.rptr, P.lptr, Lx);
}

template <typename T>
void launch_tiles(const DevPlan &P, bool external, int64_t t0, int64_t t1, T *Lx, hipStream_t st) {
    if (t1 <= t0) return;
    if (external)
        hipLaunchKernelGGL((k_tiles<T, true>), dim3((unsigned)(t1 - t0)), dim3(256), 0, st,
                           P.ext_tiles + t0, P.super_ptr, P.rptr, P.lptr, P.rows, P.colpair, P.pairs,
                           P.rel, Lx);
    else
        hipLaunchKernelGGL((k_tiles<T, false>), dim3((unsigned)(t1 - t0)), dim3(256), 0, st,
                           P.int_tiles + t0, P.super_ptr, P.rptr, P.lptr, P.rows, P.colpair, P.pairs,
                           P.rel, Lx);
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
void launch_solve_diag(const DevPlan &P, bool forward, int64_t e0, int64_t e1, const T *Lx, T *W,
                       int64_t n, int nrhs, hipStream_t st) {
    if (e1 <= e0) return;
    if (forward)
        hipLaunchKernelGGL((k_solve_diag<T, true>), dim3((unsigned)(e1 - e0)), dim3(256), 0, st,
                           P.sblock_order + e0, P.sblocks, P.super_ptr, P.rptr, P.lptr, Lx, W, n, nrhs);
    else
        hipLaunchKernelGGL((k_solve_diag<T, false>), dim3((unsigned)(e1 - e0)), dim3(256), 0, st,
                           P.sblock_order + e0, P.sblocks, P.super_ptr, P.rptr, P.lptr, Lx, W, n, nrhs);
}

template <typename T>
void launch_solve_update(const DevPlan &P, bool forward, int64_t t0, int64_t t1, const T *Lx, T *W,
                         int64_t n, int nrhs, hipStream_t st) {
    if (t1 <= t0) return;
    if (forward)
        hipLaunchKernelGGL((k_solve_update<T, true>), dim3((unsigned)(t1 - t0)), dim3(256), 0, st,
                           P.stasks + t0, P.sblocks, P.super_ptr, P.rptr, P.lptr, P.rows, Lx, W, n, nrhs);
    else
        hipLaunchKernelGGL((k_solve_update<T, false>), dim3((unsigned)(t1 - t0)), dim3(256), 0, st,
                           P.stasks + t0, P.sblocks, P.super_ptr, P.rptr, P.lptr, P.rows, Lx, W, n, nrhs);
}

#define SPC_INSTANTIATE(T)                                                                              \
    template void launch_zero<T>(T *, int64_t, hipStream_t);                                            \
    template void launch_assemble<T>(const DevPlan &, int64_t, const double *, T *, hipStream_t);       \
    template void launch_potrf<T>(const DevPlan &, int64_t, int64_t, T *, unsigned long long *,          \
                                  hipStream_t);                                                         \
    template void launch_trsm<T>(const DevPlan &, int64_t, int64_t, T *, hipStream_t);                  \
    template void launch_tiles<T>(const DevPlan &, bool, int64_t, int64_t, T *, hipStream_t);           \
    template void launch_perm_in<T>(const DevPlan &, int64_t, int, const double *, int64_t, T *,        \
                                    hipStream_t);                                                       \
    template void launch_perm_out<T>(const DevPlan &, int64_t, int, const T *, double *, int64_t,       \
                                     hipStream_t);                                                      \
    template void launch_solve_diag<T>(const DevPlan &, bool, int64_t, int64_t, const T *, T *, int64_t, \
                                       int, hipStream_t);                                               \
    template void launch_solve_update<T>(const DevPlan &, bool, int64_t, int64_t, const T *, T *,       \
                                         int64_t, int, hipStream_t);
SPC_INSTANTIATE(double)
SPC_INSTANTIATE(float)

}  // namespace spc
