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

#include <algorithm>
#include <climits>
#include <mutex>
#include <type_traits>

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

// BF16 updates (SPC_FP32_BF16UPD): D(16x16, FP32) += A(16x32) B(32x16) with
// both operands rounded to BF16 (round to nearest even).  Lane l supplies
// eight consecutive k of row l%16 of A and of column l%16 of B, k = 8 (l/16)
// .. 8 (l/16) + 7; the same k order for A and B is all a sum over k needs.
// D is laid out as in the FP32 16x16x4 shape: element v of lane l is
// D[4 (l/16) + v][l%16].
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f4 mfma_bf16(bf16x8 a, bf16x8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// Eight FP32 values as eight BF16 (16 bytes) for an LDS row of k.
__device__ __forceinline__ bf16x8 to_bf16x8(const float *v) {
    bf16x8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (__bf16)v[e];
    return r;
}

__device__ __forceinline__ bool finite_pos(double d) { return d > 0.0 && d <= 1.7976931348623157e308; }
__device__ __forceinline__ bool finite_pos(float d) { return d > 0.0f && d <= 3.402823466e38f; }

template <typename T>
__global__ void k_zero(T *x, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) x[i] = T(0);
}

__global__ void k_status_reset(unsigned long long *status, int count, int32_t *deverr, int32_t *flags, int nflags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) status[i] = ~0ull;
    if (i < nflags) flags[i] = 0;
    if (i < 2) deverr[i] = 0;  // the device-error word and the raised-pivot count
}

// Data handed from one workgroup to another inside a launch (which may run
// on another XCD, with its own L2) moves through device-scope atomic loads
// and stores, and the flag that announces it is raised only after the
// writer's own stores have completed; no cache-wide fences.
template <typename T>
__device__ __forceinline__ T dev_load(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void dev_store(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Every wait on another workgroup is bounded: after a number of polls
// chosen by the host (about a second's worth by default) it gives up, sets
// the factor's device-error word and goes on, so every wave always exits;
// the host then reports SPC_DEVICE_ERROR.  The pivot status word is never
// used for this.
__device__ __forceinline__ void flag_device_error(int32_t *deverr) {
    __hip_atomic_fetch_or(deverr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded waits: poll an int until it holds `want`; after `spin` polls
// (about a second by default) give up, flag err and go on, so every wave
// always exits.  Once any wait has given up, the others stop waiting too.
__device__ __forceinline__ void wait_value(int32_t *p, int32_t want, int32_t *err, int32_t spin) {
    for (int it = 0; it < spin; ++it) {
        if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == want) return;
        // once any wait has given up, the others stop waiting too
        if ((it & 255) == 255 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
        __builtin_amdgcn_s_sleep(2);
    }
    flag_device_error(err);
}

template <typename T>
__global__ void k_assemble(const int64_t *amap, int64_t nnz, const double *values, T *Lx) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) Lx[amap[k]] = (T)values[k];
}

// Pivot floors of the BF16-update factorization: theta times the diagonal
// entry of A of each permuted column.
template <typename T>
__global__ void k_pivot_floor(const int64_t *dsrc, int64_t n, const double *values, double theta, T *floor) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) floor[j] = (T)(theta * values[dsrc[j]]);
}

// ---------------------------------------------------------------------------
// Global loads in the kernels below are issued unconditionally from clamped,
// always valid indices and masked afterwards, in groups, so that a wave has
// many loads in flight: a load under a branch makes the compiler wait for
// memory at the join, which serializes a loop of them.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// k_potrf: one workgroup (4 waves) per diagonal block (nb <= kNB = 64), held
// in LDS.  Blocked right-looking Cholesky with 16-column panels:
//   - wave 0 factors the panel with lane = row and the panel's 16 columns in
//     registers: for column j, d = a_jj (read from lane j), 1/l_jj from a
//     reciprocal square root, l_ij = a_ij / l_jj, and the later panel
//     columns k lose l_ij l_kj (l_kj read from lane k);
//   - the four waves subtract the panel's product from the trailing lower
//     part in 16x16 MFMA tiles.
// Inverse: each wave inverts one 16x16 diagonal triangle by forward
// substitution (lane = column; the diagonal of L^{-1} is the 1/l_jj of the
// factorization), then the 2x2 block formula for a lower triangle,
//   inv [L11 0; L21 L22] = [X11 0; -X22 L21 X11  X22],
// on the 16-blocks inside each 32-block and then on the two 32-blocks, the
// products on MFMA tiles.  L stays in the lower triangle of A; the strict
// lower part of L^{-1} is kept transposed in the strict upper triangle
// (A[c][a] = Linv[a][c]) and its diagonal in rdg.  A pivot that is not
// positive and finite lowers the status word to its global column.
// L^{-1} is stored column-major: Linv[ioff + k * nb + i] = (L^{-1})_ik.
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

// Bounded wait on an LDS word written by another wave of the workgroup
// (all of whose waves are resident, so the wait ends unless the code is
// wrong; the bound keeps even that from hanging the device).
__device__ __forceinline__ bool lds_wait_geq(int *f, int v) {
    for (int it = 0; it < (1 << 22); ++it) {
        if (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= v) return true;
        __builtin_amdgcn_s_sleep(1);
    }
    return false;
}
// Completes a wave's own LDS operations (and keeps the compiler from moving
// memory accesses across), so its later LDS reads of other lanes' data, and
// other waves after a flag, see them.  Global memory operations in flight
// are not waited for.
__device__ __forceinline__ void wave_lds_sync() {
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __asm__ volatile("" ::: "memory");
}
__device__ __forceinline__ void lds_flag_store(int *f, int v) {
    wave_lds_sync();
    __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_flag_add(int *f) {
    wave_lds_sync();
    __hip_atomic_fetch_add(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Factor the block in A (nb <= 64; rows and columns >= nb hold the identity,
// the upper triangle is zero), write L into P (columns c0.., leading
// dimension m, lower triangle only) and the inverse into Vi; a failed pivot
// lowers *status to g0 + its column.  LDS scratch from the caller: rdg (64
// entries), Tf and T32 (32 x 33 each), flags (8 ints).  Called by all 256
// threads of the workgroup.  With pflags (a full block, nb = 64), each
// panel p is also handed to workgroups of the same launch: its L and the
// inverse of its 16x16 diagonal triangle go out with device-scope atomic
// stores, and each of waves 1-3 adds 1 to pflags[p] once its part has
// completed (3 when the panel is out).
//
// Blocked by 16-column panels with lookahead: wave 0 factors panel p (lane
// = row, pivots broadcast by readlane) right after bringing its columns up
// to date with panel p-1 itself (16x16x4 MFMA), while waves 1-3 apply panel
// p-1 to the columns two panels on and beyond; then wave 1 inverts its 16x16
// diagonal triangle (and merges the second 32-column block's inverse after
// the last panel), wave 2 merges the first 32-column block's inverse once
// its two triangles are inverted, and waves 2-3 store L, so that the
// inverses keep pace with the panels.  The waves hand over through LDS flags, so
// the panel chain never waits for a whole-workgroup barrier.  Each trailing
// tile belongs to one wave for all panels, so no tile is updated by two
// waves at once.
template <typename T, bool BOOST = false>
__device__ __forceinline__ void potrf_lds(T (*A)[kNB + 1], T *rdg, T (*Tf)[33], T (*T32)[33], int *flags, int nb,
                                          T *P, int64_t m, int c0, T *Vi, unsigned long long *status, int32_t *deverr,
                                          int64_t g0, int32_t *pflags, PivotFloor<T> pfl = {}) {
    constexpr int NB = kNB, PW = 16;
    using M = Mfma<T>;
    using acc_t = typename M::acc;
    int &flag_panel = flags[0];   // panels 0 .. flag_panel - 1 are factored in A
    int *flag_trail = flags + 1;  // [4] trailing waves done with panel p (0..3)
    int &flag_err = flags[5];
    int &flag_x11 = flags[6];     // inverse of the first 32-column block done
    int &flag_dinv = flags[7];    // diagonal 16x16 triangles 0 .. flag_dinv - 1 inverted
    // T32: L21 X11 of the two 32-column blocks
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int npan = (nb + PW - 1) / PW;
    if (t == 0) {
        flag_panel = 0;
        flag_trail[0] = flag_trail[1] = flag_trail[2] = flag_trail[3] = 0;
        flag_err = 0;
        flag_x11 = 0;
        flag_dinv = 0;
    }
    if (t >= PW * npan && t < NB) rdg[t] = T(1);  // identity rows past the last panel
    __syncthreads();
#define SPC_INV(a, c) ((c) < (a) ? A[c][a] : ((c) == (a) ? rdg[a] : T(0)))
    auto vi_put = [&](int64_t e, T v) { Vi[e] = v; };
    // one wave's part of a panel is out: its stores have completed
    auto panel_out = [&](int pb) {
        __builtin_amdgcn_s_waitcnt(0);
        if (lane == 0) __hip_atomic_fetch_add(pflags + pb, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // inverse of the 32-column block at o from its two 16-block inverses
    // (one wave): X21 = -X22 L21 X11, kept transposed in the upper triangle
    auto inv16 = [&](int o) {
        const int tr = o >> 1;  // Tf rows tr .. tr + 15
        acc_t acc = {0, 0, 0, 0};  // L21 X11
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4)
            acc = M::run(A[o + 16 + (lane & 15)][o + kk + (lane >> 4)], SPC_INV(o + kk + (lane >> 4), o + (lane & 15)),
                         acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) Tf[tr + M::row(lane, v)][lane & 15] = acc[v];
        wave_lds_sync();
        acc = acc_t{0, 0, 0, 0};  // X22 (L21 X11)
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4)
            acc = M::run(SPC_INV(o + 16 + (lane & 15), o + 16 + kk + (lane >> 4)), Tf[tr + kk + (lane >> 4)][lane & 15],
                         acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) A[o + (lane & 15)][o + 16 + M::row(lane, v)] = -acc[v];
        wave_lds_sync();
    };
    int bad = -1;  // wave 0: first pivot (block column) that failed
    int boosted = 0;
    if (wv == 0) {
        const int i = lane;
        // pivot floors of this block's columns (lane = column), read off the chain
        const T flo = BOOST ? pfl.v[g0 + min(lane, nb - 1)] : T(0);
        for (int pb = 0; pb < npan; ++pb) {
            const int p0 = PW * pb;
            if (pb >= 2 && !lds_wait_geq(&flag_trail[pb - 2], 3)) flag_err = 1;
            if (pb >= 1) {
                // this panel's columns (rows >= p0) minus panel pb-1's
                // product: up to three 16-row tiles, their loads, products
                // and updates each issued together
                const int q0 = p0 - PW;
                T bop[4], aop[3][4], cold[3][4];
                acc_t acc[3];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) bop[kk] = A[p0 + (lane & 15)][q0 + 4 * kk + (lane >> 4)];
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    const int tt = min(pb + x, 3);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) aop[x][kk] = A[16 * tt + (lane & 15)][q0 + 4 * kk + (lane >> 4)];
#pragma unroll
                    for (int v = 0; v < 4; ++v) cold[x][v] = A[16 * tt + M::row(lane, v)][p0 + (lane & 15)];
                }
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    acc[x] = acc_t{0, 0, 0, 0};
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) acc[x] = M::run(aop[x][kk], bop[kk], acc[x]);
                }
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    const int tt = pb + x;
                    if (tt < npan)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int r = 16 * tt + M::row(lane, v), c = p0 + (lane & 15);
                            if (r >= c) A[r][c] = cold[x][v] - acc[x][v];
                        }
                }
                wave_lds_sync();
            }
            T r[PW];
#pragma unroll
            for (int c = 0; c < PW; ++c) r[c] = A[i][p0 + c];
#pragma unroll
            for (int c = 0; c < PW; ++c) {
                const int j = p0 + c;
                T d = lane_read(r[c], j);
                if (BOOST) {
                    const T fj = lane_read(flo, j);
                    if (d < fj && j < nb) {  // a NaN compares false and still fails below
                        d = fj;
                        ++boosted;
                    }
                }
                if (bad < 0 && j < nb && !finite_pos(d)) bad = j;
                const T rs = rsqrt_nr(d);
                if (i == j) rdg[j] = rs;
                const T lij = (i == j) ? d * rs : r[c] * rs;
                r[c] = lij;
#pragma unroll
                for (int c2 = c + 1; c2 < PW; ++c2) r[c2] -= lij * lane_read(lij, p0 + c2);
            }
            // rows >= p0 in full: the entries above the diagonal hold
            // scratch until the inverse levels overwrite every one of them
            if (i >= p0)
#pragma unroll
                for (int c = 0; c < PW; ++c) A[i][p0 + c] = r[c];
            lds_flag_store(&flag_panel, pb + 1);
        }
    } else {
        const int tw = wv - 1;  // trailing wave 0..2
        for (int pb = 0; pb < npan; ++pb) {
            const int p0 = PW * pb;
            if (!lds_wait_geq(&flag_panel, pb + 1)) flag_err = 1;
            // panel pb applied to the tiles (ti, tj), tj >= pb + 2, lower part;
            // tile x = ti (ti + 1) / 2 + tj belongs to trailing wave x % 3
            for (int x = tw; x < 10; x += 3) {
                int ti = 0;
                while ((ti + 1) * (ti + 2) / 2 <= x) ++ti;
                const int tj = x - ti * (ti + 1) / 2;
                if (tj < pb + 2 || ti >= npan) continue;
                const int i0 = 16 * ti, j0 = 16 * tj;
                acc_t acc = {0, 0, 0, 0};
#pragma unroll
                for (int kk = 0; kk < PW; kk += 4)
                    acc = M::run(A[i0 + (lane & 15)][p0 + kk + (lane >> 4)], A[j0 + (lane & 15)][p0 + kk + (lane >> 4)],
                                 acc);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = i0 + M::row(lane, v), c = j0 + (lane & 15);
                    if (r >= c) A[r][c] -= acc[v];
                }
            }
            if (lane == 0) lds_flag_add(&flag_trail[pb]);
            else wave_lds_sync();
            if (wv == 1) {
                // inverse of panel pb's diagonal 16x16 triangle: 2x2 block
                // formula from the diagonal (rdg = 1/l_jj) up, h = 1, 2, 4, 8;
                // X21 is kept transposed in the upper triangle.  Scratch:
                // rows 16.. of Tf (rows 0..15 belong to the merge of the
                // first 32-column block, which wave 2 may be running)
                T *tf = &Tf[16][0];
                // fixed trip counts (h unrolled, terms masked) so each
                // level issues its LDS reads together; lanes >= 8 h compute
                // a clamped copy and store nothing
#pragma unroll
                for (int lv = 0; lv < 4; ++lv) {
                    const int h = 1 << lv, nel = 8 * h;  // 16 / (2h) blocks of h x h
                    const int ln = min(lane, nel - 1);
                    const int blk = ln / (h * h), rem = ln % (h * h), a = rem % h, b = rem / h, o = p0 + 2 * h * blk;
                    T acc = T(0);  // (L21 X11)[a][b]
#pragma unroll
                    for (int c = 0; c < h; ++c) {
                        const T l = A[o + h + a][o + c], x = SPC_INV(o + c, o + b);
                        acc += (c >= b) ? l * x : T(0);
                    }
                    if (lane < nel) tf[lane] = acc;
                    wave_lds_sync();
                    T out = T(0);  // -(X22 (L21 X11))[a][b]
#pragma unroll
                    for (int c = 0; c < h; ++c) {
                        const T x = SPC_INV(o + h + a, o + h + c), u = tf[blk * h * h + b * h + c];
                        out -= (c <= a) ? x * u : T(0);
                    }
                    wave_lds_sync();
                    if (lane < nel) A[o + b][o + h + a] = out;
                    wave_lds_sync();
                }
                lds_flag_store(&flag_dinv, pb + 1);
                if (pflags) {
                    // the panel's diagonal 16x16 block of the inverse
#pragma unroll
                    for (int q = 0; q < PW * PW / 64; ++q) {
                        const int e = lane + 64 * q, i = p0 + e % PW, k = p0 + e / PW;
                        dev_store(Vi + k * nb + i, SPC_INV(i, k));
                    }
                    panel_out(pb);
                }
                // the second 32-column block (its second 16-block may be
                // identity padding) is merged right after its last panel
                if (pb >= 2 && pb == npan - 1) inv16(32);
            } else {
                // waves 2 and 3 store L of panel pb (rows >= p0 of its
                // columns), so that wave 1 keeps up with the panels
                for (int e = lane + 64 * (wv - 2); e < PW * NB; e += 128) {
                    const int k = p0 + e / NB, row = e % NB;
                    if (k < nb && row >= k && row < nb) {
                        T *dst = P + (int64_t)(c0 + k) * m + c0 + row;
                        if (pflags) dev_store(dst, A[row][k]);
                        else *dst = A[row][k];
                    }
                }
                if (pflags) panel_out(pb);
            }
            if (pb == 1 && wv == 2) {
                // the first 32-column block: merge its two inverted
                // 16-blocks once wave 1 has both
                if (!lds_wait_geq(&flag_dinv, 2)) flag_err = 1;
                inv16(0);
                lds_flag_store(&flag_x11, 1);
            }
            if (pb == 1 && nb > 2 * PW && wv >= 2) {
                // the first 32-column block's inverse X11 is final: wave 2
                // forms L21 X11 for the last merge, wave 3 stores the
                // inverse's first 32 rows (X11, zeros to its right)
                if (!lds_wait_geq(&flag_x11, 1)) flag_err = 1;
                if (wv == 2) {
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt) {
                        const int ti = tt >> 1, tj = tt & 1;
                        acc_t acc = {0, 0, 0, 0};
#pragma unroll
                        for (int kk = 0; kk < 32; kk += 4)
                            acc = M::run(A[32 + 16 * ti + (lane & 15)][kk + (lane >> 4)],
                                         SPC_INV(kk + (lane >> 4), 16 * tj + (lane & 15)), acc);
#pragma unroll
                        for (int v = 0; v < 4; ++v) T32[16 * ti + M::row(lane, v)][16 * tj + (lane & 15)] = acc[v];
                    }
                } else {
                    for (int e = lane; e < 32 * nb; e += 64) {
                        const int i = e & 31, k = e >> 5;
                        vi_put(k * nb + i, SPC_INV(i, k));
                    }
                }
            }
        }
    }
    __syncthreads();
    if (wv == 0 && lane == 0) {
        if (bad >= 0) atomicMin(status, (unsigned long long)(g0 + bad));
        if (flag_err) flag_device_error(deverr);
        if (BOOST && boosted) atomicAdd(pfl.count, boosted);
    }
    if (nb > 32) {
        // the two 32-blocks: X21 = -X22 (L21 X11), wave w the 16x16 tile
        // (w / 2, w % 2); the first 32 rows of the inverse are stored already
        const int ti = wv >> 1, tj = wv & 1;
        acc_t acc = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 32; kk += 4)
            acc = M::run(SPC_INV(32 + 16 * ti + (lane & 15), 32 + kk + (lane >> 4)),
                         T32[kk + (lane >> 4)][16 * tj + (lane & 15)], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) A[16 * tj + (lane & 15)][32 + 16 * ti + M::row(lane, v)] = -acc[v];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 32 * NB / 256; ++q) {
            const int e = t + 256 * q, i = 32 + e % 32, k = e / 32;
            if (i < nb && k < nb) vi_put(k * nb + i, SPC_INV(i, k));
        }
    } else {
#pragma unroll
        for (int q = 0; q < NB * NB / 256; ++q) {
            const int e = t + 256 * q, i = e % NB, k = e / NB;
            if (i < nb && k < nb) vi_put(k * nb + i, SPC_INV(i, k));
        }
    }
#undef SPC_INV
}

template <typename T, bool BOOST>
__global__ __launch_bounds__(256) void k_potrf(const PanelTask *tasks, T *Lx, T *Linv,
                                               unsigned long long *status, const int32_t *status_slot,
                                               int32_t *deverr, PivotFloor<T> pfl) {
    constexpr int NB = kNB;
    __shared__ T A[NB][NB + 1];
    __shared__ T rdg[NB];
    __shared__ T Tf[32][33];
    __shared__ T T32[32][33];
    __shared__ int flags[8];
    const PanelTask tk = tasks[blockIdx.x];
    const int64_t m = tk.m;
    const int c0 = tk.c0, nb = tk.c1 - tk.c0;
    T *P = Lx + tk.loff;
    const int t = threadIdx.x;
    {
        T ld[NB * NB / 256];
#pragma unroll
        for (int q = 0; q < NB * NB / 256; ++q) {
            const int e = t + 256 * q, i = e % NB, k = e / NB;
            const int ic = min(i, nb - 1), kc = min(k, ic);
            ld[q] = P[(int64_t)(c0 + kc) * m + c0 + ic];
        }
#pragma unroll
        for (int q = 0; q < NB * NB / 256; ++q) {
            const int e = t + 256 * q, i = e % NB, k = e / NB;
            A[i][k] = (i < nb && k <= i) ? ld[q] : (i == k ? T(1) : T(0));
        }
    }
    __syncthreads();
    potrf_lds<T, BOOST>(A, rdg, Tf, T32, flags, nb, P, m, c0, Linv + tk.ioff,
                        status + (status_slot ? status_slot[tk.s] : 0), deverr, tk.g0, nullptr, pfl);
}

// ---------------------------------------------------------------------------
// k_tiny: one wave per supernode with w <= kTinyW and m <= kTinyM (four per
// workgroup, no LDS, no barriers): lane = row of the panel, the row's w
// entries in registers, values of other rows read from their lanes.
//   1. column Cholesky: l_jj = sqrt(d_j), l_ij = a_ij / l_jj, then
//      a_ik -= l_ij l_kj for the later columns;
//   2. inverse of the diagonal triangle: lane c < w forms column c by
//      forward substitution;
//   3. the update C[i][k] = sum_j l_ij l_kj of the rows below (w <= k <= i),
//      scatter-added into the ancestors: C[i][k] goes to cbase[k] +
//      rel[crel[k] + i].
// Pivots that are not positive and finite lower the status word.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t lane_read_i64(int64_t v, int src) {
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), src);
    return ((int64_t)hi << 32) | (uint32_t)lo;
}

// One wave's tiny supernode (the body of k_tiny and of the persistent
// launch).  COH: the panel is read with device-scope loads, for a launch in
// which other workgroups (on other XCDs) scatter-added into it.
template <typename T, bool COH>
__device__ __forceinline__ void tiny_body(const SmallTask &tk, const int64_t *cbase, const int64_t *crel,
                                          const int32_t *rel, T *Lx, T *Linv, unsigned long long *status,
                                          const int32_t *status_slot, PivotFloor<T> pfl) {
    constexpr int WT = kTinyW, CB = 8;  // CB: update columns per batch of loads
    const int lane = threadIdx.x & 63;
    const int m = tk.m, w = tk.w;
    T *P = Lx + tk.loff;
    const int rc = min(lane, m - 1);
    T r[WT];
#pragma unroll
    for (int c = 0; c < WT; ++c) {
        const T *src = &P[(int64_t)min(c, w - 1) * m + rc];
        r[c] = COH ? dev_load(src) : *src;
    }
    // scatter addressing of this lane's row position taken as a column
    const int64_t kpos = tk.roff + min(max(lane, w), m - 1);
    const int64_t my_cb = cbase[kpos], my_cr = crel[kpos];
    // 1. column Cholesky
    int bad = -1, boosted = 0;
    T rdg[WT];
    const T flo = pfl.v ? pfl.v[tk.g0 + min(lane, w - 1)] : T(0);
#pragma unroll
    for (int c = 0; c < WT; ++c) {
        if (c < w) {
            T d = lane_read(r[c], c);
            if (pfl.v) {
                const T fc = lane_read(flo, c);
                if (d < fc) {
                    d = fc;
                    ++boosted;
                }
            }
            if (bad < 0 && !finite_pos(d)) bad = c;
            const T rs = rsqrt_nr(d);
            rdg[c] = rs;
            const T lic = (lane == c) ? d * rs : r[c] * rs;
            r[c] = lic;
#pragma unroll
            for (int c2 = c + 1; c2 < WT; ++c2)
                if (c2 < w) r[c2] -= lic * lane_read(lic, c2);
        }
    }
    if (lane == 0 && bad >= 0)
        atomicMin(status + (status_slot ? status_slot[tk.s] : 0), (unsigned long long)(tk.g0 + bad));
    if (lane == 0 && boosted) atomicAdd(pfl.count, boosted);
    if (lane < m)
#pragma unroll
        for (int c = 0; c < WT; ++c)
            if (c < w && c <= lane) P[(int64_t)c * m + lane] = r[c];
    // 2. inverse of the diagonal triangle, column `lane`
    {
        T y[WT];
#pragma unroll
        for (int a = 0; a < WT; ++a) {
            T v = (a == lane) ? T(1) : T(0);
#pragma unroll
            for (int k = 0; k < a; ++k) v -= lane_read(r[k], a) * y[k];
            y[a] = a < w ? v * rdg[a] : T(0);
        }
        T *Vi = Linv + tk.ioff;
        if (lane < w)
#pragma unroll
            for (int a = 0; a < WT; ++a)
                if (a < w) Vi[lane * w + a] = y[a];
    }
    // 3. update of the rows below, scatter-added into the ancestors
    for (int k0 = w; k0 < m; k0 += CB) {
        int32_t rv[CB];
        int64_t cbk[CB];
        T acc[CB];
        bool ok[CB];
#pragma unroll
        for (int u = 0; u < CB; ++u) {
            const int k = k0 + u, kc = min(k, m - 1);
            cbk[u] = lane_read_i64(my_cb, kc);
            const int64_t crk = lane_read_i64(my_cr, kc);
            ok[u] = k < m && lane >= k && lane < m;
            rv[u] = rel[crk + (ok[u] ? lane : kc)];
            T a = T(0);
#pragma unroll
            for (int j = 0; j < WT; ++j)
                if (j < w) a += r[j] * lane_read(r[j], kc);
            acc[u] = a;
        }
#pragma unroll
        for (int u = 0; u < CB; ++u)
            if (ok[u]) atomicAdd(&Lx[cbk[u] + rv[u]], -acc[u]);
    }
}

// ---------------------------------------------------------------------------
// Grouped tiny supernodes (w <= kGroupW, m <= G): G = 16 or 32 lanes per
// supernode, 64 / G of them per wave, the steps of tiny_body inside each
// group; values of other rows come from their lanes by ds_bpermute (every
// lane of the wave takes part in each exchange, so a lane read is always
// active).  Groups past the end of a launch's list (live false) run on an
// identity block and store nothing.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t pull32(int32_t v, int src) {
    return __builtin_amdgcn_ds_bpermute(src << 2, v);
}
__device__ __forceinline__ double lane_pull(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = pull32((int)(b & 0xffffffffll), src), hi = pull32((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_pull(float v, int src) { return __int_as_float(pull32(__float_as_int(v), src)); }
__device__ __forceinline__ int64_t lane_pull(int64_t v, int src) {
    const int lo = pull32((int)(v & 0xffffffffll), src), hi = pull32((int)(v >> 32), src);
    return ((int64_t)hi << 32) | (uint32_t)lo;
}

template <typename T, int G, bool COH>
__device__ __forceinline__ void group_body(const SmallTask &tk, bool live, const int64_t *cbase, const int64_t *crel,
                                           const int32_t *rel, T *Lx, T *Linv, unsigned long long *status,
                                           const int32_t *status_slot, PivotFloor<T> pfl) {
    constexpr int WG = kGroupW, CB = 4;
    static_assert(G == 16 || G == 32, "group of 16 or 32 lanes");
    const int lane = threadIdx.x & 63, gi = lane & (G - 1), gb = lane - gi;
    const int m = live ? tk.m : 1, w = live ? tk.w : 1;
    T *P = Lx + tk.loff;
    const int rc = min(gi, m - 1);
    T r[WG];
#pragma unroll
    for (int c = 0; c < WG; ++c) {
        if (live) {
            const T *src = &P[(int64_t)min(c, w - 1) * m + rc];
            r[c] = COH ? dev_load(src) : *src;
        } else {
            r[c] = gi == c ? T(1) : T(0);
        }
    }
    int64_t my_cb = 0, my_cr = 0;
    if (live) {
        const int64_t kpos = tk.roff + min(max(gi, w), m - 1);
        my_cb = cbase[kpos];
        my_cr = crel[kpos];
    }
    const T flo = (live && pfl.v) ? pfl.v[tk.g0 + min(gi, w - 1)] : T(0);
    // 1. column Cholesky (columns past w are padding: left alone)
    int bad = -1, boosted = 0;
    T rdg[WG];
#pragma unroll
    for (int c = 0; c < WG; ++c) {
        const bool on = c < w;
        T d = lane_pull(r[c], gb + c);
        if (pfl.v) {
            const T fc = lane_pull(flo, gb + c);
            if (on && d < fc) {
                d = fc;
                ++boosted;
            }
        }
        if (on && bad < 0 && !finite_pos(d)) bad = c;
        const T rs = rsqrt_nr(on ? d : T(1));
        rdg[c] = rs;
        const T lic = (gi == c) ? d * rs : r[c] * rs;
        if (on) r[c] = lic;
#pragma unroll
        for (int c2 = c + 1; c2 < WG; ++c2) {
            const T lk = lane_pull(lic, gb + c2);
            if (on) r[c2] -= lic * lk;
        }
    }
    if (live && gi == 0 && bad >= 0)
        atomicMin(status + (status_slot ? status_slot[tk.s] : 0), (unsigned long long)(tk.g0 + bad));
    if (live && gi == 0 && boosted) atomicAdd(pfl.count, boosted);
    if (live && gi < m)
#pragma unroll
        for (int c = 0; c < WG; ++c)
            if (c < w && c <= gi) P[(int64_t)c * m + gi] = r[c];
    // 2. inverse of the diagonal triangle, column gi
    {
        T y[WG];
#pragma unroll
        for (int a = 0; a < WG; ++a) {
            T v = (a == gi) ? T(1) : T(0);
#pragma unroll
            for (int k = 0; k < a; ++k) v -= lane_pull(r[k], gb + a) * y[k];
            y[a] = a < w ? v * rdg[a] : T(0);
        }
        T *Vi = Linv + tk.ioff;
        if (live && gi < w)
#pragma unroll
            for (int a = 0; a < WG; ++a)
                if (a < w) Vi[gi * w + a] = y[a];
    }
    // 3. update of the rows below, scatter-added into the ancestors
#pragma unroll
    for (int k0 = 0; k0 < G; k0 += CB) {
        int32_t rv[CB];
        int64_t cbk[CB];
        T acc[CB];
        bool ok[CB];
#pragma unroll
        for (int u = 0; u < CB; ++u) {
            const int k = k0 + u, kc = min(max(k, w), m - 1);
            cbk[u] = lane_pull(my_cb, gb + kc);
            const int64_t crk = lane_pull(my_cr, gb + kc);
            ok[u] = live && k >= w && k < m && gi >= k && gi < m;
            rv[u] = ok[u] ? rel[crk + gi] : 0;
            T a = T(0);
#pragma unroll
            for (int j = 0; j < WG; ++j) {
                const T lk = lane_pull(r[j], gb + kc);
                if (j < w) a += r[j] * lk;
            }
            acc[u] = a;
        }
#pragma unroll
        for (int u = 0; u < CB; ++u)
            if (ok[u]) atomicAdd(&Lx[cbk[u] + rv[u]], -acc[u]);
    }
}

// The tiny supernodes of one level: tasks [0, n16) in groups of 16 lanes
// (16 per workgroup), [n16, n32) in groups of 32 (8 per workgroup), the
// rest one wave each (4 per workgroup); the workgroups of the three parts
// follow each other.
template <typename T>
__global__ __launch_bounds__(256) void k_tiny(const SmallTask *tasks, int64_t n16, int64_t n32, int64_t ntasks,
                                              const int64_t *cbase, const int64_t *crel, const int32_t *rel, T *Lx,
                                              T *Linv, unsigned long long *status, const int32_t *status_slot,
                                              PivotFloor<T> pfl) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int64_t b = blockIdx.x;
    const int64_t b16 = (n16 + 15) / 16, b32 = (n32 - n16 + 7) / 8;
    if (b < b16) {
        const int64_t gi = b * 16 + wv * 4 + (lane >> 4);
        const bool live = gi < n16;
        group_body<T, 16, false>(tasks[live ? gi : 0], live, cbase, crel, rel, Lx, Linv, status, status_slot, pfl);
        return;
    }
    b -= b16;
    if (b < b32) {
        const int64_t gi = n16 + b * 8 + wv * 2 + (lane >> 5);
        const bool live = gi < n32;
        group_body<T, 32, false>(tasks[live ? gi : n16], live, cbase, crel, rel, Lx, Linv, status, status_slot,
                                 pfl);
        return;
    }
    b -= b32;
    const int64_t ti = n32 + b * 4 + wv;
    if (ti >= ntasks) return;  // the whole wave
    tiny_body<T, false>(tasks[ti], cbase, crel, rel, Lx, Linv, status, status_slot, pfl);
}

// ---------------------------------------------------------------------------
// k_small: one workgroup per small supernode (w <= kSmallW, m <= kSmallM),
// the whole m x w panel in LDS:
//   1. column Cholesky of the panel, right-looking: l_jj = sqrt(d_j),
//      l_ij = a_ij / l_jj, then a_ik -= l_ij l_kj for the columns right of j
//      (POTRF of the diagonal block and TRSM of the rows below at once);
//   2. the inverse of the diagonal triangle, one column per thread by
//      forward substitution (kept for the solves);
//   3. the update C = P P^T of the rows below the block, scatter-added into
//      the ancestors: C[i][k] goes to cbase[k] + rel[crel[k] + i].
// Pivots that are not positive and finite lower the status word.
// ---------------------------------------------------------------------------
// LDS of one small supernode: A[c][i] = panel entry (row i, column c), the
// inverse Vt[c][a] = (L^{-1})_ac, and the scatter addresses of its rows.
template <typename T>
struct SmallLds {
    T A[kSmallW][kSmallM + 1];
    T Vt[kSmallW][kSmallW + 1];
    int64_t cb[kSmallM], cr[kSmallM];
};

// One workgroup's small supernode (the body of k_small and of the
// persistent launch); COH as in tiny_body.
template <typename T, bool COH>
__device__ __forceinline__ void small_body(const SmallTask &tk, SmallLds<T> &L, const int64_t *cbase,
                                           const int64_t *crel, const int32_t *rel, T *Lx, T *Linv,
                                           unsigned long long *status, const int32_t *status_slot,
                                           PivotFloor<T> pfl) {
    constexpr int MS = kSmallM, WS = kSmallW, LPT = WS * MS / 256, SB = 8;
    auto &A = L.A;
    auto &Vt = L.Vt;
    auto &cb = L.cb;
    auto &cr = L.cr;
    const int m = tk.m, w = tk.w;
    T *P = Lx + tk.loff;
    const int tid = threadIdx.x;
    {
        T ld[LPT];
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int e = tid + 256 * q, i = e % MS, c = e / MS;
            const T *src = &P[(int64_t)min(c, w - 1) * m + min(i, m - 1)];
            ld[q] = COH ? dev_load(src) : *src;
        }
        if (tid < MS) {
            const int64_t k = tk.roff + min(max(tid, w), m - 1);
            cb[tid] = cbase[k];
            cr[tid] = crel[k];
        }
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int e = tid + 256 * q, i = e % MS, c = e / MS;
            A[c][i] = (i < m && c < w) ? ld[q] : T(0);
        }
    }
    __syncthreads();
    int bad = -1, boosted = 0;
    for (int j = 0; j < w; ++j) {
        T d = A[j][j];
        if (pfl.v) {
            const T fj = pfl.v[tk.g0 + j];
            if (d < fj) {
                d = fj;
                ++boosted;
            }
        }
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
        atomicMin(status + (status_slot ? status_slot[tk.s] : 0), (unsigned long long)(tk.g0 + bad));
    if (tid == 0 && boosted) atomicAdd(pfl.count, boosted);
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
    T *Vi = Linv + tk.ioff;
    for (int e = tid; e < w * w; e += 256) Vi[e] = Vt[e / w][e % w];
    // update of the rows below, scatter-added into the ancestors
    const int mb = m - w, ne = mb * mb;
    for (int e0 = 0; e0 < ne; e0 += 256 * SB) {
        int32_t rr[SB];
        int cc_[SB];
        T vv[SB];
        bool ok[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int e = e0 + tid + 256 * u;
            const int r = w + e % mb, cc = w + e / mb;  // row, column (positions in R_s)
            ok[u] = e < ne && cc <= r;
            const int rc = ok[u] ? r : w, ccc = ok[u] ? cc : w;
            cc_[u] = ccc;
            rr[u] = rel[cr[ccc] + rc];
            T acc = T(0);
            for (int k = 0; k < w; ++k) acc += A[k][rc] * A[k][ccc];
            vv[u] = acc;
        }
#pragma unroll
        for (int u = 0; u < SB; ++u)
            if (ok[u]) atomicAdd(&Lx[cb[cc_[u]] + rr[u]], -vv[u]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_small(const SmallTask *tasks, const int64_t *cbase, const int64_t *crel,
                                               const int32_t *rel, T *Lx, T *Linv, unsigned long long *status,
                                               const int32_t *status_slot, PivotFloor<T> pfl) {
    __shared__ SmallLds<T> L;
    small_body<T, false>(tasks[blockIdx.x], L, cbase, crel, rel, Lx, Linv, status, status_slot, pfl);
}

// ---------------------------------------------------------------------------
// k_persist_small: every small subtree of the elimination forest (of every
// system of a batch), all its levels, in one launch.  Resident workgroups
// take queue entries from a work counter; the queue is in level order, so
// every supernode an entry waits for belongs to an earlier entry, which a
// running workgroup holds or has finished: no wait can deadlock.  An entry is
// one small supernode (the workgroup, small_body) or up to four tiny ones
// (one wave each, tiny_body).  Before it starts, a supernode waits until
// every source inside the launch has scatter-added its update into it
// (pdep[s] counted down to 0); after its own scatter-adds have completed
// (s_waitcnt), it counts down each of its targets inside the launch.  The
// scatter-adds are device-scope atomics and the panel is read with
// device-scope loads, so the values cross XCDs without cache-wide fences.
// ---------------------------------------------------------------------------
__global__ void k_persist_reset(const int32_t *pdep0, int64_t ns, int32_t *pdep, int32_t *qctr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns) pdep[i] = pdep0[i];
    if (i == 0) *qctr = 0;
}

// (at least six waves per SIMD where the LDS allows it, i.e. in FP32: the
// entries are latency-bound, and 4 -> 6 waves cut the 512-system batch's
// launch from 13.3 to 10.4 ms)
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_persist_small(const PersistEntry *queue, const int32_t *chunk, int64_t nc,
                                                       const SmallTask *psmall,
                                                       const SmallTask *ptiny, const int64_t *ptgt_ptr,
                                                       const int32_t *ptgt, int32_t *pdep, int32_t *qctr,
                                                       const int64_t *cbase, const int64_t *crel, const int32_t *rel,
                                                       T *Lx, T *Linv, unsigned long long *status,
                                                       const int32_t *status_slot, PivotFloor<T> pfl, WaitCtl wc) {
    __shared__ SmallLds<T> L;
    __shared__ int32_t slot;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (;;) {
        if (tid == 0) slot = atomicAdd(qctr, 1);
        __syncthreads();
        const int64_t c = slot;
        __syncthreads();  // every thread has read the slot
        if (c >= nc) return;
        // the chunk's entries in order: an entry waits only on entries before
        // it, earlier in this chunk (done) or in chunks taken before
        for (int32_t q = chunk[c]; q < chunk[c + 1]; ++q) {
        const PersistEntry e = queue[q];
        if (e.kind == 0) {
            const SmallTask tk = psmall[e.first];
            if (tid == 0) wait_value(&pdep[tk.s], 0, wc.err, wc.spin);
            __syncthreads();
            small_body<T, true>(tk, L, cbase, crel, rel, Lx, Linv, status, status_slot, pfl);
            __builtin_amdgcn_s_waitcnt(0);  // this thread's scatter-adds have completed
            __syncthreads();
            for (int64_t k = ptgt_ptr[tk.s] + tid; k < ptgt_ptr[tk.s + 1]; k += 256) atomicSub(&pdep[ptgt[k]], 1);
        } else if (e.kind == 1) {
            if (wv < e.count) {
                const SmallTask tk = ptiny[e.first + wv];
                if (lane == 0) wait_value(&pdep[tk.s], 0, wc.err, wc.spin);
                __asm__ volatile("" ::: "memory");
                tiny_body<T, true>(tk, cbase, crel, rel, Lx, Linv, status, status_slot, pfl);
                __builtin_amdgcn_s_waitcnt(0);
                for (int64_t k = ptgt_ptr[tk.s] + lane; k < ptgt_ptr[tk.s + 1]; k += 64)
                    atomicSub(&pdep[ptgt[k]], 1);
            }
        } else {
            // kind 2 (3): up to 16 (8) tiny supernodes in groups of 16 (32)
            // lanes; each group's first lane waits for its own supernode
            const int G = e.kind == 2 ? 16 : 32;
            const int gi = wv * (64 / G) + lane / G, gl = lane & (G - 1);
            const bool live = gi < e.count;
            const SmallTask tk = ptiny[e.first + (live ? gi : 0)];
            if (live && gl == 0) wait_value(&pdep[tk.s], 0, wc.err, wc.spin);
            __asm__ volatile("" ::: "memory");
            if (e.kind == 2)
                group_body<T, 16, true>(tk, live, cbase, crel, rel, Lx, Linv, status, status_slot, pfl);
            else
                group_body<T, 32, true>(tk, live, cbase, crel, rel, Lx, Linv, status, status_slot, pfl);
            __builtin_amdgcn_s_waitcnt(0);
            if (live)
                for (int64_t k = ptgt_ptr[tk.s] + gl; k < ptgt_ptr[tk.s + 1]; k += G) atomicSub(&pdep[ptgt[k]], 1);
        }
        __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// MFMA tiles.  One workgroup (4 waves) computes a 64x64 tile C = A B^T,
// each wave a 2x2 set of 16x16x4 MFMA blocks; K staged through LDS 16 at a
// time, the next chunk loaded into registers while the current one is used.
//   MODE_TRAILING: A, B = panel rows i0.., j0..; P[i][j] -= C for i >= j,
//                  j < jmax.  The diagonal tile of the next column block
//                  then factors that block (potrf_lds); a tile below it
//                  with a flag then solves X L^T = P - C for its rows,
//                  following the block's panels as they are handed out,
//                  and stores X instead.  The block's factorization is
//                  claimed by whichever of these workgroups comes first.
//   MODE_SCATTER:  A, B = panel rows i0.., j0..; C (i >= j) scatter-added
//                  atomically into the ancestors: C[i][j] goes to
//                  cbase[j] + rel[crel[j] + i].
//   MODE_TRSM:     B = inverse of block blk (at aux), stored as
//                  Q[k' * nb + c] = (L^{-1})_{c k'}; P[i][k0 + c] = C
//                  (rows times the transposed inverse: X = B L^{-T}).
// ---------------------------------------------------------------------------
enum { MODE_TRAILING = 0, MODE_SCATTER = 1, MODE_TRSM = 2 };

template <typename T, int MODE, bool BF = false>
__global__ __launch_bounds__(256, 3) void k_tiles(const TileTask *tasks, const int64_t *cbase, const int64_t *crel,
                                               const int32_t *rel, T *Linv, T *Lx, unsigned long long *status,
                                               const int32_t *status_slot, int32_t *hflags, WaitCtl wctl,
                                               PivotFloor<T> pfl) {
    constexpr int TM = kTile, KB = 16, CPT = 16;
    using acc_t = typename Mfma<T>::acc;
    __shared__ T ABs[2][KB][TM + 4];  // A and B chunks, one buffer
    __shared__ T Cs[TM][TM + 1];
    __shared__ int64_t cb[TM], cr[TM];
    __shared__ int claimed;
    T(*As)[TM + 4] = ABs[0];
    T(*Bs)[TM + 4] = ABs[1];
    const TileTask own = tasks[blockIdx.x];
    if (MODE == MODE_TRAILING && own.s < 0) return;  // a no-op entry of the launch layout
    // the claim of the next block's factorization (see below): thread 0 of
    // the diagonal tile's workgroup takes it at its start and reads the
    // outcome only before factoring, so the atomic's round trip overlaps the
    // tile's update
    int32_t *const claim = (MODE == MODE_TRAILING && own.flag >= 0) ? hflags + kFlagsPerBlock * own.flag + 4 : nullptr;
    int32_t ticket = 0;
    // one tile task (the whole body; its returns end that task); defer: the
    // diagonal tile's own task, which factors the block only if its ticket
    // won the claim
    auto body = [&](const TileTask tk, bool defer) {
    const int64_t m = tk.m;
    T *P = Lx + tk.loff;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    const int lr = tid & 63, lk = tid >> 6;
    const int kw = tk.k1 - tk.k0;
    const bool row_ok = tk.i0 + lr < m;
    const bool col_ok = (MODE == MODE_TRSM) ? lr < kw : tk.j0 + lr < tk.jmax;
    const T *pa = P + min<int64_t>(tk.i0 + lr, m - 1);
    const T *pb = (MODE == MODE_TRSM) ? Linv + tk.aux + min(lr, kw - 1) : P + min(tk.j0 + lr, tk.jmax - 1);
    const int64_t ldb = (MODE == MODE_TRSM) ? kw : m;
    const int kofs = (MODE == MODE_TRSM) ? tk.k0 : 0;
    if (MODE == MODE_SCATTER && tid < TM) {
        const int64_t k = tk.aux + min(tk.j0 + tid, tk.jmax - 1);
        cb[tid] = cbase[k];
        cr[tid] = crel[k];
    }
    // the next K chunk is loaded into registers while the current one is used
    T ra[KB / 4], rb[KB / 4];
    auto load = [&](int kb) {
#pragma unroll
        for (int e = 0; e < KB / 4; ++e) {
            const int k = min(kb + lk + 4 * e, tk.k1 - 1);
            ra[e] = pa[(int64_t)k * m];
            rb[e] = pb[(int64_t)(k - kofs) * ldb];
        }
    };
    const int r = tid & 63, cg = tid >> 6;
    const int64_t gi = tk.i0 + r;
    T old[CPT];  // trailing tiles: the tile's values before the update
    auto load_old = [&] {
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            const int64_t gj = min(tk.j0 + cg * CPT + cc, tk.jmax - 1);
            old[cc] = P[gj * m + min<int64_t>(gi, m - 1)];
        }
    };
    if (MODE == MODE_TRAILING && tk.blk >= 0 && tk.i0 == tk.j0) {
        // the diagonal tile of the next block heads the step's critical
        // path: the tile and its panel rows (A = B) are loaded with one
        // round trip, TM columns of K at a time, staged in Cs
        load_old();
        for (int kb = tk.k0; kb < tk.k1; kb += TM) {
            T xv[TM / 4];
#pragma unroll
            for (int e = 0; e < TM / 4; ++e) xv[e] = pa[(int64_t)min(kb + lk + 4 * e, tk.k1 - 1) * m];
            if (kb > tk.k0) __syncthreads();
#pragma unroll
            for (int e = 0; e < TM / 4; ++e)
                Cs[lk + 4 * e][lr] = (kb + lk + 4 * e < tk.k1 && row_ok) ? xv[e] : T(0);
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < TM; kk += 4) {
                T af[2], bf[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) af[a] = Cs[kk + (lane >> 4)][wr + a * 16 + (lane & 15)];
#pragma unroll
                for (int b = 0; b < 2; ++b) bf[b] = Cs[kk + (lane >> 4)][wc + b * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::run(af[a], bf[b], acc[a][b]);
            }
        }
        __syncthreads();
    } else if constexpr (BF) {
        // BF16 operands, FP32 accumulation, K staged 32 at a time: thread
        // (row lr, quarter lk) loads k = 8 lk .. 8 lk + 7 of its row of A
        // and of B, rounds them to BF16 and writes each as 16 bytes of an
        // LDS row (k contiguous), which a lane then reads with one load
        static_assert(sizeof(T) == 4, "BF16 updates are for FP32 panels");
        constexpr int KBB = 32, RS = KBB + 8;  // row stride in bf16 (16 bytes of padding)
        // staged in Cs, which the epilogue needs only after the last chunk
        __bf16 *Ab = reinterpret_cast<__bf16 *>(&Cs[0][0]);
        __bf16 *Bb = Ab + TM * RS;
        static_assert(2 * TM * RS * sizeof(__bf16) <= sizeof(Cs), "bf16 staging fits the output tile buffer");
        float fa[8], fb[8];
        auto loadb = [&](int kb) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = min(kb + 8 * lk + e, tk.k1 - 1);
                fa[e] = pa[(int64_t)k * m];
                fb[e] = pb[(int64_t)k * m];
            }
        };
        loadb(tk.k0);
        for (int kb = tk.k0; kb < tk.k1; kb += KBB) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const bool kin = kb + 8 * lk + e < tk.k1;
                fa[e] = (kin && row_ok) ? fa[e] : 0.0f;
                fb[e] = (kin && col_ok) ? fb[e] : 0.0f;
            }
            *reinterpret_cast<bf16x8 *>(Ab + lr * RS + 8 * lk) = to_bf16x8(fa);
            *reinterpret_cast<bf16x8 *>(Bb + lr * RS + 8 * lk) = to_bf16x8(fb);
            __syncthreads();
            if (kb + KBB < tk.k1) loadb(kb + KBB);
            bf16x8 af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                af[a] = *reinterpret_cast<const bf16x8 *>(Ab + (wr + a * 16 + (lane & 15)) * RS + 8 * (lane >> 4));
#pragma unroll
            for (int b = 0; b < 2; ++b)
                bf[b] = *reinterpret_cast<const bf16x8 *>(Bb + (wc + b * 16 + (lane & 15)) * RS + 8 * (lane >> 4));
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = mfma_bf16(af[a], bf[b], acc[a][b]);
            __syncthreads();
        }
        if (MODE == MODE_TRAILING) load_old();
    } else {
        load(tk.k0);
        for (int kb = tk.k0; kb < tk.k1; kb += KB) {
#pragma unroll
            for (int e = 0; e < KB / 4; ++e) {
                const int kk = lk + 4 * e;
                const bool kin = kb + kk < tk.k1;
                As[kk][lr] = (kin && row_ok) ? ra[e] : T(0);
                Bs[kk][lr] = (kin && col_ok) ? rb[e] : T(0);
            }
            __syncthreads();
            if (kb + KB < tk.k1) load(kb + KB);
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
        // epilogue: thread = row r, columns cg*16 .. cg*16+15
        if (MODE == MODE_TRAILING) load_old();
    }
    int32_t rv[CPT];
    if (MODE == MODE_SCATTER) {
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            const int c = cg * CPT + cc;
            const int64_t gj = min(tk.j0 + c, tk.jmax - 1);
            rv[cc] = rel[cr[c] + max(min<int64_t>(gi, m - 1), gj)];
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = wr + a * 16 + Mfma<T>::row(lane, v);
                const int c = wc + b * 16 + (lane & 15);
                Cs[c][rr] = acc[a][b][v];
            }
    __syncthreads();
    if (MODE == MODE_TRAILING && tk.blk >= 0 && tk.i0 == tk.j0) {
        // diagonal tile of the next column block: its rows r < nb2 form the
        // block, final after this update; factor it here (rows below it are
        // stored as in any other tile)
        const int nb2 = min(TM, tk.jmax - tk.j0);
        T nv[CPT];
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) nv[cc] = old[cc] - Cs[cg * CPT + cc][r];
        if (r >= nb2 && gi < m)
#pragma unroll
            for (int cc = 0; cc < CPT; ++cc) {
                const int64_t gj = tk.j0 + cg * CPT + cc;
                if (gj < tk.jmax) P[gj * m + gi] = nv[cc];
            }
        if (defer) {
            if (tid == 0) claimed = ticket == 0;
            __syncthreads();
            if (!claimed) return;  // a tile below took the factorization
        }
        __syncthreads();
        // LDS for the factorization: the tile buffers, free now (cb and cr
        // hold no scatter addresses in this mode)
        T(*A)[TM + 1] = Cs;
        T *rdg = reinterpret_cast<T *>(cb);
        int *flags = reinterpret_cast<int *>(cr);
        T(*Tf)[33] = reinterpret_cast<T(*)[33]>(&Bs[0][0]);
        T(*T32)[33] = reinterpret_cast<T(*)[33]>(&As[0][0]);
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            const int c = cg * CPT + cc;
            A[r][c] = (r < nb2 && c <= r) ? nv[cc] : (r == c ? T(1) : T(0));
        }
        __syncthreads();
        // with a flag, each panel goes to the tiles below as it comes out
        // (also after a failed pivot, which the status word reports, so
        // that no tile waits in vain)
        potrf_lds<T, BF>(A, rdg, Tf, T32, flags, nb2, P, m, tk.j0, Linv + tk.aux,
                         status + (status_slot ? status_slot[tk.s] : 0), wctl.err, tk.blk,
                         tk.flag >= 0 ? hflags + kFlagsPerBlock * tk.flag : nullptr, pfl);
        return;
    }
    if (MODE == MODE_TRAILING && tk.flag >= 0) {
        // below the diagonal tile of a block factored in this launch: the
        // block's TRSM on this tile, X L^T = C (C the updated tile), 16
        // columns at a time as the block's panels come out: X_p = C_p
        // L_pp^{-T}, then C_q -= X_p L_qp^T for the later panels q.  Each
        // wave owns 16 rows of the tile, so the waves never wait for each
        // other, only for the panel flags (3 once a panel is out).
        static_assert(TM == kNB && TM == 64, "four 16-column panels per block");
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) Cs[cg * CPT + cc][r] = old[cc] - Cs[cg * CPT + cc][r];
        __syncthreads();
        const T *Vi = Linv + tk.aux;                        // (L^{-1})_{jk} at Vi[k * TM + j]
        const T *Lb = P + (int64_t)tk.j0 * m + tk.j0;       // block-local L[i][k] at Lb[k * m + i]
        int32_t *pf = hflags + kFlagsPerBlock * tk.flag;
        const int w16 = wave * 16, l16 = lane & 15, lk4 = lane >> 4;
        bool ok = true;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            // wait for panel p (every lane reads the same word: one load)
            bool ready = false;
            for (int it = 0; ok && it < wctl.spin; ++it) {
                if (__builtin_amdgcn_readfirstlane(dev_load(pf + p)) >= 3) {
                    ready = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            ok = ok && ready;
            __asm__ volatile("" ::: "memory");
            // B operands: the inverse of the panel's diagonal triangle,
            // B[k][j] = (L^{-1})_{16p+j,16p+k}, and L below it, B[k][j] =
            // L[16q+j][16p+k]
            T bi[4], bl[3][4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 16 * p + 4 * kk + lk4;
                bi[kk] = dev_load(Vi + k * TM + 16 * p + l16);
#pragma unroll
                for (int q = p + 1; q < 4; ++q) bl[q - p - 1][kk] = dev_load(Lb + (int64_t)k * m + 16 * q + l16);
            }
            // X_p for this wave's rows, staged over C_p in Cs
            acc_t x = {0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) x = Mfma<T>::run(Cs[16 * p + 4 * kk + lk4][w16 + l16], bi[kk], x);
#pragma unroll
            for (int v = 0; v < 4; ++v) Cs[16 * p + l16][w16 + Mfma<T>::row(lane, v)] = x[v];
            wave_lds_sync();
#pragma unroll
            for (int q = p + 1; q < 4; ++q) {
                acc_t u = {0, 0, 0, 0};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    u = Mfma<T>::run(Cs[16 * p + 4 * kk + lk4][w16 + l16], bl[q - p - 1][kk], u);
#pragma unroll
                for (int v = 0; v < 4; ++v) Cs[16 * q + l16][w16 + Mfma<T>::row(lane, v)] -= u[v];
            }
            wave_lds_sync();
        }
        if (!ok && lane == 0) flag_device_error(wctl.err);
        __syncthreads();
        if (gi < m)
#pragma unroll
            for (int cc = 0; cc < CPT; ++cc) P[(tk.j0 + cg * CPT + cc) * m + gi] = Cs[cg * CPT + cc][r];
        return;
    }
    if (gi >= m) return;
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
        const int c = cg * CPT + cc;
        const int64_t gj = tk.j0 + c;
        if (gj >= tk.jmax) continue;
        const T v = Cs[c][r];
        if (MODE == MODE_TRSM) {
            P[gj * m + gi] = v;
        } else if (MODE == MODE_TRAILING) {
            if (gj <= gi) P[gj * m + gi] = old[cc] - v;
        } else {
            if (gj <= gi) atomicAdd(&Lx[cb[c] + rv[cc]], -v);
        }
    }
    };
    if (MODE == MODE_TRAILING && own.flag >= 0) {
        // The factorization of the next block (its diagonal tile's update,
        // POTRF and the panels handed out) is one job that the first
        // workgroup of the hand-over to arrive claims: the diagonal tile's,
        // or, if that one has not started yet, a tile below it, which does
        // the job before its own work.  A tile that waits for the panels
        // thus always waits for a workgroup that is running and never waits
        // itself, whatever the dispatch order, the XCDs or other launches.
        // The claim word is cleared with the factorization's status.  The
        // diagonal tile starts at once and looks at its ticket before it
        // factors; a tile below first reads the word and takes a ticket
        // only while nobody has (the diagonal tile, first in the launch,
        // nearly always has).
        if (own.i0 == own.j0) {
            if (threadIdx.x == 0) ticket = __hip_atomic_fetch_add(claim, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            body(own, true);
            return;
        }
        if (threadIdx.x == 0)
            claimed = dev_load(claim) == 0 &&
                      __hip_atomic_fetch_add(claim, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
        __syncthreads();
        const bool mine = claimed;
        __syncthreads();
        if (mine) {
            TileTask d = own;
            d.i0 = d.j0;
            body(d, false);
            __syncthreads();
        }
    }
    body(own, false);
}

// ---------------------------------------------------------------------------
// k_tiles128: the scatter update on 128x128 tiles for the large supernodes
// (same operation as k_tiles in MODE_SCATTER), or, with TRAIL, the bulk
// trailing update inside a wide supernode (as MODE_TRAILING without the
// next block's factorization: P[i][j] -= C for i >= j, j < jmax, in place).
// 8 waves in a 2x4 grid of 64x32 sub-tiles, each a 4x2 set of 16x16x4 MFMA
// blocks, so two waves share each SIMD and hide each other's MFMA latency; K
// staged through LDS 16 at a time with the next chunk in registers while the
// current one is consumed.  The epilogue goes through LDS in four passes of
// 32 columns.
// ---------------------------------------------------------------------------
template <typename T, bool BF = false, bool TRAIL = false>
__global__ __launch_bounds__(512) void k_tiles128(const TileTask *tasks, const int64_t *cbase, const int64_t *crel,
                                                  const int32_t *rel, T *Lx) {
    constexpr int TM = 128, KB = 16, PADA = 4, CPT = 8, NT = 512;
    constexpr int KBB = 32, RS = KBB + 8;  // BF16: K per chunk, LDS row stride (bf16)
    using acc_t = typename Mfma<T>::acc;
    constexpr int kSmem = BF ? (2 * TM * RS * 2 + sizeof(T) - 1) / sizeof(T) : 2 * KB * (TM + PADA);
    __shared__ T smem[kSmem];
    __shared__ int64_t cb[TM], cr[TM];
    T(*As)[TM + PADA] = reinterpret_cast<T(*)[TM + PADA]>(smem);
    T(*Bs)[TM + PADA] = reinterpret_cast<T(*)[TM + PADA]>(smem + KB * (TM + PADA));
    const TileTask tk = tasks[blockIdx.x];
    const int64_t m = tk.m;
    T *P = Lx + tk.loff;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 2) * 64, wc = (wave & 3) * 32;
    acc_t acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    // loader: thread covers row lr (0..127) and k-rows lk, lk+4, lk+8, lk+12
    const int lr = tid & 127, lk = tid >> 7;
    const bool row_ok = tk.i0 + lr < m;
    const bool col_ok = tk.j0 + lr < tk.jmax;
    const T *pa = P + min<int64_t>(tk.i0 + lr, m - 1);
    const T *pb = P + min(tk.j0 + lr, tk.jmax - 1);
    if (!TRAIL && tid < TM) {
        const int64_t k = tk.aux + min(tk.j0 + tid, tk.jmax - 1);
        cb[tid] = cbase[k];
        cr[tid] = crel[k];
    }
    if constexpr (BF) {
        // BF16 operands, FP32 accumulation (as in k_tiles): thread (row lr,
        // quarter lk) stages k = 8 lk .. 8 lk + 7 of its rows of A and B
        static_assert(sizeof(T) == 4, "BF16 updates are for FP32 panels");
        __bf16 *Ab = reinterpret_cast<__bf16 *>(smem);
        __bf16 *Bb = Ab + TM * RS;
        float fa[8], fb[8];
        auto loadb = [&](int kb) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t k = min(kb + 8 * lk + e, tk.k1 - 1);
                fa[e] = pa[k * m];
                fb[e] = pb[k * m];
            }
        };
        loadb(tk.k0);
        for (int kb = tk.k0; kb < tk.k1; kb += KBB) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const bool kin = kb + 8 * lk + e < tk.k1;
                fa[e] = (kin && row_ok) ? fa[e] : 0.0f;
                fb[e] = (kin && col_ok) ? fb[e] : 0.0f;
            }
            *reinterpret_cast<bf16x8 *>(Ab + lr * RS + 8 * lk) = to_bf16x8(fa);
            *reinterpret_cast<bf16x8 *>(Bb + lr * RS + 8 * lk) = to_bf16x8(fb);
            __syncthreads();
            if (kb + KBB < tk.k1) loadb(kb + KBB);
            bf16x8 af[4], bf[2];
#pragma unroll
            for (int a = 0; a < 4; ++a)
                af[a] = *reinterpret_cast<const bf16x8 *>(Ab + (wr + a * 16 + (lane & 15)) * RS + 8 * (lane >> 4));
#pragma unroll
            for (int b = 0; b < 2; ++b)
                bf[b] = *reinterpret_cast<const bf16x8 *>(Bb + (wc + b * 16 + (lane & 15)) * RS + 8 * (lane >> 4));
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = mfma_bf16(af[a], bf[b], acc[a][b]);
            __syncthreads();
        }
    } else {
    T ra[KB / 4], rb[KB / 4];
    auto load = [&](int kb) {
#pragma unroll
        for (int e = 0; e < KB / 4; ++e) {
            const int64_t k = min(kb + lk + 4 * e, tk.k1 - 1);
            ra[e] = pa[k * m];
            rb[e] = pb[k * m];
        }
    };
    load(tk.k0);
    for (int kb = tk.k0; kb < tk.k1; kb += KB) {
#pragma unroll
        for (int e = 0; e < KB / 4; ++e) {
            const bool kin = kb + lk + 4 * e < tk.k1;
            As[lk + 4 * e][lr] = (kin && row_ok) ? ra[e] : T(0);
            Bs[lk + 4 * e][lr] = (kin && col_ok) ? rb[e] : T(0);
        }
        __syncthreads();
        if (kb + KB < tk.k1) load(kb + KB);
#pragma unroll
        for (int kk = 0; kk < KB; kk += 4) {
            T af[4], bf[2];
#pragma unroll
            for (int a = 0; a < 4; ++a) af[a] = As[kk + (lane >> 4)][wr + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bf[b] = Bs[kk + (lane >> 4)][wc + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::run(af[a], bf[b], acc[a][b]);
        }
        __syncthreads();
    }
    }
    // epilogue: 4 passes of 32 columns staged as Cs[32][128 + 1]; in pass p
    // the two waves with wc = 32 p stage their columns, then thread (row r,
    // quarter cq) adds 8 of them
    static_assert(32 * (TM + 1) <= kSmem, "the epilogue's staging fits");
    T(*Cs)[TM + 1] = reinterpret_cast<T(*)[TM + 1]>(smem);
    const int r = tid & 127, cq = tid >> 7;
    const int64_t gi = tk.i0 + r;
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        int32_t rv[CPT];
        T old[CPT];
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            const int c = 32 * pass + cq * CPT + cc;
            const int64_t gj = min(tk.j0 + c, tk.jmax - 1);
            if constexpr (TRAIL) {
                old[cc] = P[gj * m + min<int64_t>(gi, m - 1)];
                rv[cc] = 0;
            } else {
                rv[cc] = rel[cr[c] + max(min<int64_t>(gi, m - 1), gj)];
                old[cc] = T(0);
            }
        }
        if (wc == 32 * pass)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        Cs[b * 16 + (lane & 15)][wr + a * 16 + Mfma<T>::row(lane, v)] = acc[a][b][v];
        __syncthreads();
        if (gi < m) {
#pragma unroll
            for (int cc = 0; cc < CPT; ++cc) {
                const int c = 32 * pass + cq * CPT + cc;
                const int64_t gj = tk.j0 + c;
                if (gj >= tk.jmax || gj > gi) continue;
                if constexpr (TRAIL)
                    P[gj * m + gi] = old[cc] - Cs[c & 31][r];
                else
                    atomicAdd(&Lx[cb[c] + rv[cc]], -Cs[c & 31][r]);
            }
        }
        __syncthreads();
    }
    (void)NT;
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
    int64_t k = i / nrhs, r = i % nrhs;
    W[i] = (T)B[perm[k] + r * ldb];
}

template <typename T>
__global__ void k_perm_out(const int32_t *perm, int64_t n, int nrhs, const T *W, double *B, int64_t ldb) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    int64_t k = i / nrhs, r = i % nrhs;
    B[perm[k] + r * ldb] = (double)W[i];
}

constexpr int kMaxRhs = 16;

// Persistent sweeps: instead of one launch per block-tree level, a grid of
// resident workgroups takes tasks from an atomic counter in an order where
// every task's dependencies come first, so a task waits only on tasks that
// running workgroups already hold and the sweep cannot deadlock.  Forward:
// a block's tasks wait until every task updating its rows has counted down
// dep[block]; backward: a task waits until the blocks owning its rows are
// done (bounded waits, wait_value).

// Data handed between workgroups of one persistent sweep moves through
// device-scope atomics (loads after a wait, stores before a flag is raised),
// and a workgroup raises a flag after waiting for its own memory operations;
// no cache-wide fences, whose writeback and invalidation cost more than the
// data.
template <typename T>
__device__ __forceinline__ T shared_load(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void shared_store(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void release_own() { __builtin_amdgcn_s_waitcnt(0); }
__device__ __forceinline__ void acquire_after_wait() {}

// Hand-over buffers between consecutive blocks of a supernode: filled with
// a signalling-NaN pattern before the sweep, which no arithmetic result
// takes (a NaN that arithmetic yields is quiet), so a reader polls the
// value itself and the writer needs no flag after it.
template <typename T>
struct Unset;
template <>
struct Unset<double> {
    using bits_t = unsigned long long;
    static constexpr bits_t bits = 0x7ff5a5a5a5a5a5a5ull;
};
template <>
struct Unset<float> {
    using bits_t = unsigned int;
    static constexpr bits_t bits = 0x7fa5a5a5u;
};
template <typename T>
__device__ __forceinline__ bool is_unset(T v) {
    return __builtin_bit_cast(typename Unset<T>::bits_t, v) == Unset<T>::bits;
}
// Bounded wait for a handed-over value (0 once a wait gave up).
template <typename T>
__device__ __forceinline__ T wait_handed(const T *p, int32_t *err, int32_t spin) {
    for (int it = 0; it < spin; ++it) {
        const T v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!is_unset(v)) return v;
        if ((it & 255) == 255 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return T(0);
        __builtin_amdgcn_s_sleep(1);
    }
    flag_device_error(err);
    return T(0);
}

// Next task of a workgroup: the persistent grid takes it from the work
// counter (through `order` when given), the level-launch grid takes its
// own index once.  Returns -1 when there is none.
template <bool PERSIST>
__device__ __forceinline__ int64_t next_task(int pass, const int32_t *order, int32_t *queue, int64_t ntasks,
                                             int32_t *slot) {
    if (!PERSIST) return pass == 0 ? (int64_t)blockIdx.x : -1;
    if (threadIdx.x == 0) *slot = atomicAdd(queue, 1);
    __syncthreads();
    const int64_t i = *slot;
    if (i >= ntasks) return -1;
    return order ? order[i] : i;
}

// Forward, one task = rows r0..r1-1 below block q:
//   x_q = Linv_q y_q (every task; the first task stores it in X), then
//   Y[rows[r]] -= sum_k L[r][c0+k] x_q[k] (atomic).
// One right-hand side: thread = row for the update; for x_q four threads
// share a row of Linv (16 columns each, held in registers) and add up by
// lane shuffles.  Everything a task reads besides y (its panel rows, its
// part of Linv, its target blocks) is loaded before it waits.
// A persistent task's rows fall in at most 256 blocks (one per row), so
// each thread holds at most one target block to count down.
// Persistent sweep, inside a supernode: the first task of block q - 1 puts
// its sums for q's rows into H (as values, not subtracted from Y) instead
// of counting q down, and q's tasks take y_q = Y - H once those values are
// there (hand bits).
template <typename T, bool PERSIST>
__global__ __launch_bounds__(256) void k_solve_fwd(const SolveTask *tasks, int64_t ntasks, const int32_t *rows,
                                                   const T *Lx, const T *Linv, T *Y, T *X, T *H, int64_t n,
                                                   const int64_t *tgt_ptr, const int32_t *tgt, SolveSync sy) {
    constexpr int NB = kNB, QW = NB / 4;
    __shared__ T yq[NB];
    __shared__ T xq[NB];
    __shared__ int32_t slot;
    const int tid = threadIdx.x;
    const int vi = tid >> 2, vp = tid & 3;  // x: row vi of Linv, columns QW vp .. QW vp + QW - 1
    for (int pass = 0;; ++pass) {
        const int64_t t = next_task<PERSIST>(pass, nullptr, sy.queue, ntasks, &slot);
        if (t < 0) return;
        const SolveTask tk = tasks[t];
        const int nb = tk.nb;
        const int64_t m = tk.m;
        const T *P = Lx + tk.loff;
        const T *Q = Linv + tk.ioff;
        const int64_t r = tk.r0 + tid;
        const int64_t rc = min(r, m - 1);
        T qv[QW], pv[NB];
        const int qi = min(vi, nb - 1);
#pragma unroll
        for (int k = 0; k < QW; ++k) qv[k] = Q[qi + (int64_t)min(QW * vp + k, nb - 1) * nb];
        const int64_t gr = rows[tk.roff + rc];
#pragma unroll
        for (int k = 0; k < NB; ++k) pv[k] = P[(int64_t)(tk.c0 + min(k, nb - 1)) * m + rc];
        int32_t my_tgt = -1;
        if (PERSIST) {
            const int64_t tb = tgt_ptr[t], te = tgt_ptr[t + 1];
            if (tid < te - tb) my_tgt = tgt[tb + tid];
            if (tid == 0) wait_value(&sy.dep[tk.blk], 0, sy.err, sy.spin);
            __syncthreads();
            acquire_after_wait();
        }
        if (tid < NB) {
            const T *py = &Y[tk.g0 + min(tid, nb - 1)];
            T yv = PERSIST ? shared_load(py) : *py;
            if (PERSIST && (tk.hand & kHandIn) && tid < nb) yv -= wait_handed(&H[tk.g0 + tid], sy.err, sy.spin);
            yq[tid] = tid < nb ? yv : T(0);
        }
        __syncthreads();
        {
            T a0 = T(0), a1 = T(0);
#pragma unroll
            for (int k = 0; k < QW; k += 2) {
                const int c = QW * vp + k;
                a0 += (c <= vi ? qv[k] : T(0)) * yq[c];
                a1 += (c + 1 <= vi ? qv[k + 1] : T(0)) * yq[c + 1];
            }
            T a = a0 + a1;
            a += __shfl_xor(a, 1);
            a += __shfl_xor(a, 2);
            if (vp == 0) {
                xq[vi] = vi < nb ? a : T(0);
                if (tk.first && vi < nb) X[tk.g0 + vi] = a;
            }
        }
        __syncthreads();
        if (r < tk.r1) {
            // entries of x_q beyond nb are zero, so clamped columns add nothing
            T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
#pragma unroll
            for (int k = 0; k < NB; k += 4) {
                a0 += pv[k] * xq[k];
                a1 += pv[k + 1] * xq[k + 1];
                a2 += pv[k + 2] * xq[k + 2];
                a3 += pv[k + 3] * xq[k + 3];
            }
            const T v = (a0 + a1) + (a2 + a3);
            if (PERSIST && (tk.hand & kHandOut) && tid < (tk.hand >> 8)) shared_store(&H[gr], v);
            else atomicAdd(&Y[gr], -v);
        }
        if (PERSIST) {
            release_own();
            __syncthreads();
            if (my_tgt >= 0 && !((tk.hand & kHandOut) && my_tgt == tk.blk + 1)) atomicSub(&sy.dep[my_tgt], 1);
        }
    }
}

// Several right-hand sides (up to kMaxRhs): the update of the task's rows
// is the product (rows x 64) (64 x 16) on 16x16x4 MFMA blocks, wave w
// taking the 16-row tiles w, w + 4, w + 8 and w + 12 in that order (so the
// first 64 rows, handed over to the next block in the persistent sweep, are
// done first, by all four waves); the A operand comes straight from the
// panel, the B operand (x_q) from LDS.  Two workgroups per CU (the FP64
// form then keeps 256 registers with a spill of two): the persistent sweep
// runs twice as many resident workgroups, so the tasks waiting on a block
// leave room for the ones on the chain.
template <typename T, bool PERSIST>
__global__ __launch_bounds__(256, 2) void k_solve_fwd_multi(const SolveTask *tasks, int64_t ntasks,
                                                         const int32_t *rows, const T *Lx, const T *Linv, T *Y,
                                                         T *X, T *H, int64_t n, int nrhs, const int64_t *tgt_ptr,
                                                         const int32_t *tgt, SolveSync sy) {
    constexpr int NB = kNB, NR = kMaxRhs, YPT = NB * NR / 256, KS = NB / 4;
    using acc_t = typename Mfma<T>::acc;
    __shared__ T yq[NB][NR + 1];
    __shared__ T xq[NB][NR + 1];
    __shared__ int64_t grs[256];
    __shared__ int32_t slot;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int pass = 0;; ++pass) {
        const int64_t t = next_task<PERSIST>(pass, nullptr, sy.queue, ntasks, &slot);
        if (t < 0) return;
        const SolveTask tk = tasks[t];
        const int nb = tk.nb;
        const int64_t m = tk.m;
        const T *P = Lx + tk.loff;
        const T *Q = Linv + tk.ioff;
        // x = Linv y on MFMA as well: wave w the rows 16 w .. 16 w + 15 of x,
        // lane bringing Linv[16 w + lane % 16][4 s + lane / 16]
        // Level launches: K-steps of 4 columns that reach the block's nb
        // columns, and the row tiles of 16 that reach the task's rows; the
        // clamped operands beyond them only ever meet zeros, so the narrow
        // blocks and short tasks of the bottom levels skip their loads and
        // products (same for every lane of a wave).  The persistent sweep,
        // of mostly full blocks, keeps the unconditional form.
        const int ksn = (nb + 3) >> 2;
        const int64_t nrows = tk.r1 - tk.r0;
        T qv[KS], yv[YPT], av[4][KS];
        if constexpr (PERSIST) {
#pragma unroll
            for (int s2 = 0; s2 < KS; ++s2) {
                const int i = 16 * wave + (lane & 15), c = 4 * s2 + (lane >> 4);
                const T v = Q[min(i, nb - 1) + (int64_t)min(c, nb - 1) * nb];
                qv[s2] = (c <= i && i < nb) ? v : T(0);
            }
        } else {
#pragma unroll
            for (int s2 = 0; s2 < KS; ++s2) {
                const int i = 16 * wave + (lane & 15), c = 4 * s2 + (lane >> 4);
                const T v = s2 < ksn ? Q[min(i, nb - 1) + (int64_t)min(c, nb - 1) * nb] : T(0);
                qv[s2] = (c <= i && i < nb) ? v : T(0);
            }
        }
        grs[tid] = rows[tk.roff + min<int64_t>(tk.r0 + tid, m - 1)];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            const int64_t row = min<int64_t>(tk.r0 + 16 * (4 * tt + wave) + (lane & 15), m - 1);
            if constexpr (PERSIST) {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
                    av[tt][ks] = P[(int64_t)(tk.c0 + min(4 * ks + (lane >> 4), nb - 1)) * m + row];
            } else {
                const bool live = 16 * (4 * tt + wave) < nrows;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
                    av[tt][ks] = live && ks < ksn
                                     ? P[(int64_t)(tk.c0 + min(4 * ks + (lane >> 4), nb - 1)) * m + row]
                                     : T(0);
            }
        }
        int32_t my_tgt = -1;
        if (PERSIST) {
            // at most one target block per row of the task
            const int64_t tb = tgt_ptr[t], te = tgt_ptr[t + 1];
            if (tid < te - tb) my_tgt = tgt[tb + tid];
            if (tid == 0) wait_value(&sy.dep[tk.blk], 0, sy.err, sy.spin);
            __syncthreads();
            acquire_after_wait();
        }
#pragma unroll
        for (int u = 0; u < YPT; ++u) {
            const int e = tid + 256 * u, i = e / NR, q = e % NR;
            const T *py = &Y[(tk.g0 + min(i, nb - 1)) * nrhs + min(q, nrhs - 1)];
            yv[u] = PERSIST ? shared_load(py) : *py;
        }
#pragma unroll
        for (int u = 0; u < YPT; ++u) {
            const int e = tid + 256 * u, i = e / NR, q = e % NR;
            if (PERSIST && (tk.hand & kHandIn) && i < nb && q < nrhs)
                yv[u] -= wait_handed(&H[(tk.g0 + i) * nrhs + q], sy.err, sy.spin);
            yq[i][q] = (i < nb && q < nrhs) ? yv[u] : T(0);
        }
        __syncthreads();
        {
            acc_t xa = {0, 0, 0, 0};
#pragma unroll
            for (int s2 = 0; s2 < KS; ++s2)
                if (PERSIST || s2 < ksn) xa = Mfma<T>::run(qv[s2], yq[4 * s2 + (lane >> 4)][lane & 15], xa);
#pragma unroll
            for (int v = 0; v < 4; ++v) xq[16 * wave + Mfma<T>::row(lane, v)][lane & 15] = xa[v];
        }
        __syncthreads();
        if (tk.first)
            for (int e = tid; e < nb * nrhs; e += 256) {
                const int i = e / nrhs, q = e % nrhs;
                X[(tk.g0 + i) * nrhs + q] = xq[i][q];
            }
        // rows of x_q beyond nb are zero, so the clamped columns contribute nothing
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            if constexpr (!PERSIST) {
                if (16 * (4 * tt + wave) >= nrows) continue;  // no row of this tile is the task's
            }
            acc_t acc = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                if (PERSIST || ks < ksn) acc = Mfma<T>::run(av[tt][ks], xq[4 * ks + (lane >> 4)][lane & 15], acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = 16 * (4 * tt + wave) + Mfma<T>::row(lane, v), q = lane & 15;
                if (tk.r0 + rr < tk.r1 && q < nrhs) {
                    if (PERSIST && (tk.hand & kHandOut) && rr < (tk.hand >> 8))
                        shared_store(&H[grs[rr] * nrhs + q], acc[v]);
                    else
                        atomicAdd(&Y[grs[rr] * nrhs + q], -acc[v]);
                }
            }
        }
        if (PERSIST) {
            release_own();
            __syncthreads();
            if (my_tgt >= 0 && !((tk.hand & kHandOut) && my_tgt == tk.blk + 1)) atomicSub(&sy.dep[my_tgt], 1);
        }
        __syncthreads();
    }
}

// Backward, one task = rows r0..r1-1 below block q: thread (k, g) sums
// L[r][c0+k] X[rows[r]] over the rows r of group g (64 rows each); the four
// groups are added through LDS.  A block with one task finishes itself:
//   t = X_q - sum,  x_q = Linv_q^T t.
// A block split over several tasks adds its sums into Acc.  In a level
// launch the last task to arrive (sy.cnt) finishes the block.  In the
// persistent sweep the block's first task does: it holds the rows nearest
// the block, whose x are final last, and it is queued after the block's
// other tasks, so it collects their sums (waiting on sy.cnt) before its own
// rows are ready, which keeps that exchange off the chain of blocks.
// Rows below the block belong to ancestors, whose x is final before the
// block's tasks read it (level order, or the done flags of the persistent
// sweep).  Persistent sweep, inside a supernode: the task finishing block
// q also puts x_q into XB, and the first task of block q - 1 (whose first
// rows are q's) polls XB for those rows instead of q's done flag (hand bits).
template <typename T, int NR, bool PERSIST>
__global__ __launch_bounds__(256) void k_solve_bwd(const SolveTask *tasks, int64_t ntasks, const int32_t *order,
                                                   const int32_t *rows, const T *Lx, const T *Linv, T *X, T *Acc,
                                                   T *XB, int64_t n, int nrhs, const int64_t *tgt_ptr,
                                                   const int32_t *tgt, SolveSync sy) {
    constexpr int NB = kNB, QW = 16, RG = 64;
    constexpr int XR = 256 * (NR + 1), SM = 4 * NB * NR, VT = NR == 1 ? 0 : NB * (NB + 1);
    constexpr int SH = XR > SM ? (XR > VT ? XR : VT) : (SM > VT ? SM : VT);
    __shared__ T sh[SH];
    __shared__ T tq[NB][NR];
    __shared__ T ao[NB][NR];  // persistent finisher: the other tasks' sums
    __shared__ int last;
    __shared__ int32_t slot;
    T(*xr)[NR + 1] = reinterpret_cast<T(*)[NR + 1]>(sh);   // x of the task's rows
    T(*Sm)[NB][NR] = reinterpret_cast<T(*)[NB][NR]>(sh);    // sums of the 4 groups
    T(*Vt)[NB + 1] = reinterpret_cast<T(*)[NB + 1]>(sh);    // block inverse (several RHS)
    const int tid = threadIdx.x, k = tid & 63, g = tid >> 6;
    // x_q = Linv^T t, with (Linv^T)[c][i] = Linv[i][c] nonzero for i >= c.
    // One right-hand side: four threads per output c, 16 rows i each, that
    // part of Linv held in registers.  Several: Linv is loaded coalesced and
    // staged in LDS, then 16x16x4 MFMA, wave g the outputs 16 g .. 16 g + 15,
    // lane bringing A[c][i] for c = 16 g + lane % 16, i = 4 s + lane / 16.
    const int oc = tid >> 2;
    auto inv_row = [&](int s2) { return QW * (tid & 3) + s2; };
    for (int pass = 0;; ++pass) {
        const int64_t t = next_task<PERSIST>(pass, order, sy.queue + 1, ntasks, &slot);
        if (t < 0) return;
        const SolveTask tk = tasks[t];
        const int nb = tk.nb;
        const int64_t m = tk.m;
        const T *P = Lx + tk.loff;
        const T *Q = Linv + tk.ioff;
        const int64_t rown = tk.r0 + tid;
        const int64_t gr = rows[tk.roff + min(rown, m - 1)];
        T qv[QW], pv[RG];
#pragma unroll
        for (int u = 0; u < RG; ++u)
            pv[u] = P[(int64_t)(tk.c0 + min(k, nb - 1)) * m + min<int64_t>(tk.r0 + g * RG + u, m - 1)];
        if constexpr (NR == 1) {
#pragma unroll
            for (int s2 = 0; s2 < QW; ++s2) {
                const int i = inv_row(s2);
                const T v = Q[min(i, nb - 1) + (int64_t)min(oc, nb - 1) * nb];
                qv[s2] = (i >= oc && i < nb && oc < nb) ? v : T(0);
            }
        } else {
#pragma unroll
            for (int u = 0; u < QW; ++u) qv[u] = Q[min(tid + 256 * u, nb * nb - 1)];
        }
        int32_t my_tgt = -1;
        if (PERSIST) {
            // at most one target block per row of the task
            const int64_t tb = tgt_ptr[t], te = tgt_ptr[t + 1];
            if (tid < te - tb) my_tgt = tgt[tb + tid];
        }
        // the block's own forward values: final since the forward sweep, and
        // overwritten only by the task that finishes this block, so a task
        // known to finish it loads them before it waits
        constexpr int XPT = NB * NR / 256 > 0 ? NB * NR / 256 : 1;
        T xb[XPT];
        auto load_xb = [&]() {
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int e = tid + 256 * u, i = min(e / nrhs, nb - 1), q = min(e % nrhs, nrhs - 1);
                xb[u] = X[(tk.g0 + i) * nrhs + q];
            }
        };
        if (tk.ntasks == 1 || (PERSIST && tk.first)) load_xb();
        const bool finisher = PERSIST && tk.first && tk.ntasks > 1;
        if (finisher) {
            // every other task of the block was dequeued before this one
            if (tid == 0) wait_value(&sy.cnt[tk.blk], tk.ntasks - 1, sy.err, sy.spin);
            __syncthreads();
            acquire_after_wait();
            for (int e = tid; e < nb * nrhs; e += 256) {
                const int i = e / nrhs, q = e % nrhs;
                ao[i][q] = __hip_atomic_exchange(&Acc[(tk.g0 + i) * nrhs + q], T(0), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // rows of the next block of the supernode: their x come through XB
        const bool handed = PERSIST && (tk.hand & kHandOut) && tid < (tk.hand >> 8);
        if (PERSIST) {
            if (my_tgt >= 0 && !((tk.hand & kHandOut) && my_tgt == tk.blk + 1))
                wait_value(&sy.done[my_tgt], 1, sy.err, sy.spin);
            __syncthreads();
            acquire_after_wait();
        }
        T xv[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int64_t e = gr * nrhs + min(q, nrhs - 1);
            xv[q] = handed ? (q < nrhs ? wait_handed(&XB[e], sy.err, sy.spin) : T(0))
                           : (PERSIST ? shared_load(&X[e]) : X[e]);
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) xr[tid][q] = (rown < tk.r1 && q < nrhs) ? xv[q] : T(0);
        __syncthreads();
        T acc[NR];
        if constexpr (NR == 1) {
            T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
#pragma unroll
            for (int u = 0; u < RG; u += 4) {
                a0 += pv[u] * xr[g * RG + u][0];
                a1 += pv[u + 1] * xr[g * RG + u + 1][0];
                a2 += pv[u + 2] * xr[g * RG + u + 2][0];
                a3 += pv[u + 3] * xr[g * RG + u + 3][0];
            }
            acc[0] = (a0 + a1) + (a2 + a3);
        } else {
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[q] = T(0);
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                const T l = pv[u];
#pragma unroll
                for (int q = 0; q < NR; ++q) acc[q] += l * xr[g * RG + u][q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NR; ++q) Sm[g][k][q] = acc[q];
        __syncthreads();
        for (int e = tid; e < NB * NR; e += 256) {
            const int i = e % NB, q = e / NB;
            tq[i][q] = Sm[0][i][q] + Sm[1][i][q] + Sm[2][i][q] + Sm[3][i][q];
        }
        __syncthreads();
        bool fin = true;
        if (tk.ntasks == 1) {
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int e = tid + 256 * u, i = e / nrhs, q = e % nrhs;
                if (e < nb * nrhs) tq[i][q] = xb[u] - tq[i][q];
            }
        } else if (finisher) {
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int e = tid + 256 * u, i = e / nrhs, q = e % nrhs;
                if (e < nb * nrhs) tq[i][q] = xb[u] - (tq[i][q] + ao[i][q]);
            }
            if (tid == 0) sy.cnt[tk.blk] = 0;
        } else if (PERSIST) {
            for (int e = tid; e < nb * nrhs; e += 256) {
                const int i = e / nrhs, q = e % nrhs;
                atomicAdd(&Acc[(tk.g0 + i) * nrhs + q], tq[i][q]);
            }
            release_own();
            __syncthreads();
            if (tid == 0) atomicAdd(&sy.cnt[tk.blk], 1);
            fin = false;
        } else {
            if (tk.r1 > tk.r0)
                for (int e = tid; e < nb * nrhs; e += 256) {
                    const int i = e / nrhs, q = e % nrhs;
                    atomicAdd(&Acc[(tk.g0 + i) * nrhs + q], tq[i][q]);
                }
            // the partial sums are device-scope atomics and the last task
            // reads them back with atomic exchanges: each thread only waits
            // for its own atomics to be performed before the count goes up
            release_own();
            __syncthreads();
            if (tid == 0) last = (atomicAdd(&sy.cnt[tk.blk], 1) == tk.ntasks - 1);
            __syncthreads();
            fin = last;
            if (fin) {
                load_xb();
#pragma unroll
                for (int u = 0; u < XPT; ++u) {
                    const int e = tid + 256 * u, i = e / nrhs, q = e % nrhs;
                    if (e < nb * nrhs) {
                        const T a = __hip_atomic_exchange(&Acc[(tk.g0 + i) * nrhs + q], T(0), __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                        tq[i][q] = xb[u] - a;
                    }
                }
                if (tid == 0) sy.cnt[tk.blk] = 0;
            }
        }
        if (fin) {
            // x_q = Linv^T t (rows of t beyond nb meet zero entries of qv)
            __syncthreads();
            if constexpr (NR == 1) {
                T a0 = T(0), a1 = T(0);
#pragma unroll
                for (int s2 = 0; s2 < QW; s2 += 2) {
                    a0 += qv[s2] * tq[inv_row(s2)][0];
                    a1 += qv[s2 + 1] * tq[inv_row(s2 + 1)][0];
                }
                T a = a0 + a1;
                a += __shfl_xor(a, 1);
                a += __shfl_xor(a, 2);
                if ((tid & 3) == 0 && oc < nb) {
                    if (PERSIST) {
                        shared_store(&X[tk.g0 + oc], a);
                        if (tk.hand & kHandIn) shared_store(&XB[tk.g0 + oc], a);
                    } else {
                        X[tk.g0 + oc] = a;
                    }
                }
            } else if constexpr (NR < kMaxRhs) {
                // a few right-hand sides: the inverse staged in LDS, each
                // thread one or two outputs (c, q) as a dot product over the
                // rows i >= c of the inverse's column c
#pragma unroll
                for (int u = 0; u < QW; ++u) {
                    const int e = tid + 256 * u;
                    if (e < nb * nb) Vt[e % nb][e / nb] = qv[u];
                }
                __syncthreads();
#pragma unroll
                for (int u = 0; u < (NB * NR + 255) / 256; ++u) {
                    const int e = tid + 256 * u, c = e / NR, q = e % NR;
                    if (c < nb && q < nrhs) {
                        T a0 = T(0), a1 = T(0);
                        int i = c;
                        for (; i + 1 < nb; i += 2) {
                            a0 += Vt[i][c] * tq[i][q];
                            a1 += Vt[i + 1][c] * tq[i + 1][q];
                        }
                        if (i < nb) a0 += Vt[i][c] * tq[i][q];
                        const T a = a0 + a1;
                        if (PERSIST) {
                            shared_store(&X[(tk.g0 + c) * nrhs + q], a);
                            if (tk.hand & kHandIn) shared_store(&XB[(tk.g0 + c) * nrhs + q], a);
                        } else {
                            X[(tk.g0 + c) * nrhs + q] = a;
                        }
                    }
                }
            } else {
                using acc_t = typename Mfma<T>::acc;
#pragma unroll
                for (int u = 0; u < QW; ++u) {
                    const int e = tid + 256 * u;
                    if (e < nb * nb) Vt[e % nb][e / nb] = qv[u];
                }
                __syncthreads();
                const int c0 = 16 * g + (k & 15);
                acc_t xa = {0, 0, 0, 0};
#pragma unroll
                for (int s2 = 0; s2 < QW; ++s2) {
                    const int i = 4 * s2 + (k >> 4);
                    const T a = (i >= c0 && i < nb && c0 < nb) ? Vt[min(i, nb - 1)][min(c0, nb - 1)] : T(0);
                    xa = Mfma<T>::run(a, tq[i][k & 15], xa);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = 16 * g + Mfma<T>::row(k, v), q = k & 15;
                    if (c < nb && q < nrhs) {
                        if (PERSIST) {
                            shared_store(&X[(tk.g0 + c) * nrhs + q], xa[v]);
                            if (tk.hand & kHandIn) shared_store(&XB[(tk.g0 + c) * nrhs + q], xa[v]);
                        } else {
                            X[(tk.g0 + c) * nrhs + q] = xa[v];
                        }
                    }
                }
            }
            if (PERSIST) {
                release_own();
                __syncthreads();
                if (tid == 0) atomicExch(&sy.done[tk.blk], 1);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// One-wave solves of tiny supernodes (w <= kTinyW, m <= kTinyM), four per
// workgroup, for the wide bottom levels where nearly every supernode is
// tiny: a supernode costs one wave instead of a workgroup sized for a
// 64-column block.  Right-hand sides are interleaved by row (entry (k, q) at
// k * nrhs + q), so the values of one row sit together.
// Forward: x = Linv y for the w diagonal rows, stored in X; then each row
// i >= w below takes
//   Y[rows[i]] -= sum_c L[i][c] x_c      (atomic, as in the block sweep).
// One right-hand side: lane i holds row position i, y_c and x_c are
// broadcast from lane c.  Several: x goes through LDS and the update is the
// product (rows x w)(w x 16) on 16x16x4 MFMA (four row tiles, two steps of
// the contraction), so the 16 lanes of one output row write its 16
// consecutive values.
// ---------------------------------------------------------------------------
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_solve_tiny_fwd(const SmallTask *tasks, int64_t ntasks, const int32_t *rows,
                                                        const T *Lx, const T *Linv, T *Y, T *X, int64_t n,
                                                        int nrhs) {
    constexpr int WT = kTinyW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t ti = (int64_t)blockIdx.x * 4 + wv;
    if constexpr (NR == 1) {
        if (ti >= ntasks) return;  // the whole wave
        const SmallTask tk = tasks[ti];
        const int m = tk.m, w = tk.w;
        const T *P = Lx + tk.loff;
        const T *Q = Linv + tk.ioff;
        const int rc = min(lane, m - 1), dc = min(lane, w - 1);
        T l[WT], vi[WT];
#pragma unroll
        for (int c = 0; c < WT; ++c) l[c] = P[(int64_t)min(c, w - 1) * m + rc];
#pragma unroll
        for (int c = 0; c < WT; ++c) vi[c] = Q[dc + min(c, w - 1) * w];  // (L^{-1})[dc][c]
        const int64_t g = rows[tk.roff + rc];
        const T y = Y[tk.g0 + dc];
        T x = T(0), acc = T(0);
#pragma unroll
        for (int c = 0; c < WT; ++c)
            if (c < w) x += (c <= lane ? vi[c] : T(0)) * lane_read(y, c);
#pragma unroll
        for (int c = 0; c < WT; ++c)
            if (c < w) acc += l[c] * lane_read(x, c);
        if (lane < w) X[tk.g0 + lane] = x;
        else if (lane < m) atomicAdd(&Y[g], -acc);
    } else {
        using acc_t = typename Mfma<T>::acc;
        __shared__ T ys[4][WT][kMaxRhs + 1];
        __shared__ T xs[4][WT][kMaxRhs + 1];
        const bool active = ti < ntasks;
        const SmallTask tk = tasks[active ? ti : ntasks - 1];  // idle waves mirror a task, store nothing
        const int m = tk.m, w = tk.w;
        const T *P = Lx + tk.loff;
        const T *Q = Linv + tk.ioff;
        const int kq = lane & 15, kr = lane >> 4;
        const int64_t g = rows[tk.roff + min(lane, m - 1)];  // lane = row position
        // A operands: row 16 tt + kq of the panel, columns 4 s + kr
        T a[4][2];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
                a[tt][s2] = P[(int64_t)min(4 * s2 + kr, w - 1) * m + min(16 * tt + kq, m - 1)];
        // y of the diagonal rows, two (c, q) slots per lane: c = kr + 4 h
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = kr + 4 * h;
            const T yv = Y[(tk.g0 + min(c, w - 1)) * nrhs + min(kq, nrhs - 1)];
            ys[wv][c][kq] = (c < w && kq < nrhs) ? yv : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = kr + 4 * h;
            T xv = T(0);
#pragma unroll
            for (int j = 0; j < WT; ++j) {
                const T vq = Q[min(c, w - 1) + (int64_t)min(j, w - 1) * w];  // (L^{-1})[c][j]
                xv += (j <= c && c < w) ? vq * ys[wv][j][kq] : T(0);
            }
            xs[wv][c][kq] = xv;
            if (active && c < w && kq < nrhs) X[(tk.g0 + c) * nrhs + kq] = xv;
        }
        __syncthreads();
        // B operands: x[4 s + kr][kq] (zero beyond w)
        const T b0 = xs[wv][kr][kq], b1 = xs[wv][4 + kr][kq];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            if (16 * tt >= m) break;  // uniform
            acc_t acc = {0, 0, 0, 0};
            acc = Mfma<T>::run(4 * 0 + kr < w ? a[tt][0] : T(0), b0, acc);
            acc = Mfma<T>::run(4 + kr < w ? a[tt][1] : T(0), b1, acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * tt + Mfma<T>::row(lane, v);
                const int64_t gr = __shfl(g, min(r, 63));
                if (active && r >= w && r < m && kq < nrhs) atomicAdd(&Y[gr * nrhs + kq], -acc[v]);
            }
        }
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Backward: t_c = X[g0 + c] - sum_{i >= w} L[i][c] X[rows[i]] for the w
// columns c (the rows below are ancestors, final already), then
// x = Linv^T t.  One right-hand side: the sums are wave reductions.
// Several: the sums form the product (L_below^T)(X_rows), w x 16 with up to
// 64 rows of contraction, on 16x16x4 MFMA (A: lane l brings L[k][l%16],
// B: X[rows[k]][l%16], k = 4 s + l/16); t goes through LDS for the final
// small product with the inverse.
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_solve_tiny_bwd(const SmallTask *tasks, int64_t ntasks, const int32_t *rows,
                                                        const T *Lx, const T *Linv, T *X, int64_t n, int nrhs) {
    constexpr int WT = kTinyW;
    __shared__ T ts[4][WT][kMaxRhs + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t tr = (int64_t)blockIdx.x * 4 + wv;
    const bool active = tr < ntasks;
    const SmallTask tk = tasks[active ? tr : ntasks - 1];  // idle waves mirror a task, store nothing
    const int m = tk.m, w = tk.w;
    const T *P = Lx + tk.loff;
    const T *Q = Linv + tk.ioff;
    const int rc = min(lane, m - 1), dc = min(lane, w - 1);
    const int64_t g = rows[tk.roff + rc];
    if constexpr (NR == 1) {
        T l[WT], vt[WT];
#pragma unroll
        for (int c = 0; c < WT; ++c) l[c] = P[(int64_t)min(c, w - 1) * m + rc];
#pragma unroll
        for (int i = 0; i < WT; ++i) vt[i] = Q[min(i, w - 1) + dc * w];  // (L^{-1})[i][dc]
        const T xr = (lane >= w && lane < m) ? X[g] : T(0);
        T t = X[tk.g0 + dc];
#pragma unroll
        for (int c = 0; c < WT; ++c)
            if (c < w) {
                const T sc = wave_sum(l[c] * xr);
                if (lane == c) t -= sc;
            }
        T xv = T(0);
#pragma unroll
        for (int i = 0; i < WT; ++i)
            if (i < w) xv += (i >= lane ? vt[i] : T(0)) * lane_read(t, i);
        if (active && lane < w) X[tk.g0 + lane] = xv;
    } else {
        using acc_t = typename Mfma<T>::acc;
        const int kq = lane & 15, kr = lane >> 4;
        T a[16], b[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int k = 4 * s + kr, kc = min(k, m - 1);
            const int64_t gk = __shfl(g, kc);
            const bool row_ok = k >= w && k < m;
            const T av = P[(int64_t)min(kq, w - 1) * m + kc];
            const T bv = X[gk * nrhs + min(kq, nrhs - 1)];
            a[s] = (row_ok && kq < w) ? av : T(0);
            b[s] = (row_ok && kq < nrhs) ? bv : T(0);
        }
        acc_t acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 16; ++s) acc = Mfma<T>::run(a[s], b[s], acc);
        // element v of this lane: row c of (L_below^T X_rows), column kq
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = Mfma<T>::row(lane, v);
            const T xo = X[(tk.g0 + min(c, w - 1)) * nrhs + min(kq, nrhs - 1)];
            if (c < WT) ts[wv][c][kq] = (c < w && kq < nrhs) ? xo - acc[v] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = kr + 4 * h;
            T xv = T(0);
#pragma unroll
            for (int i = 0; i < WT; ++i) {
                const T vq = Q[min(i, w - 1) + (int64_t)min(c, w - 1) * w];  // (L^{-1})[i][c]
                xv += (i >= c && i < w) ? vq * ts[wv][i][kq] : T(0);
            }
            if (active && c < w && kq < nrhs) X[(tk.g0 + c) * nrhs + kq] = xv;
        }
    }
}

// Per solve: dep <- the forward counts, done and cnt <- 0, queues <- 0.  The
// error word is the factor's, cleared only by a factorization, so a wait
// that gave up stays reported.
__global__ void k_solve_reset(const int32_t *fdep, int64_t nblocks, SolveSync sy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nblocks) {
        sy.dep[i] = fdep[i];
        sy.done[i] = 0;
        sy.cnt[i] = 0;
    }
    if (i < 2) sy.queue[i] = 0;
}

// The hand-over buffers of a solve: every entry unset.
template <typename T>
__global__ void k_fill_unset(T *p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = __builtin_bit_cast(T, Unset<T>::bits);
}

// |v| for the maxima of refinement, with NaN mapped to +Inf: fmax drops a
// NaN operand, and a NaN in a residual or solution must not vanish from
// its norm (the bit patterns of non-negative doubles order as unsigned
// integers, so the maxima run as integer atomicMax on them).
__device__ __forceinline__ double abs_key(double v) { return v != v ? __longlong_as_double(0x7ff0000000000000ll) : fabs(v); }

// ---------------------------------------------------------------------------
// FP64 kernels of iterative refinement.  A is applied in full through a CSR
// of the symmetric pattern whose entries point into the caller's lower-CSC
// values (valmap), so refinement always uses the values given.  Vectors are
// n x nrhs column-major with leading dimension ld.
// ---------------------------------------------------------------------------
// Y = B - A X (beta = -1, with B) or Y = A X (B == nullptr).  LPR
// consecutive lanes share a row (LPR a power of two <= 64, so a group never
// straddles a wave): lane j of the group takes entries j, j + LPR, ... of
// the row, so a group's index and value loads are contiguous, and the
// group's partial sums meet by shuffles.
template <int LPR>
__global__ __launch_bounds__(256) void k_spmv(const int64_t *rowptr, const int32_t *colidx, const int64_t *valmap,
                                              const double *values, const double *X, const double *B, double *Y,
                                              int64_t n, int nrhs, int64_t ld) {
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LPR;
    const int j = threadIdx.x % LPR;
    double acc[kMaxRhs];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) acc[q] = 0.0;
    if (i < n)
        for (int64_t e = rowptr[i] + j; e < rowptr[i + 1]; e += LPR) {
            const double a = values[valmap[e]];
            const int64_t c = colidx[e];
#pragma unroll
            for (int q = 0; q < kMaxRhs; ++q)
                if (q < nrhs) acc[q] += a * X[c + q * ld];
        }
    // every lane takes part in the shuffles (nrhs is the same for all)
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q)
        if (q < nrhs)
#pragma unroll
            for (int off = LPR / 2; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off);
    if (i < n && j == 0)
        for (int q = 0; q < nrhs; ++q) Y[i + q * ld] = B ? B[i + q * ld] - acc[q] : acc[q];
}

// out = max_i sum_j |a_ij| (as the bit pattern of a non-negative double):
// LPR lanes per row as in k_spmv (so a group's loads are contiguous), rows
// taken grid-stride by a capped grid, one atomic per workgroup
template <int LPR>
__global__ __launch_bounds__(256) void k_norm_inf_A(const int64_t *rowptr, const int64_t *valmap,
                                                    const double *values, int64_t n, unsigned long long *out) {
    __shared__ double wmax[4];
    const int j = threadIdx.x % LPR;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / LPR);
    double mx = 0.0;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LPR;; i += stride) {
        // every lane takes part in the shuffles: the loop ends for a whole
        // wave at once (i advances by the same stride in all its groups)
        if (__builtin_amdgcn_ballot_w64(i < n) == 0) break;
        double sum = 0.0;
        if (i < n)
            for (int64_t e = rowptr[i] + j; e < rowptr[i + 1]; e += LPR) sum += fabs(values[valmap[e]]);
#pragma unroll
        for (int off = LPR / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
        mx = fmax(mx, abs_key(sum));  // NaN as +Inf
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(out, (unsigned long long)__double_as_longlong(fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]))));
}

// out[q] = max_i |V[i, q]| (bit patterns), grid.y = q, 256 threads: one
// atomic per workgroup (same-address atomics serialize at L2)
__global__ __launch_bounds__(256) void k_colmax(const double *V, int64_t n, int64_t ld, unsigned long long *out) {
    __shared__ double wmax[4];
    const int q = blockIdx.y;
    double mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        mx = fmax(mx, abs_key(V[i + q * ld]));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(&out[q], (unsigned long long)__double_as_longlong(fmax(fmax(wmax[0], wmax[1]),
                                                                           fmax(wmax[2], wmax[3]))));
}

// out[q] += sum_i U[i, q] V[i, q], grid.y = q, 256 threads: one atomic per
// workgroup, as in k_colmax
__global__ __launch_bounds__(256) void k_coldot(const double *U, const double *V, int64_t n, int64_t ld,
                                                double *out) {
    __shared__ double wsum[4];
    const int q = blockIdx.y;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += U[i + q * ld] * V[i + q * ld];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&out[q], (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]));
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

// Conjugate-gradient coefficients per (column, system) slot j < K, formed
// on the device so that a step needs no host round trip.  alpha: coef[j] =
// rho[j] / dots[j] and coef[K + j] = -coef[j]; beta: coef[2K + j] =
// dots[j] / rho[j], then rho[j] = dots[j].  A frozen slot (its column has
// met the tolerance) and a quotient that is not finite give 0, and a frozen
// slot keeps its rho.
__global__ void k_cg_coef(const double *dots, double *rho, const double *frozen, double *coef, int64_t K, int alpha) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    const bool fz = frozen[j] != 0.0;
    if (alpha) {
        const double a = (!fz && dots[j] > 0.0 && isfinite(rho[j] / dots[j])) ? rho[j] / dots[j] : 0.0;
        coef[j] = a;
        coef[K + j] = -a;
    } else {
        const double bt = (rho[j] != 0.0 && isfinite(dots[j] / rho[j])) ? dots[j] / rho[j] : 0.0;
        coef[2 * K + j] = fz ? 0.0 : bt;
        if (!fz) rho[j] = dots[j];
    }
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

// Segmented forms for batches: row i belongs to system seg[i] (the rows of
// a system are contiguous and the ids ascend), and every reduction or
// coefficient is kept per (column q, system) at index q * nseg + seg[i].
// One row per thread: a wave whose rows all lie in one system reduces in
// registers and makes one atomic; a wave across a boundary makes one per
// row.  Lanes past n contribute the identity (0 for max of magnitudes and
// for sums).
__device__ inline bool wave_in_one_segment(int s) { return __shfl(s, 0) == __shfl(s, 63); }

__global__ void k_seg_norm_inf_A(const int64_t *rowptr, const int64_t *valmap, const double *values,
                                 const int32_t *seg, int64_t n, unsigned long long *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = seg[i < n ? i : n - 1];
    double sum = 0.0;
    if (i < n)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) sum += fabs(values[valmap[e]]);
    sum = abs_key(sum);
    if (wave_in_one_segment(s)) {
        for (int off = 32; off > 0; off >>= 1) sum = fmax(sum, __shfl_xor(sum, off));
        if ((threadIdx.x & 63) == 0) atomicMax(&out[s], (unsigned long long)__double_as_longlong(sum));
    } else if (i < n) {
        atomicMax(&out[s], (unsigned long long)__double_as_longlong(sum));
    }
}

// The segmented column reductions give each workgroup of 256 threads
// kSegRows consecutive rows.  A system's rows are contiguous, so when the
// first and last row of the chunk belong to one system the whole chunk does:
// one atomic per workgroup.  A chunk that spans systems falls back to one
// atomic per wave (or per row where a wave spans systems).
constexpr int kSegRows = 256 * 8;

__global__ __launch_bounds__(256) void k_seg_colmax(const double *V, const int32_t *seg, int64_t n, int64_t ld,
                                                    int nseg, unsigned long long *out) {
    __shared__ double wm[4];
    const int q = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * kSegRows;
    const int64_t last = (base + kSegRows < n ? base + kSegRows : n) - 1;
    if (seg[base] == seg[last]) {  // the same for every thread of the workgroup
        double mx = 0.0;
        for (int r = 0; r < kSegRows / 256; ++r) {
            const int64_t i = base + r * 256 + threadIdx.x;
            if (i < n) mx = fmax(mx, abs_key(V[i + q * ld]));
        }
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
        if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0)
            atomicMax(out + (int64_t)q * nseg + seg[base],
                      (unsigned long long)__double_as_longlong(fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]))));
        return;
    }
    for (int r = 0; r < kSegRows / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        const int64_t ic = i < n ? i : n - 1;
        const int s = seg[ic];
        double mx = i < n ? abs_key(V[ic + q * ld]) : 0.0;
        unsigned long long *o = out + (int64_t)q * nseg + s;
        if (wave_in_one_segment(s)) {
            for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
            if ((threadIdx.x & 63) == 0) atomicMax(o, (unsigned long long)__double_as_longlong(mx));
        } else if (i < n) {
            atomicMax(o, (unsigned long long)__double_as_longlong(mx));
        }
    }
}

__global__ __launch_bounds__(256) void k_seg_coldot(const double *U, const double *V, const int32_t *seg, int64_t n,
                                                    int64_t ld, int nseg, double *out) {
    __shared__ double ws[4];
    const int q = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * kSegRows;
    const int64_t last = (base + kSegRows < n ? base + kSegRows : n) - 1;
    if (seg[base] == seg[last]) {  // the same for every thread of the workgroup
        double acc = 0.0;
        for (int r = 0; r < kSegRows / 256; ++r) {
            const int64_t i = base + r * 256 + threadIdx.x;
            if (i < n) acc += U[i + q * ld] * V[i + q * ld];
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(out + (int64_t)q * nseg + seg[base], (ws[0] + ws[1]) + (ws[2] + ws[3]));
        return;
    }
    for (int r = 0; r < kSegRows / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        const int64_t ic = i < n ? i : n - 1;
        const int s = seg[ic];
        double acc = i < n ? U[ic + q * ld] * V[ic + q * ld] : 0.0;
        double *o = out + (int64_t)q * nseg + s;
        if (wave_in_one_segment(s)) {
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
            if ((threadIdx.x & 63) == 0) atomicAdd(o, acc);
        } else if (i < n) {
            atomicAdd(o, acc);
        }
    }
}

// Y[:, q] = a X[:, q] + b Y[:, q] with a = a[q * nseg + seg[i]] (or a0 when
// a is null), likewise b; b = 0 does not read Y.
__global__ void k_seg_axpby(const double *a, double a0, const double *X, const double *b, double b0, double *Y,
                            const int32_t *seg, int64_t n, int64_t ld, int nseg) {
    const int q = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t k = (int64_t)q * nseg + seg[i];
    const double aq = a ? a[k] : a0, bq = b ? b[k] : b0;
    Y[i + q * ld] = (bq == 0.0) ? aq * X[i + q * ld] : aq * X[i + q * ld] + bq * Y[i + q * ld];
}

inline unsigned grid1(int64_t count, int block) {
    int64_t g = (count + block - 1) / block;
    return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

void launch_status_reset(unsigned long long *status, int count, int32_t *deverr, int32_t *flags, int nflags,
                         hipStream_t st) {
    const int n = count > nflags ? count : nflags;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_status_reset, dim3((n + 255) / 256), dim3(256), 0, st, status, count, deverr, flags, nflags);
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
void launch_pivot_floor(const DevPlan &P, int64_t n, const double *values, double theta, T *floor, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pivot_floor<T>, dim3(grid1(n, 256)), dim3(256), 0, st, P.dsrc, n, values, theta, floor);
}

template <typename T>
void launch_potrf(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, T *Linv, unsigned long long *status,
                  int32_t *deverr, PivotFloor<T> pfl, hipStream_t st) {
    if (t1 <= t0) return;
    if (pfl.v)
        hipLaunchKernelGGL((k_potrf<T, true>), dim3((unsigned)(t1 - t0)), dim3(256), 0, st, P.potrf_tasks + t0, Lx,
                           Linv, status, P.status_slot, deverr, pfl);
    else
        hipLaunchKernelGGL((k_potrf<T, false>), dim3((unsigned)(t1 - t0)), dim3(256), 0, st, P.potrf_tasks + t0, Lx,
                           Linv, status, P.status_slot, deverr, pfl);
}

template <typename T>
void launch_tiny(const DevPlan &P, int64_t t0, int64_t t16, int64_t t32, int64_t t1, T *Lx, T *Linv,
                 unsigned long long *status, PivotFloor<T> pfl, hipStream_t st) {
    if (t1 <= t0) return;
    const int64_t n16 = t16 - t0, n32 = t32 - t0, nt = t1 - t0;
    const int64_t blocks = (n16 + 15) / 16 + (n32 - n16 + 7) / 8 + (nt - n32 + 3) / 4;
    hipLaunchKernelGGL(k_tiny<T>, dim3((unsigned)blocks), dim3(256), 0, st, P.tiny_tasks + t0, n16, n32, nt,
                       P.cbase, P.crel, P.rel, Lx, Linv, status, P.status_slot, pfl);
}

template <typename T>
void launch_small(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, T *Linv, unsigned long long *status,
                  PivotFloor<T> pfl, hipStream_t st) {
    if (t1 <= t0) return;
    hipLaunchKernelGGL(k_small<T>, dim3((unsigned)(t1 - t0)), dim3(256), 0, st, P.small_tasks + t0, P.cbase,
                       P.crel, P.rel, Lx, Linv, status, P.status_slot, pfl);
}

template <typename T>
void launch_tiles(const DevPlan &P, int mode, int64_t t0, int64_t t1, T *Lx, T *Linv, unsigned long long *status,
                  int32_t *hflags, WaitCtl wc, bool bf16, PivotFloor<T> pfl, hipStream_t st) {
    if (t1 <= t0) return;
    const dim3 g((unsigned)(t1 - t0)), b(256);
    if constexpr (std::is_same<T, float>::value) {
        if (bf16 && mode == kTilesTrailing) {
            hipLaunchKernelGGL((k_tiles<T, MODE_TRAILING, true>), g, b, 0, st, P.int_tiles + t0, P.cbase, P.crel,
                               P.rel, Linv, Lx, status, P.status_slot, hflags, wc, pfl);
            return;
        }
        if (bf16 && mode == kTilesScatter) {
            hipLaunchKernelGGL((k_tiles<T, MODE_SCATTER, true>), g, b, 0, st, P.ext_tiles + t0, P.cbase, P.crel,
                               P.rel, Linv, Lx, status, P.status_slot, (int32_t *)nullptr, wc, pfl);
            return;
        }
    }
    if (mode == kTilesTrailing)
        hipLaunchKernelGGL((k_tiles<T, MODE_TRAILING>), g, b, 0, st, P.int_tiles + t0, P.cbase, P.crel, P.rel,
                           Linv, Lx, status, P.status_slot, hflags, wc, PivotFloor<T>{});
    else if (mode == kTilesScatter)
        hipLaunchKernelGGL((k_tiles<T, MODE_SCATTER>), g, b, 0, st, P.ext_tiles + t0, P.cbase, P.crel, P.rel,
                           Linv, Lx, status, P.status_slot, (int32_t *)nullptr, wc, PivotFloor<T>{});
    else
        hipLaunchKernelGGL((k_tiles<T, MODE_TRSM>), g, b, 0, st, P.trsm_tiles + t0, P.cbase, P.crel, P.rel,
                           Linv, Lx, status, P.status_slot, (int32_t *)nullptr, wc, PivotFloor<T>{});
}

template <typename T>
void launch_tiles128(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, bool bf16, hipStream_t st) {
    if (t1 <= t0) return;
    if constexpr (std::is_same<T, float>::value) {
        if (bf16) {
            hipLaunchKernelGGL((k_tiles128<T, true>), dim3((unsigned)(t1 - t0)), dim3(512), 0, st,
                               P.ext_tiles_big + t0, P.cbase, P.crel, P.rel, Lx);
            return;
        }
    }
    hipLaunchKernelGGL((k_tiles128<T, false>), dim3((unsigned)(t1 - t0)), dim3(512), 0, st,
                       P.ext_tiles_big + t0, P.cbase, P.crel, P.rel, Lx);
}

template <typename T>
void launch_trail128(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, bool bf16, hipStream_t st) {
    if (t1 <= t0) return;
    if constexpr (std::is_same<T, float>::value) {
        if (bf16) {
            hipLaunchKernelGGL((k_tiles128<T, true, true>), dim3((unsigned)(t1 - t0)), dim3(512), 0, st,
                               P.trail_big + t0, P.cbase, P.crel, P.rel, Lx);
            return;
        }
    }
    hipLaunchKernelGGL((k_tiles128<T, false, true>), dim3((unsigned)(t1 - t0)), dim3(512), 0, st,
                       P.trail_big + t0, P.cbase, P.crel, P.rel, Lx);
}

template <typename T>
void launch_persist_small(const DevPlan &P, int64_t nchunks, int64_t nsuper, int32_t *pdep, int32_t *qctr, T *Lx,
                          T *Linv, unsigned long long *status, PivotFloor<T> pfl, WaitCtl wc, hipStream_t st) {
    if (nchunks <= 0) return;
    hipLaunchKernelGGL(k_persist_reset, dim3(grid1(std::max<int64_t>(nsuper, 1), 256)), dim3(256), 0, st, P.pdep0,
                       nsuper, pdep, qctr);
    // as many workgroups as can be resident at once (the kernel's occupancy
    // times the CUs), measured once per precision: the entries are short and
    // latency-bound, so every resident slot counts
    static int resident[2] = {0, 0};
    int &r = resident[sizeof(T) == 8 ? 1 : 0];
    if (r == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist_small<T>, 256, 0) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1 ||
            cus < 1)
            r = 768;
        else
            r = per_cu * cus;
    }
    const unsigned g = (unsigned)std::min<int64_t>(nchunks, r);
    hipLaunchKernelGGL(k_persist_small<T>, dim3(g), dim3(256), 0, st, P.pqueue, P.pchunk, nchunks, P.psmall, P.ptiny,
                       P.ptgt_ptr,
                       P.ptgt, pdep, qctr, P.cbase, P.crel, P.rel, Lx, Linv, status, P.status_slot, pfl, wc);
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

inline unsigned persist_grid(int64_t ntasks) {
    // two resident workgroups per CU on 256 CUs; more only queue behind them
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ntasks, 512));
}

void launch_solve_reset(const DevPlan &P, int64_t nblocks, SolveSync sy, hipStream_t st) {
    hipLaunchKernelGGL(k_solve_reset, dim3(grid1(std::max<int64_t>(nblocks, 2), 256)), dim3(256), 0, st, P.fdep,
                       nblocks, sy);
}

template <typename T>
void launch_fill_unset(T *p, int64_t count, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill_unset<T>, dim3(grid1(count, 256)), dim3(256), 0, st, p, count);
}

template <typename T>
void launch_solve_fwd(const DevPlan &P, int64_t t0, int64_t t1, const T *Lx, const T *Linv, T *Y, T *X, T *H,
                      int64_t n, int nrhs, SolveSync sy, bool persist, hipStream_t st) {
    if (t1 <= t0) return;
    const int64_t nt = t1 - t0;
    const dim3 g(persist ? persist_grid(nt) : (unsigned)nt), b(256);
    const SolveTask *tk = P.stasks + t0;
    const int64_t *tp = P.stgt_ptr + t0;
    if (nrhs == 1) {
        if (persist)
            hipLaunchKernelGGL((k_solve_fwd<T, true>), g, b, 0, st, tk, nt, P.rows, Lx, Linv, Y, X, H, n, tp, P.stgt,
                               sy);
        else
            hipLaunchKernelGGL((k_solve_fwd<T, false>), g, b, 0, st, tk, nt, P.rows, Lx, Linv, Y, X, H, n, tp, P.stgt,
                               sy);
    } else {
        if (persist)
            hipLaunchKernelGGL((k_solve_fwd_multi<T, true>), g, b, 0, st, tk, nt, P.rows, Lx, Linv, Y, X, H, n, nrhs,
                               tp, P.stgt, sy);
        else
            hipLaunchKernelGGL((k_solve_fwd_multi<T, false>), g, b, 0, st, tk, nt, P.rows, Lx, Linv, Y, X, H, n, nrhs,
                               tp, P.stgt, sy);
    }
}

template <typename T>
void launch_solve_tiny_fwd(const DevPlan &P, int64_t t0, int64_t t1, const T *Lx, const T *Linv, T *Y, T *X,
                           int64_t n, int nrhs, hipStream_t st) {
    if (t1 <= t0) return;
    const dim3 g((unsigned)((t1 - t0 + 3) / 4)), b(256);
    if (nrhs == 1)
        hipLaunchKernelGGL((k_solve_tiny_fwd<T, 1>), g, b, 0, st, P.stiny + t0, t1 - t0, P.rows, Lx, Linv, Y, X, n,
                           nrhs);
    else
        hipLaunchKernelGGL((k_solve_tiny_fwd<T, kMaxRhs>), g, b, 0, st, P.stiny + t0, t1 - t0, P.rows, Lx, Linv, Y,
                           X, n, nrhs);
}

template <typename T>
void launch_solve_tiny_bwd(const DevPlan &P, int64_t t0, int64_t t1, const T *Lx, const T *Linv, T *X, int64_t n,
                           int nrhs, hipStream_t st) {
    if (t1 <= t0) return;
    const dim3 g((unsigned)((t1 - t0 + 3) / 4)), b(256);
    if (nrhs == 1)
        hipLaunchKernelGGL((k_solve_tiny_bwd<T, 1>), g, b, 0, st, P.stiny + t0, t1 - t0, P.rows, Lx, Linv, X, n,
                           nrhs);
    else
        hipLaunchKernelGGL((k_solve_tiny_bwd<T, kMaxRhs>), g, b, 0, st, P.stiny + t0, t1 - t0, P.rows, Lx, Linv, X,
                           n, nrhs);
}

template <typename T>
void launch_solve_bwd(const DevPlan &P, int64_t t0, int64_t t1, const T *Lx, const T *Linv, T *X, T *Acc, T *XB,
                      int64_t n, int nrhs, SolveSync sy, bool persist, hipStream_t st) {
    if (t1 <= t0) return;
    const int64_t nt = t1 - t0;
    const dim3 g(persist ? persist_grid(nt) : (unsigned)nt), b(256);
    // the persistent sweep takes its tasks (global indices) from bwd_order
    const SolveTask *tk = persist ? P.stasks : P.stasks + t0;
    const int64_t *tp = persist ? P.stgt_ptr : P.stgt_ptr + t0;
    const int32_t *ord = persist ? P.bwd_order : nullptr;
    // the instantiation for the fewest right-hand sides that holds nrhs
#define SPC_BWD(NRV)                                                                                          \
    do {                                                                                                      \
        if (persist)                                                                                          \
            hipLaunchKernelGGL((k_solve_bwd<T, NRV, true>), g, b, 0, st, tk, nt, ord, P.rows, Lx, Linv, X, Acc, \
                               XB, n, nrhs, tp, P.stgt, sy);                                                  \
        else                                                                                                  \
            hipLaunchKernelGGL((k_solve_bwd<T, NRV, false>), g, b, 0, st, tk, nt, ord, P.rows, Lx, Linv, X,    \
                               Acc, XB, n, nrhs, tp, P.stgt, sy);                                             \
    } while (0)
    if (nrhs == 1) {
        SPC_BWD(1);
    } else if (nrhs <= 4) {
        SPC_BWD(4);
    } else if (nrhs <= 8) {
        SPC_BWD(8);
    } else {
        SPC_BWD(kMaxRhs);
    }
#undef SPC_BWD
}

void launch_spmv(const int64_t *rowptr, const int32_t *colidx, const int64_t *valmap, const double *values,
                 const double *X, const double *B, double *Y, int64_t n, int64_t nnz, int nrhs, int64_t ld,
                 hipStream_t st) {
    if (n <= 0) return;
    // lanes per row: the power of two (4..32) at or above the mean row length
    const int64_t avg = (nnz + n - 1) / n;
    if (avg <= 4)
        hipLaunchKernelGGL(k_spmv<4>, dim3(grid1(n * 4, 256)), dim3(256), 0, st, rowptr, colidx, valmap, values, X,
                           B, Y, n, nrhs, ld);
    else if (avg <= 8)
        hipLaunchKernelGGL(k_spmv<8>, dim3(grid1(n * 8, 256)), dim3(256), 0, st, rowptr, colidx, valmap, values, X,
                           B, Y, n, nrhs, ld);
    else if (avg <= 16)
        hipLaunchKernelGGL(k_spmv<16>, dim3(grid1(n * 16, 256)), dim3(256), 0, st, rowptr, colidx, valmap, values,
                           X, B, Y, n, nrhs, ld);
    else
        hipLaunchKernelGGL(k_spmv<32>, dim3(grid1(n * 32, 256)), dim3(256), 0, st, rowptr, colidx, valmap, values,
                           X, B, Y, n, nrhs, ld);
}
void launch_norm_inf_A(const int64_t *rowptr, const int64_t *valmap, const double *values, int64_t n, int64_t nnz,
                       unsigned long long *out, hipStream_t st) {
    if (n <= 0) return;
    const int64_t avg = (nnz + n - 1) / n;
    const unsigned g4 = (unsigned)std::min<int64_t>(grid1(n * 4, 256), 1024);
    const unsigned g32 = (unsigned)std::min<int64_t>(grid1(n * 32, 256), 1024);
    if (avg <= 8)
        hipLaunchKernelGGL(k_norm_inf_A<4>, dim3(g4), dim3(256), 0, st, rowptr, valmap, values, n, out);
    else
        hipLaunchKernelGGL(k_norm_inf_A<32>, dim3(g32), dim3(256), 0, st, rowptr, valmap, values, n, out);
}
static unsigned red_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}
void launch_colmax(const double *V, int64_t n, int nrhs, int64_t ld, unsigned long long *out, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_colmax, dim3(std::min(red_grid(n), 128u), nrhs), dim3(256), 0, st, V, n, ld, out);
}
void launch_coldot(const double *U, const double *V, int64_t n, int nrhs, int64_t ld, double *out, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_coldot, dim3(std::min(red_grid(n), 128u), nrhs), dim3(256), 0, st, U, V, n, ld, out);
}
void launch_cg_coef(const double *dots, double *rho, const double *frozen, double *coef, int64_t K, bool alpha,
                    hipStream_t st) {
    if (K <= 0) return;
    hipLaunchKernelGGL(k_cg_coef, dim3(grid1(K, 256)), dim3(256), 0, st, dots, rho, frozen, coef, K, alpha ? 1 : 0);
}
void launch_axpby(const double *a, double a0, const double *X, const double *b, double b0, double *Y, int64_t n,
                  int nrhs, int64_t ld, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_axpby, dim3(red_grid(n), nrhs), dim3(256), 0, st, a, a0, X, b, b0, Y, n, ld);
}
void launch_seg_norm_inf_A(const int64_t *rowptr, const int64_t *valmap, const double *values, const int32_t *seg,
                           int64_t n, unsigned long long *out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_seg_norm_inf_A, dim3(grid1(n, 256)), dim3(256), 0, st, rowptr, valmap, values, seg, n,
                       out);
}
void launch_seg_colmax(const double *V, const int32_t *seg, int64_t n, int nrhs, int64_t ld, int nseg,
                       unsigned long long *out, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_seg_colmax, dim3(grid1(n, kSegRows), nrhs), dim3(256), 0, st, V, seg, n, ld, nseg, out);
}
void launch_seg_coldot(const double *U, const double *V, const int32_t *seg, int64_t n, int nrhs, int64_t ld,
                       int nseg, double *out, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_seg_coldot, dim3(grid1(n, kSegRows), nrhs), dim3(256), 0, st, U, V, seg, n, ld, nseg, out);
}
void launch_seg_axpby(const double *a, double a0, const double *X, const double *b, double b0, double *Y,
                      const int32_t *seg, int64_t n, int nrhs, int64_t ld, int nseg, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_seg_axpby, dim3(grid1(n, 256), nrhs), dim3(256), 0, st, a, a0, X, b, b0, Y, seg, n, ld,
                       nseg);
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
                                  int32_t *, PivotFloor<T>, hipStream_t);                                   \
    template void launch_pivot_floor<T>(const DevPlan &, int64_t, const double *, double, T *, hipStream_t); \
    template void launch_tiles<T>(const DevPlan &, int, int64_t, int64_t, T *, T *, unsigned long long *,    \
                                  int32_t *, WaitCtl, bool, PivotFloor<T>, hipStream_t);                    \
    template void launch_small<T>(const DevPlan &, int64_t, int64_t, T *, T *, unsigned long long *,         \
                                  PivotFloor<T>, hipStream_t);                                              \
    template void launch_tiny<T>(const DevPlan &, int64_t, int64_t, int64_t, int64_t, T *, T *,             \
                                 unsigned long long *, PivotFloor<T>, hipStream_t);                         \
    template void launch_tiles128<T>(const DevPlan &, int64_t, int64_t, T *, bool, hipStream_t);            \
    template void launch_trail128<T>(const DevPlan &, int64_t, int64_t, T *, bool, hipStream_t);            \
    template void launch_persist_small<T>(const DevPlan &, int64_t, int64_t, int32_t *, int32_t *, T *, T *, \
                                          unsigned long long *, PivotFloor<T>, WaitCtl, hipStream_t);       \
    template void launch_perm_in<T>(const DevPlan &, int64_t, int, const double *, int64_t, T *,            \
                                    hipStream_t);                                                           \
    template void launch_perm_out<T>(const DevPlan &, int64_t, int, const T *, double *, int64_t,           \
                                     hipStream_t);                                                          \
    template void launch_fill_unset<T>(T *, int64_t, hipStream_t);                                         \
    template void launch_solve_fwd<T>(const DevPlan &, int64_t, int64_t, const T *, const T *, T *, T *, T *, \
                                      int64_t, int, SolveSync, bool, hipStream_t);                          \
    template void launch_solve_bwd<T>(const DevPlan &, int64_t, int64_t, const T *, const T *, T *, T *, T *, \
                                      int64_t, int, SolveSync, bool, hipStream_t);                          \
    template void launch_solve_tiny_fwd<T>(const DevPlan &, int64_t, int64_t, const T *, const T *, T *, T *, \
                                           int64_t, int, hipStream_t);                                      \
    template void launch_solve_tiny_bwd<T>(const DevPlan &, int64_t, int64_t, const T *, const T *, T *,     \
                                           int64_t, int, hipStream_t);
SPC_INSTANTIATE(double)
SPC_INSTANTIATE(float)

// ---------------------------------------------------------------------------
// Scratch for callers that cannot allocate (spc_solve_noalloc): a fixed
// array in device memory, one copy per device, held until the process ends.
// Every call on a device shares it.
// ---------------------------------------------------------------------------
}  // namespace spc

static __device__ __align__(256) unsigned char scratch[spc::kScratchBytes];

namespace spc {

int scratch_address(int device, void **out) {
    static std::mutex mu;
    static void *addr[64] = {};
    if (device < 0 || device >= 64) return -5;  // SPC_DEVICE_ERROR
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return -5;
        if (cur != device && hipSetDevice(device) != hipSuccess) return -5;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return -5;
        addr[device] = p;
    }
    *out = addr[device];
    return 0;
}

}  // namespace spc
