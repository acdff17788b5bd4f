// capi.cpp -- the extern "C" entry points declared in include/spchol.h.
//
// A symbolic handle owns the host analysis and, after the first numeric
// call, one device allocation holding every array the kernels read.  A
// factor handle owns its panels, a status word and a solve work area.
#include <hip/hip_runtime.h>

#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/spchol.h"
#include "kernels.h"
#include "plan.h"

namespace {

constexpr uint32_t kSymMagic = 0x53594d31u, kFacMagic = 0x46414331u, kDead = 0xdeadbeefu;

struct DeviceArrays {
    void *base = nullptr;
    size_t bytes = 0;
    int device = -1;
    spc::DevPlan plan{};
};

}  // namespace

struct spc_symbolic_s {
    uint32_t magic = kSymMagic;
    std::atomic<int> refs{1};
    spc::Symbolic S;
    DeviceArrays dev;
    // full-A CSR for refinement, uploaded on first use
    void *csr_base = nullptr;
    const int64_t *d_csr_ptr = nullptr, *d_csr_val = nullptr;
    const int32_t *d_csr_col = nullptr;
    int64_t hbm_budget = 0;  // bytes per factorization; <= 0: none
    std::mutex mu;
};

struct spc_factor_s {
    uint32_t magic = kFacMagic;
    spc_symbolic_s *sym = nullptr;
    int precision = SPC_FP64;
    int device = -1;
    void *Lx = nullptr;
    void *Linv = nullptr;       // inverses of the diagonal blocks (factor precision)
    unsigned long long *status = nullptr;
    // device-error word: set by a bounded wait on another workgroup that gave
    // up (factor hand-over, persistent solve sweeps), cleared by every
    // factorization; after the status words in their allocation
    int32_t *deverr = nullptr;
    int32_t spin = spc::kSpinDefault;  // polls before such a wait gives up
    // BF16 updates: pivot floors (n entries, factor precision); the count of
    // pivots raised to their floor is the word after deverr
    void *pfloor = nullptr;
    // hand-over flags of the trailing launches, one per 16-column panel of
    // each column block (in the status allocation, after the error word)
    int32_t *hflags = nullptr;
    int nflags = 0;
    // persistent launch over the small subtrees: its work counter and one
    // dependency counter per supernode (after the flags)
    int32_t *qctr = nullptr;
    int32_t *pdep = nullptr;
    void *work = nullptr;       // solve vectors Y, X, Acc (factor precision) + block counters
    size_t work_bytes = 0;
    double *refine = nullptr;   // refinement vectors (FP64)
    size_t refine_bytes = 0;
    void *refine_host = nullptr;  // pinned: the maxima read back each step, the converged flags sent down
    size_t refine_host_bytes = 0;
    // a refined solve with this factorization switched to CG, so the next
    // ones start there (cleared by every factorization)
    std::atomic<bool> refine_cg{false};
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // status words (one per system of a batch) and, for a view into a
    // batch, the owning batch, the system index and its first column
    int nstatus = 1;
    bool owns_storage = true;
    struct spc_batch_s *batch = nullptr;
    int batch_index = -1;
    int64_t status_col_off = 0;
    // graph replay of the factorization: captured once on cap_stream (a
    // graph cannot be captured on the legacy default stream), then launched
    // on the caller's stream; recaptured when the values pointer changes
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const double *graph_values = nullptr;
    // per-launch profiling
    bool profiling = false;
    std::vector<hipEvent_t> prof_ev;     // pairs
    std::vector<int> prof_cls;
    std::vector<int> prof_lvl;   // etree level of each launch (-1: assembly)
    std::vector<double> prof_flops;
    size_t prof_used = 0;
};

// A batch: the disjoint union of several analyses, factored and solved by
// one level schedule.  It owns the merged plan and the merged factor; views
// of single systems (spc_batch_factor) share that storage and keep the batch
// alive until they are freed.
struct spc_batch_s {
    uint32_t magic = 0x42415431u;
    std::atomic<int> refs{1};
    int count = 0;
    int precision = SPC_FP64;
    std::vector<spc_symbolic_s *> members;
    spc_symbolic_s *merged = nullptr;
    spc_factor_s *F = nullptr;
    std::vector<int64_t> col_off, panel_off, inv_base, val_off;
    double *vbuf = nullptr;      // concatenated values
    double *bbuf = nullptr;      // merged right-hand sides
    size_t bbuf_bytes = 0;
    void *meta = nullptr;        // device: pointer table, leading dims, row offsets, second pointer table
    size_t meta_bytes = 0;
    int32_t *rowseg = nullptr;   // device: system of each merged row (refinement)
};

namespace {

thread_local char g_last_error[256] = "";

int record_error(hipError_t e, const char *what, int line) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s (%s) at capi.cpp:%d", hipGetErrorString(e), what, line);
    return e == hipErrorOutOfMemory ? SPC_OUT_OF_MEMORY : SPC_DEVICE_ERROR;
}

#define HIP_TRY(expr)                                          \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return record_error(e_, #expr, __LINE__); \
    } while (0)

bool sym_ok(spc_symbolic s) { return s && s->magic == kSymMagic; }

// Host-synchronous copies on a non-blocking stream of the calling thread's
// own (one per thread and device, kept for the process): the legacy default
// stream is never used, so these copies neither wait for other threads'
// blocking streams nor collide with a graph capture running in another
// thread (the HIP runtime refuses legacy-stream work while any capture is
// in progress).  Callers synchronize the stream that produced the data
// first.
constexpr int kMaxDevices = 64;
hipError_t copy_sync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
    thread_local hipStream_t streams[kMaxDevices] = {};
    if (bytes == 0) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (!streams[dev]) {
        e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    e = hipMemcpyAsync(dst, src, bytes, kind, streams[dev]);
    if (e == hipSuccess) e = hipStreamSynchronize(streams[dev]);
    return e;
}

// The factor whose storage, status words and device-error word a handle
// uses: itself, or for a view into a batch, the batch's merged factor.
spc_factor_s *owner_of(spc_factor_s *f) { return f->batch ? f->batch->F : f; }
spc::WaitCtl wait_of(spc_factor_s *f) {
    spc_factor_s *o = owner_of(f);
    return spc::WaitCtl{o->deverr, o->spin};
}

// SPC_DEVICE_ERROR if a bounded wait of f's work gave up (the stream must
// have drained), else SPC_OK.
int check_deverr(spc_factor_s *f) {
    int32_t v = 0;
    HIP_TRY(copy_sync(&v, owner_of(f)->deverr, sizeof(v), hipMemcpyDeviceToHost));
    if (v == 0) return SPC_OK;
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "a wait on another workgroup gave up after its poll limit; the factor and the solves since "
                  "its factorization are unreliable until it is factored again");
    return SPC_DEVICE_ERROR;
}
bool fac_ok(spc_factor f) { return f && f->magic == kFacMagic && sym_ok(f->sym); }

void sym_release(spc_symbolic_s *s) {
    if (s && s->refs.fetch_sub(1) == 1) {
        if (s->dev.base || s->csr_base) {
            int cur = -1;
            (void)hipGetDevice(&cur);
            if (s->dev.device >= 0) (void)hipSetDevice(s->dev.device);
            if (s->dev.base) (void)hipFree(s->dev.base);
            if (s->csr_base) (void)hipFree(s->csr_base);
            if (cur >= 0) (void)hipSetDevice(cur);
        }
        s->magic = kDead;
        delete s;
    }
}

int check_device(int *dev_out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SPC_NO_DEVICE;
    *dev_out = dev;
    return SPC_OK;
}

template <typename V>
size_t bytes_of(const std::vector<V> &v) {
    return v.size() * sizeof(V);
}

// Upload the schedule once per symbolic handle and device.
int ensure_device_plan(spc_symbolic_s *sym, int device) {
    std::lock_guard<std::mutex> lk(sym->mu);
    if (sym->dev.base) return sym->dev.device == device ? SPC_OK : SPC_INVALID_INPUT;
    const spc::Symbolic &S = sym->S;
    struct Piece {
        const void *src;
        size_t bytes;
        const void **dst;
    };
    spc::DevPlan &P = sym->dev.plan;
    std::vector<Piece> pieces = {
        {S.rows.data(), bytes_of(S.rows), (const void **)&P.rows},
        {S.rel.data(), bytes_of(S.rel), (const void **)&P.rel},
        {S.cbase.data(), bytes_of(S.cbase), (const void **)&P.cbase},
        {S.crel.data(), bytes_of(S.crel), (const void **)&P.crel},
        {S.amap.data(), bytes_of(S.amap), (const void **)&P.amap},
        {S.perm.data(), bytes_of(S.perm), (const void **)&P.perm},
        {S.dsrc.data(), bytes_of(S.dsrc), (const void **)&P.dsrc},
        {S.potrf_tasks.data(), bytes_of(S.potrf_tasks), (const void **)&P.potrf_tasks},
        {S.small_tasks.data(), bytes_of(S.small_tasks), (const void **)&P.small_tasks},
        {S.tiny_tasks.data(), bytes_of(S.tiny_tasks), (const void **)&P.tiny_tasks},
        {S.trsm_tiles.data(), bytes_of(S.trsm_tiles), (const void **)&P.trsm_tiles},
        {S.int_tiles.data(), bytes_of(S.int_tiles), (const void **)&P.int_tiles},
        {S.ext_tiles.data(), bytes_of(S.ext_tiles), (const void **)&P.ext_tiles},
        {S.ext_tiles_big.data(), bytes_of(S.ext_tiles_big), (const void **)&P.ext_tiles_big},
        {S.trail_big.data(), bytes_of(S.trail_big), (const void **)&P.trail_big},
        {S.stasks.data(), bytes_of(S.stasks), (const void **)&P.stasks},
        {S.stiny.data(), bytes_of(S.stiny), (const void **)&P.stiny},
        {S.status_slot.data(), bytes_of(S.status_slot), (const void **)&P.status_slot},
        {S.stgt_ptr.data(), bytes_of(S.stgt_ptr), (const void **)&P.stgt_ptr},
        {S.stgt.data(), bytes_of(S.stgt), (const void **)&P.stgt},
        {S.fdep.data(), bytes_of(S.fdep), (const void **)&P.fdep},
        {S.bwd_order.data(), bytes_of(S.bwd_order), (const void **)&P.bwd_order},
        {S.pqueue.data(), bytes_of(S.pqueue), (const void **)&P.pqueue},
        {S.pchunk.data(), bytes_of(S.pchunk), (const void **)&P.pchunk},
        {S.psmall.data(), bytes_of(S.psmall), (const void **)&P.psmall},
        {S.ptiny.data(), bytes_of(S.ptiny), (const void **)&P.ptiny},
        {S.pdep0.data(), bytes_of(S.pdep0), (const void **)&P.pdep0},
        {S.ptgt_ptr.data(), bytes_of(S.ptgt_ptr), (const void **)&P.ptgt_ptr},
        {S.ptgt.data(), bytes_of(S.ptgt), (const void **)&P.ptgt},
    };
    size_t total = 0;
    for (auto &p : pieces) total += (p.bytes + 255) & ~size_t(255);
    void *base = nullptr;
    HIP_TRY(hipMalloc(&base, total ? total : 256));
    std::vector<char> host(total ? total : 256, 0);
    size_t off = 0;
    for (auto &p : pieces) {
        if (p.bytes) std::memcpy(host.data() + off, p.src, p.bytes);
        *p.dst = (const char *)base + off;
        off += (p.bytes + 255) & ~size_t(255);
    }
    hipError_t e = copy_sync(base, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(base);
        return record_error(e, "plan upload", __LINE__);
    }
    if (S.status_slot.empty()) P.status_slot = nullptr;
    sym->dev.base = base;
    sym->dev.bytes = total;
    sym->dev.device = device;
    return SPC_OK;
}

size_t plan_bytes(const spc::Symbolic &S) {
    return bytes_of(S.rows) + bytes_of(S.rel) + bytes_of(S.cbase) + bytes_of(S.crel) + bytes_of(S.amap) +
           bytes_of(S.perm) + bytes_of(S.dsrc) + bytes_of(S.potrf_tasks) + bytes_of(S.small_tasks) + bytes_of(S.tiny_tasks) + bytes_of(S.trsm_tiles) + bytes_of(S.trail_big) +
           bytes_of(S.int_tiles) + bytes_of(S.ext_tiles) + bytes_of(S.ext_tiles_big) +
           bytes_of(S.stasks) + bytes_of(S.stiny) + bytes_of(S.status_slot) + bytes_of(S.stgt_ptr) + bytes_of(S.stgt) +
           bytes_of(S.fdep) + bytes_of(S.bwd_order) + bytes_of(S.pqueue) + bytes_of(S.pchunk) + bytes_of(S.psmall) + bytes_of(S.ptiny) +
           bytes_of(S.pdep0) + bytes_of(S.ptgt_ptr) + bytes_of(S.ptgt);
}

// Device bytes of one factor (panels and block inverses at esz bytes per
// entry) plus the device plan: the footprint the budget and
// spc_symbolic_info use.
int64_t factor_footprint(const spc::Symbolic &S, int64_t esz) {
    const int64_t entries = S.panel_entries() + (S.inv_off.empty() ? 0 : S.inv_off.back());
    return entries * esz + (int64_t)plan_bytes(S);
}

// Brackets one launch with a pair of events (on the launch's stream) when
// profiling is on.
struct Prof {
    spc_factor_s *f;
    int level = -1;  // etree level of the launches that follow
    template <typename Fn>
    void run(int cls, double flops, hipStream_t st, Fn &&fn) {
        if (!f || !f->profiling) {
            fn();
            return;
        }
        size_t i = f->prof_used++;
        while (f->prof_ev.size() < 2 * (i + 1)) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                f->prof_used--;
                fn();
                return;
            }
            f->prof_ev.push_back(e);
        }
        if (f->prof_cls.size() <= i) {
            f->prof_cls.resize(i + 1);
            f->prof_lvl.resize(i + 1);
            f->prof_flops.resize(i + 1);
        }
        f->prof_cls[i] = cls;
        f->prof_lvl[i] = level;
        f->prof_flops[i] = flops;
        (void)hipEventRecord(f->prof_ev[2 * i], st);
        fn();
        (void)hipEventRecord(f->prof_ev[2 * i + 1], st);
    }
};

// The numeric factorization, level by level (Sec. 3, Fig. 1).  Inside a
// level, step b runs TRSM of block b, then one launch of the trailing update
// by panel b: the tiles of block b+1's columns first (the diagonal-tile
// workgroup also factors block b+1), then the columns beyond, so that
// factoring the next block overlaps the bulk of the update.
template <typename T>
void enqueue_factor(const spc::Symbolic &S, const spc::DevPlan &P, const double *d_values, T *Lx, T *Linv,
                    unsigned long long *status, int32_t *hflags, int32_t *qctr, int32_t *pdep, spc::WaitCtl wc,
                    bool bf16, T *pfloor, hipStream_t st, Prof &prof) {
    spc::PivotFloor<T> pfl;
    if (bf16) {
        pfl.v = pfloor;
        pfl.count = wc.err + 1;
    }
    prof.run(SPC_K_ASSEMBLE, 0.0, st, [&] {
        spc::launch_zero<T>(Lx, S.panel_entries(), st);
        spc::launch_assemble<T>(P, S.nnzA, d_values, Lx, st);
        if (bf16) spc::launch_pivot_floor<T>(P, S.n, d_values, spc::kBf16PivotTheta, pfloor, st);
    });
    if (!S.pqueue.empty()) {
        prof.level = -2;
        prof.run(SPC_K_SMALL_TREES, S.persist_flops, st, [&] {
            spc::launch_persist_small<T>(P, (int64_t)S.pchunk.size() - 1, S.nsuper, pdep, qctr, Lx, Linv, status, pfl,
                                         wc, st);
        });
    }
    for (int32_t l = 0; l < S.nlevels; ++l) {
        prof.level = l;
        if (S.tiny_ptr[l + 1] > S.tiny_ptr[l])
            prof.run(SPC_K_TINY, S.tiny_flops[l], st, [&] {
                spc::launch_tiny<T>(P, S.tiny_ptr[l], S.tiny_e16[l], S.tiny_e32[l], S.tiny_ptr[l + 1], Lx, Linv,
                                    status, pfl, st);
            });
        if (S.small_ptr[l + 1] > S.small_ptr[l])
            prof.run(SPC_K_SMALL, S.small_flops[l], st, [&] {
                spc::launch_small<T>(P, S.small_ptr[l], S.small_ptr[l + 1], Lx, Linv, status, pfl, st);
            });
        for (int64_t k = S.level_step_ptr[l]; k < S.level_step_ptr[l + 1]; ++k) {
            const auto &stp = S.steps[k];
            if (stp.f1 > stp.f0)
                prof.run(SPC_K_POTRF, stp.potrf_flops, st,
                         [&] { spc::launch_potrf<T>(P, stp.f0, stp.f1, Lx, Linv, status, wc.err, pfl, st); });
            if (stp.p1 > stp.p0)
                prof.run(SPC_K_TRSM, stp.trsm_flops, st, [&] {
                    spc::launch_tiles<T>(P, spc::kTilesTrsm, stp.p0, stp.p1, Lx, Linv, status, nullptr, wc, false, pfl,
                                         st);
                });
            if (stp.t1 > stp.t0)
                prof.run(SPC_K_TRAILING, stp.look_flops + stp.rest_flops, st, [&] {
                    spc::launch_tiles<T>(P, spc::kTilesTrailing, stp.t0, stp.t1, Lx, Linv, status, hflags, wc, bf16,
                                         pfl, st);
                });
            if (stp.q1 > stp.q0)
                prof.run(SPC_K_TRAILING, stp.big_flops, st,
                         [&] { spc::launch_trail128<T>(P, stp.q0, stp.q1, Lx, bf16, st); });
        }
        if (S.ext_big_ptr[l + 1] > S.ext_big_ptr[l])
            prof.run(SPC_K_SCATTER_BIG, S.ext_big_flops[l], st, [&] {
                spc::launch_tiles128<T>(P, S.ext_big_ptr[l], S.ext_big_ptr[l + 1], Lx, bf16, st);
            });
        if (S.ext_tile_ptr[l + 1] > S.ext_tile_ptr[l])
            prof.run(SPC_K_SCATTER, S.ext_flops[l], st, [&] {
                spc::launch_tiles<T>(P, spc::kTilesScatter, S.ext_tile_ptr[l], S.ext_tile_ptr[l + 1], Lx, Linv,
                                     status, nullptr, wc, bf16, pfl, st);
            });
    }
}

// Y holds the permuted right-hand sides on entry (and is overwritten); X
// receives the solution.
// sync points to kSolveSyncInts(blocks) words of workspace.  Each sweep runs
// one launch per wide block-tree level, and the narrow levels at the top
// (levels solve_split..) as one persistent launch per sweep, which removes
// a launch per level from the long chains of the top supernodes.
template <typename T>
void enqueue_solve(const spc::Symbolic &S, const spc::DevPlan &P, const T *Lx, const T *Linv, T *Y, T *X,
                   T *Acc, int32_t *sync, spc::WaitCtl wc, int nrhs, hipStream_t st) {
    const int64_t n = S.n, nb = (int64_t)S.sblocks.size(), nt = (int64_t)S.stasks.size();
    const spc::SolveSync sy = spc::make_solve_sync(sync, nb, wc);
    const int32_t split = S.solve_split;
    // the persistent sweeps' hand-over buffers: Acc (unused until the
    // backward sweep) for the forward one, Y (spent by then) for the
    // backward one
    const bool persist = split < S.nslevels;
    if (persist) spc::launch_fill_unset<T>(Acc, n * nrhs, st);
    else spc::launch_zero<T>(Acc, n * nrhs, st);
    spc::launch_solve_reset(P, nb, sy, st);
    // below solve_split the tiny supernodes of a level have their own
    // (one-wave) launch beside the level's task launch
    const int32_t tsplit = S.solve_split;
    for (int32_t l = 0; l < split; ++l) {
        if (l < tsplit)
            spc::launch_solve_tiny_fwd<T>(P, S.stiny_ptr[l], S.stiny_ptr[l + 1], Lx, Linv, Y, X, n, nrhs, st);
        spc::launch_solve_fwd<T>(P, S.stask_ptr[l], S.stask_ptr[l + 1], Lx, Linv, Y, X, nullptr, n, nrhs, sy, false,
                                 st);
    }
    if (persist) {
        spc::launch_solve_fwd<T>(P, S.stask_ptr[split], nt, Lx, Linv, Y, X, Acc, n, nrhs, sy, true, st);
        spc::launch_fill_unset<T>(Y, n * nrhs, st);
        spc::launch_zero<T>(Acc, n * nrhs, st);
        spc::launch_solve_bwd<T>(P, S.stask_ptr[split], nt, Lx, Linv, X, Acc, Y, n, nrhs, sy, true, st);
    }
    for (int32_t l = split - 1; l >= 0; --l) {
        if (l < tsplit)
            spc::launch_solve_tiny_bwd<T>(P, S.stiny_ptr[l], S.stiny_ptr[l + 1], Lx, Linv, X, n, nrhs, st);
        spc::launch_solve_bwd<T>(P, S.stask_ptr[l], S.stask_ptr[l + 1], Lx, Linv, X, Acc, nullptr, n, nrhs, sy, false,
                                 st);
    }
}

void drop_graph(spc_factor_s *f) {
    if (f->gexec) (void)hipGraphExecDestroy(f->gexec);
    if (f->graph) (void)hipGraphDestroy(f->graph);
    f->gexec = nullptr;
    f->graph = nullptr;
    f->graph_values = nullptr;
}

// Capture the status reset and every launch of the factorization (kernels
// only: the fills are kernels too) into f's graph.
int capture_factor(spc_factor f, const double *d_values) {
    const spc::Symbolic &S = f->sym->S;
    const spc::DevPlan &P = f->sym->dev.plan;
    drop_graph(f);
    if (!f->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&f->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(f->cap_stream, hipStreamCaptureModeRelaxed));
    spc::launch_status_reset(f->status, f->nstatus, f->deverr, f->hflags, f->nflags, f->cap_stream);
    Prof none{nullptr};
    const spc::WaitCtl wc{f->deverr, f->spin};
    if (f->precision == SPC_FP64)
        enqueue_factor<double>(S, P, d_values, (double *)f->Lx, (double *)f->Linv, f->status, f->hflags, f->qctr,
                               f->pdep, wc, false, nullptr, f->cap_stream, none);
    else
        enqueue_factor<float>(S, P, d_values, (float *)f->Lx, (float *)f->Linv, f->status, f->hflags, f->qctr,
                              f->pdep, wc, f->precision == SPC_FP32_BF16UPD, (float *)f->pfloor, f->cap_stream, none);
    hipGraph_t g = nullptr;
    const hipError_t e0 = hipGetLastError();
    const hipError_t e1 = hipStreamEndCapture(f->cap_stream, &g);
    if (e0 != hipSuccess || e1 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return record_error(e0 != hipSuccess ? e0 : e1, "factor capture", __LINE__);
    }
    f->graph = g;
    HIP_TRY(hipGraphInstantiate(&f->gexec, g, nullptr, nullptr, 0));
    f->graph_values = d_values;
    return SPC_OK;
}

int run_factor(spc_factor f, const double *d_values, hipStream_t st) {
    const spc::Symbolic &S = f->sym->S;
    const spc::DevPlan &P = f->sym->dev.plan;
    f->refine_cg = false;
    (void)hipGetLastError();  // report only the launches below
    if (f->use_graph && !f->profiling) {
        if (!f->gexec || f->graph_values != d_values) {
            int rc = capture_factor(f, d_values);
            if (rc) return rc;
        }
        HIP_TRY(hipEventRecord(f->ev0, st));
        HIP_TRY(hipGraphLaunch(f->gexec, st));
        HIP_TRY(hipEventRecord(f->ev1, st));
        f->stream = st;
        return SPC_OK;
    }
    spc::launch_status_reset(f->status, f->nstatus, f->deverr, f->hflags, f->nflags, st);
    HIP_TRY(hipEventRecord(f->ev0, st));
    f->prof_used = 0;
    Prof prof{f};
    const spc::WaitCtl wc{f->deverr, f->spin};
    if (f->precision == SPC_FP64)
        enqueue_factor<double>(S, P, d_values, (double *)f->Lx, (double *)f->Linv, f->status, f->hflags, f->qctr,
                               f->pdep, wc, false, nullptr, st, prof);
    else
        enqueue_factor<float>(S, P, d_values, (float *)f->Lx, (float *)f->Linv, f->status, f->hflags, f->qctr,
                              f->pdep, wc, f->precision == SPC_FP32_BF16UPD, (float *)f->pfloor, st, prof);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(f->ev1, st));
    f->stream = st;
    return SPC_OK;
}

int create_factor(spc_symbolic sym, int precision, spc_factor *out, int nstatus = 1) {
    if (precision != SPC_FP64 && precision != SPC_FP32 && precision != SPC_FP32_BF16UPD) return SPC_INVALID_INPUT;
    if (sym->hbm_budget > 0) {
        const int64_t need = factor_footprint(sym->S, precision == SPC_FP64 ? 8 : 4);
        if (need > sym->hbm_budget) {
            std::snprintf(g_last_error, sizeof(g_last_error),
                          "factorization needs %lld device bytes, over the budget of %lld", (long long)need,
                          (long long)sym->hbm_budget);
            return SPC_OUT_OF_MEMORY;
        }
    }
    int dev = -1;
    int rc = check_device(&dev);
    if (rc) return rc;
    rc = ensure_device_plan(sym, dev);
    if (rc) return rc;
    spc_factor f = new (std::nothrow) spc_factor_s;
    if (!f) return SPC_OUT_OF_MEMORY;
    f->sym = sym;
    sym->refs.fetch_add(1);
    f->precision = precision;
    f->device = dev;
    f->nstatus = nstatus;
    size_t esz = precision == SPC_FP64 ? sizeof(double) : sizeof(float);
    size_t bytes = std::max<size_t>(1, (size_t)sym->S.panel_entries()) * esz;
    hipError_t e = hipMalloc(&f->Lx, bytes);
    size_t inv_bytes = std::max<size_t>(1, (size_t)sym->S.inv_off.back()) * esz;
    if (e == hipSuccess) e = hipMalloc(&f->Linv, inv_bytes);
    f->nflags = spc::kFlagsPerBlock * (int)sym->S.sblocks.size();  // panel flags and claim of each block
    // status words, the device-error word and the raised-pivot count,
    // hand-over flags, the persistent launch's work counter (padded to 8
    // bytes) and its dependency counters
    if (e == hipSuccess)
        e = hipMalloc((void **)&f->status, sizeof(unsigned long long) * (nstatus + 1) +
                                               sizeof(int32_t) * (f->nflags + 2 + (size_t)sym->S.nsuper));
    if (e == hipSuccess) {
        f->deverr = reinterpret_cast<int32_t *>(f->status + nstatus);
        f->hflags = reinterpret_cast<int32_t *>(f->status + nstatus + 1);
        f->qctr = f->hflags + f->nflags;
        f->pdep = f->qctr + 2;
    }
    if (e == hipSuccess && precision == SPC_FP32_BF16UPD)
        e = hipMalloc(&f->pfloor, std::max<size_t>(1, (size_t)sym->S.n) * sizeof(float));
    if (e == hipSuccess) e = hipEventCreate(&f->ev0);
    if (e == hipSuccess) e = hipEventCreate(&f->ev1);

    if (e != hipSuccess) {
        spc_free_factor(f);
        return record_error(e, "factor allocation", __LINE__);
    }
    *out = f;
    return SPC_OK;
}

int ensure_bytes(void **p, size_t *have, size_t need) {
    if (*have >= need) return SPC_OK;
    if (*p) HIP_TRY(hipFree(*p));
    *p = nullptr;
    *have = 0;
    HIP_TRY(hipMalloc(p, need));
    *have = need;
    return SPC_OK;
}


// ---------------------------------------------------------------------------
// Iterative refinement (FP64 on the device).
// ---------------------------------------------------------------------------
constexpr int kRefineChunk = 16;

int ensure_csr(spc_symbolic_s *sym) {
    std::lock_guard<std::mutex> lk(sym->mu);
    if (sym->csr_base) return SPC_OK;
    const spc::Symbolic &S = sym->S;
    const size_t b0 = (bytes_of(S.csr_ptr) + 255) & ~size_t(255);
    const size_t b1 = (bytes_of(S.csr_val) + 255) & ~size_t(255);
    const size_t b2 = (bytes_of(S.csr_col) + 255) & ~size_t(255);
    void *base = nullptr;
    HIP_TRY(hipMalloc(&base, b0 + b1 + b2 + 256));
    char *c = (char *)base;
    hipError_t e = copy_sync(c, S.csr_ptr.data(), bytes_of(S.csr_ptr), hipMemcpyHostToDevice);
    if (e == hipSuccess && !S.csr_val.empty())
        e = copy_sync(c + b0, S.csr_val.data(), bytes_of(S.csr_val), hipMemcpyHostToDevice);
    if (e == hipSuccess && !S.csr_col.empty())
        e = copy_sync(c + b0 + b1, S.csr_col.data(), bytes_of(S.csr_col), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(base);
        return record_error(e, "csr upload", __LINE__);
    }
    sym->csr_base = base;
    sym->d_csr_ptr = (const int64_t *)c;
    sym->d_csr_val = (const int64_t *)(c + b0);
    sym->d_csr_col = (const int32_t *)(c + b0 + b1);
    return SPC_OK;
}

struct RefineResult {
    int iterations = 0;
    bool converged = false;
    double berr = 0.0;
};

double bits_to_double(unsigned long long b) {
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

// What one refinement runs on: the factor whose solve is the
// preconditioner, the full-A CSR with the caller values it points into,
// and, for a batch, the system of every row (the rows of a system are
// contiguous); every norm, dot product and coefficient is then kept per
// system and column, so each system refines as if it were alone.
struct RefineTarget {
    spc_factor f = nullptr;
    const int64_t *rp = nullptr, *vm = nullptr;
    const int32_t *ci = nullptr;
    const double *values = nullptr;
    int64_t n = 0;
    int64_t nnz = 0;  // entries of the full-A CSR
    const int32_t *seg = nullptr;  // row -> system, or null (one system)
    int nseg = 1;
};

// One chunk of q <= kRefineChunk right-hand sides.  x0 = low-precision
// solve; then each step computes r = b - A x in FP64 and the backward error
//   eta_k = ||r_k||_inf / (||A||_inf ||x_k||_inf + ||b_k||_inf)
// per system and column.  Classical refinement (x += solve(r)) runs while
// each step cuts the largest eta at least tenfold; after that, conjugate
// gradients in FP64 preconditioned by the factor (M^{-1} = solve) continue
// from the current x, with alpha and beta per system and column (the
// preconditioner is block diagonal over the systems, so the iterations of
// different systems do not mix).  Stops when every eta <= tol or after
// maxit steps of either kind.  res[s] receives system s's result; its
// iteration count is the step at which all its columns first met tol.
// Once a refined solve with a factorization has switched to CG, the next
// ones with it start with CG: the classical step would only show again
// that the factor is too weak for it.
int refine_chunk(const RefineTarget &T, const double *B, double *X, int q, int64_t ld, double tol, int maxit,
                 hipStream_t st, RefineResult *res) {
    const int64_t n = T.n;
    const int ns = T.nseg;
    constexpr int C = kRefineChunk;
    const int64_t K = (int64_t)C * ns;  // (column, system) slots
    // workspace: 7 vectors of n x C (leading dimension n), then scalars
    const size_t vec = ((size_t)n * C * sizeof(double) + 255) & ~size_t(255);
    const size_t scal = (size_t)(9 * K + ns) * sizeof(double);
    int rc = ensure_bytes((void **)&T.f->refine, &T.f->refine_bytes, 7 * vec + scal);
    if (rc) return rc;
    char *base = (char *)T.f->refine;
    double *Bw = (double *)base, *Xw = (double *)(base + vec), *Tv = (double *)(base + 2 * vec),
           *Rv = (double *)(base + 3 * vec), *Zv = (double *)(base + 4 * vec), *Pv = (double *)(base + 5 * vec),
           *Qv = (double *)(base + 6 * vec);
    unsigned long long *umax = (unsigned long long *)(base + 7 * vec);  // r[K], x[K], b[K], |A|[ns]
    double *dots = (double *)(umax + 3 * K + ns);                          // [K]
    double *coef = dots + K;                                               // alpha[K], -alpha[K], beta[K]
    double *rho = coef + 3 * K;                                            // [K] r.z of the current step
    double *frz = rho + K;                                                 // [K] 1 for a converged slot
    auto colmax = [&](const double *V, unsigned long long *out) {
        if (T.seg) spc::launch_seg_colmax(V, T.seg, n, q, n, ns, out, st);
        else spc::launch_colmax(V, n, q, n, out, st);
    };
    auto axpby = [&](const double *a, double a0, const double *Xv, const double *bb, double b0, double *Y) {
        if (T.seg) spc::launch_seg_axpby(a, a0, Xv, bb, b0, Y, T.seg, n, q, n, ns, st);
        else spc::launch_axpby(a, a0, Xv, bb, b0, Y, n, q, n, st);
    };

    spc::launch_copy_cols(B, ld, Bw, n, n, q, st);
    spc::launch_copy_cols(Bw, n, Xw, n, n, q, st);
    rc = spc_solve(T.f, Xw, q, n, st);
    if (rc) return rc;
    spc::launch_zero<unsigned long long>(umax, 3 * K + ns, st);
    if (T.seg) spc::launch_seg_norm_inf_A(T.rp, T.vm, T.values, T.seg, n, umax + 3 * K, st);
    else spc::launch_norm_inf_A(T.rp, T.vm, T.values, n, T.nnz, umax + 3 * K, st);
    colmax(Bw, umax + 2 * K);

    // the per-step copies go through pinned host memory (no staging)
    const size_t host_need = (3 * K + ns) * sizeof(unsigned long long) + K * sizeof(double);
    if (T.f->refine_host_bytes < host_need) {
        if (T.f->refine_host) HIP_TRY(hipHostFree(T.f->refine_host));
        T.f->refine_host = nullptr;
        T.f->refine_host_bytes = 0;
        HIP_TRY(hipHostMalloc(&T.f->refine_host, host_need, hipHostMallocDefault));
        T.f->refine_host_bytes = host_need;
    }
    unsigned long long *hb = (unsigned long long *)T.f->refine_host;  // r[K], x[K], b[K], |A|[ns]
    double *frozen = (double *)(hb + 3 * K + ns);                       // [K]
    std::fill(frozen, frozen + K, 0.0);
    std::vector<double> eta_hist, eta_s(ns);
    std::vector<char> done(ns, 0);
    std::atomic<bool> &start_cg = owner_of(T.f)->refine_cg;  // per factorization (a batch's for a view)
    bool cg = start_cg, cg_started = false;
    int it = 0;
    // dot products per slot into dots, left on the device: the CG
    // coefficients are formed there too, so a step synchronizes only for
    // its backward errors
    auto dot = [&](const double *U, const double *V) {
        spc::launch_zero<double>(dots, K, st);
        if (T.seg) spc::launch_seg_coldot(U, V, T.seg, n, q, n, ns, dots, st);
        else spc::launch_coldot(U, V, n, q, n, dots, st);
    };
    std::vector<double> e_slot(K, 0.0);
    for (;;) {
        // Once CG runs, its recursive residual r tracks b - A x to rounding,
        // so a step's backward error is first estimated from r; the true
        // residual (one more SpMV) is taken before any column counts as
        // converged and at the step limit, so every reported backward error
        // is the true one.  After a true residual, r is replaced by it.
        bool est = cg_started;
        double eta = 0.0;
        for (;;) {
            if (!est) spc::launch_spmv(T.rp, T.ci, T.vm, T.values, Xw, Bw, Tv, n, T.nnz, q, n, st);  // T = b - A x
            spc::launch_zero<unsigned long long>(umax, 2 * K, st);
            colmax(est ? Rv : Tv, umax);
            colmax(Xw, umax + K);
            HIP_TRY(hipMemcpyAsync(hb, umax, (3 * K + ns) * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if ((rc = check_deverr(T.f))) return rc;
            eta = 0.0;
            std::fill(eta_s.begin(), eta_s.end(), 0.0);
            bool newly = false;
            for (int k = 0; k < q; ++k)
                for (int sg = 0; sg < ns; ++sg) {
                    const int64_t j = (int64_t)k * ns + sg;
                    const double normA = bits_to_double(hb[3 * K + sg]);
                    const double rn = bits_to_double(hb[j]), xn = bits_to_double(hb[K + j]),
                                 bn = bits_to_double(hb[2 * K + j]);
                    const double den = normA * xn + bn;
                    double e = den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
                    // a NaN or Inf anywhere (the maxima carry NaN as +Inf) is
                    // never converged
                    if (std::isnan(e) || !std::isfinite(rn) || !std::isfinite(xn) || !std::isfinite(bn) ||
                        !std::isfinite(normA))
                        e = INFINITY;
                    e_slot[j] = e;
                    if (e <= tol && frozen[j] == 0.0) newly = true;
                    eta_s[sg] = std::max(eta_s[sg], e);
                    eta = std::max(eta, e);
                }
            if (est && (newly || it >= maxit)) {
                est = false;  // confirm on the true residual
                continue;
            }
            break;
        }
        if (cg_started && !est) spc::launch_copy_cols(Tv, n, Rv, n, n, q, st);  // residual replacement
        for (int64_t j = 0; j < (int64_t)q * ns; ++j) frozen[j] = e_slot[j] <= tol ? 1.0 : 0.0;
        for (int sg = 0; sg < ns; ++sg) {
            res[sg].berr = eta_s[sg];
            res[sg].converged = eta_s[sg] <= tol;
            if (!done[sg]) res[sg].iterations = it;
            if (res[sg].converged) done[sg] = 1;
        }
        eta_hist.push_back(eta);
        if (eta <= tol || it >= maxit) break;
        const size_t h = eta_hist.size();
        // A classical step contracts eta by about the spectral radius rho of
        // I - M^{-1} A.  Once a step contracts it by less than 10x, CG takes
        // over: its rate bound (sqrt(k) - 1) / (sqrt(k) + 1), with
        // k <= (1 + rho) / (1 - rho), is then well below rho, which pays for
        // its dot products and its true residuals near convergence.
        if (!cg && h >= 2 && !(eta_hist[h - 1] <= 0.1 * eta_hist[h - 2])) cg = start_cg = true;
        ++it;
        if (!cg) {
            spc::launch_copy_cols(Tv, n, Zv, n, n, q, st);
            rc = spc_solve(T.f, Zv, q, n, st);  // d = M^{-1} r
            if (rc) return rc;
            axpby(nullptr, 1.0, Zv, nullptr, 1.0, Xw);  // x += d
            continue;
        }
        // frozen is next written after the next step's synchronization,
        // so this copy from it has finished by then
        HIP_TRY(hipMemcpyAsync(frz, frozen, K * sizeof(double), hipMemcpyHostToDevice, st));
        if (!cg_started) {
            // r = b - A x, z = M^{-1} r, p = z, rho = r.z
            spc::launch_copy_cols(Tv, n, Rv, n, n, q, st);
            spc::launch_copy_cols(Rv, n, Zv, n, n, q, st);
            rc = spc_solve(T.f, Zv, q, n, st);
            if (rc) return rc;
            spc::launch_copy_cols(Zv, n, Pv, n, n, q, st);
            dot(Rv, Zv);
            HIP_TRY(hipMemcpyAsync(rho, dots, K * sizeof(double), hipMemcpyDeviceToDevice, st));
            cg_started = true;
        } else {
            // the preconditioner solve of the last step's residual comes
            // after that step's convergence check, so the step that
            // converges makes none
            spc::launch_copy_cols(Rv, n, Zv, n, n, q, st);
            rc = spc_solve(T.f, Zv, q, n, st);  // z = M^{-1} r
            if (rc) return rc;
            dot(Rv, Zv);
            spc::launch_cg_coef(dots, rho, frz, coef, K, false, st);  // beta = r.z / rho, rho = r.z
            axpby(nullptr, 1.0, Zv, coef + 2 * K, 0.0, Pv);  // p = z + beta p
        }
        spc::launch_spmv(T.rp, T.ci, T.vm, T.values, Pv, nullptr, Qv, n, T.nnz, q, n, st);  // q = A p
        dot(Pv, Qv);
        spc::launch_cg_coef(dots, rho, frz, coef, K, true, st);  // alpha = rho / p.q
        axpby(coef, 0.0, Pv, nullptr, 1.0, Xw);      // x += alpha p
        axpby(coef + K, 0.0, Qv, nullptr, 1.0, Rv);  // r -= alpha q
    }
    spc::launch_copy_cols(Xw, n, X, ld, n, q, st);
    HIP_TRY(hipGetLastError());
    return SPC_OK;
}


// ---------------------------------------------------------------------------
// Triangular solves in chunks of right-hand sides over a work area of
// solve_work_bytes(S, chunk, esz): Y, X, Acc (n x chunk each, factor
// precision) then the persistent sweeps' counters.  The kernels clear what
// they need (Acc and the counters) at the start of every chunk.
// ---------------------------------------------------------------------------
constexpr int kSolveChunk = 16;

size_t solve_vec_bytes(const spc::Symbolic &S, int chunk, size_t esz) { return (size_t)S.n * chunk * esz; }
size_t solve_work_bytes(const spc::Symbolic &S, int chunk, size_t esz) {
    const size_t cnt_off = (3 * solve_vec_bytes(S, chunk, esz) + 255) & ~size_t(255);
    return cnt_off + sizeof(int32_t) * spc::kSolveSyncInts((int64_t)S.sblocks.size());
}

int solve_chunks(spc_factor f, double *d_B, int nrhs, int64_t ldb, hipStream_t st, char *base, int chunk) {
    const spc::Symbolic &S = f->sym->S;
    const spc::DevPlan &P = f->sym->dev.plan;
    const size_t esz = f->precision == SPC_FP64 ? sizeof(double) : sizeof(float);
    (void)hipGetLastError();  // report only the launches below
    const size_t vec = solve_vec_bytes(S, chunk, esz);
    const size_t cnt_off = (3 * vec + 255) & ~size_t(255);
    int32_t *counters = (int32_t *)(base + cnt_off);
    const spc::WaitCtl wc = wait_of(f);
    for (int q0 = 0; q0 < nrhs; q0 += chunk) {
        const int q = std::min(chunk, nrhs - q0);
        double *B = d_B + (int64_t)q0 * ldb;
        if (f->precision == SPC_FP64) {
            double *Y = (double *)base, *X = (double *)(base + vec), *Acc = (double *)(base + 2 * vec);
            spc::launch_perm_in<double>(P, S.n, q, B, ldb, Y, st);
            enqueue_solve<double>(S, P, (const double *)f->Lx, (const double *)f->Linv, Y, X, Acc, counters, wc, q,
                                  st);
            spc::launch_perm_out<double>(P, S.n, q, X, B, ldb, st);
        } else {
            float *Y = (float *)base, *X = (float *)(base + vec), *Acc = (float *)(base + 2 * vec);
            spc::launch_perm_in<float>(P, S.n, q, B, ldb, Y, st);
            enqueue_solve<float>(S, P, (const float *)f->Lx, (const float *)f->Linv, Y, X, Acc, counters, wc, q,
                                 st);
            spc::launch_perm_out<float>(P, S.n, q, X, B, ldb, st);
        }
    }
    HIP_TRY(hipGetLastError());
    return SPC_OK;
}

void batch_release(spc_batch_s *b) {
    if (!b || b->refs.fetch_sub(1) != 1) return;
    if (b->F) spc_free_factor(b->F);
    if (b->vbuf) (void)hipFree(b->vbuf);
    if (b->bbuf) (void)hipFree(b->bbuf);
    if (b->meta) (void)hipFree(b->meta);
    if (b->rowseg) (void)hipFree(b->rowseg);
    if (b->merged) sym_release(b->merged);
    for (spc_symbolic_s *m : b->members) sym_release(m);
    b->magic = kDead;
    delete b;
}

bool batch_ok(spc_batch b) { return b && b->magic == 0x42415431u; }

}  // namespace

extern "C" {

int spc_analyze(int64_t n, const int64_t *h_colptr, const int32_t *h_rowidx, const int32_t *h_perm,
                const spc_options *opts, spc_symbolic *out) {
    if (!out) return SPC_INVALID_INPUT;
    *out = nullptr;
    spc_symbolic s = new (std::nothrow) spc_symbolic_s;
    if (!s) return SPC_OUT_OF_MEMORY;
    double z = opts ? opts->amalg_z : 0.05;
    if (std::isnan(z)) {
        delete s;
        return SPC_INVALID_INPUT;
    }
    spc::Tuning tu;
    if (opts) {
        // 0: default; < 0: off; > limit: invalid
        auto pick = [](int32_t v, int32_t def, int32_t lim, int32_t off, int32_t *out) {
            if (v == 0) *out = def;
            else if (v < 0) *out = off;
            else if (v > lim) return false;
            else *out = v;
            return true;
        };
        constexpr int32_t kNone = INT32_MAX;
        const bool ok = pick(opts->tiny_w, spc::kTinyW, spc::kTinyW, 0, &tu.tiny_w) &&
                        pick(opts->tiny_m, spc::kTinyM, spc::kTinyM, 0, &tu.tiny_m) &&
                        pick(opts->small_w, spc::kSmallW, spc::kSmallW, 0, &tu.small_w) &&
                        pick(opts->small_m, spc::kSmallM, spc::kSmallM, 0, &tu.small_m) &&
                        pick(opts->big_min, spc::kBigMin, kNone, kNone, &tu.big_min) &&
                        pick(opts->big_min_k, spc::kBigMinK, kNone, kNone, &tu.big_min_k) &&
                        pick(opts->solve_persist_max, spc::kSolvePersistMax, kNone, 0, &tu.solve_persist_max) &&
                        pick(opts->handover, 1, 2, 0, &tu.handover) &&
                        pick(opts->delay, spc::kDelay, spc::kDelayMax, spc::kDelay, &tu.delay) &&
                        pick(opts->persist, 0, 1, 0, &tu.persist) &&
                        pick(opts->ordering, 0, 2, 0, &tu.ordering) &&
                        pick(opts->group, 1, 1, 0, &tu.group) &&
                        pick(opts->bulk128, 0, 1, 0, &tu.bulk128) &&
                        pick(opts->lookahead, 0, 1, 0, &tu.lookahead);
        if (!ok) {
            delete s;
            return SPC_INVALID_INPUT;
        }
        s->hbm_budget = opts->hbm_budget;
    }
    int rc;
    std::vector<int32_t> computed;
    if (!h_perm && tu.ordering != 0 && n > 0) {
        if (!h_colptr || !h_rowidx) {
            delete s;
            return SPC_INVALID_INPUT;
        }
        try {
            computed.resize(n);
        } catch (const std::bad_alloc &) {
            delete s;
            return SPC_OUT_OF_MEMORY;
        }
        rc = spc_order(n, h_colptr, h_rowidx, tu.ordering, computed.data());
        if (rc != SPC_OK) {
            delete s;
            return rc;
        }
        h_perm = computed.data();
    }
    try {
        rc = spc::analyze(n, h_colptr, h_rowidx, h_perm, z, tu, s->S);
    } catch (const std::bad_alloc &) {
        rc = SPC_OUT_OF_MEMORY;
    } catch (...) {
        rc = SPC_INVALID_INPUT;
    }
    if (rc != SPC_OK) {
        delete s;
        return rc;
    }
    *out = s;
    return SPC_OK;
}

int spc_order(int64_t n, const int64_t *h_colptr, const int32_t *h_rowidx, int method, int32_t *h_perm) {
    if (n < 0 || (n > 0 && (!h_colptr || !h_rowidx || !h_perm)) || method < 0 || method > 2) return SPC_INVALID_INPUT;
    if (n == 0) return SPC_OK;
    if (n > INT32_MAX - 1 || h_colptr[0] != 0) return SPC_INVALID_INPUT;
    for (int64_t c = 0; c < n; ++c)
        if (h_colptr[c + 1] < h_colptr[c]) return SPC_INVALID_INPUT;
    int rc;
    try {
        rc = spc::order_graph(n, h_colptr, h_rowidx, method, h_perm);
    } catch (const std::bad_alloc &) {
        return SPC_OUT_OF_MEMORY;
    }
    if (rc != 0) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      method == 2 && n > 10000 ? "spc_order: minimum degree is for n <= 10000"
                                               : "spc_order: malformed pattern");
        return SPC_INVALID_INPUT;
    }
    return SPC_OK;
}

int spc_symbolic_info(spc_symbolic sym, spc_info *out) {
    if (!sym_ok(sym)) return SPC_BAD_HANDLE;
    if (!out) return SPC_INVALID_INPUT;
    const spc::Symbolic &S = sym->S;
    out->n = S.n;
    out->nnz_a = S.nnzA;
    out->nsuper = S.nsuper;
    out->nnz_l = S.nnzL;
    out->panel_entries = S.panel_entries();
    out->flops = S.flops;
    out->levels = S.nlevels;
    out->rows_total = S.rows_total();
    out->max_width = S.max_w;
    out->max_rows = S.max_m;
    out->factor_bytes_fp64 = factor_footprint(S, 8);
    out->factor_bytes_fp32 = factor_footprint(S, 4);
    out->solve_levels = S.nslevels;
    out->solve_persistent_levels = S.nslevels - S.solve_split;
    out->solve_block_tasks = (int64_t)S.stasks.size();
    out->solve_tiny_tasks = (int64_t)S.stiny.size();
    out->updates_total = (int64_t)S.pairs.size();
    out->solve_handovers = 0;
    for (const spc::SolveTask &t : S.stasks)
        if (t.first && (t.hand & spc::kHandOut)) out->solve_handovers++;
    return SPC_OK;
}

int spc_symbolic_verify(spc_symbolic sym) {
    if (!sym_ok(sym)) return SPC_BAD_HANDLE;
    std::string msg;
    if (spc::verify_schedule(sym->S, msg) == 0) return SPC_OK;
    std::snprintf(g_last_error, sizeof(g_last_error), "schedule: %s", msg.c_str());
    return SPC_INVALID_INPUT;
}

int spc_symbolic_export(spc_symbolic sym, int which, void *h_dst) {
    if (!sym_ok(sym)) return SPC_BAD_HANDLE;
    if (!h_dst) return SPC_INVALID_INPUT;
    const spc::Symbolic &S = sym->S;
    auto put = [&](const auto &v) {
        if (!v.empty()) std::memcpy(h_dst, v.data(), bytes_of(v));
        return SPC_OK;
    };
    switch (which) {
    case 0: return put(S.perm);
    case 1: return put(S.parent);
    case 2: return put(S.colcount);
    case 3: return put(S.super_ptr);
    case 4: return put(S.sparent);
    case 5: return put(S.rptr);
    case 6: return put(S.rows);
    case 7: return put(S.lptr);
    case 8: return put(S.level);
    case 9:
    case 10: {
        // the update lists U_t (Sec. 3, Listing 1: every earlier supernode
        // whose rows meet t's columns), ascending, as the transpose of the
        // scatter pairs (source s -> ancestor t)
        const int32_t ns = S.nsuper;
        std::vector<int64_t> uptr(ns + 1, 0);
        for (const spc::UpdatePair &q : S.pairs) uptr[q.target + 1]++;
        for (int32_t t = 0; t < ns; ++t) uptr[t + 1] += uptr[t];
        if (which == 9) return put(uptr);
        std::vector<int32_t> ulist(S.pairs.size());
        std::vector<int64_t> fill(uptr.begin(), uptr.end() - 1);
        for (int32_t src = 0; src < ns; ++src)  // ascending sources: each list comes out sorted
            for (int64_t k = S.pair_ptr[src]; k < S.pair_ptr[src + 1]; ++k) ulist[fill[S.pairs[k].target]++] = src;
        return put(ulist);
    }
    default: return SPC_INVALID_INPUT;
    }
}

int spc_factorize(spc_symbolic sym, const double *d_values, int precision, void *stream,
                  spc_factor *out) {
    if (!out) return SPC_INVALID_INPUT;
    *out = nullptr;
    if (!sym_ok(sym)) return SPC_BAD_HANDLE;
    if (!d_values && sym->S.nnzA > 0) return SPC_INVALID_INPUT;
    spc_factor f = nullptr;
    int rc = create_factor(sym, precision, &f);
    if (rc) return rc;
    rc = run_factor(f, d_values, (hipStream_t)stream);
    if (rc) {
        spc_free_factor(f);
        return rc;
    }
    *out = f;
    return SPC_OK;
}

int spc_refactorize(spc_factor f, const double *d_values, void *stream) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    if (f->batch) return SPC_INVALID_INPUT;  // refactor the batch instead
    if (!d_values && f->sym->S.nnzA > 0) return SPC_INVALID_INPUT;
    return run_factor(f, d_values, (hipStream_t)stream);
}

int spc_factorize_batch(int count, const spc_symbolic *syms, const double *const *d_values,
                        int precision, void *stream, spc_factor *outs) {
    if (count < 0 || (count > 0 && (!syms || !d_values || !outs))) return SPC_INVALID_INPUT;
    for (int i = 0; i < count; ++i) outs[i] = nullptr;
    if (count == 0) return SPC_OK;
    spc_batch b = nullptr;
    int rc = spc_batch_create(count, syms, precision, &b);
    if (rc) return rc;
    rc = spc_batch_factorize(b, d_values, stream);
    for (int i = 0; rc == SPC_OK && i < count; ++i) rc = spc_batch_factor(b, i, &outs[i]);
    if (rc)
        for (int i = 0; i < count; ++i) {
            spc_free_factor(outs[i]);
            outs[i] = nullptr;
        }
    spc_free_batch(b);  // the views keep the storage alive
    return rc;
}

int spc_solve(spc_factor f, double *d_B, int nrhs, int64_t ldb, void *stream) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    const spc::Symbolic &S = f->sym->S;
    if (nrhs < 0 || ldb < S.n || (!d_B && nrhs > 0 && S.n > 0)) return SPC_INVALID_INPUT;
    if (nrhs == 0 || S.n == 0) return SPC_OK;
    const size_t esz = f->precision == SPC_FP64 ? sizeof(double) : sizeof(float);
    const size_t need = solve_work_bytes(S, kSolveChunk, esz);
    int rc = ensure_bytes(&f->work, &f->work_bytes, need);
    if (rc) return rc;
    return solve_chunks(f, d_B, nrhs, ldb, (hipStream_t)stream, (char *)f->work, kSolveChunk);
}

int spc_solve_noalloc(spc_factor f, double *d_B, int nrhs, int64_t ldb, void *stream) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    const spc::Symbolic &S = f->sym->S;
    if (nrhs < 0 || ldb < S.n || (!d_B && nrhs > 0 && S.n > 0)) return SPC_INVALID_INPUT;
    if (nrhs == 0 || S.n == 0) return SPC_OK;
    const size_t esz = f->precision == SPC_FP64 ? sizeof(double) : sizeof(float);
    // the most right-hand sides per chunk whose work fits the scratch array
    int chunk = 0;
    while (chunk < kSolveChunk && solve_work_bytes(S, chunk + 1, esz) <= spc::kScratchBytes) ++chunk;
    if (chunk == 0) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "spc_solve_noalloc: one right-hand side needs %zu bytes of work, more than the %zu-byte "
                      "scratch array",
                      solve_work_bytes(S, 1, esz), (size_t)spc::kScratchBytes);
        return SPC_INVALID_INPUT;
    }
    void *scratch = nullptr;
    int rc = spc::scratch_address(f->device, &scratch);
    if (rc) {
        std::snprintf(g_last_error, sizeof(g_last_error), "spc_solve_noalloc: hipGetSymbolAddress of the scratch "
                                                          "array failed on device %d", f->device);
        return rc;
    }
    return solve_chunks(f, d_B, nrhs, ldb, (hipStream_t)stream, (char *)scratch, chunk);
}

int spc_solve_refined(spc_factor f, const double *d_values, const double *d_B, double *d_X, int nrhs,
                      int64_t ld, double tol, int maxit, void *stream, spc_refine_info *info) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    const spc::Symbolic &S = f->sym->S;
    const int64_t n = S.n;
    if (nrhs < 0 || ld < n || maxit < 0 || !(tol >= 0.0) || (n > 0 && nrhs > 0 && (!d_values || !d_B || !d_X)))
        return SPC_INVALID_INPUT;
    if (info) {
        info->iterations = 0;
        info->converged = 1;
        info->berr = 0.0;
    }
    if (n == 0 || nrhs == 0) return SPC_OK;
    hipStream_t st = (hipStream_t)stream;
    int rc = ensure_csr(f->sym);
    if (rc) return rc;
    int worst = 0;
    double worst_berr = 0.0;
    bool all_conv = true;
    for (int q0 = 0; q0 < nrhs; q0 += kRefineChunk) {
        const int q = std::min(kRefineChunk, nrhs - q0);
        RefineResult res;
        RefineTarget T;
        T.f = f;
        T.rp = f->sym->d_csr_ptr;
        T.vm = f->sym->d_csr_val;
        T.ci = f->sym->d_csr_col;
        T.values = d_values;
        T.n = n;
        T.nnz = f->sym->S.csr_ptr.empty() ? 0 : f->sym->S.csr_ptr.back();
        rc = refine_chunk(T, d_B + (int64_t)q0 * ld, d_X + (int64_t)q0 * ld, q, ld, tol, maxit, st, &res);
        if (rc) return rc;
        worst = std::max(worst, res.iterations);
        worst_berr = std::max(worst_berr, res.berr);
        all_conv = all_conv && res.converged;
    }
    if (info) {
        info->iterations = worst;
        info->converged = all_conv ? 1 : 0;
        info->berr = worst_berr;
    }
    return all_conv ? SPC_OK : SPC_NO_CONVERGENCE;
}

int spc_sync(spc_factor f, int64_t *bad_pivot) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    if (bad_pivot) *bad_pivot = -1;
    HIP_TRY(hipStreamSynchronize(f->batch ? f->batch->F->stream : f->stream));
    int rc = check_deverr(f);
    if (rc) return rc;
    unsigned long long v = 0;
    HIP_TRY(copy_sync(&v, f->status, sizeof(v), hipMemcpyDeviceToHost));
    if (v != ~0ull) {
        if (bad_pivot) *bad_pivot = (int64_t)v - f->status_col_off;
        return SPC_NOT_SPD;
    }
    return SPC_OK;
}

int spc_factor_export(spc_factor f, double *h_dst) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    if (!h_dst) return SPC_INVALID_INPUT;
    const spc::Symbolic &S = f->sym->S;
    HIP_TRY(hipStreamSynchronize(f->batch ? f->batch->F->stream : f->stream));
    int64_t cnt = S.panel_entries();
    if (f->precision == SPC_FP64) {
        HIP_TRY(copy_sync(h_dst, f->Lx, cnt * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(cnt);
        HIP_TRY(copy_sync(tmp.data(), f->Lx, cnt * sizeof(float), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < cnt; ++i) h_dst[i] = tmp[i];
    }
    for (int32_t s = 0; s < S.nsuper; ++s) {
        int64_t w = S.super_ptr[s + 1] - S.super_ptr[s], m = S.rptr[s + 1] - S.rptr[s];
        double *Pn = h_dst + S.lptr[s];
        for (int64_t c = 1; c < w; ++c)
            for (int64_t i = 0; i < c; ++i) Pn[c * m + i] = 0.0;
    }
    return SPC_OK;
}

int spc_factor_last_ms(spc_factor f, float *ms) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    if (!ms) return SPC_INVALID_INPUT;
    HIP_TRY(hipEventSynchronize(f->ev1));
    HIP_TRY(hipEventElapsedTime(ms, f->ev0, f->ev1));
    return SPC_OK;
}

int spc_factor_set_profiling(spc_factor f, int on) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    f->profiling = on != 0;
    return SPC_OK;
}

int spc_factor_kernel_stats(spc_factor f, int kernel_class, spc_kernel_stats *out) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    if (!out || kernel_class < 0 || kernel_class >= SPC_K_COUNT) return SPC_INVALID_INPUT;
    out->launches = 0;
    out->total_ms = 0.0;
    out->flops = 0.0;
    if (f->prof_used) HIP_TRY(hipEventSynchronize(f->prof_ev[2 * f->prof_used - 1]));
    for (size_t i = 0; i < f->prof_used; ++i) {
        if (f->prof_cls[i] != kernel_class) continue;
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, f->prof_ev[2 * i], f->prof_ev[2 * i + 1]));
        out->launches++;
        out->total_ms += ms;
        out->flops += f->prof_flops[i];
    }
    return SPC_OK;
}

int spc_factor_level_stats(spc_factor f, int level, spc_kernel_stats *out) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    if (!out || level < -2 || level >= f->sym->S.nlevels) return SPC_INVALID_INPUT;
    out->launches = 0;
    out->total_ms = 0.0;
    out->flops = 0.0;
    if (f->prof_used) HIP_TRY(hipEventSynchronize(f->prof_ev[2 * f->prof_used - 1]));
    for (size_t i = 0; i < f->prof_used; ++i) {
        if (f->prof_lvl[i] != level) continue;
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, f->prof_ev[2 * i], f->prof_ev[2 * i + 1]));
        out->launches++;
        out->total_ms += ms;
        out->flops += f->prof_flops[i];
    }
    return SPC_OK;
}

void spc_free_symbolic(spc_symbolic sym) {
    if (!sym_ok(sym)) return;
    sym_release(sym);
}

void spc_free_factor(spc_factor f) {
    if (!f || f->magic != kFacMagic) return;
    if (f->batch) {
        spc_batch_s *b = f->batch;
        if (f->work) (void)hipFree(f->work);
        if (f->refine) (void)hipFree(f->refine);
        if (f->refine_host) (void)hipHostFree(f->refine_host);
        spc_symbolic_s *s = f->sym;
        f->magic = kDead;
        delete f;
        if (s) sym_release(s);
        batch_release(b);
        return;
    }
    if (f->stream || f->Lx) (void)hipStreamSynchronize(f->stream);
    if (f->Lx) (void)hipFree(f->Lx);
    if (f->Linv) (void)hipFree(f->Linv);
    if (f->pfloor) (void)hipFree(f->pfloor);
    if (f->status) (void)hipFree(f->status);
    if (f->work) (void)hipFree(f->work);
    if (f->refine) (void)hipFree(f->refine);
    if (f->refine_host) (void)hipHostFree(f->refine_host);
    if (f->ev0) (void)hipEventDestroy(f->ev0);
    if (f->ev1) (void)hipEventDestroy(f->ev1);
    for (hipEvent_t e : f->prof_ev) (void)hipEventDestroy(e);
    drop_graph(f);
    if (f->cap_stream) (void)hipStreamDestroy(f->cap_stream);
    spc_symbolic_s *s = f->sym;
    f->magic = kDead;
    delete f;
    if (s) sym_release(s);
}

int spc_factor_set_graph(spc_factor f, int on) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    if (f->batch) return SPC_INVALID_INPUT;  // a batch view: spc_batch_set_graph
    f->use_graph = on != 0;
    if (!f->use_graph) drop_graph(f);
    return SPC_OK;
}

int spc_factor_pivot_floors(spc_factor f, int64_t *raised) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    if (!raised) return SPC_INVALID_INPUT;
    *raised = 0;
    spc_factor_s *o = owner_of(f);
    if (o->precision != SPC_FP32_BF16UPD) return SPC_OK;
    HIP_TRY(hipStreamSynchronize(o->stream));
    int32_t v = 0;
    HIP_TRY(copy_sync(&v, o->deverr + 1, sizeof(v), hipMemcpyDeviceToHost));
    *raised = v;
    return SPC_OK;
}

int spc_factor_set_wait_limit(spc_factor f, int32_t polls) {
    if (!fac_ok(f)) return SPC_BAD_HANDLE;
    if (f->batch || polls < 0) return SPC_INVALID_INPUT;
    f->spin = polls;
    drop_graph(f);  // a captured graph holds the old limit
    return SPC_OK;
}

int spc_batch_set_graph(spc_batch b, int on) {
    if (!batch_ok(b)) return SPC_BAD_HANDLE;
    b->F->use_graph = on != 0;
    if (!b->F->use_graph) drop_graph(b->F);
    return SPC_OK;
}


int spc_batch_create(int count, const spc_symbolic *syms, int precision, spc_batch *out) {
    if (!out) return SPC_INVALID_INPUT;
    *out = nullptr;
    if (count <= 0 || !syms || (precision != SPC_FP64 && precision != SPC_FP32 && precision != SPC_FP32_BF16UPD))
        return SPC_INVALID_INPUT;
    for (int i = 0; i < count; ++i)
        if (!sym_ok(syms[i])) return SPC_BAD_HANDLE;
    int dev = -1;
    int rc = check_device(&dev);
    if (rc) return rc;
    spc_batch_s *b = new (std::nothrow) spc_batch_s;
    if (!b) return SPC_OUT_OF_MEMORY;
    b->count = count;
    b->precision = precision;
    std::vector<const spc::Symbolic *> parts;
    for (int i = 0; i < count; ++i) {
        syms[i]->refs.fetch_add(1);
        b->members.push_back(syms[i]);
        parts.push_back(&syms[i]->S);
    }
    b->merged = new (std::nothrow) spc_symbolic_s;
    if (!b->merged) {
        batch_release(b);
        return SPC_OUT_OF_MEMORY;
    }
    try {
        rc = spc::merge(parts, b->merged->S, b->col_off, b->panel_off, b->inv_base, b->val_off);
    } catch (const std::bad_alloc &) {
        rc = SPC_OUT_OF_MEMORY;
    }
    for (int i = 0; i < count; ++i) {
        const int64_t bud = syms[i]->hbm_budget;
        if (bud > 0 && (b->merged->hbm_budget <= 0 || bud < b->merged->hbm_budget)) b->merged->hbm_budget = bud;
    }
    if (rc == SPC_OK) rc = create_factor(b->merged, precision, &b->F, count);
    if (rc == SPC_OK && hipMalloc((void **)&b->vbuf, std::max<int64_t>(1, b->val_off[count]) * sizeof(double)) !=
                            hipSuccess)
        rc = SPC_OUT_OF_MEMORY;
    // meta: pointer table [count], leading dims [count], row offsets
    // [count + 1], second pointer table [count]
    b->meta_bytes = 2 * sizeof(double *) * count + sizeof(int64_t) * (2 * count + 1);
    if (rc == SPC_OK && hipMalloc(&b->meta, b->meta_bytes) != hipSuccess) rc = SPC_OUT_OF_MEMORY;
    if (rc == SPC_OK &&
        copy_sync((char *)b->meta + sizeof(double *) * count + sizeof(int64_t) * count, b->col_off.data(),
                  sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice) != hipSuccess)
        rc = SPC_DEVICE_ERROR;
    if (rc) {
        batch_release(b);
        return rc;
    }
    *out = b;
    return SPC_OK;
}

int spc_batch_factorize(spc_batch b, const double *const *d_values, void *stream) {
    if (!batch_ok(b)) return SPC_BAD_HANDLE;
    if (!d_values) return SPC_INVALID_INPUT;
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < b->count; ++i) {
        const int64_t cnt = b->val_off[i + 1] - b->val_off[i];
        if (cnt == 0) continue;
        if (!d_values[i]) return SPC_INVALID_INPUT;
        HIP_TRY(hipMemcpyAsync(b->vbuf + b->val_off[i], d_values[i], cnt * sizeof(double), hipMemcpyDeviceToDevice,
                               st));
    }
    return run_factor(b->F, b->vbuf, st);
}

int spc_batch_factor(spc_batch b, int i, spc_factor *out) {
    if (!out) return SPC_INVALID_INPUT;
    *out = nullptr;
    if (!batch_ok(b)) return SPC_BAD_HANDLE;
    if (i < 0 || i >= b->count) return SPC_INVALID_INPUT;
    spc_symbolic_s *sym = b->members[i];
    int rc = ensure_device_plan(sym, b->F->device);
    if (rc) return rc;
    spc_factor f = new (std::nothrow) spc_factor_s;
    if (!f) return SPC_OUT_OF_MEMORY;
    const size_t esz = b->precision == SPC_FP64 ? sizeof(double) : sizeof(float);
    f->sym = sym;
    sym->refs.fetch_add(1);
    f->precision = b->precision;
    f->device = b->F->device;
    f->owns_storage = false;
    f->batch = b;
    b->refs.fetch_add(1);
    f->batch_index = i;
    f->Lx = (char *)b->F->Lx + b->panel_off[i] * esz;
    f->Linv = (char *)b->F->Linv + b->inv_base[i] * esz;
    f->status = b->F->status + i;
    f->status_col_off = b->col_off[i];
    f->stream = b->F->stream;
    *out = f;
    return SPC_OK;
}

int spc_batch_solve(spc_batch b, double *const *d_B, int nrhs, const int64_t *ldb, void *stream) {
    if (!batch_ok(b)) return SPC_BAD_HANDLE;
    if (nrhs < 0 || (nrhs > 0 && (!d_B || !ldb))) return SPC_INVALID_INPUT;
    if (nrhs == 0) return SPC_OK;
    for (int i = 0; i < b->count; ++i)
        if (ldb[i] < b->col_off[i + 1] - b->col_off[i] || (!d_B[i] && b->col_off[i + 1] > b->col_off[i]))
            return SPC_INVALID_INPUT;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = b->col_off[b->count];
    int rc = ensure_bytes((void **)&b->bbuf, &b->bbuf_bytes, (size_t)std::max<int64_t>(n, 1) * nrhs * sizeof(double));
    if (rc) return rc;
    char *meta = (char *)b->meta;
    double **ptrs = (double **)meta;
    int64_t *lds = (int64_t *)(meta + sizeof(double *) * b->count);
    int64_t *offs = lds + b->count;
    HIP_TRY(hipMemcpyAsync(ptrs, d_B, sizeof(double *) * b->count, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(lds, ldb, sizeof(int64_t) * b->count, hipMemcpyHostToDevice, st));
    spc::launch_batch_move(ptrs, lds, offs, b->bbuf, n, b->count, nrhs, true, st);
    rc = spc_solve(b->F, b->bbuf, nrhs, n, st);
    if (rc) return rc;
    spc::launch_batch_move(ptrs, lds, offs, b->bbuf, n, b->count, nrhs, false, st);
    HIP_TRY(hipGetLastError());
    // the pointer tables are read by the kernels above: wait before returning
    // so the caller may reuse its host arrays
    HIP_TRY(hipStreamSynchronize(st));
    return check_deverr(b->F);
}

int spc_batch_solve_refined(spc_batch b, const double *const *d_B, double *const *d_X, int nrhs, const int64_t *ld,
                            double tol, int maxit, void *stream, spc_refine_info *infos) {
    if (!batch_ok(b)) return SPC_BAD_HANDLE;
    if (nrhs < 0 || maxit < 0 || !(tol >= 0.0) || (nrhs > 0 && (!d_B || !d_X || !ld))) return SPC_INVALID_INPUT;
    const int cnt = b->count;
    if (nrhs > 0)
        for (int i = 0; i < cnt; ++i) {
            const int64_t ni = b->col_off[i + 1] - b->col_off[i];
            if (ld[i] < ni || (ni > 0 && (!d_B[i] || !d_X[i]))) return SPC_INVALID_INPUT;
        }
    if (infos)
        for (int i = 0; i < cnt; ++i) infos[i] = spc_refine_info{0, 1, 0.0};
    const int64_t n = b->col_off[cnt];
    if (nrhs == 0 || n == 0) return SPC_OK;
    hipStream_t st = (hipStream_t)stream;
    int rc = ensure_csr(b->merged);
    if (rc) return rc;
    if (!b->rowseg) {
        std::vector<int32_t> seg(n);
        for (int i = 0; i < cnt; ++i)
            std::fill(seg.begin() + b->col_off[i], seg.begin() + b->col_off[i + 1], (int32_t)i);
        int32_t *d = nullptr;
        HIP_TRY(hipMalloc((void **)&d, n * sizeof(int32_t)));
        hipError_t e = copy_sync(d, seg.data(), n * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return record_error(e, "row systems upload", __LINE__);
        }
        b->rowseg = d;
    }
    rc = ensure_bytes((void **)&b->bbuf, &b->bbuf_bytes, (size_t)n * nrhs * sizeof(double));
    if (rc) return rc;
    char *meta = (char *)b->meta;
    double **ptrs = (double **)meta;
    int64_t *lds = (int64_t *)(meta + sizeof(double *) * cnt);
    int64_t *offs = lds + cnt;
    double **xptrs = (double **)(offs + cnt + 1);
    HIP_TRY(hipMemcpyAsync(ptrs, d_B, sizeof(double *) * cnt, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(xptrs, d_X, sizeof(double *) * cnt, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(lds, ld, sizeof(int64_t) * cnt, hipMemcpyHostToDevice, st));
    spc::launch_batch_move(ptrs, lds, offs, b->bbuf, n, cnt, nrhs, true, st);
    RefineTarget T;
    T.f = b->F;
    T.rp = b->merged->d_csr_ptr;
    T.vm = b->merged->d_csr_val;
    T.ci = b->merged->d_csr_col;
    T.values = b->vbuf;
    T.n = n;
    T.nnz = b->merged->S.csr_ptr.empty() ? 0 : b->merged->S.csr_ptr.back();
    T.seg = b->rowseg;
    T.nseg = cnt;
    std::vector<RefineResult> res(cnt);
    bool all_conv = true;
    for (int q0 = 0; q0 < nrhs; q0 += kRefineChunk) {
        const int q = std::min(kRefineChunk, nrhs - q0);
        std::vector<RefineResult> part(cnt);
        double *Bq = b->bbuf + (int64_t)q0 * n;
        rc = refine_chunk(T, Bq, Bq, q, n, tol, maxit, st, part.data());
        if (rc) return rc;
        for (int i = 0; i < cnt; ++i) {
            res[i].iterations = std::max(res[i].iterations, part[i].iterations);
            res[i].berr = std::max(res[i].berr, part[i].berr);
            res[i].converged = (q0 == 0 || res[i].converged) && part[i].converged;
            all_conv = all_conv && part[i].converged;
        }
    }
    spc::launch_batch_move(xptrs, lds, offs, b->bbuf, n, cnt, nrhs, false, st);
    HIP_TRY(hipGetLastError());
    // the pointer tables are read by the kernels above
    HIP_TRY(hipStreamSynchronize(st));
    if (infos)
        for (int i = 0; i < cnt; ++i)
            infos[i] = spc_refine_info{res[i].iterations, res[i].converged ? 1 : 0, res[i].berr};
    return all_conv ? SPC_OK : SPC_NO_CONVERGENCE;
}

int spc_batch_sync(spc_batch b, int64_t *bad_system, int64_t *bad_pivot) {
    if (!batch_ok(b)) return SPC_BAD_HANDLE;
    if (bad_system) *bad_system = -1;
    if (bad_pivot) *bad_pivot = -1;
    HIP_TRY(hipStreamSynchronize(b->F->stream));
    int rc = check_deverr(b->F);
    if (rc) return rc;
    std::vector<unsigned long long> v(b->count);
    HIP_TRY(copy_sync(v.data(), b->F->status, sizeof(unsigned long long) * b->count, hipMemcpyDeviceToHost));
    for (int i = 0; i < b->count; ++i)
        if (v[i] != ~0ull) {
            if (bad_system) *bad_system = i;
            if (bad_pivot) *bad_pivot = (int64_t)v[i] - b->col_off[i];
            return SPC_NOT_SPD;
        }
    return SPC_OK;
}

int spc_batch_last_ms(spc_batch b, float *ms) {
    if (!batch_ok(b)) return SPC_BAD_HANDLE;
    return spc_factor_last_ms(b->F, ms);
}

int spc_batch_set_profiling(spc_batch b, int on) {
    if (!batch_ok(b)) return SPC_BAD_HANDLE;
    return spc_factor_set_profiling(b->F, on);
}

int spc_batch_kernel_stats(spc_batch b, int kernel_class, spc_kernel_stats *out) {
    if (!batch_ok(b)) return SPC_BAD_HANDLE;
    return spc_factor_kernel_stats(b->F, kernel_class, out);
}

int spc_batch_level_stats(spc_batch b, int level, spc_kernel_stats *out) {
    if (!batch_ok(b)) return SPC_BAD_HANDLE;
    return spc_factor_level_stats(b->F, level, out);
}

int spc_batch_info(spc_batch b, spc_info *out) {
    if (!batch_ok(b)) return SPC_BAD_HANDLE;
    return spc_symbolic_info(b->merged, out);
}

void spc_free_batch(spc_batch b) {
    if (!batch_ok(b)) return;
    batch_release(b);
}

const char *spc_last_error_message(void) { return g_last_error; }

const char *spc_status_string(int status) {
    switch (status) {
    case SPC_OK: return "ok";
    case SPC_INVALID_INPUT: return "invalid input";
    case SPC_NOT_SPD: return "matrix is not positive definite";
    case SPC_OUT_OF_MEMORY: return "out of memory";
    case SPC_NO_CONVERGENCE: return "refinement did not converge";
    case SPC_DEVICE_ERROR: return "device error";
    case SPC_BAD_HANDLE: return "bad handle";
    case SPC_NO_DEVICE: return "no gfx950 device";
    default: return "unknown status";
    }
}

}  // extern "C"
