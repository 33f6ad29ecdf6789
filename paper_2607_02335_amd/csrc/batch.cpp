// Batched launches over independent problems, the tile-shape autotuner, and
// the continuous-batching solve server.
//
// A batched launch covers many problems: one launch per degree (the kernels
// walk a concatenated tile range and find each tile's problem in a device
// table), or, for the degrees 2, 3 and 7, one mixed-degree launch per phase
// whose workgroups each run one degree's kernel body.  The server keeps every
// admitted solve's vectors and scalars on the device and advances all of
// them with such launches; requests are admitted in arrival order as slots
// and device memory free up.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "fem_internal.h"
#include "host_api.h"
#include "launch.h"

using namespace fem;

static void destroy_problem_internal(fem_problem* P) {
    if (!P) return;
    P->owned_by_batch = false;
    fem_problem_destroy(P);
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
static size_t pbytes(int prec) { return prec == FEM_F64 ? 8 : prec == FEM_F32 ? 4 : 2; }

static ProbEntry pi_entry(fem_problem* P, const void* r, void* z, int prec, double alpha) {
    ProbEntry e = entry_of(P);
    e.a = r;
    e.c = z;
    e.d = P->d_patch;
    e.e = P->d_glob;
    e.alpha = alpha;
    for (int k = 0; k < 3; ++k)
        e.fd[k] = prec == FEM_F64 ? (const void*)(P->d_fd64 + k * P->fd_dir_stride)
                                  : (const void*)(P->d_fd32 + k * P->fd_dir_stride);
    return e;
}

// ===================================================================== batch
struct fem_batch {
    int count = 0;
    hipStream_t stream = nullptr;
    std::vector<fem_problem*> probs;
    std::vector<int> group[kMaxP + 1];
    LaunchCfg cfg_apply[kMaxP + 1];
    LaunchCfg cfg_pi[kMaxP + 1];
    int mixed = 1;          // mixed-degree launches (default kernel shapes) where the degrees allow
    TableStager st;
};

// The batch's degrees allow a mixed launch: two or three of {2, 3, 7} and no other.
static bool batch_mixable(const fem_batch* B) {
    int present = 0;
    for (int p = 1; p <= kMaxP; ++p) {
        if (B->group[p].empty()) continue;
        if (p != 2 && p != 3 && p != 7) return false;
        ++present;
    }
    return present >= 2;
}

extern "C" fem_status fem_batch_create(int count, const fem_desc* descs, void* stream, fem_batch** out) {
    if (!out) return set_error(FEM_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !descs) return set_error(FEM_EINVAL, "fem_batch_create: count >= 1 and descs required");
    for (int i = 0; i < count; ++i) {
        fem_status st = check_desc(&descs[i]);
        if (st != FEM_OK) return st;
    }
    fem_batch* B = new (std::nothrow) fem_batch();
    if (!B) return set_error(FEM_ENOMEM, "host allocation failed");
    B->count = count;
    B->stream = static_cast<hipStream_t>(stream);
    hipError_t e = B->st.init(2 * count);
    if (e != hipSuccess) {
        B->st.destroy();
        delete B;
        return set_error(FEM_ENOMEM, "fem_batch_create: table staging allocation failed");
    }
    for (int i = 0; i < count; ++i) {
        fem_problem* P = nullptr;
        fem_status st = create_problem(&descs[i], B->stream, &P);
        if (st != FEM_OK) {
            for (fem_problem* Q : B->probs) destroy_problem_internal(Q);
            B->st.destroy();
            delete B;
            return st;
        }
        P->owned_by_batch = true;
        B->probs.push_back(P);
        B->group[P->p].push_back(i);
    }
    *out = B;
    return FEM_OK;
}

extern "C" fem_status fem_batch_destroy(fem_batch* B) {
    if (!B) return FEM_OK;
    hipStreamSynchronize(B->stream);
    for (fem_problem* P : B->probs) destroy_problem_internal(P);
    B->st.destroy();
    delete B;
    return FEM_OK;
}

extern "C" fem_status fem_batch_problem(fem_batch* B, int i, fem_problem** out) {
    if (!B || !out || i < 0 || i >= B->count) return set_error(FEM_EINVAL, "fem_batch_problem: bad index");
    *out = B->probs[i];
    return FEM_OK;
}

static fem_status batch_apply_cfg(fem_batch* B, void* const* x, void* const* y, int prec, const LaunchCfg* cfgs) {
    std::vector<ProbEntry> ents;
    if (B->mixed && batch_mixable(B)) {
        for (int i = 0; i < B->count; ++i) {
            if (!x[i] || !y[i] || x[i] == y[i]) return set_error(FEM_EINVAL, "fem_batch_apply: bad vector pointers");
            ProbEntry e = entry_of(B->probs[i]);
            e.a = x[i];
            e.c = y[i];
            ents.push_back(e);
        }
        FEM_HIP(launch_apply_any(prec, 0, ents.data(), (int)ents.size(), &B->st, B->stream), "fem_batch_apply");
        return FEM_OK;
    }
    for (int p = 1; p <= kMaxP; ++p) {
        if (B->group[p].empty()) continue;
        ents.clear();
        for (int i : B->group[p]) {
            if (!x[i] || !y[i] || x[i] == y[i]) return set_error(FEM_EINVAL, "fem_batch_apply: bad vector pointers");
            ProbEntry e = entry_of(B->probs[i]);
            e.a = x[i];
            e.c = y[i];
            ents.push_back(e);
        }
        FEM_HIP(launch_apply(p, prec, 0, ents.data(), (int)ents.size(), &B->st, B->stream, cfgs[p]),
                "fem_batch_apply");
    }
    return FEM_OK;
}

static fem_status batch_pi_cfg(fem_batch* B, void* const* r, void* const* z, int prec, const LaunchCfg* cfgs) {
    std::vector<ProbEntry> ents;
    if (B->mixed && batch_mixable(B)) {
        for (int i = 0; i < B->count; ++i) {
            if (!r[i] || !z[i] || r[i] == z[i]) return set_error(FEM_EINVAL, "fem_batch_patch_inverse: bad pointers");
            ents.push_back(pi_entry(B->probs[i], r[i], z[i], prec, 1.0));
        }
        FEM_HIP(launch_patch_inverse_any(prec, 0, ents.data(), (int)ents.size(), &B->st, B->stream),
                "fem_batch_patch_inverse");
        return FEM_OK;
    }
    for (int p = 1; p <= kMaxP; ++p) {
        if (B->group[p].empty()) continue;
        ents.clear();
        for (int i : B->group[p]) {
            if (!r[i] || !z[i] || r[i] == z[i]) return set_error(FEM_EINVAL, "fem_batch_patch_inverse: bad pointers");
            ents.push_back(pi_entry(B->probs[i], r[i], z[i], prec, 1.0));
        }
        FEM_HIP(launch_patch_inverse(p, prec, 0, ents.data(), (int)ents.size(), &B->st, B->stream, cfgs[p]),
                "fem_batch_patch_inverse");
    }
    return FEM_OK;
}

extern "C" fem_status fem_batch_set_mixed(fem_batch* B, int mixed) {
    if (!B) return set_error(FEM_EINVAL, "fem_batch_set_mixed: NULL batch");
    B->mixed = mixed ? 1 : 0;
    return FEM_OK;
}

extern "C" int fem_batch_mixed(const fem_batch* B) { return B && B->mixed && batch_mixable(B) ? 1 : 0; }

extern "C" fem_status fem_batch_apply(fem_batch* B, void* const* x, void* const* y, int prec) {
    if (!B || !x || !y) return set_error(FEM_EINVAL, "fem_batch_apply: NULL argument");
    if (prec < FEM_F64 || prec > FEM_F16) return set_error(FEM_EINVAL, "unknown precision");
    return batch_apply_cfg(B, x, y, prec, B->cfg_apply);
}

extern "C" fem_status fem_batch_patch_inverse(fem_batch* B, void* const* r, void* const* z, int prec) {
    if (!B || !r || !z) return set_error(FEM_EINVAL, "fem_batch_patch_inverse: NULL argument");
    if (prec < FEM_F64 || prec > FEM_F16) return set_error(FEM_EINVAL, "unknown precision");
    return batch_pi_cfg(B, r, z, prec, B->cfg_pi);
}

// Autotuner: for each degree present, time every candidate kernel shape on
// this batch's own problems (all problems of that degree in one launch) and
// keep the fastest.  Candidates: apply = {register/LDS kernel} x {grid cap};
// patch inverse = {two-phase, fused sweep (p <= 3)} x {grid cap}.
extern "C" fem_status fem_batch_autotune(fem_batch* B, int prec, int* choice) {
    if (!B) return set_error(FEM_EINVAL, "fem_batch_autotune: NULL batch");
    if (prec < FEM_F64 || prec > FEM_F16) return set_error(FEM_EINVAL, "unknown precision");
    const int caps[2] = {kMaxGrid, 4 * 256};
    std::vector<void*> x(B->count), y(B->count);
    for (int i = 0; i < B->count; ++i) {
        const size_t bytes = align256(B->probs[i]->cell_len * pbytes(prec));
        if (hipMalloc(&x[i], bytes) != hipSuccess || hipMalloc(&y[i], bytes) != hipSuccess) {
            for (void* v : x) hipFree(v);
            for (void* v : y) hipFree(v);
            return set_error(FEM_ENOMEM, "fem_batch_autotune: scratch allocation failed");
        }
        hipMemsetAsync(x[i], 0, bytes, B->stream);
        hipMemsetAsync(y[i], 0, bytes, B->stream);
    }
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    fem_status result = FEM_OK;
    B->mixed = 0;                 // per-degree shapes are tuned with one launch per degree
    for (int p = 1; p <= kMaxP && result == FEM_OK; ++p) {
        if (B->group[p].empty()) continue;
        for (int which = 0; which < 2 && result == FEM_OK; ++which) {
            // apply: 0 = register (p <= 3) / plane-streamed (p >= 4; matrix-core
            //        for p = 7 in FP64) kernel, 1 = LDS line kernel,
            //        2 = plane-streamed (p = 7);
            // patch inverse, p <= 3: 0 = two launches through the patch buffer,
            //        1 = fused sweep summing cell copies, 2 = fused sweep from the
            //        assembled residual, 3 = solves with the in-tile x-combine,
            //        4 = the same with one wavefront per tile;
            //        p >= 4: 0 = MFMA solves, 2 = line solves
            std::vector<int> kinds = which == 0 ? (p == 7 ? std::vector<int>{0, 1, 2} : std::vector<int>{0, 1})
                                   : (p <= 3 ? std::vector<int>{0, 1, 2, 3, 4} : std::vector<int>{0, 2});
            std::vector<LaunchCfg> cand;
            for (int kind : kinds) {
                for (int c : caps) {
                    LaunchCfg cfg;
                    cfg.grid_cap = c;
                    if (which == 0) cfg.apply_lds = kind; else cfg.pi_fused = kind;
                    cand.push_back(cfg);
                }
            }
            float best = 1e30f;
            int best_i = 0;
            for (size_t ci = 0; ci < cand.size(); ++ci) {
                LaunchCfg cfgs[kMaxP + 1];
                for (int q = 0; q <= kMaxP; ++q) cfgs[q] = which == 0 ? B->cfg_apply[q] : B->cfg_pi[q];
                cfgs[p] = cand[ci];
                // only this degree's problems take part
                std::vector<int> saved[kMaxP + 1];
                for (int q = 1; q <= kMaxP; ++q)
                    if (q != p) std::swap(saved[q], B->group[q]);
                auto run = [&]() {
                    return which == 0 ? batch_apply_cfg(B, x.data(), y.data(), prec, cfgs)
                                      : batch_pi_cfg(B, x.data(), y.data(), prec, cfgs);
                };
                fem_status st = run();                                // warm
                const int reps = 3;
                hipEventRecord(e0, B->stream);
                for (int r = 0; r < reps && st == FEM_OK; ++r) st = run();
                hipEventRecord(e1, B->stream);
                hipEventSynchronize(e1);
                for (int q = 1; q <= kMaxP; ++q)
                    if (q != p) std::swap(saved[q], B->group[q]);
                if (st != FEM_OK) {
                    result = st;
                    break;
                }
                float ms = 0;
                hipEventElapsedTime(&ms, e0, e1);
                if (ms < best) {
                    best = ms;
                    best_i = (int)ci;
                }
            }
            if (result != FEM_OK) break;
            if (which == 0) B->cfg_apply[p] = cand[best_i]; else B->cfg_pi[p] = cand[best_i];
            if (choice) choice[2 * (p - 1) + which] = best_i;
        }
    }
    // then the whole pass (apply + patch inverse): the tuned per-degree
    // launches against the mixed-degree launches, the faster one is kept
    if (result == FEM_OK && batch_mixable(B)) {
        float t[2] = {0.f, 0.f};
        for (int m = 0; m < 2 && result == FEM_OK; ++m) {
            B->mixed = m;
            auto run = [&]() {
                fem_status st = batch_apply_cfg(B, x.data(), y.data(), prec, B->cfg_apply);
                return st == FEM_OK ? batch_pi_cfg(B, y.data(), x.data(), prec, B->cfg_pi) : st;
            };
            fem_status st = run();
            hipEventRecord(e0, B->stream);
            for (int r = 0; r < 3 && st == FEM_OK; ++r) st = run();
            hipEventRecord(e1, B->stream);
            hipEventSynchronize(e1);
            if (st != FEM_OK) result = st;
            hipEventElapsedTime(&t[m], e0, e1);
        }
        B->mixed = t[1] <= t[0] ? 1 : 0;
    } else {
        B->mixed = 1;
    }
    hipStreamSynchronize(B->stream);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    for (void* v : x) hipFree(v);
    for (void* v : y) hipFree(v);
    return result;
}

// ===================================================================== server
namespace {

struct Request {
    uint64_t ticket = 0;
    fem_desc desc{};
    std::vector<double> widths[3];
    std::vector<double> f;
    double rtol = 1e-8;
    int maxit = 1000;
    size_t footprint = 0;
    std::chrono::steady_clock::time_point t_admit;
};

struct Active {
    Request req;
    fem_problem* P = nullptr;
    char* mem = nullptr;        // solve vectors, after the problem workspace in the block
    size_t block_off = 0;       // the solve's block in the server arena
    size_t block_bytes = 0;
    double *u = nullptr, *b = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
    void* z = nullptr;
    void* rs = nullptr;
    int iters = 0;
    bool finished = false;
    int status = FEM_OK;
    double relres = 1.0;
};

struct Done {
    std::vector<double> u;
    fem_solve_info info{};
};

}  // namespace

struct fem_server {
    // guards the request queue, the ticket states, the finished results and
    // the memory counters: submit/poll/finished/memory may run on other host
    // threads than fem_server_step (which holds it only for short updates)
    std::mutex mu;
    size_t budget = 0, in_use = 0, high_water = 0;
    int max_active = 0;
    int sp = FEM_F32, sweeps = 2, variant = FEM_CG_FCG;
    int pc = FEM_PC_SCHWARZ;       // FEM_PC_SCHWARZ or FEM_PC_TWO_LEVEL
    double omega = 0.125;
    std::atomic<int> mix{1};       // mixed-degree launches (set from any thread)
    hipStream_t stream = nullptr;
    uint64_t next_ticket = 1;
    std::deque<Request> queue;
    std::vector<Active*> active;
    std::unordered_map<uint64_t, Done> done;
    std::unordered_map<uint64_t, int> state;      // 0 queued, 1 active, 2 done
    TableStager st;
    double* d_collect = nullptr;
    double* h_collect = nullptr;
    // device arena (one allocation of the budget) with a first-fit free list
    // of (offset -> bytes), coalesced on release
    char* arena = nullptr;
    std::map<size_t, size_t> free_blocks;
    // pinned staging for uploads (request right-hand sides at admission,
    // set-up data at activation): two bump regions used by alternate steps.
    // A step's region is free again two steps later, its copies having been
    // consumed before that step's scalar read-back completed.
    char* stage_buf[2] = {nullptr, nullptr};
    size_t stage_capv[2] = {0, 0};
    int cur = 0;
    char* stage = nullptr;
    size_t stage_cap = 0, stage_used = 0;
    // admitted solves whose right-hand sides are being uploaded (event ev_up)
    std::vector<Active*> staged;
    // solves whose solutions are being copied out: one batch per step, each
    // with its own pinned buffer and event, handed over once complete
    struct RetireBatch {
        std::vector<Active*> fin;
        std::vector<size_t> at;        // offset of each solution in buf
        char* buf = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
    };
    std::deque<RetireBatch> rbatches;
    std::vector<std::pair<char*, size_t>> rpool;   // free pinned download buffers
    std::vector<hipEvent_t> evpool;
    hipEvent_t ev_scalars = nullptr;
    // request uploads and solution downloads run on their own stream (at the
    // default priority), ordered against the compute stream by events, so
    // the copy engine overlaps the iterations of the other solves
    hipStream_t copy = nullptr;
    hipEvent_t ev_up = nullptr, ev_ext = nullptr;
    // host seconds per step phase: admission, launches, waits for the
    // scalars, retirement hand-over, retirement start; and steps taken
    double t_phase[5] = {0, 0, 0, 0, 0};
    long steps = 0;
};

namespace {
struct PhaseClock {
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    double lap() {
        const auto n = std::chrono::steady_clock::now();
        const double d = std::chrono::duration<double>(n - t).count();
        t = n;
        return d;
    }
};
}  // namespace

static bool arena_alloc(fem_server* S, size_t bytes, size_t* off) {
    for (auto it = S->free_blocks.begin(); it != S->free_blocks.end(); ++it) {
        if (it->second < bytes) continue;
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        S->free_blocks.erase(it);
        if (rest) S->free_blocks[at] = rest;
        return true;
    }
    return false;
}

static void arena_free(fem_server* S, size_t off, size_t bytes) {
    auto it = S->free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != S->free_blocks.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        S->free_blocks.erase(nx);
    }
    if (it != S->free_blocks.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            S->free_blocks.erase(it);
        }
    }
}

// Reserve pinned staging bytes for this step; grows the staging (after a
// stream synchronisation, so no copy still reads the old one).
static char* stage_take(fem_server* S, size_t bytes) {
    bytes = align256(bytes);
    if (S->stage_used + bytes > S->stage_cap) {
        if (S->stage_used > 0) return nullptr;          // caller retries next step
        if (hipStreamSynchronize(S->stream) != hipSuccess || hipStreamSynchronize(S->copy) != hipSuccess)
            return nullptr;
        if (S->stage) hipHostFree(S->stage);
        S->stage = nullptr;
        S->stage_cap = 0;
        size_t cap = std::max<size_t>(bytes, 64u << 20);
        if (hipHostMalloc((void**)&S->stage, cap, hipHostMallocDefault) != hipSuccess) {
            S->stage_buf[S->cur] = nullptr;
            S->stage_capv[S->cur] = 0;
            return nullptr;
        }
        S->stage_cap = cap;
        S->stage_buf[S->cur] = S->stage;
        S->stage_capv[S->cur] = cap;
    }
    char* q = S->stage + S->stage_used;
    S->stage_used += bytes;
    return q;
}

// Bytes of one solve's block: problem workspace, then u, b, r, p, q (FP64)
// and z, rs (smoother precision).
static size_t solve_block_bytes(const fem_desc* d, int sp) { return fem_footprint_bytes(d, sp); }

extern "C" fem_status fem_server_create(size_t hbm_budget, int max_active, int smoother_prec, int sweeps,
                                        double omega, void* stream, fem_server** out) {
    return fem_server_create_pc(hbm_budget, max_active, FEM_PC_SCHWARZ, smoother_prec, sweeps, omega, stream, out);
}

extern "C" fem_status fem_server_create_pc(size_t hbm_budget, int max_active, int precond, int smoother_prec,
                                           int sweeps, double omega, void* stream, fem_server** out) {
    if (!out) return set_error(FEM_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_active < 1 || sweeps < 1 || smoother_prec < FEM_F64 || smoother_prec > FEM_F16 || !std::isfinite(omega))
        return set_error(FEM_EINVAL, "fem_server_create: bad arguments");
    if (precond != FEM_PC_SCHWARZ && precond != FEM_PC_TWO_LEVEL)
        return set_error(FEM_EINVAL, "fem_server_create: preconditioner must be FEM_PC_SCHWARZ or FEM_PC_TWO_LEVEL");
    fem_server* S = new (std::nothrow) fem_server();
    if (!S) return set_error(FEM_ENOMEM, "host allocation failed");
    S->pc = precond;
    S->budget = hbm_budget;
    S->max_active = max_active;
    S->sp = smoother_prec;
    S->sweeps = sweeps;
    S->omega = omega;
    S->variant = smoother_prec == FEM_F64 ? FEM_CG_PCG : FEM_CG_FCG;
    S->stream = static_cast<hipStream_t>(stream);
    const char* what = nullptr;
    hipError_t herr = hipSuccess;
    if ((herr = S->st.init(2 * max_active)) != hipSuccess) what = "entry tables";
    else if ((herr = hipMalloc((void**)&S->d_collect, sizeof(double) * 4 * max_active)) != hipSuccess)
        what = "scalar read-back";
    else if ((herr = hipHostMalloc((void**)&S->h_collect, sizeof(double) * 4 * max_active, hipHostMallocDefault)) !=
             hipSuccess)
        what = "pinned scalar read-back";
    else if ((herr = hipMalloc((void**)&S->arena, hbm_budget)) != hipSuccess) what = "arena of hbm_budget bytes";
    else if ((herr = hipEventCreateWithFlags(&S->ev_scalars, hipEventDisableTiming)) != hipSuccess ||
             (herr = hipEventCreateWithFlags(&S->ev_up, hipEventDisableTiming)) != hipSuccess ||
             (herr = hipEventCreateWithFlags(&S->ev_ext, hipEventDisableTiming)) != hipSuccess)
        what = "events";
    else if ((herr = hipStreamCreateWithFlags(&S->copy, hipStreamNonBlocking)) != hipSuccess) what = "copy stream";
    if (what) {
        hipGetLastError();
        const std::string msg =
            std::string("fem_server_create: allocation failed (") + what + ": " + hipGetErrorString(herr) + ")";
        S->st.destroy();
        hipFree(S->d_collect);
        if (S->h_collect) hipHostFree(S->h_collect);
        if (S->arena) hipFree(S->arena);
        if (S->ev_scalars) hipEventDestroy(S->ev_scalars);
        if (S->ev_up) hipEventDestroy(S->ev_up);
        if (S->ev_ext) hipEventDestroy(S->ev_ext);
        if (S->copy) hipStreamDestroy(S->copy);
        delete S;
        return set_error(FEM_ENOMEM, msg.c_str());
    }
    S->free_blocks[0] = hbm_budget;
    *out = S;
    return FEM_OK;
}

static void release_active(fem_server* S, Active* A) {
    // the solve's last work (its download) has completed: no stream wait
    destroy_problem_nosync(A->P);
    arena_free(S, A->block_off, A->block_bytes);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->in_use -= A->block_bytes;
    }
    delete A;
}

extern "C" fem_status fem_server_destroy(fem_server* S) {
    if (!S) return FEM_OK;
    hipStreamSynchronize(S->stream);
    hipStreamSynchronize(S->copy);
    for (Active* A : S->active) release_active(S, A);
    S->st.destroy();
    hipFree(S->d_collect);
    hipHostFree(S->h_collect);
    for (auto& b : S->rbatches) {
        for (Active* A : b.fin) release_active(S, A);
        hipHostFree(b.buf);
        hipEventDestroy(b.ev);
    }
    for (auto& pb : S->rpool) hipHostFree(pb.first);
    for (hipEvent_t e : S->evpool) hipEventDestroy(e);
    for (Active* A : S->staged) release_active(S, A);
    hipFree(S->arena);
    for (int k = 0; k < 2; ++k)
        if (S->stage_buf[k]) hipHostFree(S->stage_buf[k]);
    hipEventDestroy(S->ev_scalars);
    hipEventDestroy(S->ev_up);
    hipEventDestroy(S->ev_ext);
    hipStreamDestroy(S->copy);
    delete S;
    return FEM_OK;
}

extern "C" fem_status fem_server_submit(fem_server* S, const fem_desc* desc, const double* f_glob, double rtol,
                                        int maxit, uint64_t* ticket) {
    if (!S || !desc || !f_glob || !ticket) return set_error(FEM_EINVAL, "fem_server_submit: NULL argument");
    fem_status st = check_desc(desc);
    if (st != FEM_OK) return st;
    if (!(rtol > 0) || maxit < 1) return set_error(FEM_EINVAL, "fem_server_submit: rtol > 0 and maxit >= 1");
    if (desc->bc != FEM_BC_DIRICHLET) return set_error(FEM_EINVAL, "fem_server_submit: Dirichlet problems only");
    Request R;
    R.desc = *desc;
    for (int k = 0; k < 3; ++k) {
        if (desc->widths[k]) {
            R.widths[k].assign(desc->widths[k], desc->widths[k] + desc->n[k]);
            R.desc.widths[k] = nullptr;
        }
    }
    R.footprint = fem_footprint_bytes(desc, S->sp);
    if (R.footprint > S->budget) return set_error(FEM_ENOMEM, "fem_server_submit: request exceeds the memory budget");
    const size_t glen = (size_t)(desc->n[0] * desc->p + 1) * (desc->n[1] * desc->p + 1) * (desc->n[2] * desc->p + 1);
    R.f.assign(f_glob, f_glob + glen);
    R.rtol = rtol;
    R.maxit = maxit;
    std::lock_guard<std::mutex> lk(S->mu);
    R.ticket = S->next_ticket++;
    *ticket = R.ticket;
    S->state[R.ticket] = 0;
    S->queue.push_back(std::move(R));
    return FEM_OK;
}

// Admission: carve the solve's block from the arena, form b = P_I M f, and
// run the iteration's start (r = b, z = P(r), p = z, <r,z>) with
// single-problem launches on the server stream.  Returns FEM_EAGAIN (and
// leaves R untouched) when the arena has no free block of the size yet or
// this step's pinned staging is used up.
static fem_status admit(fem_server* S, Request& R) {
    fem_desc d = R.desc;
    for (int k = 0; k < 3; ++k) d.widths[k] = R.widths[k].empty() ? nullptr : R.widths[k].data();
    const size_t need = solve_block_bytes(&d, S->sp);
    size_t off = 0;
    if (S->in_use + need > S->budget || !arena_alloc(S, need, &off)) return FEM_EAGAIN;
    char* hf = stage_take(S, sizeof(double) * R.f.size());
    if (!hf) {
        arena_free(S, off, need);
        return FEM_EAGAIN;
    }
    Active* A = new (std::nothrow) Active();
    if (!A) {
        arena_free(S, off, need);
        return set_error(FEM_ENOMEM, "host allocation failed");
    }
    A->req = std::move(R);
    A->block_off = off;
    A->block_bytes = need;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->in_use += need;
        S->high_water = std::max(S->high_water, S->in_use);
        S->state[A->req.ticket] = 1;
    }
    A->req.t_admit = std::chrono::steady_clock::now();
    // f goes to the tail of the block (the solve's q vector) on the copy
    // stream; the solve starts in the next step, when the copy is done
    const size_t len = desc_cell_len(&d);
    const size_t wsb = workspace_bytes(&d), v64 = align256(8 * len);
    double* q = reinterpret_cast<double*>(S->arena + off + wsb + 4 * v64);
    std::memcpy(hf, A->req.f.data(), sizeof(double) * A->req.f.size());
    FEM_HIP(hipMemcpyAsync(q, hf, sizeof(double) * A->req.f.size(), hipMemcpyHostToDevice, S->copy),
            "server upload");
    A->req.f.clear();
    A->req.f.shrink_to_fit();
    S->staged.push_back(A);
    return FEM_OK;
}

// Start the solves whose right-hand sides were uploaded in the previous
// step: set up the problem in its block, form b = P_I M f, and run the
// iteration's start (r = b, z = P(r), p = z, <r,z>) with single-problem
// launches on the server stream.
static fem_status activate(fem_server* S, Active* A) {
    fem_desc d = A->req.desc;
    for (int k = 0; k < 3; ++k) d.widths[k] = A->req.widths[k].empty() ? nullptr : A->req.widths[k].data();
    char* hs = stage_take(S, problem_stage_bytes(&d));
    if (!hs) {
        // this step's staging is full: free it after the copies reading it
        FEM_HIP(hipStreamSynchronize(S->stream), "server activate");
        FEM_HIP(hipStreamSynchronize(S->copy), "server activate");
        S->stage_used = 0;
        hs = stage_take(S, problem_stage_bytes(&d));
        if (!hs) return set_error(FEM_ENOMEM, "server activate: pinned staging allocation failed");
    }
    const size_t wsb = workspace_bytes(&d);
    ProblemMem pm{S->arena + A->block_off, wsb, hs, problem_stage_bytes(&d)};
    fem_status st = create_problem(&d, S->stream, &A->P, &pm);
    if (st != FEM_OK) return st;
    A->P->owned_by_batch = true;
    fem_problem* P = A->P;
    const size_t len = P->cell_len;
    const size_t v64 = align256(8 * len), vs = align256(pbytes(S->sp) * len);
    A->mem = S->arena + A->block_off + wsb;
    A->u = reinterpret_cast<double*>(A->mem);
    A->b = reinterpret_cast<double*>(A->mem + v64);
    A->r = reinterpret_cast<double*>(A->mem + 2 * v64);
    A->p = reinterpret_cast<double*>(A->mem + 3 * v64);
    A->q = reinterpret_cast<double*>(A->mem + 4 * v64);
    A->z = A->mem + 5 * v64;
    A->rs = S->sp == FEM_F64 ? (void*)A->r : (void*)(A->mem + 5 * v64 + vs);

    hipStream_t s = S->stream;
    // f (global, uploaded into q), gathered into p, b = P_I M f
    FEM_HIP(run_gather(P, A->q, A->p, FEM_F64), "server gather");
    {
        ProbEntry e = entry_of(P);
        e.a = A->p;
        e.c = A->b;
        FEM_HIP(launch_apply(P->p, FEM_F64, 2, &e, 1, nullptr, s), "server rhs");
    }
    FEM_HIP(run_fill_zero(P, A->u, FEM_F64), "server init");
    {
        ProbEntry e = entry_of(P);
        e.alpha = A->req.rtol;
        e.zchunk = A->req.maxit;
        FEM_HIP(launch_solve_init(&e, 1, nullptr, s), "server init");
    }
    FEM_HIP(hipMemcpyAsync(A->r, A->b, sizeof(double) * len, hipMemcpyDeviceToDevice, s), "server init");
    FEM_HIP(run_assembled_norm2(P, A->b, FEM_F64, kSlotB2), "server norm");
    // the residual norm first (FP16 copies take their scale from it), then the
    // smoother's copy: the same sequence as pcg_solve, so a served solve's
    // iterates equal the standalone ones bit for bit
    FEM_HIP(run_assembled_norm2(P, A->r, FEM_F64, kSlotRN), "server norm");
    if (S->sp != FEM_F64) FEM_HIP(run_distribute(P, A->r, A->rs, S->sp, kSlotTmp, true), "server distribute");
    st = S->pc == FEM_PC_TWO_LEVEL ? two_level_run(P, A->rs, A->z, S->sp, S->sweeps, S->omega)
                                   : smoother_run(P, A->rs, A->z, S->sp, S->sweeps, S->omega);
    if (st != FEM_OK) return st;
    FEM_HIP(run_convert(P, A->z, S->sp, A->p, FEM_F64), "server p0");
    FEM_HIP(run_dot(P, A->r, FEM_F64, A->z, S->sp, kSlotRZ), "server dot");
    S->active.push_back(A);
    return FEM_OK;
}

// Retire finished solves: start moves every solution to global order
// (compute stream) and downloads it into a pinned buffer of the batch (copy
// stream, after an event), then records the batch's event; collect hands
// the solutions of completed batches to the host and frees the solves'
// arena blocks, waiting only when asked to (or when many batches are open).
static fem_status retire_collect(fem_server* S, bool block) {
    while (!S->rbatches.empty()) {
        fem_server::RetireBatch& b = S->rbatches.front();
        if (block || S->rbatches.size() > 8) {
            FEM_HIP(hipEventSynchronize(b.ev), "server retire");
        } else {
            const hipError_t q = hipEventQuery(b.ev);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) return hip_error(q, "server retire");
        }
        for (size_t i = 0; i < b.fin.size(); ++i) {
            Active* A = b.fin[i];
            Done D;
            const double* src = reinterpret_cast<const double*>(b.buf + b.at[i]);
            D.u.assign(src, src + A->P->global_len);
            D.info.iters = A->iters;
            D.info.status = A->status;
            D.info.relres = A->relres;
            D.info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - A->req.t_admit).count();
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->done[A->req.ticket] = std::move(D);
                S->state[A->req.ticket] = 2;
            }
            release_active(S, A);
        }
        S->rpool.emplace_back(b.buf, b.cap);
        S->evpool.push_back(b.ev);
        S->rbatches.pop_front();
    }
    return FEM_OK;
}

static fem_status retire_start(fem_server* S, std::vector<Active*>& fin) {
    if (fin.empty()) return FEM_OK;
    fem_server::RetireBatch b;
    size_t bytes = 0;
    for (Active* A : fin) {
        b.at.push_back(bytes);
        bytes += align256(sizeof(double) * A->P->global_len);
    }
    // a pooled pinned buffer that is large enough, else a new one
    for (size_t k = 0; k < S->rpool.size(); ++k) {
        if (S->rpool[k].second >= bytes) {
            b.buf = S->rpool[k].first;
            b.cap = S->rpool[k].second;
            S->rpool.erase(S->rpool.begin() + k);
            break;
        }
    }
    if (!b.buf) {
        b.cap = std::max<size_t>(bytes, 32u << 20);
        FEM_HIP(hipHostMalloc((void**)&b.buf, b.cap, hipHostMallocDefault), "server retire buffer");
    }
    if (!S->evpool.empty()) {
        b.ev = S->evpool.back();
        S->evpool.pop_back();
    } else {
        FEM_HIP(hipEventCreateWithFlags(&b.ev, hipEventDisableTiming), "server retire event");
    }
    for (Active* A : fin) FEM_HIP(run_extract(A->P, A->u, A->q, FEM_F64), "server extract");
    FEM_HIP(hipEventRecord(S->ev_ext, S->stream), "server retire");
    FEM_HIP(hipStreamWaitEvent(S->copy, S->ev_ext, 0), "server retire");
    for (size_t i = 0; i < fin.size(); ++i)
        FEM_HIP(hipMemcpyAsync(b.buf + b.at[i], fin[i]->q, sizeof(double) * fin[i]->P->global_len,
                               hipMemcpyDeviceToHost, S->copy),
                "server download");
    FEM_HIP(hipEventRecord(b.ev, S->copy), "server retire");
    b.fin = fin;
    S->rbatches.push_back(std::move(b));
    return FEM_OK;
}

extern "C" fem_status fem_server_step(fem_server* S, int* n_active, int* n_queued, int* n_done) {
    if (!S) return set_error(FEM_EINVAL, "fem_server_step: NULL server");
    PhaseClock clk;
    S->steps += 1;
    // 1. admission in arrival order, staged in this step's region
    S->cur ^= 1;
    S->stage = S->stage_buf[S->cur];
    S->stage_cap = S->stage_capv[S->cur];
    S->stage_used = 0;
    if (!S->staged.empty()) {
        FEM_HIP(hipStreamWaitEvent(S->stream, S->ev_up, 0), "server activate");
        std::vector<Active*> staged;
        staged.swap(S->staged);
        for (Active* A : staged) {
            fem_status st = activate(S, A);
            if (st != FEM_OK) return st;
        }
    }
    const size_t nstaged0 = S->staged.size();
    while ((int)(S->active.size() + S->staged.size()) < S->max_active) {
        Request R;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->queue.empty()) break;
            R = std::move(S->queue.front());
            S->queue.pop_front();
        }
        fem_status st = admit(S, R);
        if (st == FEM_EAGAIN) {
            // not yet: back to the head of the queue (only this thread pops)
            std::lock_guard<std::mutex> lk(S->mu);
            S->queue.push_front(std::move(R));
            break;
        }
        if (st != FEM_OK) return st;
    }
    if (S->staged.size() > nstaged0) FEM_HIP(hipEventRecord(S->ev_up, S->copy), "server upload");
    hipStream_t s = S->stream;
    const int na = (int)S->active.size();
    S->t_phase[0] += clk.lap();
    if (na > 0) {
        std::vector<ProbEntry> ents;
        // 2. iterations.  Every active solve takes one (F)PCG iteration per
        //    step; a solve smaller than the largest active one takes up to
        //    kInnerMax, as many as its size fits into the largest one's, so
        //    small requests do not advance at the pace of the large ones.
        //    Convergence is decided on the device after every iteration
        //    (launch_cg_check), so the host waits once per step; a solve that
        //    finishes early in a step runs its remaining iterations in vain
        //    with u kept.
        constexpr int kInnerMax = 8;
        size_t maxlen = 1;
        for (Active* A : S->active) maxlen = std::max(maxlen, A->P->cell_len);
        std::vector<int> reps(na);
        int kmax = 1;
        for (int i = 0; i < na; ++i) {
            const size_t len = std::max<size_t>(S->active[i]->P->cell_len, 1);
            reps[i] = (int)std::min<size_t>(kInnerMax, std::max<size_t>(1, maxlen / len));
            kmax = std::max(kmax, reps[i]);
        }
        const bool mix = S->mix.load(std::memory_order_relaxed) != 0;
        for (int it = 0; it < kmax; ++it) {
            // the solves taking this inner iteration, all degrees together:
            // the degree-dependent kernels run as mixed-degree launches
            // (degrees 2, 3, 7; else one launch per degree), the vector
            // kernels over all of them at once
            std::vector<Active*> g;
            for (int i = 0; i < na; ++i)
                if (reps[i] > it) g.push_back(S->active[i]);
            const int n = (int)g.size();
            ents.resize(n);
            // q = A p, <q,p>, r -= alpha q, residual norm (and the smoother's
            // copy of r), the convergence test
            for (int i = 0; i < n; ++i) {
                ents[i] = entry_of(g[i]->P);
                ents[i].a = g[i]->p;
                ents[i].c = g[i]->q;
            }
            FEM_HIP(launch_apply_any(FEM_F64, 0, ents.data(), n, &S->st, s, mix), "server apply");
            for (int i = 0; i < n; ++i) {
                ents[i] = entry_of(g[i]->P);
                ents[i].a = g[i]->q;
                ents[i].b = g[i]->p;
            }
            FEM_HIP(launch_dot(FEM_F64, FEM_F64, ents.data(), n, &S->st, s, kSlotQP), "server dot");
            for (int i = 0; i < n; ++i) {
                ents[i] = entry_of(g[i]->P);
                ents[i].b = g[i]->q;
                ents[i].d = g[i]->r;
            }
            FEM_HIP(launch_cg_ur(ents.data(), n, &S->st, s), "server update");
            for (int i = 0; i < n; ++i) {
                ents[i] = entry_of(g[i]->P);
                ents[i].a = g[i]->r;
                ents[i].c = g[i]->rs;
                ents[i].alpha = 1.0;                // a solver's residual copy (FP16: scaled)
            }
            FEM_HIP(launch_norm_any(S->sp, ents.data(), n, &S->st, s, kSlotRN, mix), "server norm");
            for (int i = 0; i < n; ++i) ents[i] = entry_of(g[i]->P);
            FEM_HIP(launch_cg_check(ents.data(), n, &S->st, s), "server convergence");
            // smoother, pairings and the new direction (with the u step of
            // this iteration's r update, which completes a finishing solve's u)
            // z = P(rs): Schwarz sweeps, or for the two-level method
            // pre-sweeps, the coarse correction and post-sweeps
            auto residual = [&]() -> fem_status {       // tmp = rs - A z
                for (int i = 0; i < n; ++i) {
                    ents[i] = entry_of(g[i]->P);
                    ents[i].a = g[i]->z;
                    ents[i].b = g[i]->rs;
                    ents[i].c = g[i]->P->d_tmp;
                }
                FEM_HIP(launch_apply_any(S->sp, 1, ents.data(), n, &S->st, s, mix), "server smoother residual");
                return FEM_OK;
            };
            auto sweep_acc = [&]() -> fem_status {      // z += omega P_AS tmp
                for (int i = 0; i < n; ++i) ents[i] = pi_entry(g[i]->P, g[i]->P->d_tmp, g[i]->z, S->sp, S->omega);
                FEM_HIP(launch_patch_inverse_any(S->sp, 1, ents.data(), n, &S->st, s, mix), "server smoother");
                return FEM_OK;
            };
            for (int i = 0; i < n; ++i) ents[i] = pi_entry(g[i]->P, g[i]->rs, g[i]->z, S->sp, S->omega);
            FEM_HIP(launch_patch_inverse_any(S->sp, 0, ents.data(), n, &S->st, s, mix), "server smoother");
            for (int sw = 1; sw < S->sweeps; ++sw) {
                fem_status sst = residual();
                if (sst == FEM_OK) sst = sweep_acc();
                if (sst != FEM_OK) return sst;
            }
            if (S->pc == FEM_PC_TWO_LEVEL) {
                fem_status sst = residual();
                if (sst != FEM_OK) return sst;
                for (int i = 0; i < n; ++i) ents[i] = coarse_entry(g[i]->P, g[i]->P->d_tmp, g[i]->z);
                FEM_HIP(launch_coarse_any(S->sp, ents.data(), n, &S->st, s, mix), "server coarse correction");
                for (int sw = 0; sw < S->sweeps; ++sw) {
                    sst = residual();
                    if (sst == FEM_OK) sst = sweep_acc();
                    if (sst != FEM_OK) return sst;
                }
            }
            if (S->variant == FEM_CG_PCG) {
                for (int i = 0; i < n; ++i) ents[i] = entry_of(g[i]->P);
                FEM_HIP(launch_slot_copy(ents.data(), n, &S->st, s, kSlotRZOld, kSlotRZ), "server slots");
                for (int i = 0; i < n; ++i) {
                    ents[i] = entry_of(g[i]->P);
                    ents[i].a = g[i]->r;
                    ents[i].b = g[i]->z;
                }
                FEM_HIP(launch_dot(FEM_F64, S->sp, ents.data(), n, &S->st, s, kSlotRZ), "server dot");
            } else {
                for (int i = 0; i < n; ++i) {
                    ents[i] = entry_of(g[i]->P);
                    ents[i].a = g[i]->q;
                    ents[i].d = g[i]->r;
                    ents[i].b = g[i]->z;
                }
                FEM_HIP(launch_dot_qz_rz(S->sp, ents.data(), n, &S->st, s), "server dots");
            }
            for (int i = 0; i < n; ++i) {
                ents[i] = entry_of(g[i]->P);
                ents[i].a = g[i]->z;
                ents[i].c = g[i]->p;
                ents[i].d = g[i]->u;
            }
            FEM_HIP(launch_cg_p(S->sp, S->variant, ents.data(), n, &S->st, s), "server direction");
        }
        // 3. one read-back of every solve's convergence state
        ents.resize(na);
        for (int i = 0; i < na; ++i) ents[i] = entry_of(S->active[i]->P);
        FEM_HIP(launch_collect_slots(ents.data(), na, &S->st, s, kSlotState, kSlotIters, S->d_collect),
                "server collect");
        FEM_HIP(launch_collect_slots(ents.data(), na, &S->st, s, kSlotRel, kSlotStatus, S->d_collect + 2 * na),
                "server collect");
        FEM_HIP(hipMemcpyAsync(S->h_collect, S->d_collect, sizeof(double) * 4 * na, hipMemcpyDeviceToHost, s),
                "server read-back");
        FEM_HIP(hipEventRecord(S->ev_scalars, s), "server read-back");
        S->t_phase[1] += clk.lap();
        // completed downloads of earlier steps reach the host while the GPU
        // runs this step's work
        fem_status stf = retire_collect(S, false);
        if (stf != FEM_OK) return stf;
        S->t_phase[3] += clk.lap();
        FEM_HIP(hipEventSynchronize(S->ev_scalars), "server read-back");
        S->t_phase[2] += clk.lap();
        for (int i = 0; i < na; ++i) {
            Active* A = S->active[i];
            const double state = S->h_collect[2 * i], iters = S->h_collect[2 * i + 1];
            const double rel = S->h_collect[2 * na + 2 * i], status = S->h_collect[2 * na + 2 * i + 1];
            A->iters = (int)iters;
            A->relres = rel;
            if (state != 0.0) {
                A->finished = true;
                A->status = (int)status;
            }
        }
        // 4. retire finished solves (frees their memory for the next admissions)
        std::vector<Active*> keep, fin;
        for (Active* A : S->active) (A->finished ? fin : keep).push_back(A);
        S->active.swap(keep);
        fem_status st = retire_start(S, fin);
        if (st != FEM_OK) return st;
        S->t_phase[4] += clk.lap();
    }
    if (na == 0) {
        // nothing ran this step: hand over what is pending (waiting for it)
        fem_status stf = retire_collect(S, true);
        if (stf != FEM_OK) return stf;
    }
    if (n_active) *n_active = (int)S->active.size();
    std::lock_guard<std::mutex> lk(S->mu);
    if (n_queued) *n_queued = (int)S->queue.size();
    if (n_done) *n_done = (int)S->done.size();
    return FEM_OK;
}

extern "C" fem_status fem_server_set_mixed(fem_server* S, int mixed) {
    if (!S) return set_error(FEM_EINVAL, "fem_server_set_mixed: NULL server");
    S->mix.store(mixed ? 1 : 0, std::memory_order_relaxed);
    return FEM_OK;
}

extern "C" fem_status fem_server_poll(fem_server* S, uint64_t ticket, double* u_glob, fem_solve_info* info) {
    if (!S) return set_error(FEM_EINVAL, "fem_server_poll: NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->state.find(ticket);
    if (it == S->state.end()) return set_error(FEM_ENOTFOUND, "fem_server_poll: unknown ticket");
    if (it->second != 2) return FEM_EAGAIN;
    Done& D = S->done[ticket];
    if (u_glob) std::memcpy(u_glob, D.u.data(), sizeof(double) * D.u.size());
    if (info) *info = D.info;
    S->done.erase(ticket);
    S->state.erase(it);
    return FEM_OK;
}

extern "C" fem_status fem_server_stats(fem_server* S, double* out, int n) {
    if (!S || !out) return set_error(FEM_EINVAL, "fem_server_stats: NULL argument");
    const double v[6] = {S->t_phase[0], S->t_phase[1], S->t_phase[2], S->t_phase[3], S->t_phase[4],
                         (double)S->steps};
    for (int i = 0; i < n && i < 6; ++i) out[i] = v[i];
    return FEM_OK;
}

extern "C" int fem_server_finished(fem_server* S, uint64_t* out, int max_tickets) {
    if (!S) return 0;
    std::vector<uint64_t> t;
    std::lock_guard<std::mutex> lk(S->mu);
    t.reserve(S->done.size());
    for (const auto& kv : S->done) t.push_back(kv.first);
    std::sort(t.begin(), t.end());
    if (out)
        for (int i = 0; i < (int)t.size() && i < max_tickets; ++i) out[i] = t[i];
    return (int)t.size();
}

extern "C" fem_status fem_server_memory(fem_server* S, size_t* in_use, size_t* high_water) {
    if (!S) return set_error(FEM_EINVAL, "fem_server_memory: NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (in_use) *in_use = S->in_use;
    if (high_water) *high_water = S->high_water;
    return FEM_OK;
}
