// C-ABI entry points: problem lifecycle, converters, operators, smoother,
// reductions and the primal-dual (flexible) PCG.
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fem_internal.h"
#include "host_api.h"
#include "launch.h"

using namespace fem;

namespace fem {

static size_t prec_bytes(int prec) { return prec == FEM_F64 ? 8 : prec == FEM_F32 ? 4 : 2; }

fem_status check_desc(const fem_desc* d) {
    if (!d) return set_error(FEM_EINVAL, "fem_desc is NULL");
    if (d->p < 1 || d->p > kMaxP) return set_error(FEM_EINVAL, "degree p must be in 1..7");
    for (int k = 0; k < 3; ++k) {
        if (d->n[k] < 1) return set_error(FEM_EINVAL, "cells per direction must be >= 1");
        if ((long long)d->n[0] * d->n[1] * d->n[2] > (1LL << 26))
            return set_error(FEM_EINVAL, "mesh too large (more than 2^26 cells)");
        if (d->widths[k])
            for (int i = 0; i < d->n[k]; ++i)
                if (!(d->widths[k][i] > 0) || !std::isfinite(d->widths[k][i]))
                    return set_error(FEM_EINVAL, "cell widths must be positive and finite");
    }
    if (d->bc != FEM_BC_DIRICHLET && d->bc != FEM_BC_NEUMANN) return set_error(FEM_EINVAL, "unknown bc");
    // the p >= 4 patch solves address a patch's box with 32-bit offsets
    if (d->p >= 4 && (unsigned long long)(d->n[0] * d->p + 1) * (d->n[1] * d->p + 1) * (2 * d->p - 1) >= (1ULL << 32))
        return set_error(FEM_EINVAL, "mesh too wide: (n0 p + 1)(n1 p + 1)(2p - 1) must stay below 2^32 for p >= 4");
    return FEM_OK;
}

size_t desc_cell_len(const fem_desc* d) {
    const size_t nc = (size_t)d->n[0] * d->n[1] * d->n[2];
    const size_t nn = (size_t)(d->p + 1) * (d->p + 1) * (d->p + 1);
    return (nc + kLanes - 1) / kLanes * nn * kLanes;
}

static size_t desc_patch_len(const fem_desc* d) {
    const size_t np = (size_t)(d->n[0] > 1 ? d->n[0] - 1 : 0) * (d->n[1] > 1 ? d->n[1] - 1 : 0) *
                      (d->n[2] > 1 ? d->n[2] - 1 : 0);
    const size_t nP = 2 * d->p - 1;
    return (np + kLanes - 1) / kLanes * nP * nP * nP * kLanes;
}

static size_t fd_stride(const fem_desc* d) {
    int nmax = std::max(d->n[0], std::max(d->n[1], d->n[2]));
    return (size_t)std::max(nmax - 1, 1) * fd_record(d->p);
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t coarse_fd_len(const fem_desc* d) {
    size_t c = 0;
    for (int k = 0; k < 3; ++k) {
        const size_t m = d->n[k] > 1 ? d->n[k] - 1 : 0;
        c += m * m + m;
    }
    return c;
}

static size_t coarse_len(const fem_desc* d) {
    size_t c = 1;
    for (int k = 0; k < 3; ++k) c *= d->n[k] > 1 ? d->n[k] - 1 : 0;
    return c;
}

static size_t corner_len(const fem_desc* d) {
    const size_t nc = (size_t)d->n[0] * d->n[1] * d->n[2];
    return 8 * ((nc + kLanes - 1) / kLanes * kLanes);
}

size_t workspace_bytes(const fem_desc* d) {
    size_t b = 0;
    b += align256(sizeof(double) * std::max<size_t>(coarse_fd_len(d), 1));
    b += align256(sizeof(double) * std::max<size_t>(2 * coarse_len(d), 1));
    b += align256(sizeof(double) * corner_len(d));
    b += align256(sizeof(double) * (d->n[0] + d->n[1] + d->n[2]));
    b += align256(sizeof(double) * 3 * fd_stride(d));
    b += align256(sizeof(float) * 3 * fd_stride(d));
    b += align256(sizeof(double) * kRedStride);
    b += align256(sizeof(double) * std::max<size_t>(desc_patch_len(d), 1));
    b += align256(sizeof(double) * desc_cell_len(d));
    b += align256(sizeof(double) * (size_t)(d->n[0] * d->p + 1) * (d->n[1] * d->p + 1) * (d->n[2] * d->p + 1));
    return b;
}

size_t solve_vector_bytes(const fem_desc* d, int sp) {
    const size_t len = desc_cell_len(d);
    return align256(3 * 8 * len) + align256(2 * prec_bytes(sp) * len);
}

}  // namespace fem

// ------------------------------------------------------------------ setup
extern "C" size_t fem_prec_bytes(int prec) { return prec_bytes(prec); }

extern "C" size_t fem_footprint_bytes(const fem_desc* d, int smoother_prec) {
    if (check_desc(d) != FEM_OK) return 0;
    // workspace, then u, b, r, p, q (FP64) and z, rs (smoother precision):
    // exactly the block the solve server carves for a request
    const size_t len = desc_cell_len(d);
    return workspace_bytes(d) + 5 * align256(8 * len) + 2 * align256(prec_bytes(smoother_prec) * len);
}

static void free_problem(fem_problem* P) {
    if (!P) return;
    if (P->external_mem) {
        delete P;
        return;
    }
    hipFree(P->d_h);
    hipFree(P->d_fd64);
    hipFree(P->d_fd32);
    hipFree(P->d_red);
    hipFree(P->d_patch);
    hipFree(P->d_tmp);
    hipFree(P->d_glob);
    hipFree(P->d_solve);
    hipFree(P->d_cfd);
    hipFree(P->d_cvec);
    hipFree(P->d_corner);
    if (P->h_red) hipHostFree(P->h_red);
    delete P;
}

namespace fem {
size_t problem_stage_bytes(const fem_desc* d) {
    return align256(sizeof(double) * (d->n[0] + d->n[1] + d->n[2])) + align256(sizeof(double) * 3 * fd_stride(d)) +
           align256(sizeof(float) * 3 * fd_stride(d)) + align256(sizeof(double) * std::max<size_t>(coarse_fd_len(d), 1));
}

fem_status create_problem(const fem_desc* d, hipStream_t stream, fem_problem** out, const ProblemMem* mem) {
    if (!out) return set_error(FEM_EINVAL, "out is NULL");
    *out = nullptr;
    fem_status st = check_desc(d);
    if (st != FEM_OK) return st;
    fem_problem* P = new (std::nothrow) fem_problem();
    if (!P) return set_error(FEM_ENOMEM, "host allocation failed");
    std::memset(P, 0, sizeof(*P));
    P->p = d->p;
    for (int k = 0; k < 3; ++k) P->n[k] = d->n[k];
    P->bc = d->bc;
    P->ncells = d->n[0] * d->n[1] * d->n[2];
    P->nblk = (P->ncells + kLanes - 1) / kLanes;
    P->cell_len = desc_cell_len(d);
    P->global_len = (size_t)(d->n[0] * d->p + 1) * (d->n[1] * d->p + 1) * (d->n[2] * d->p + 1);
    P->npatch = (size_t)(d->n[0] - 1) * (d->n[1] - 1) * (d->n[2] - 1);
    P->npblk = (int)((P->npatch + kLanes - 1) / kLanes);
    P->patch_len = desc_patch_len(d);
    P->stream = stream;
    hipGetDevice(&P->device);
    P->fd_dir_stride = fd_stride(d);
    if (entry_of(P).ntiles_red > kRedParts) {
        // reduction partials would run past their group in the workspace
        free_problem(P);
        return set_error(FEM_EINVAL, "create_problem: reduction tiling exceeds kRedParts");
    }

    // geometry
    std::vector<double> h;
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < d->n[k]; ++i) h.push_back(d->widths[k] ? d->widths[k][i] : 1.0 / d->n[k]);
    // FD data per direction and vertex line
    const int rec = fd_record(d->p), nP = 2 * d->p - 1;
    std::vector<double> fd(3 * P->fd_dir_stride, 0.0);
    std::vector<float> fd32(3 * P->fd_dir_stride, 0.0f);
    size_t off = 0;
    for (int k = 0; k < 3; ++k) {
        const double* w = &h[off];
        for (int v = 1; v < d->n[k]; ++v) {
            double* r = &fd[k * P->fd_dir_stride + (size_t)(v - 1) * rec];
            if (host_fd_1d(d->p, w[v - 1], w[v], r, r + nP * nP) != 0) {
                free_problem(P);
                return set_error(FEM_EINVAL, "1D patch eigenproblem failed");
            }
        }
        off += d->n[k];
    }
    for (size_t i = 0; i < fd.size(); ++i) fd32[i] = (float)fd[i];
    // coarse level: Q1 fast-diagonalisation data per direction
    std::vector<double> cfd(std::max<size_t>(coarse_fd_len(d), 1), 0.0);
    {
        size_t o = 0, hoff = 0;
        for (int k = 0; k < 3; ++k) {
            P->cm[k] = d->n[k] > 1 ? d->n[k] - 1 : 0;
            P->cfd_off[k] = o;
            const int m = P->cm[k];
            if (m > 0 && host_coarse_1d(d->n[k], &h[hoff], &cfd[o], &cfd[o + (size_t)m * m]) != 0) {
                free_problem(P);
                return set_error(FEM_EINVAL, "coarse 1D eigenproblem failed");
            }
            o += (size_t)m * m + m;
            hoff += d->n[k];
        }
    }

    hipError_t e;
    if (mem) {
        // carve the workspace from the caller's block, in workspace_bytes order
        if (mem->dev_bytes < workspace_bytes(d) || mem->stage_bytes < problem_stage_bytes(d)) {
            free_problem(P);
            return set_error(FEM_EINVAL, "create_problem: caller memory too small");
        }
        P->external_mem = true;
        size_t off = 0;
        auto take = [&](size_t bytes) {
            char* q = mem->dev + off;
            off += align256(bytes);
            return q;
        };
        P->d_cfd = reinterpret_cast<double*>(take(sizeof(double) * cfd.size()));
        P->d_cvec = reinterpret_cast<double*>(take(sizeof(double) * std::max<size_t>(2 * coarse_len(d), 1)));
        P->d_corner = reinterpret_cast<double*>(take(sizeof(double) * corner_len(d)));
        P->d_h = reinterpret_cast<double*>(take(sizeof(double) * h.size()));
        P->d_fd64 = reinterpret_cast<double*>(take(sizeof(double) * fd.size()));
        P->d_fd32 = reinterpret_cast<float*>(take(sizeof(float) * fd32.size()));
        P->d_red = reinterpret_cast<double*>(take(sizeof(double) * kRedStride));
        P->d_patch = take(sizeof(double) * std::max<size_t>(P->patch_len, 1));
        P->d_tmp = take(sizeof(double) * P->cell_len);
        P->d_glob = take(sizeof(double) * P->global_len);
        char* hs = mem->stage;
        std::memcpy(hs, h.data(), sizeof(double) * h.size());
        char* hf = hs + align256(sizeof(double) * h.size());
        std::memcpy(hf, fd.data(), sizeof(double) * fd.size());
        char* hf32 = hf + align256(sizeof(double) * fd.size());
        std::memcpy(hf32, fd32.data(), sizeof(float) * fd32.size());
        char* hc = hf32 + align256(sizeof(float) * fd32.size());
        std::memcpy(hc, cfd.data(), sizeof(double) * cfd.size());
        e = hipMemcpyAsync(P->d_h, hs, sizeof(double) * h.size(), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(P->d_cfd, hc, sizeof(double) * cfd.size(), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(P->d_fd64, hf, sizeof(double) * fd.size(), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(P->d_fd32, hf32, sizeof(float) * fd32.size(), hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) {
            free_problem(P);
            return hip_error(e, "create_problem upload");
        }
        *out = P;
        return FEM_OK;
    }
#define ALLOC(ptr, bytes)                                                    \
    e = hipMalloc((void**)&(ptr), (bytes));                                  \
    if (e != hipSuccess) {                                                   \
        free_problem(P);                                                     \
        return set_error(FEM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)); \
    }
    ALLOC(P->d_h, sizeof(double) * h.size());
    ALLOC(P->d_fd64, sizeof(double) * fd.size());
    ALLOC(P->d_fd32, sizeof(float) * fd32.size());
    ALLOC(P->d_red, sizeof(double) * kRedStride);
    ALLOC(P->d_patch, sizeof(double) * std::max<size_t>(P->patch_len, 1));
    ALLOC(P->d_tmp, sizeof(double) * P->cell_len);
    ALLOC(P->d_glob, sizeof(double) * P->global_len);
    ALLOC(P->d_cfd, sizeof(double) * cfd.size());
    ALLOC(P->d_cvec, sizeof(double) * std::max<size_t>(2 * coarse_len(d), 1));
    ALLOC(P->d_corner, sizeof(double) * corner_len(d));
#undef ALLOC
    e = hipHostMalloc((void**)&P->h_red, sizeof(double) * kSlotCount, hipHostMallocDefault);
    if (e != hipSuccess) {
        free_problem(P);
        return set_error(FEM_ENOMEM, "hipHostMalloc failed");
    }
    e = hipMemcpyAsync(P->d_h, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(P->d_fd64, fd.data(), sizeof(double) * fd.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(P->d_fd32, fd32.data(), sizeof(float) * fd32.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(P->d_cfd, cfd.data(), sizeof(double) * cfd.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        free_problem(P);
        return hip_error(e, "fem_problem_create upload");
    }
    *out = P;
    return FEM_OK;
}
}  // namespace fem

extern "C" fem_status fem_problem_create(const fem_desc* d, void* stream, fem_problem** out) {
    return create_problem(d, static_cast<hipStream_t>(stream), out, nullptr);
}

namespace fem {
// Free a problem without waiting for its stream: for callers that know no
// queued work still uses it (the solve server, after a solve's last copy).
void destroy_problem_nosync(fem_problem* P) { free_problem(P); }
}  // namespace fem

extern "C" fem_status fem_problem_destroy(fem_problem* P) {
    if (!P) return FEM_OK;
    if (P->owned_by_batch) return set_error(FEM_EINVAL, "problem belongs to a batch");
    hipStreamSynchronize(P->stream);
    free_problem(P);
    return FEM_OK;
}

extern "C" fem_status fem_set_stream(fem_problem* P, void* stream) {
    if (!P) return set_error(FEM_EINVAL, "problem is NULL");
    P->stream = static_cast<hipStream_t>(stream);
    return FEM_OK;
}

extern "C" size_t fem_cell_len(const fem_problem* P) { return P ? P->cell_len : 0; }
extern "C" size_t fem_global_len(const fem_problem* P) { return P ? P->global_len : 0; }
extern "C" size_t fem_num_cells(const fem_problem* P) { return P ? (size_t)P->ncells : 0; }
extern "C" size_t fem_num_patches(const fem_problem* P) { return P ? P->npatch : 0; }

// -------------------------------------------------------------- helpers
static fem_status check_prec(int prec) {
    if (prec != FEM_F64 && prec != FEM_F32 && prec != FEM_BF16 && prec != FEM_F16)
        return set_error(FEM_EINVAL, "unknown precision");
    return FEM_OK;
}
#define CHECK_P(P) \
    if (!(P)) return set_error(FEM_EINVAL, "problem is NULL")
#define CHECK_PTR(x) \
    if (!(x)) return set_error(FEM_EINVAL, #x " is NULL")

extern "C" fem_status fem_gather(fem_problem* P, const double* xg, void* xc, int prec) {
    CHECK_P(P); CHECK_PTR(xg); CHECK_PTR(xc);
    if (check_prec(prec)) return FEM_EINVAL;
    FEM_HIP(run_gather(P, xg, xc, prec), "fem_gather");
    return FEM_OK;
}
extern "C" fem_status fem_scatter(fem_problem* P, const void* yc, double* yg, int prec) {
    CHECK_P(P); CHECK_PTR(yc); CHECK_PTR(yg);
    if (check_prec(prec)) return FEM_EINVAL;
    FEM_HIP(run_scatter(P, yc, yg, prec), "fem_scatter");
    return FEM_OK;
}
extern "C" fem_status fem_extract(fem_problem* P, const void* uc, double* ug, int prec) {
    CHECK_P(P); CHECK_PTR(uc); CHECK_PTR(ug);
    if (check_prec(prec)) return FEM_EINVAL;
    FEM_HIP(run_extract(P, uc, ug, prec), "fem_extract");
    return FEM_OK;
}
extern "C" fem_status fem_pack(fem_problem* P, const double* canon, void* vc, int prec) {
    CHECK_P(P); CHECK_PTR(canon); CHECK_PTR(vc);
    if (check_prec(prec)) return FEM_EINVAL;
    FEM_HIP(run_pack(P, canon, vc, prec, 0), "fem_pack");
    return FEM_OK;
}
extern "C" fem_status fem_unpack(fem_problem* P, const void* vc, double* canon, int prec) {
    CHECK_P(P); CHECK_PTR(canon); CHECK_PTR(vc);
    if (check_prec(prec)) return FEM_EINVAL;
    FEM_HIP(run_pack(P, canon, const_cast<void*>(vc), prec, 1), "fem_unpack");
    return FEM_OK;
}
extern "C" fem_status fem_distribute_assembled(fem_problem* P, const double* r, void* out, int prec) {
    CHECK_P(P); CHECK_PTR(r); CHECK_PTR(out);
    if (check_prec(prec)) return FEM_EINVAL;
    if ((const void*)r == out) return set_error(FEM_EINVAL, "fem_distribute_assembled: r and out alias");
    FEM_HIP(run_distribute(P, r, out, prec, kSlotTmp), "fem_distribute_assembled");
    return FEM_OK;
}

extern "C" fem_status fem_convert(fem_problem* P, const void* src, int sp, void* dst, int dp) {
    CHECK_P(P); CHECK_PTR(src); CHECK_PTR(dst);
    if (check_prec(sp) || check_prec(dp)) return FEM_EINVAL;
    if (src == dst) return set_error(FEM_EINVAL, "fem_convert: src and dst alias");
    FEM_HIP(run_convert(P, src, sp, dst, dp), "fem_convert");
    return FEM_OK;
}

// ------------------------------------------------------------ operators
static fem_status apply_mode(fem_problem* P, const void* x, const void* b, void* y, int prec, int mode,
                             const char* what) {
    CHECK_P(P); CHECK_PTR(x); CHECK_PTR(y);
    if (check_prec(prec)) return FEM_EINVAL;
    if (x == y) return set_error(FEM_EINVAL, std::string(what) + ": input and output alias");
    ProbEntry e = entry_of(P);
    e.a = x;
    e.b = b;
    e.c = y;
    FEM_HIP(launch_apply(P->p, prec, mode, &e, 1, nullptr, P->stream), what);
    return FEM_OK;
}

extern "C" fem_status fe_apply(fem_problem* P, const void* x, void* y, int prec) {
    return apply_mode(P, x, nullptr, y, prec, 0, "fe_apply");
}
extern "C" fem_status fe_mass_apply(fem_problem* P, const void* x, void* y, int prec) {
    return apply_mode(P, x, nullptr, y, prec, 2, "fe_mass_apply");
}

extern "C" fem_status fem_dss_axis(fem_problem* P, void* v, int axis, int prec) {
    CHECK_P(P); CHECK_PTR(v);
    if (check_prec(prec)) return FEM_EINVAL;
    if (axis < 0 || axis > 2) return set_error(FEM_EINVAL, "axis must be 0, 1 or 2");
    FEM_HIP(run_dss_axis(P, v, axis, prec), "fem_dss_axis");
    return FEM_OK;
}

extern "C" fem_status fem_dss(fem_problem* P, const void* v, void* s, int prec) {
    CHECK_P(P); CHECK_PTR(v); CHECK_PTR(s);
    if (check_prec(prec)) return FEM_EINVAL;
    if (v != s)
        FEM_HIP(hipMemcpyAsync(s, v, P->cell_len * prec_bytes(prec), hipMemcpyDeviceToDevice, P->stream),
                "fem_dss copy");
    for (int axis = 2; axis >= 0; --axis) FEM_HIP(run_dss_axis(P, s, axis, prec), "fem_dss");
    return FEM_OK;
}

namespace fem {
static fem_status pi_run(fem_problem* P, const void* r, void* z, int prec, int acc, double alpha) {
    ProbEntry e = entry_of(P);
    e.a = r;
    e.c = z;
    e.d = P->d_patch;
    e.e = P->d_glob;
    e.alpha = alpha;
    for (int k = 0; k < 3; ++k)
        e.fd[k] = prec == FEM_F64 ? (const void*)(P->d_fd64 + k * P->fd_dir_stride)
                                  : (const void*)(P->d_fd32 + k * P->fd_dir_stride);
    FEM_HIP(launch_patch_inverse(P->p, prec, acc, &e, 1, nullptr, P->stream), "patch_inverse");
    return FEM_OK;
}

// t = r - A z into the scratch vector
static fem_status residual_to_tmp(fem_problem* P, const void* r, const void* z, int prec) {
    ProbEntry e = entry_of(P);
    e.a = z;
    e.b = r;
    e.c = P->d_tmp;
    FEM_HIP(launch_apply(P->p, prec, 1, &e, 1, nullptr, P->stream), "smoother residual");
    return FEM_OK;
}

fem_status smoother_run(fem_problem* P, const void* r, void* z, int prec, int sweeps, double omega) {
    fem_status st = pi_run(P, r, z, prec, 0, omega);
    if (st != FEM_OK) return st;
    for (int s = 1; s < sweeps; ++s) {
        // t = r - A z (scratch), z += omega P_AS t
        st = residual_to_tmp(P, r, z, prec);
        if (st != FEM_OK) return st;
        st = pi_run(P, P->d_tmp, z, prec, 1, omega);
        if (st != FEM_OK) return st;
    }
    return FEM_OK;
}

fem_status two_level_run(fem_problem* P, const void* r, void* z, int prec, int sweeps, double omega) {
    fem_status st = smoother_run(P, r, z, prec, sweeps, omega);
    if (st != FEM_OK) return st;
    st = residual_to_tmp(P, r, z, prec);
    if (st != FEM_OK) return st;
    FEM_HIP(run_coarse_correction(P, P->d_tmp, z, prec), "coarse correction");
    for (int s = 0; s < sweeps; ++s) {
        st = residual_to_tmp(P, r, z, prec);
        if (st != FEM_OK) return st;
        st = pi_run(P, P->d_tmp, z, prec, 1, omega);
        if (st != FEM_OK) return st;
    }
    return FEM_OK;
}
}  // namespace fem

extern "C" fem_status patch_inverse(fem_problem* P, const void* r, void* z, int prec) {
    CHECK_P(P); CHECK_PTR(r); CHECK_PTR(z);
    if (check_prec(prec)) return FEM_EINVAL;
    if (r == z) return set_error(FEM_EINVAL, "patch_inverse: r and z alias");
    return pi_run(P, r, z, prec, 0, 1.0);
}

extern "C" fem_status fem_two_level(fem_problem* P, const void* r, void* z, int prec, int sweeps, double omega) {
    CHECK_P(P); CHECK_PTR(r); CHECK_PTR(z);
    if (check_prec(prec)) return FEM_EINVAL;
    if (r == z) return set_error(FEM_EINVAL, "fem_two_level: r and z alias");
    if (sweeps < 1) return set_error(FEM_EINVAL, "fem_two_level: sweeps >= 1");
    if (!std::isfinite(omega)) return set_error(FEM_EINVAL, "fem_two_level: omega must be finite");
    return two_level_run(P, r, z, prec, sweeps, omega);
}

extern "C" fem_status smoother_step(fem_problem* P, const void* r, void* z, int prec, int sweeps, double omega) {
    CHECK_P(P); CHECK_PTR(r); CHECK_PTR(z);
    if (check_prec(prec)) return FEM_EINVAL;
    if (r == z) return set_error(FEM_EINVAL, "smoother_step: r and z alias");
    if (sweeps < 1) return set_error(FEM_EINVAL, "smoother_step: sweeps >= 1");
    if (!std::isfinite(omega)) return set_error(FEM_EINVAL, "smoother_step: omega must be finite");
    return smoother_run(P, r, z, prec, sweeps, omega);
}

// ------------------------------------------------------------ reductions
static fem_status read_slots(fem_problem* P) {
    FEM_HIP(hipMemcpyAsync(P->h_red, red_slots(P->d_red), sizeof(double) * kSlotCount, hipMemcpyDeviceToHost,
                           P->stream),
            "read scalars");
    FEM_HIP(hipStreamSynchronize(P->stream), "read scalars");
    return FEM_OK;
}

extern "C" fem_status fem_dot(fem_problem* P, const void* a, int pa, const void* b, int pb, double* result) {
    CHECK_P(P); CHECK_PTR(a); CHECK_PTR(b); CHECK_PTR(result);
    if (check_prec(pa) || check_prec(pb)) return FEM_EINVAL;
    FEM_HIP(run_dot(P, a, pa, b, pb, kSlotTmp), "fem_dot");
    fem_status st = read_slots(P);
    if (st != FEM_OK) return st;
    *result = P->h_red[kSlotTmp];
    return FEM_OK;
}

extern "C" fem_status fem_assembled_norm(fem_problem* P, const void* r, int prec, double* result) {
    CHECK_P(P); CHECK_PTR(r); CHECK_PTR(result);
    if (check_prec(prec)) return FEM_EINVAL;
    FEM_HIP(run_assembled_norm2(P, r, prec, kSlotTmp), "fem_assembled_norm");
    fem_status st = read_slots(P);
    if (st != FEM_OK) return st;
    *result = std::sqrt(P->h_red[kSlotTmp]);
    return FEM_OK;
}

// ---------------------------------------------------------------- solver
namespace fem {
// Bytes of the solver's own vectors r, p, q (FP64) and z, rs (preconditioner
// precision) for a cell length.
static size_t solve_bytes_for(size_t len, int sp) { return align256(3 * 8 * len) + align256(2 * prec_bytes(sp) * len); }

// The (F)PCG of Algorithm "Communication-Free (F)PCG" on the handle's
// stream, its vectors carved from `work` (solve_bytes_for bytes).  pc picks
// the preconditioner: the Schwarz smoother (smoother_run), or one pass of
// S or D_cell^{-1} S (Section 3.3), which also yields ||G^T r|| for the
// stopping test.
static fem_status pcg_core(fem_problem* P, const double* b, double* u, double rtol, int maxit, int pc, int sp,
                           int sweeps, double omega, int variant, char* work, fem_solve_info* info,
                           std::chrono::steady_clock::time_point t0) {
    const size_t len = P->cell_len;
    double* r = reinterpret_cast<double*>(work);
    double* p = r + len;
    double* q = p + len;
    void* z = work + align256(3 * 8 * len);
    void* rs = sp == FEM_F64 ? (void*)r : (void*)(static_cast<char*>(z) + align256(prec_bytes(sp) * len));
    // the smoother-type preconditioners see the residual as the smoother does
    const bool schwarz = pc == FEM_PC_SCHWARZ || pc == FEM_PC_TWO_LEVEL;

    auto finish = [&](fem_status st, int iters, double relres) {
        info->iters = iters;
        info->status = st;
        info->relres = relres;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (st != FEM_OK && st != FEM_ENOTCONV && st != FEM_EBREAKDOWN) return st;
        if (st == FEM_ENOTCONV) set_error(st, "pcg_solve: not converged at maxit");
        if (st == FEM_EBREAKDOWN) set_error(st, "pcg_solve: breakdown (<q,p> not positive and finite)");
        return st;
    };
    auto precondition = [&]() -> fem_status {
        if (pc == FEM_PC_SCHWARZ) return smoother_run(P, rs, z, sp, sweeps, omega);
        if (pc == FEM_PC_TWO_LEVEL) return two_level_run(P, rs, z, sp, sweeps, omega);
        return FEM_OK;      // the simple preconditioners ran with the norm
    };

    // the solve is running (the state the r and p updates consult)
    {
        ProbEntry e = entry_of(P);
        e.alpha = rtol;
        e.zchunk = maxit;
        FEM_HIP(launch_solve_init(&e, 1, nullptr, P->stream), "pcg_solve init");
    }
    // r = b - A u
    {
        ProbEntry e = entry_of(P);
        e.a = u;
        e.b = b;
        e.c = r;
        FEM_HIP(launch_apply(P->p, FEM_F64, 1, &e, 1, nullptr, P->stream), "pcg_solve residual");
    }
    FEM_HIP(run_assembled_norm2(P, b, FEM_F64, kSlotB2), "pcg_solve norm");
    // (FP16 copies take their scale from the norm slot: fill it first)
    if (schwarz || sp == FEM_F16) FEM_HIP(run_assembled_norm2(P, r, FEM_F64, kSlotRN), "pcg_solve norm");
    if (!schwarz) FEM_HIP(run_simple_precond(P, pc, r, z, sp, kSlotRN, true), "pcg_solve preconditioner");
    fem_status st = read_slots(P);
    if (st != FEM_OK) return finish(st, 0, NAN);
    const double bn = std::sqrt(P->h_red[kSlotB2]);
    double rel = bn > 0 ? std::sqrt(P->h_red[kSlotRN]) / bn : 0.0;
    // a non-finite right-hand side or initial residual: no iteration on it
    if (!std::isfinite(bn) || !std::isfinite(rel)) return finish(FEM_EBREAKDOWN, 0, rel);
    if (bn == 0.0 || rel <= rtol) return finish(FEM_OK, 0, rel);
    // reduced-precision smoothers get the residual assembled in FP64 first
    if (schwarz && sp != FEM_F64) FEM_HIP(run_distribute(P, r, rs, sp, kSlotTmp, true), "pcg_solve distribute");

    st = precondition();
    if (st != FEM_OK) return finish(st, 0, rel);
    FEM_HIP(run_convert(P, z, sp, p, FEM_F64), "pcg_solve p0");
    FEM_HIP(run_dot(P, r, FEM_F64, z, sp, kSlotRZ), "pcg_solve dot");

    int k = 0;
    while (k < maxit) {
        ProbEntry e = entry_of(P);
        e.a = p;
        e.c = q;
        FEM_HIP(launch_apply(P->p, FEM_F64, 0, &e, 1, nullptr, P->stream), "pcg_solve apply");
        FEM_HIP(run_dot(P, q, FEM_F64, p, FEM_F64, kSlotQP), "pcg_solve dot");
        FEM_HIP(run_cg_update_r(P, r, q, nullptr, FEM_F64), "pcg_solve update");
        if (!schwarz) FEM_HIP(run_simple_precond(P, pc, r, z, sp, kSlotRN, true), "pcg_solve preconditioner");
        else if (sp == FEM_F64) FEM_HIP(run_assembled_norm2(P, r, FEM_F64, kSlotRN), "pcg_solve norm");
        else FEM_HIP(run_distribute(P, r, rs, sp, kSlotRN, true), "pcg_solve distribute");
        st = read_slots(P);
        if (st != FEM_OK) return finish(st, k, rel);
        ++k;
        const double qp = P->h_red[kSlotQP];
        if (!(qp > 0) || !std::isfinite(qp)) return finish(FEM_EBREAKDOWN, k, rel);
        rel = std::sqrt(P->h_red[kSlotRN]) / bn;
        if (!std::isfinite(rel)) return finish(FEM_EBREAKDOWN, k, rel);
        if (rel <= rtol || k >= maxit) {
            // the last r update's u step (u catches up one update late)
            FEM_HIP(run_cg_update_u(P, u, p), "pcg_solve update u");
            FEM_HIP(hipStreamSynchronize(P->stream), "pcg_solve");
            return finish(rel <= rtol ? FEM_OK : FEM_ENOTCONV, k, rel);
        }
        st = precondition();
        if (st != FEM_OK) return finish(st, k, rel);
        if (variant == FEM_CG_PCG) {
            FEM_HIP(run_slot_copy(P, kSlotRZOld, kSlotRZ), "pcg_solve slots");
            FEM_HIP(run_dot(P, r, FEM_F64, z, sp, kSlotRZ), "pcg_solve dot");
        } else {
            FEM_HIP(run_dot_qz_rz(P, q, r, z, sp), "pcg_solve dot");
        }
        FEM_HIP(run_cg_update_p(P, p, u, z, sp, variant), "pcg_solve update p");
    }
    return finish(FEM_ENOTCONV, k, rel);
}

// Argument checks shared by the solve entry points; resolves FEM_CG_AUTO.
static fem_status check_solve_args(fem_problem* P, const double* b, const double* u, double rtol, int maxit,
                                   int pc, int sp, int sweeps, int* variant) {
    CHECK_P(P); CHECK_PTR(b); CHECK_PTR(u);
    if (check_prec(sp)) return FEM_EINVAL;
    if (pc != FEM_PC_SCHWARZ && pc != FEM_PC_DSS && pc != FEM_PC_JACOBI && pc != FEM_PC_TWO_LEVEL)
        return set_error(FEM_EINVAL, "pcg_solve: unknown preconditioner");
    if (!(rtol > 0) || maxit < 0 || sweeps < 1) return set_error(FEM_EINVAL, "pcg_solve: rtol > 0, maxit >= 0, sweeps >= 1");
    if (b == u) return set_error(FEM_EINVAL, "pcg_solve: b and u alias");
    if (*variant == FEM_CG_AUTO)
        *variant = (sp == FEM_F64 || pc == FEM_PC_DSS || pc == FEM_PC_JACOBI) ? FEM_CG_PCG : FEM_CG_FCG;
    if (*variant != FEM_CG_PCG && *variant != FEM_CG_FCG) return set_error(FEM_EINVAL, "pcg_solve: unknown variant");
    return FEM_OK;
}
}  // namespace fem

extern "C" fem_status pcg_solve_pc(fem_problem* P, const double* b, double* u, double rtol, int maxit, int pc,
                                   int sp, int sweeps, double omega, int variant, fem_solve_info* info) {
    const auto t0 = std::chrono::steady_clock::now();
    fem_solve_info loc{};
    if (!info) info = &loc;
    *info = fem_solve_info{};
    fem_status st = check_solve_args(P, b, u, rtol, maxit, pc, sp, sweeps, &variant);
    if (st != FEM_OK) return st;
    const size_t need = solve_bytes_for(P->cell_len, sp);
    if (P->solve_bytes < need) {
        hipFree(P->d_solve);
        P->d_solve = nullptr;
        P->solve_bytes = 0;
        hipError_t e = hipMalloc(&P->d_solve, need);
        if (e != hipSuccess) return set_error(FEM_ENOMEM, "pcg_solve: workspace allocation failed");
        P->solve_bytes = need;
    }
    return pcg_core(P, b, u, rtol, maxit, pc, sp, sweeps, omega, variant, static_cast<char*>(P->d_solve), info, t0);
}

extern "C" fem_status pcg_solve(fem_problem* P, const double* b, double* u, double rtol, int maxit,
                                int sp, int sweeps, double omega, int variant, fem_solve_info* info) {
    return pcg_solve_pc(P, b, u, rtol, maxit, FEM_PC_SCHWARZ, sp, sweeps, omega, variant, info);
}

extern "C" fem_status fem_precond_apply(fem_problem* P, int pc, const void* r, void* z, int prec) {
    CHECK_P(P); CHECK_PTR(r); CHECK_PTR(z);
    if (check_prec(prec)) return FEM_EINVAL;
    if (pc != FEM_PC_DSS && pc != FEM_PC_JACOBI) return set_error(FEM_EINVAL, "fem_precond_apply: kind must be FEM_PC_DSS or FEM_PC_JACOBI");
    if (r == z) return set_error(FEM_EINVAL, "fem_precond_apply: r and z alias");
    FEM_HIP(run_simple_precond(P, pc, static_cast<const double*>(r), z, prec, kSlotTmp), "fem_precond_apply");
    return FEM_OK;
}

// ------------------------------------------------ solve without allocation
// The solver vectors of pcg_solve_noalloc live in one file-scope device
// array, resolved per device on the first call there (hipGetSymbolAddress
// with that device current); host code uses only the resolved address.
namespace fem {
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
}  // namespace fem

static __device__ __align__(256) char scratch[fem::kNoAllocScratchBytes];

namespace {
std::once_flag g_scratch_once[fem::kMaxDevices];
void* g_scratch_ptr[fem::kMaxDevices];
hipError_t g_scratch_err[fem::kMaxDevices];
}  // namespace

extern "C" size_t fem_noalloc_scratch_bytes(void) { return fem::kNoAllocScratchBytes; }

extern "C" fem_status pcg_solve_noalloc(fem_problem* P, const double* b, double* u, double rtol, int maxit, int pc,
                                        int sp, int sweeps, double omega, int variant, fem_solve_info* info) {
    const auto t0 = std::chrono::steady_clock::now();
    fem_solve_info loc{};
    if (!info) info = &loc;
    *info = fem_solve_info{};
    fem_status st = check_solve_args(P, b, u, rtol, maxit, pc, sp, sweeps, &variant);
    if (st != FEM_OK) return st;
    const size_t need = solve_bytes_for(P->cell_len, sp);
    if (need > kNoAllocScratchBytes)
        return set_error(FEM_EINVAL, "pcg_solve_noalloc: the solver vectors need " + std::to_string(need) +
                                         " bytes, more than the " + std::to_string(kNoAllocScratchBytes) +
                                         "-byte device scratch");
    int dev = -1;
    FEM_HIP(hipGetDevice(&dev), "pcg_solve_noalloc");
    if (dev != P->device) return set_error(FEM_EINVAL, "pcg_solve_noalloc: call with the problem's device current");
    if (dev < 0 || dev >= kMaxDevices) return set_error(FEM_EINVAL, "pcg_solve_noalloc: device index out of range");
    std::call_once(g_scratch_once[dev], [dev]() {
        g_scratch_err[dev] = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
    });
    if (g_scratch_err[dev] != hipSuccess) return hip_error(g_scratch_err[dev], "pcg_solve_noalloc: scratch address");
    if (!g_scratch_ptr[dev]) return set_error(FEM_EHIP, "pcg_solve_noalloc: scratch address is null");
    return pcg_core(P, b, u, rtol, maxit, pc, sp, sweeps, omega, variant, static_cast<char*>(g_scratch_ptr[dev]),
                    info, t0);
}
