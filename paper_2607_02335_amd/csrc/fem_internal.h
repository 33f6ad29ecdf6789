// Internal declarations shared by the host library and the HIP kernels.
//
// Cell-wise storage layout (private to the library): cells are grouped in
// blocks of kLanes = 64 consecutive cells (lexicographic cell order, x
// fastest); a block stores its (p+1)^3 local nodes one after another and, for
// each node, the 64 cells of the block contiguously:
//
//     offset(e, l) = (e / 64) * (p+1)^3 * 64 + l * 64 + (e % 64)
//
// so a wavefront that walks 64 consecutive cells at one local node reads one
// contiguous 512-byte (FP64) segment.  This is the blocked element-fastest
// layout of Section 5.1 with the block size fixed to the wavefront width.
// Padding cells of the last block are zero in every vector.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <stddef.h>
#include <string>

#include "../../include/fem.h"

namespace fem {

constexpr int kLanes = 64;          // cells per storage block
constexpr int kMaxP = 7;

// --------------------------------------------------------------------------
// Storage precisions.  BF16 is stored as its 16-bit pattern and computed in
// FP32; conversions round to nearest even.
struct bf16_t { uint16_t bits; };

// FP16 (IEEE binary16) is stored as its bit pattern and computed in FP32;
// its range ends at 65504 and its normal range at 6.1e-5, so the solver
// stores FP16 copies of residuals scaled by a power of two (k_distribute).
struct f16_t { uint16_t bits; };

template <typename S> struct Prec;
template <> struct Prec<double> { using C = double; static constexpr int id = FEM_F64; };
template <> struct Prec<float>  { using C = float;  static constexpr int id = FEM_F32; };
template <> struct Prec<bf16_t> { using C = float;  static constexpr int id = FEM_BF16; };
template <> struct Prec<f16_t>  { using C = float;  static constexpr int id = FEM_F16; };

__host__ __device__ inline float bf16_to_f32(uint16_t b) {
    uint32_t u = static_cast<uint32_t>(b) << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))   // NaN stays NaN
        return static_cast<uint16_t>((u >> 16) | 0x0040u);
    uint32_t rounding = 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>((u + rounding) >> 16);
}

template <typename C> __device__ __forceinline__ C load_as(const double* p) { return (C)*p; }
template <typename C> __device__ __forceinline__ C load_as(const float* p) { return (C)*p; }
template <typename C> __device__ __forceinline__ C load_as(const bf16_t* p) { return (C)bf16_to_f32(p->bits); }
__device__ __forceinline__ float f16_to_f32(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
__device__ __forceinline__ uint16_t f32_to_f16(float f) { return __builtin_bit_cast(uint16_t, (_Float16)f); }
template <typename C> __device__ __forceinline__ C load_as(const f16_t* p) { return (C)f16_to_f32(p->bits); }
__device__ __forceinline__ void store_from(double* p, double v) { *p = v; }
__device__ __forceinline__ void store_from(double* p, float v) { *p = (double)v; }
__device__ __forceinline__ void store_from(float* p, float v) { *p = v; }
__device__ __forceinline__ void store_from(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ void store_from(bf16_t* p, float v) { p->bits = f32_to_bf16(v); }
__device__ __forceinline__ void store_from(bf16_t* p, double v) { p->bits = f32_to_bf16((float)v); }
__device__ __forceinline__ void store_from(f16_t* p, float v) { p->bits = f32_to_f16(v); }
__device__ __forceinline__ void store_from(f16_t* p, double v) { p->bits = f32_to_f16((float)v); }

// Streaming (nontemporal) access for FP64 data that one pass reads or writes
// once and that the next kernels do not read back soon: the patch inverse's
// cell-wise input in the assembly and its cell-wise output in the row
// combine.  Keeping those lines out of the Infinity Cache leaves it to the
// intermediate arrays that are re-read (measured on the Q3 64^3 FP64 step:
// 286 -> 267 us).  The other precisions keep cached accesses: their arrays
// are a half or a quarter of the size, and streaming was not measured there.
template <typename C> __device__ __forceinline__ C load_stream(const double* p) {
    return (C)__builtin_nontemporal_load(p);
}
template <typename C, typename S> __device__ __forceinline__ C load_stream(const S* p) { return load_as<C>(p); }
__device__ __forceinline__ void store_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }
template <typename S, typename C> __device__ __forceinline__ void store_stream(S* p, C v) { store_from(p, v); }

// --------------------------------------------------------------------------
// One problem's entry in a launch.  Kernels walk a flat range of tiles; a
// launch over several problems (of one degree) concatenates their tile
// ranges, and each tile finds its problem by binary search on tile_begin.
struct ProbEntry {
    int n[3];            // cells per direction
    int p;               // degree
    size_t len;          // elements of a cell-wise vector (nblk * (p+1)^3 * 64)
    int ncells;
    int nblk;            // storage blocks (ceil(ncells / 64))
    int dirichlet;       // 1: mask boundary copies
    int tile_begin;      // first tile of this problem in the launch
    int ntiles;
    const double* h[3];  // cell widths per direction (device)
    const void* fd[3];   // per-direction fast-diagonalisation data (device)
    const void* a;       // operands; meaning defined by each kernel
    const void* b;
    void* c;
    void* d;
    void* e;
    void* f;
    double* red;         // per-problem reduction partials / scalars
    double alpha;        // scalar operand (e.g. damping)
    int ntiles_red;      // tiles of the reduction kernels (<= kRedParts)
    int blocks_per_red;  // storage blocks per reduction tile (red_lsplit == 1)
    int red_lsplit;      // reduction tiles per storage block (blocks_per_red == 1)
    int zchunk;          // cell layers per z-chunk of the fused patch sweep
};

struct LaunchTable {
    int nprob;
    int total_tiles;
    const ProbEntry* tab;   // device array of nprob entries (nprob > 1)
    ProbEntry one;          // used when nprob == 1
};

// Entry of the problem owning `tile`.  Single-problem launches (MULTI =
// false) read the entry from the kernel arguments, multi-problem launches
// from the device table; keeping the two apart lets the compiler read fields
// with scalar loads instead of copying the struct to scratch.
template <bool MULTI>
__device__ __forceinline__ const ProbEntry& entry(const LaunchTable& L, int tile) {
    if constexpr (!MULTI) {
        return L.one;
    } else {
        int lo = 0, hi = L.nprob - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (L.tab[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
        }
        return L.tab[lo];
    }
}
// Entry of problem i (one workgroup per problem).
template <bool MULTI>
__device__ __forceinline__ const ProbEntry& entry_at(const LaunchTable& L, int i) {
    if constexpr (!MULTI) return L.one; else return L.tab[i];
}

__host__ __device__ inline size_t cell_offset(int e, int l, int nn) {
    return (size_t)(e / kLanes) * nn * kLanes + (size_t)l * kLanes + (e % kLanes);
}

// Reference 1D matrices of one degree, passed by value to kernels.
template <int P, typename C> struct RefMats {
    C M[(P + 1) * (P + 1)];
    C K[(P + 1) * (P + 1)];
};

// Size of the per-direction FD record of one vertex line: S (nP x nP, row
// major, columns are eigenvectors) followed by lambda (nP), padded.
__host__ __device__ constexpr int fd_record(int p) {
    return ((2 * p - 1) * (2 * p - 1) + (2 * p - 1) + 3) & ~3;
}

}  // namespace fem

// ---------------------------------------------------------------------------
// The problem handle.
struct fem_problem {
    int p;
    int n[3];
    int bc;
    int ncells;
    int nblk;
    size_t cell_len;       // nblk * (p+1)^3 * 64
    size_t global_len;
    size_t npatch;
    int npblk;             // patch storage blocks (ceil(npatch / 64))
    hipStream_t stream;
    int device;
    bool owned_by_batch;
    double* d_h;           // widths: [n0 | n1 | n2]
    double* d_fd64;        // FD data FP64: [3][nmax-1 lines][fd_record(p)]
    float* d_fd32;         // FD data FP32, same layout
    size_t fd_dir_stride;  // elements between directions in d_fd64/d_fd32
    double* d_red;         // reduction partials and scalar slots
    void* d_patch;         // patch-result buffer (sized for FP64)
    size_t patch_len;      // elements of the patch buffer
    void* d_tmp;           // smoother scratch: one cell vector (sized for FP64)
    void* d_glob;          // assembled residual in global-node order (FP64 size; p >= 4 patch solves)
    void* d_solve;         // pcg_solve vectors, allocated on first use
    size_t solve_bytes;
    double* h_red;         // pinned host mirror of the scalar slots (null for arena problems)
    bool external_mem;     // buffers carved from caller memory (freed with it)
    // coarse (Q1 on the interior vertices) level of the two-level preconditioner
    int cm[3];             // interior vertices per direction (n - 1)
    double* d_cfd;         // per direction: S (cm x cm, row-major) then lambda (cm)
    size_t cfd_off[3];     // offsets of the directions in d_cfd
    double* d_cvec;        // two coarse vectors of cm[0] cm[1] cm[2] values
    double* d_corner;      // per-cell corner sums of a restriction: [8][nblk * 64]
};

// Caller-provided memory for a problem (the solve server's arena): device
// bytes for the workspace (at least workspace_bytes) and pinned host bytes
// (at least problem_stage_bytes) from which the set-up data is uploaded
// asynchronously; the caller keeps the staging alive until the stream has
// passed the uploads.
struct ProblemMem {
    char* dev;
    size_t dev_bytes;
    char* stage;
    size_t stage_bytes;
};
