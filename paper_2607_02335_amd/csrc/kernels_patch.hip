// Additive Schwarz over 2x2x2-cell vertex patches with fast-diagonalisation
// patch inverses.
//
// Patch of interior vertex (vi, vj, vk): the (2p-1)^3 nodes strictly inside
// the cells [vi-1, vi] x [vj-1, vj] x [vk-1, vk]; patch-local node
// (qx, qy, qz), qx = I - (vi-1) p - 1 for global node plane I.
//
// Phase 1 (k_pi_solve), one workgroup per CBP consecutive patches along x:
//   restrict:  r_P(q) = sum of the coincident cell copies of node q among the
//              patch's eight cells (= (G^T r)(q): every cell holding q lies in
//              the patch), so the smoother sees r only through its assembly,
//              the consistency the paper's equivalence theorem asks of a
//              preconditioner (Section 3.2, Remarks after the theorem);
//   solve:     z_P = (Sx (x) Sy (x) Sz) diag(1/(lx+ly+lz)) (Sx (x) Sy (x) Sz)^T r_P,
//              six 1D contractions staged in LDS, one thread per line;
//   store z_P in a patch buffer.
// Phase 2 (k_pi_combine), one thread per cell copy:
//   z(node) = sum of z_P(node) over the patches whose interior contains the
//   node, added in increasing vertex order.  That order depends only on the
//   global node, so all copies of a node receive bitwise identical values:
//   the output is continuous exactly, not just to rounding.
#include <algorithm>
#include <atomic>

#include "fem_internal.h"
#include "launch.h"
#include "mfma.h"
#include "mixed.h"
#include "trace.h"

namespace fem {

// Process-wide kernel-variant switches (fem_set_option, for comparisons),
// atomic because any thread may set them while others launch.
// Patch-inverse variant: -1 picks by degree and precision, else the
// FEM_OPT_PI_FUSED value.
std::atomic<int> g_pi_fused{-1};
// 1: combine the two-phase patch results with one wavefront per storage
// block (all planes) instead of one per (block, plane).
std::atomic<int> g_combine_per_cell{0};
// 1: phase 1 of the p <= 3 patch inverse sums the copies from the cell-wise
// vector itself instead of reading the owner-assembled global-node array.
std::atomic<int> g_restrict_from_cells{0};
// Patch results per z-slab (MB) of the single-problem two-phase patch
// inverse for p <= 3; 0 runs one solve and one combine launch.
std::atomic<int> g_pi_slab_mb{0};

// Reciprocal of a positive normal value (the FD eigenvalue sums): the
// hardware estimate refined by Newton-Raphson steps r <- r + r (1 - d r),
// two for FP64 and one for FP32 (each step doubles the correct bits), so the
// FD scaling multiplies instead of running the full IEEE division sequence.
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float d) {
    const float r = __builtin_amdgcn_rcpf(d);
    const float e = __builtin_fmaf(-d, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

template <int P, typename C> constexpr int pi_patches_per_tile() {
    constexpr int nP = 2 * P - 1;
    int cb = 64;
    while (cb > 1 && cb * nP * nP * nP * (int)sizeof(C) > 40 * 1024) cb >>= 1;
    return cb;
}

// pe: a = r (S), d = patch buffer (C), fd[0..2] = FD records (C) per
// direction, indexed by vertex line v-1.
template <int P, typename S, int CBP, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_solve(LaunchTable L) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, NN = N * N * N;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    constexpr int REC = fd_record(P);
    constexpr int NT = 256, LPT = NT / CBP;     // lines per tile-thread stride
    static_assert(NT % CBP == 0, "patches per tile must divide the workgroup");
    __shared__ C sv[nP3 * CBP];
    __shared__ C sS[3][CBP][nP2];
    __shared__ C sL[3][CBP][nP];
    const int tid = threadIdx.x;
    const int pc = tid % CBP;
    for (int tile = blockIdx.x; tile < L.total_tiles; tile += gridDim.x) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        const int npx = pe.n[0] - 1, npy = pe.n[1] - 1;
        const int tpr = (npx + CBP - 1) / CBP;
        const int row = t / tpr, xt = t % tpr;
        const int vj = 1 + row % npy, vk = 1 + row / npy;
        const int vi = 1 + xt * CBP + pc;
        const bool valid = vi <= npx;
        // FD data of this patch's three vertex lines
        for (int idx = tid / CBP; idx < 3 * (nP2 + nP); idx += LPT) {
            const int d = idx / (nP2 + nP), w = idx % (nP2 + nP);
            const int line = (d == 0 ? (valid ? vi : npx) : d == 1 ? vj : vk) - 1;
            const C v = static_cast<const C*>(pe.fd[d])[(size_t)line * REC + w];
            if (w < nP2) sS[d][pc][w] = v; else sL[d][pc][w - nP2] = v;
        }
        // restrict: sum coincident copies from the eight cells
        const S* r = static_cast<const S*>(pe.a);
        const int n0 = pe.n[0], n1 = pe.n[1];
        for (int q = tid / CBP; q < nP3; q += LPT) {
            const int qx = q % nP, qy = (q / nP) % nP, qz = q / nP2;
            C s = 0;
            if (valid) {
#pragma unroll
                for (int s3 = 0; s3 < 2; ++s3) {
                    const int c = qz + 1 - s3 * P;
                    if (c < 0 || c > P) continue;
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2) {
                        const int b = qy + 1 - s2 * P;
                        if (b < 0 || b > P) continue;
#pragma unroll
                        for (int s1 = 0; s1 < 2; ++s1) {
                            const int a = qx + 1 - s1 * P;
                            if (a < 0 || a > P) continue;
                            const int e = (vi - 1 + s1) + n0 * ((vj - 1 + s2) + n1 * (vk - 1 + s3));
                            s += load_as<C>(r + cell_offset(e, a + N * (b + N * c), NN));
                        }
                    }
                }
            }
            sv[q * CBP + pc] = s;
        }
        __syncthreads();
        // forward z: v <- Sz^T v along z lines
        for (int ln = tid / CBP; ln < nP2; ln += LPT) {
            C v[nP];
#pragma unroll
            for (int i = 0; i < nP; ++i) v[i] = sv[(ln + nP2 * i) * CBP + pc];
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += sS[2][pc][i * nP + j] * v[i];
                sv[(ln + nP2 * j) * CBP + pc] = s;
            }
        }
        __syncthreads();
        // forward y
        for (int ln = tid / CBP; ln < nP2; ln += LPT) {
            const int qx = ln % nP, qz = ln / nP;
            C v[nP];
#pragma unroll
            for (int i = 0; i < nP; ++i) v[i] = sv[(qx + nP * i + nP2 * qz) * CBP + pc];
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += sS[1][pc][i * nP + j] * v[i];
                sv[(qx + nP * j + nP2 * qz) * CBP + pc] = s;
            }
        }
        __syncthreads();
        // forward x, scale by 1/(lx+ly+lz), backward x (same line, no sync)
        for (int ln = tid / CBP; ln < nP2; ln += LPT) {
            const int qy = ln % nP, qz = ln / nP;
            C v[nP], w[nP];
#pragma unroll
            for (int i = 0; i < nP; ++i) v[i] = sv[(i + nP * ln) * CBP + pc];
            const C lyz = sL[1][pc][qy] + sL[2][pc][qz];
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += sS[0][pc][i * nP + j] * v[i];
                w[j] = s * recip(sL[0][pc][j] + lyz);
            }
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += sS[0][pc][i * nP + j] * w[j];
                sv[(i + nP * ln) * CBP + pc] = s;
            }
        }
        __syncthreads();
        // backward y
        for (int ln = tid / CBP; ln < nP2; ln += LPT) {
            const int qx = ln % nP, qz = ln / nP;
            C v[nP];
#pragma unroll
            for (int j = 0; j < nP; ++j) v[j] = sv[(qx + nP * j + nP2 * qz) * CBP + pc];
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += sS[1][pc][i * nP + j] * v[j];
                sv[(qx + nP * i + nP2 * qz) * CBP + pc] = s;
            }
        }
        __syncthreads();
        // backward z and store to the patch buffer
        C* pbuf = static_cast<C*>(pe.d);
        const int pidx = (vi - 1) + npx * ((vj - 1) + npy * (vk - 1));
        C* out = pbuf + (size_t)(pidx / kLanes) * nP3 * kLanes + (pidx % kLanes);
        for (int ln = tid / CBP; ln < nP2; ln += LPT) {
            C v[nP];
#pragma unroll
            for (int j = 0; j < nP; ++j) v[j] = sv[(ln + nP2 * j) * CBP + pc];
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += sS[2][pc][i * nP + j] * v[j];
                if (valid) out[(size_t)(ln + nP2 * i) * kLanes] = s;
            }
        }
        __syncthreads();
    }
}

// pe: c = z (S), d = patch buffer (C), alpha = damping; ACC: z += alpha sum.
template <int P, typename S, int ACC, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_combine(LaunchTable L) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, NN = N * N * N;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    for (int tile = blockIdx.x; tile < L.total_tiles; tile += gridDim.x) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int blk = tile - pe.tile_begin;
        const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
        const int npx = n0 - 1, npy = n1 - 1;
        const C* pbuf = static_cast<const C*>(pe.d);
        S* z = static_cast<S*>(pe.c) + (size_t)blk * NN * kLanes;
        const C alpha = (C)pe.alpha;
        for (int idx = threadIdx.x; idx < NN * kLanes; idx += 256) {
            const int l = idx / kLanes, lane = idx % kLanes;
            const int e = blk * kLanes + lane;
            C sum = 0;
            if (e < pe.ncells) {
                const int i = e % n0, j = (e / n0) % n1, k = e / (n0 * n1);
                const int a = l % N, b = (l / N) % N, c = l / (N * N);
                // per direction: up to two (vertex, patch-local index) pairs,
                // increasing vertex order
                int vx[2], qx[2], nx = 0, vy[2], qy[2], ny = 0, vz[2], qz[2], nz = 0;
                if (a == 0) { vx[0] = i; qx[0] = P - 1; nx = 1; }
                else if (a == P) { vx[0] = i + 1; qx[0] = P - 1; nx = 1; }
                else { vx[0] = i; qx[0] = P - 1 + a; vx[1] = i + 1; qx[1] = a - 1; nx = 2; }
                if (b == 0) { vy[0] = j; qy[0] = P - 1; ny = 1; }
                else if (b == P) { vy[0] = j + 1; qy[0] = P - 1; ny = 1; }
                else { vy[0] = j; qy[0] = P - 1 + b; vy[1] = j + 1; qy[1] = b - 1; ny = 2; }
                if (c == 0) { vz[0] = k; qz[0] = P - 1; nz = 1; }
                else if (c == P) { vz[0] = k + 1; qz[0] = P - 1; nz = 1; }
                else { vz[0] = k; qz[0] = P - 1 + c; vz[1] = k + 1; qz[1] = c - 1; nz = 2; }
                for (int sz = 0; sz < nz; ++sz) {
                    if (vz[sz] < 1 || vz[sz] > n2 - 1) continue;
                    for (int sy = 0; sy < ny; ++sy) {
                        if (vy[sy] < 1 || vy[sy] > npy) continue;
                        for (int sx = 0; sx < nx; ++sx) {
                            if (vx[sx] < 1 || vx[sx] > npx) continue;
                            const int pidx = (vx[sx] - 1) + npx * ((vy[sy] - 1) + npy * (vz[sz] - 1));
                            const int q = qx[sx] + nP * (qy[sy] + nP * qz[sz]);
                            sum += pbuf[(size_t)(pidx / kLanes) * nP3 * kLanes + (size_t)q * kLanes + (pidx % kLanes)];
                        }
                    }
                }
            }
            C out = alpha * sum;
            if (ACC) out = load_as<C>(z + idx) + out;
            if (e >= pe.ncells) out = (C)0;
            store_from(z + idx, out);
        }
    }
}

// ---------------------------------------------------------------------------
// Low-degree variants (p <= 4): the 1D eigenbasis of the current direction is
// held in registers during each pass (the y and z bases are shared by the
// whole tile and read as LDS broadcasts), so LDS carries only line data.
// Tiles are spread so that consecutive tiles (neighbouring patch rows that
// share cells) run on the same XCD and reuse its L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
    const int per = G / 8;               // G is a multiple of 8
    return (b % 8) * per + b / 8;
}

template <int P, typename S, int CBP, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_solve_r(LaunchTable L) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, NN = N * N * N;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    constexpr int REC = fd_record(P);
    constexpr int NT = 256, LPT = NT / CBP;
    static_assert(NT % CBP == 0, "patches per tile must divide the workgroup");
    __shared__ C sv[nP3 * CBP];
    __shared__ C sSx[CBP][nP2 + 1];
    __shared__ C sLx[CBP][nP];
    __shared__ C sSyz[2][nP2];
    __shared__ C sLyz[2][nP];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= L.total_tiles) return;
    const int tid = threadIdx.x;
    const int pc = tid % CBP;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int t = tile - pe.tile_begin;
    const int npx = pe.n[0] - 1, npy = pe.n[1] - 1;
    const int tpr = (npx + CBP - 1) / CBP;
    const int row = t / tpr, xt = t % tpr;
    const int vj = 1 + row % npy, vk = 1 + row / npy;
    const int vi = 1 + xt * CBP + pc;
    const bool valid = vi <= npx;
    {
        const C* fx = static_cast<const C*>(pe.fd[0]) + (size_t)((valid ? vi : npx) - 1) * REC;
        for (int w = tid / CBP; w < nP2 + nP; w += LPT) {
            const C v = fx[w];
            if (w < nP2) sSx[pc][w] = v; else sLx[pc][w - nP2] = v;
        }
        for (int w = tid; w < 2 * (nP2 + nP); w += NT) {
            const int d = w / (nP2 + nP), o = w % (nP2 + nP);
            const C v = static_cast<const C*>(pe.fd[1 + d])[(size_t)((d == 0 ? vj : vk) - 1) * REC + o];
            if (o < nP2) sSyz[d][o] = v; else sLyz[d][o - nP2] = v;
        }
    }
    const S* r = static_cast<const S*>(pe.a);
    const int n0 = pe.n[0], n1 = pe.n[1];
    for (int q = tid / CBP; q < nP3; q += LPT) {
        const int qx = q % nP, qy = (q / nP) % nP, qz = q / nP2;
        C s = 0;
        if (valid) {
#pragma unroll
            for (int s3 = 0; s3 < 2; ++s3) {
                const int c = qz + 1 - s3 * P;
                if (c < 0 || c > P) continue;
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) {
                    const int b = qy + 1 - s2 * P;
                    if (b < 0 || b > P) continue;
#pragma unroll
                    for (int s1 = 0; s1 < 2; ++s1) {
                        const int a = qx + 1 - s1 * P;
                        if (a < 0 || a > P) continue;
                        const int e = (vi - 1 + s1) + n0 * ((vj - 1 + s2) + n1 * (vk - 1 + s3));
                        s += load_as<C>(r + cell_offset(e, a + N * (b + N * c), NN));
                    }
                }
            }
        }
        sv[q * CBP + pc] = s;
    }
    __syncthreads();
    C Sm[nP2];
    // forward z (broadcast basis)
#pragma unroll
    for (int i = 0; i < nP2; ++i) Sm[i] = sSyz[1][i];
    for (int ln = tid / CBP; ln < nP2; ln += LPT) {
        C v[nP];
#pragma unroll
        for (int i = 0; i < nP; ++i) v[i] = sv[(ln + nP2 * i) * CBP + pc];
#pragma unroll
        for (int j = 0; j < nP; ++j) {
            C s = 0;
#pragma unroll
            for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i];
            sv[(ln + nP2 * j) * CBP + pc] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < nP2; ++i) Sm[i] = sSyz[0][i];
    for (int ln = tid / CBP; ln < nP2; ln += LPT) {                 // forward y
        const int qx = ln % nP, qz = ln / nP;
        C v[nP];
#pragma unroll
        for (int i = 0; i < nP; ++i) v[i] = sv[(qx + nP * i + nP2 * qz) * CBP + pc];
#pragma unroll
        for (int j = 0; j < nP; ++j) {
            C s = 0;
#pragma unroll
            for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i];
            sv[(qx + nP * j + nP2 * qz) * CBP + pc] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < nP2; ++i) Sm[i] = sSx[pc][i];
    for (int ln = tid / CBP; ln < nP2; ln += LPT) {                 // x: forward, scale, backward
        const int qy = ln % nP, qz = ln / nP;
        C v[nP], w[nP];
#pragma unroll
        for (int i = 0; i < nP; ++i) v[i] = sv[(i + nP * ln) * CBP + pc];
        const C lyz = sLyz[0][qy] + sLyz[1][qz];
#pragma unroll
        for (int j = 0; j < nP; ++j) {
            C s = 0;
#pragma unroll
            for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i];
            w[j] = s * recip(sLx[pc][j] + lyz);
        }
#pragma unroll
        for (int i = 0; i < nP; ++i) {
            C s = 0;
#pragma unroll
            for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * w[j];
            sv[(i + nP * ln) * CBP + pc] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < nP2; ++i) Sm[i] = sSyz[0][i];
    for (int ln = tid / CBP; ln < nP2; ln += LPT) {                 // backward y
        const int qx = ln % nP, qz = ln / nP;
        C v[nP];
#pragma unroll
        for (int j = 0; j < nP; ++j) v[j] = sv[(qx + nP * j + nP2 * qz) * CBP + pc];
#pragma unroll
        for (int i = 0; i < nP; ++i) {
            C s = 0;
#pragma unroll
            for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * v[j];
            sv[(qx + nP * i + nP2 * qz) * CBP + pc] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < nP2; ++i) Sm[i] = sSyz[1][i];
    C* pbuf = static_cast<C*>(pe.d);
    const int pidx = (vi - 1) + npx * ((vj - 1) + npy * (vk - 1));
    C* out = pbuf + (size_t)(pidx / kLanes) * nP3 * kLanes + (pidx % kLanes);
    for (int ln = tid / CBP; ln < nP2; ln += LPT) {                 // backward z, store
        C v[nP];
#pragma unroll
        for (int j = 0; j < nP; ++j) v[j] = sv[(ln + nP2 * j) * CBP + pc];
#pragma unroll
        for (int i = 0; i < nP; ++i) {
            C s = 0;
#pragma unroll
            for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * v[j];
            if (valid) out[(size_t)(ln + nP2 * i) * kLanes] = s;
        }
    }
}

// One thread per cell (p <= 3): the eight corner patches' buffer addresses
// are formed once per cell, node loops are unrolled at compile time.
template <int P, typename S, int ACC, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_combine_cell(LaunchTable L) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int tile = blockIdx.x * 4 + wv;
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int blk = tile - pe.tile_begin;
    const int e = blk * kLanes + lane;
    S* z = static_cast<S*>(pe.c) + (size_t)blk * NN * kLanes + lane;
    if (e >= pe.ncells) {
#pragma unroll
        for (int l = 0; l < NN; ++l) store_from(z + l * kLanes, (C)0);
        return;
    }
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int npx = n0 - 1, npy = n1 - 1;
    const int i = e % n0, j = (e / n0) % n1, k = e / (n0 * n1);
    const C* pbuf = static_cast<const C*>(pe.d);
    const C* corner[2][2][2];
#pragma unroll
    for (int sz = 0; sz < 2; ++sz)
#pragma unroll
        for (int sy = 0; sy < 2; ++sy)
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
                const int vx = i + sx, vy = j + sy, vz = k + sz;
                const bool ok = vx >= 1 && vx <= npx && vy >= 1 && vy <= npy && vz >= 1 && vz <= n2 - 1;
                const int pidx = ok ? (vx - 1) + npx * ((vy - 1) + npy * (vz - 1)) : 0;
                corner[sz][sy][sx] = ok ? pbuf + (size_t)(pidx / kLanes) * nP3 * kLanes + (pidx % kLanes) : nullptr;
            }
    const C alpha = (C)pe.alpha;
#pragma unroll
    for (int c = 0; c < N; ++c)
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
            for (int a = 0; a < N; ++a) {
                C sum = 0;
#pragma unroll
                for (int sz = 0; sz < 2; ++sz) {
                    if ((sz == 0 && c == P) || (sz == 1 && c == 0)) continue;
                    const int qz = sz == 0 ? P - 1 + c : c - 1;
#pragma unroll
                    for (int sy = 0; sy < 2; ++sy) {
                        if ((sy == 0 && b == P) || (sy == 1 && b == 0)) continue;
                        const int qy = sy == 0 ? P - 1 + b : b - 1;
#pragma unroll
                        for (int sx = 0; sx < 2; ++sx) {
                            if ((sx == 0 && a == P) || (sx == 1 && a == 0)) continue;
                            const int qx = sx == 0 ? P - 1 + a : a - 1;
                            const C* src = corner[sz][sy][sx];
                            if (src) sum += src[(size_t)(qx + nP * (qy + nP * qz)) * kLanes];
                        }
                    }
                }
                const int l = a + N * b + N2 * c;
                C out = alpha * sum;
                if (ACC) out = load_as<C>(z + l * kLanes) + out;
                store_from(z + l * kLanes, out);
            }
}

// ---------------------------------------------------------------------------
// Fused sweep (p <= 3): no patch buffer.  A workgroup owns TX x TY cell
// columns and a chunk of cell layers [k0, k1) and walks the vertex layers
// k0..k1 in order.  Per vertex layer vk:
//   * cell layers vk-1 and vk sit in an LDS ring (TX+2 x TY+2 cells each,
//     loaded with coalesced reads); the next cell layer is fetched into
//     registers while this layer is solved, hiding its latency;
//   * the (TX+1) x (TY+1) patches of the layer are restricted from the ring,
//     solved by fast diagonalisation (five LDS passes) and combined at once:
//     cell layer vk-1 is finished (its partial sum from vertex layer vk-1
//     plus this layer's terms) and written out, and cell layer vk starts a
//     partial sum with this layer's terms.
// Terms are added in ascending vertex order along z, y and x for every copy
// of a node, so the copies of a node stay bitwise equal.  Patches on the
// border of a tile are solved by both neighbouring tiles; that extra
// arithmetic is the price of never writing patch results to memory.
template <int P, typename S, int TX, int TY, int NST, int ACC, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_sweep(LaunchTable L) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    constexpr int REC = fd_record(P);
    constexpr int NPL = (TX + 1) * (TY + 1);      // patches per vertex layer
    constexpr int LG = 256 / NST;                 // line groups
    constexpr int CX = TX + 2, CY = TY + 2;       // cell window per layer
    constexpr int NCW = CX * CY;
    constexpr int NLOAD = NCW * NN;               // values per cell layer
    constexpr int PF = (NLOAD + 255) / 256;       // prefetch registers per thread
    static_assert(NPL <= NST && 256 % NST == 0, "patch slots must cover a layer and divide the workgroup");
    __shared__ C cells[2][NLOAD];                 // [node][cell window] per layer
    __shared__ C pv[nP3 * NPL];                   // current patch layer [q][patch]
    __shared__ C part[TX * TY * NN];              // partial sums of the open cell layer
    __shared__ C sSx[TX + 1][nP2 + 1];
    __shared__ C sSy[TY + 1][nP2 + 1];
    __shared__ C sSz[nP2];
    __shared__ C sLx[TX + 1][nP];
    __shared__ C sLy[TY + 1][nP];
    __shared__ C sLz[nP];

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int ntx = (n0 + TX - 1) / TX, nty = (n1 + TY - 1) / TY;
    int t = tile - pe.tile_begin;
    const int tx = t % ntx;
    t /= ntx;
    const int ty = t % nty;
    const int kc = t / nty;
    const int i0 = tx * TX, j0 = ty * TY;
    const int k0 = kc * pe.zchunk;
    const int k1 = min(k0 + pe.zchunk, n2);
    const int tid = threadIdx.x, ps = tid % NST, lg = tid / NST;
    const int pxo = ps % (TX + 1), pyo = min(ps / (TX + 1), TY);
    const int vi = i0 + pxo, vj = j0 + pyo;
    const bool slot_ok = ps < NPL && vi >= 1 && vi <= n0 - 1 && vj >= 1 && vj <= n1 - 1;
    const S* r = static_cast<const S*>(pe.a);
    S* zout = static_cast<S*>(pe.c);
    const C alpha = (C)pe.alpha;

    for (int w = tid; w < (TX + 1) * (nP2 + nP); w += 256) {
        const int col = w / (nP2 + nP), o = w % (nP2 + nP);
        const int line = max(0, min(i0 + col, n0 - 1) - 1);
        const C v = static_cast<const C*>(pe.fd[0])[(size_t)line * REC + o];
        if (o < nP2) sSx[col][o] = v; else sLx[col][o - nP2] = v;
    }
    for (int w = tid; w < (TY + 1) * (nP2 + nP); w += 256) {
        const int col = w / (nP2 + nP), o = w % (nP2 + nP);
        const int line = max(0, min(j0 + col, n1 - 1) - 1);
        const C v = static_cast<const C*>(pe.fd[1])[(size_t)line * REC + o];
        if (o < nP2) sSy[col][o] = v; else sLy[col][o - nP2] = v;
    }

    // load of one cell layer: item = window cell + NCW * node (x fastest)
    auto fetch = [&](int k, C* regs) {
#pragma unroll
        for (int m = 0; m < PF; ++m) {
            const int item = tid + 256 * m;
            C v = 0;
            if (item < NLOAD && k >= 0 && k < n2) {
                const int w = item % NCW, l = item / NCW;
                const int i = i0 - 1 + w % CX, j = j0 - 1 + w / CX;
                if (i >= 0 && i < n0 && j >= 0 && j < n1)
                    v = load_as<C>(r + cell_offset(i + n0 * (j + n1 * k), l, NN));
            }
            regs[m] = v;
        }
    };
    auto stash = [&](C* dst, const C* regs) {
#pragma unroll
        for (int m = 0; m < PF; ++m) {
            const int item = tid + 256 * m;
            if (item < NLOAD) dst[item] = regs[m];
        }
    };
    {
        C reg[PF];
        fetch(k0 - 1, reg);
        stash(cells[(k0 + 1) & 1], reg);           // slot of layer k0-1
        fetch(k0, reg);
        stash(cells[k0 & 1], reg);
    }
    __syncthreads();

    for (int vk = k0; vk <= k1; ++vk) {
        C nxt[PF];
        fetch(vk + 1, nxt);                            // in flight during this layer
        const bool layer_ok = vk >= 1 && vk <= n2 - 1; // uniform over the workgroup
        if (layer_ok) {
            for (int w = tid; w < nP2 + nP; w += 256) {
                const C v = static_cast<const C*>(pe.fd[2])[(size_t)(vk - 1) * REC + w];
                if (w < nP2) sSz[w] = v; else sLz[w - nP2] = v;
            }
            // restrict from the ring: layer vk-1 is s3 = 0, layer vk is s3 = 1
            if (ps < NPL) {
                const C* lay[2] = {cells[(vk + 1) & 1], cells[vk & 1]};
                for (int q = lg; q < nP3; q += LG) {
                    const int qx = q % nP, qy = (q / nP) % nP, qz = q / nP2;
                    C s = 0;
                    if (slot_ok) {
#pragma unroll
                        for (int s3 = 0; s3 < 2; ++s3) {
                            const int c = qz + 1 - s3 * P;
                            if (c < 0 || c > P) continue;
#pragma unroll
                            for (int s2 = 0; s2 < 2; ++s2) {
                                const int b = qy + 1 - s2 * P;
                                if (b < 0 || b > P) continue;
#pragma unroll
                                for (int s1 = 0; s1 < 2; ++s1) {
                                    const int a = qx + 1 - s1 * P;
                                    if (a < 0 || a > P) continue;
                                    const int wcell = (pxo + s1) + CX * (pyo + s2);
                                    s += lay[s3][(a + N * (b + N * c)) * NCW + wcell];
                                }
                            }
                        }
                    }
                    pv[q * NPL + ps] = s;
                }
            }
            __syncthreads();
            if (ps < NPL) {
                C Sm[nP2];
#pragma unroll
                for (int i = 0; i < nP2; ++i) Sm[i] = sSz[i];
                for (int ln = lg; ln < nP2; ln += LG) {                 // forward z
                    C v[nP];
#pragma unroll
                    for (int i = 0; i < nP; ++i) v[i] = pv[(ln + nP2 * i) * NPL + ps];
#pragma unroll
                    for (int j = 0; j < nP; ++j) {
                        C s = 0;
#pragma unroll
                        for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i];
                        pv[(ln + nP2 * j) * NPL + ps] = s;
                    }
                }
            }
            __syncthreads();
            if (ps < NPL) {
                C Sm[nP2];
#pragma unroll
                for (int i = 0; i < nP2; ++i) Sm[i] = sSy[pyo][i];
                for (int ln = lg; ln < nP2; ln += LG) {                 // forward y
                    const int qx = ln % nP, qz = ln / nP;
                    C v[nP];
#pragma unroll
                    for (int i = 0; i < nP; ++i) v[i] = pv[(qx + nP * i + nP2 * qz) * NPL + ps];
#pragma unroll
                    for (int j = 0; j < nP; ++j) {
                        C s = 0;
#pragma unroll
                        for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i];
                        pv[(qx + nP * j + nP2 * qz) * NPL + ps] = s;
                    }
                }
            }
            __syncthreads();
            if (ps < NPL) {
                C Sm[nP2];
#pragma unroll
                for (int i = 0; i < nP2; ++i) Sm[i] = sSx[pxo][i];
                for (int ln = lg; ln < nP2; ln += LG) {                 // x: forward, scale, back
                    const int qy = ln % nP, qz = ln / nP;
                    C v[nP], w[nP];
#pragma unroll
                    for (int i = 0; i < nP; ++i) v[i] = pv[(i + nP * ln) * NPL + ps];
                    const C lyz = sLy[pyo][qy] + sLz[qz];
#pragma unroll
                    for (int j = 0; j < nP; ++j) {
                        C s = 0;
#pragma unroll
                        for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i];
                        w[j] = s * recip(sLx[pxo][j] + lyz);
                    }
#pragma unroll
                    for (int i = 0; i < nP; ++i) {
                        C s = 0;
#pragma unroll
                        for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * w[j];
                        pv[(i + nP * ln) * NPL + ps] = s;
                    }
                }
            }
            __syncthreads();
            if (ps < NPL) {
                C Sm[nP2];
#pragma unroll
                for (int i = 0; i < nP2; ++i) Sm[i] = sSy[pyo][i];
                for (int ln = lg; ln < nP2; ln += LG) {                 // backward y
                    const int qx = ln % nP, qz = ln / nP;
                    C v[nP];
#pragma unroll
                    for (int j = 0; j < nP; ++j) v[j] = pv[(qx + nP * j + nP2 * qz) * NPL + ps];
#pragma unroll
                    for (int i = 0; i < nP; ++i) {
                        C s = 0;
#pragma unroll
                        for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * v[j];
                        pv[(qx + nP * i + nP2 * qz) * NPL + ps] = s;
                    }
                }
            }
            __syncthreads();
            if (ps < NPL) {
                C Sm[nP2];
#pragma unroll
                for (int i = 0; i < nP2; ++i) Sm[i] = sSz[i];
                for (int ln = lg; ln < nP2; ln += LG) {                 // backward z
                    C v[nP];
#pragma unroll
                    for (int j = 0; j < nP; ++j) v[j] = pv[(ln + nP2 * j) * NPL + ps];
#pragma unroll
                    for (int i = 0; i < nP; ++i) {
                        C s = 0;
#pragma unroll
                        for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * v[j];
                        pv[(ln + nP2 * i) * NPL + ps] = s;
                    }
                }
            }
            __syncthreads();
        }
        // finish cell layer vk-1, open cell layer vk
        for (int item = tid; item < TX * TY * NN; item += 256) {
            const int cx = item % TX;
            const int cy = (item / TX) % TY;
            const int l = item / (TX * TY);
            const int i = i0 + cx, j = j0 + cy;
            const int a = l % N, b = (l / N) % N, c = l / N2;
            // this layer's terms for a node of cell layer k at plane offset sz
            auto terms = [&](int sz, C acc) -> C {
#pragma unroll
                for (int sy = 0; sy < 2; ++sy) {
                    if ((sy == 0 && b == P) || (sy == 1 && b == 0)) continue;
                    const int vy = j + sy;
                    if (vy < 1 || vy > n1 - 1) continue;
                    const int qy = sy == 0 ? P - 1 + b : b - 1;
#pragma unroll
                    for (int sx = 0; sx < 2; ++sx) {
                        if ((sx == 0 && a == P) || (sx == 1 && a == 0)) continue;
                        const int vx = i + sx;
                        if (vx < 1 || vx > n0 - 1) continue;
                        const int qx = sx == 0 ? P - 1 + a : a - 1;
                        const int qz = sz == 0 ? P - 1 + c : c - 1;
                        acc += pv[(qx + nP * (qy + nP * qz)) * NPL + (vx - i0) + (TX + 1) * (vy - j0)];
                    }
                }
                return acc;
            };
            if (i >= n0 || j >= n1) continue;
            if (vk > k0) {
                C sum = part[item];
                if (layer_ok && c >= 1) sum = terms(1, sum);
                const int e = i + n0 * (j + n1 * (vk - 1));
                S* dst = zout + cell_offset(e, l, NN);
                C out = alpha * sum;
                if (ACC) out = load_as<C>(dst) + out;
                store_from(dst, out);
            }
            if (vk < k1) part[item] = (layer_ok && c <= P - 1) ? terms(0, (C)0) : (C)0;
        }
        // cell layer vk-1 is no longer read: the prefetched layer vk+1 takes its slot
        stash(cells[(vk + 1) & 1], nxt);
        __syncthreads();
    }
}

// Zero the padding cells of the last storage block.
template <typename S>
__global__ void k_zero_padding(S* v, int ncells, int nblk, int nn) {
    const int lane = threadIdx.x;                  // 64 threads
    const int e = (nblk - 1) * kLanes + lane;
    if (e < ncells) return;
    for (int l = blockIdx.x; l < nn; l += gridDim.x)
        store_from(v + (size_t)(nblk - 1) * nn * kLanes + (size_t)l * kLanes + lane, (typename Prec<S>::C)0);
}

template <int P, typename S> struct SweepShape;
template <typename S> struct SweepShape<1, S> { static constexpr int TX = 16, TY = 4, NS = 128; };
template <typename S> struct SweepShape<2, S> { static constexpr int TX = 16, TY = 4, NS = 128; };
template <> struct SweepShape<2, double> { static constexpr int TX = 16, TY = 2, NS = 64; };
template <> struct SweepShape<3, double> { static constexpr int TX = 8, TY = 2, NS = 32; };
template <> struct SweepShape<3, float> { static constexpr int TX = 8, TY = 4, NS = 64; };
template <> struct SweepShape<3, bf16_t> { static constexpr int TX = 8, TY = 4, NS = 64; };
template <> struct SweepShape<3, f16_t> { static constexpr int TX = 8, TY = 4, NS = 64; };

// Phase 1 for p <= 3 reading the assembled residual.  A tile is CBP patches
// along x sharing one (y, z) vertex; thread (pc, group) takes patch pc and
// every LPT-th line.  The five 1D passes run x forward (a line of a patch is
// 2p-1 consecutive nodes of the global-node array, loaded into registers
// before the x bases are staged, so both loads are in flight together), y
// forward, z forward + eigenvalue scaling + z backward (in registers), y
// backward, and x backward (straight to the patch buffer).  The y and z
// eigenbases are the same for the whole tile and are read as uniform
// (scalar) loads; the per-patch x bases sit in LDS rows of odd stride so the
// lanes of a wavefront hit distinct banks.
template <int P> constexpr int solve_g_tile() { return P >= 3 ? 32 : 64; }

template <int P, typename C, int CBP> constexpr int solve_g_lds() {
    return ((2 * P - 1) * (2 * P - 1) * (2 * P - 1) * CBP + CBP * (((2 * P - 1) * (2 * P - 1)) | 1) + CBP * (2 * P - 1)) *
           (int)sizeof(C);
}

template <int P, typename S, int CBP, bool MULTI>
__device__ __forceinline__ void pi_solve_g_body(const LaunchTable& L, int item, int items, char* smem) {
    using C = typename Prec<S>::C;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    constexpr int REC = fd_record(P);
    constexpr int NT = 256, LPT = NT / CBP;
    constexpr int KL = (nP2 + LPT - 1) / LPT;       // lines per thread (upper bound)
    constexpr int SXS = nP2 | 1;                    // odd row stride of the x bases
    static_assert(NT % CBP == 0, "patches per tile must divide the workgroup");
    C* sv = reinterpret_cast<C*>(smem);
    C* sSx = sv + nP3 * CBP;
    C* sLx = sSx + CBP * SXS;
    const int tile = xcd_tile(item, items);
    if (tile >= L.total_tiles) return;
    const int tid = threadIdx.x;
    const int pc = tid % CBP, grp = tid / CBP;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int t = tile - pe.tile_begin;
    const int npx = pe.n[0] - 1, npy = pe.n[1] - 1;
    const int tpr = (npx + CBP - 1) / CBP;
    const int row = t / tpr, xt = t % tpr;
    const int vj = 1 + row % npy, vk = 1 + row / npy;
    const int vi0 = 1 + xt * CBP;
    const int vi = vi0 + pc;
    const bool valid = vi <= npx;
    const C* fy = static_cast<const C*>(pe.fd[1]) + (size_t)(vj - 1) * REC;
    const C* fz = static_cast<const C*>(pe.fd[2]) + (size_t)(vk - 1) * REC;
    C lines[KL][nP];
    {
        const C* g = static_cast<const C*>(pe.e);
        const size_t G0 = (size_t)pe.n[0] * P + 1, G1 = (size_t)pe.n[1] * P + 1;
        const size_t base = (size_t)(vi - 1) * P + 1 + G0 * (((size_t)(vj - 1) * P + 1) + G1 * ((size_t)(vk - 1) * P + 1));
#pragma unroll
        for (int k = 0; k < KL; ++k) {
            const int ln = grp + LPT * k;
            const int qy = ln % nP, qz = ln / nP;
            const C* src = g + base + G0 * (qy + G1 * qz);
#pragma unroll
            for (int i = 0; i < nP; ++i) lines[k][i] = (valid && ln < nP2) ? src[i] : (C)0;
        }
    }
    {
        // x bases and eigenvalues of the tile's patches (clamped past the end)
        const C* fx0 = static_cast<const C*>(pe.fd[0]);
        for (int w = tid; w < CBP * (nP2 + nP); w += NT) {
            const int c = w / (nP2 + nP), o = w % (nP2 + nP);
            const int line = min(vi0 + c, npx) - 1;
            const C v = fx0[(size_t)line * REC + o];
            if (o < nP2) sSx[c * SXS + o] = v; else sLx[c * nP + o - nP2] = v;
        }
    }
    __syncthreads();
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = sSx[pc * SXS + i];
#pragma unroll
        for (int k = 0; k < KL; ++k) {                              // x forward
            const int ln = grp + LPT * k;
            if (ln >= nP2) break;
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * lines[k][i];
                sv[(j + nP * ln) * CBP + pc] = s;
            }
        }
    }
    __syncthreads();
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = fy[i];
#pragma unroll
        for (int k = 0; k < KL; ++k) {                              // y forward
            const int ln = grp + LPT * k;
            if (ln >= nP2) break;
            const int qx = ln % nP, qz = ln / nP;
            C v[nP];
#pragma unroll
            for (int i = 0; i < nP; ++i) v[i] = sv[(qx + nP * i + nP2 * qz) * CBP + pc];
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i];
                sv[(qx + nP * j + nP2 * qz) * CBP + pc] = s;
            }
        }
    }
    __syncthreads();
    {
        C Sm[nP2], lz[nP];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = fz[i];
#pragma unroll
        for (int i = 0; i < nP; ++i) lz[i] = fz[nP2 + i];
#pragma unroll
        for (int k = 0; k < KL; ++k) {                              // z: forward, scale, backward
            const int ln = grp + LPT * k;
            if (ln >= nP2) break;
            const int qx = ln % nP, qy = ln / nP;
            const C lxy = sLx[pc * nP + qx] + fy[nP2 + qy];
            C v[nP], w[nP];
#pragma unroll
            for (int i = 0; i < nP; ++i) v[i] = sv[(ln + nP2 * i) * CBP + pc];
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i];
                w[j] = s * recip(lxy + lz[j]);
            }
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * w[j];
                sv[(ln + nP2 * i) * CBP + pc] = s;
            }
        }
    }
    __syncthreads();
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = fy[i];
#pragma unroll
        for (int k = 0; k < KL; ++k) {                              // y backward
            const int ln = grp + LPT * k;
            if (ln >= nP2) break;
            const int qx = ln % nP, qz = ln / nP;
            C v[nP];
#pragma unroll
            for (int j = 0; j < nP; ++j) v[j] = sv[(qx + nP * j + nP2 * qz) * CBP + pc];
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * v[j];
                sv[(qx + nP * i + nP2 * qz) * CBP + pc] = s;
            }
        }
    }
    __syncthreads();
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = sSx[pc * SXS + i];
        C* pbuf = static_cast<C*>(pe.d);
        const int pidx = (vi - 1) + npx * ((vj - 1) + npy * (vk - 1));
        C* out = pbuf + (size_t)(pidx / kLanes) * nP3 * kLanes + (pidx % kLanes);
#pragma unroll
        for (int k = 0; k < KL; ++k) {                              // x backward to the patch buffer
            const int ln = grp + LPT * k;
            if (ln >= nP2) break;
            C v[nP];
#pragma unroll
            for (int j = 0; j < nP; ++j) v[j] = sv[(j + nP * ln) * CBP + pc];
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * v[j];
                if (valid) out[(size_t)(i + nP * ln) * kLanes] = s;
            }
        }
    }
}

template <int P, typename S, int CBP, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_solve_g(LaunchTable L) {
    __shared__ __align__(16) char smem[solve_g_lds<P, typename Prec<S>::C, CBP>()];
    pi_solve_g_body<P, S, CBP, MULTI>(L, blockIdx.x, gridDim.x, smem);
}

// ---------------------------------------------------------------------------
// Patch inverse for p <= 3 through an x-combined buffer (two launches after
// the assembly).  k_pi_solve_x solves a tile of CBP patches along x that
// share one (y, z) vertex, as k_pi_solve_g does, then adds the x-overlaps
// of neighbouring patches of the tile in LDS: for every patch line (qy, qz)
// the tile writes one run of global x-nodes, each the sum of its (one or
// two) patch values in ascending vertex order, instead of every patch's
// full (2p-1)^3 box.  Layout, per problem: row (vj, vk) of patch rows, line
// ln = qy + (2p-1) qz, then the tiles of the row one after another; tile tx
// (patches 1 + tx CBP ...) covers the x-nodes X0 = tx CBP p + 1 ... X0 +
// w p + p - 2 (w = its valid patches), so consecutive tiles overlap in
// p - 1 nodes:
//   xoff(tx) = tx (CBP p + p - 1),  row length RL = npx p + ntx (p - 1).
// k_pi_combine_x then adds, per global node, the tile overlap, the y- and
// the z-patches in ascending order and writes every cell copy.
__host__ __device__ constexpr int xrow_len(int npx, int ntx, int P) { return npx * P + ntx * (P - 1); }

template <int P, typename C, int CBP> constexpr int solve_x_lds() { return solve_g_lds<P, C, CBP>(); }

template <int P, typename S, int CBP, bool MULTI>
__device__ __forceinline__ void pi_solve_x_body(const LaunchTable& L, int item, int items, char* smem) {
    using C = typename Prec<S>::C;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    constexpr int REC = fd_record(P);
    constexpr int NT = 256, LPT = NT / CBP;
    constexpr int KL = (nP2 + LPT - 1) / LPT;       // lines per thread (upper bound)
    constexpr int SXS = nP2 | 1;                    // odd row stride of the x bases
    constexpr int SPAN = CBP * P + P - 1;           // x-nodes of a full tile
    static_assert(NT % CBP == 0, "patches per tile must divide the workgroup");
    C* sv = reinterpret_cast<C*>(smem);
    C* sSx = sv + nP3 * CBP;
    C* sLx = sSx + CBP * SXS;
    const int tile = xcd_tile(item, items);
    if (tile >= L.total_tiles) return;
    const int tid = threadIdx.x;
    const int pc = tid % CBP, grp = tid / CBP;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int t = tile - pe.tile_begin;
    const int npx = pe.n[0] - 1, npy = pe.n[1] - 1;
    const int tpr = (npx + CBP - 1) / CBP;
    const int row = t / tpr, xt = t % tpr;
    const int vj = 1 + row % npy, vk = 1 + row / npy;
    const int vi0 = 1 + xt * CBP;
    const int vi = vi0 + pc;
    const bool valid = vi <= npx;
    const int nvalid = min(CBP, npx - vi0 + 1);
    const C* fy = static_cast<const C*>(pe.fd[1]) + (size_t)(vj - 1) * REC;
    const C* fz = static_cast<const C*>(pe.fd[2]) + (size_t)(vk - 1) * REC;
    C lines[KL][nP];
    {
        const C* g = static_cast<const C*>(pe.e);
        const size_t G0 = (size_t)pe.n[0] * P + 1, G1 = (size_t)pe.n[1] * P + 1;
        const size_t base = (size_t)(vi - 1) * P + 1 + G0 * (((size_t)(vj - 1) * P + 1) + G1 * ((size_t)(vk - 1) * P + 1));
#pragma unroll
        for (int k = 0; k < KL; ++k) {
            const int ln = grp + LPT * k;
            const int qy = ln % nP, qz = ln / nP;
            const C* src = g + base + G0 * (qy + G1 * qz);
#pragma unroll
            for (int i = 0; i < nP; ++i) lines[k][i] = (valid && ln < nP2) ? src[i] : (C)0;
        }
    }
    {
        const C* fx0 = static_cast<const C*>(pe.fd[0]);
        for (int w = tid; w < CBP * (nP2 + nP); w += NT) {
            const int c = w / (nP2 + nP), o = w % (nP2 + nP);
            const int line = min(vi0 + c, npx) - 1;
            const C v = fx0[(size_t)line * REC + o];
            if (o < nP2) sSx[c * SXS + o] = v; else sLx[c * nP + o - nP2] = v;
        }
    }
    __syncthreads();
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = sSx[pc * SXS + i];
#pragma unroll
        for (int k = 0; k < KL; ++k) {                              // x forward
            const int ln = grp + LPT * k;
            if (ln >= nP2) break;
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * lines[k][i];
                sv[(j + nP * ln) * CBP + pc] = s;
            }
        }
    }
    __syncthreads();
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = fy[i];
#pragma unroll
        for (int k = 0; k < KL; ++k) {                              // y forward
            const int ln = grp + LPT * k;
            if (ln >= nP2) break;
            const int qx = ln % nP, qz = ln / nP;
            C v[nP];
#pragma unroll
            for (int i = 0; i < nP; ++i) v[i] = sv[(qx + nP * i + nP2 * qz) * CBP + pc];
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i];
                sv[(qx + nP * j + nP2 * qz) * CBP + pc] = s;
            }
        }
    }
    __syncthreads();
    {
        C Sm[nP2], lz[nP];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = fz[i];
#pragma unroll
        for (int i = 0; i < nP; ++i) lz[i] = fz[nP2 + i];
#pragma unroll
        for (int k = 0; k < KL; ++k) {                              // z: forward, scale, backward
            const int ln = grp + LPT * k;
            if (ln >= nP2) break;
            const int qx = ln % nP, qy = ln / nP;
            const C lxy = sLx[pc * nP + qx] + fy[nP2 + qy];
            C v[nP], w[nP];
#pragma unroll
            for (int i = 0; i < nP; ++i) v[i] = sv[(ln + nP2 * i) * CBP + pc];
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i];
                w[j] = s * recip(lxy + lz[j]);
            }
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * w[j];
                sv[(ln + nP2 * i) * CBP + pc] = s;
            }
        }
    }
    __syncthreads();
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = fy[i];
#pragma unroll
        for (int k = 0; k < KL; ++k) {                              // y backward
            const int ln = grp + LPT * k;
            if (ln >= nP2) break;
            const int qx = ln % nP, qz = ln / nP;
            C v[nP];
#pragma unroll
            for (int j = 0; j < nP; ++j) v[j] = sv[(qx + nP * j + nP2 * qz) * CBP + pc];
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * v[j];
                sv[(qx + nP * i + nP2 * qz) * CBP + pc] = s;
            }
        }
    }
    __syncthreads();
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = sSx[pc * SXS + i];
#pragma unroll
        for (int k = 0; k < KL; ++k) {                              // x backward, in place (own line)
            const int ln = grp + LPT * k;
            if (ln >= nP2) break;
            C v[nP];
#pragma unroll
            for (int j = 0; j < nP; ++j) v[j] = sv[(j + nP * ln) * CBP + pc];
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * v[j];
                sv[(i + nP * ln) * CBP + pc] = s;
            }
        }
    }
    __syncthreads();
    // x-combine: node s of the tile's span = patch pc_hi = s / p at
    // qx = s % p, plus patch pc_hi - 1 at qx + p when that is inside it
    const int span = nvalid * P + P - 1;
    const int RL = xrow_len(npx, tpr, P);
    C* xb = static_cast<C*>(pe.d) + ((size_t)row * nP2) * RL + (size_t)xt * SPAN;
    for (int item = tid; item < nP2 * span; item += NT) {
        const int ln = item / span, sx = item % span;
        const int hi = sx / P, q = sx % P;
        C v = 0;
        if (hi >= 1 && q <= P - 2) v = sv[(q + P + nP * ln) * CBP + hi - 1];
        if (hi < nvalid) v = v + sv[(q + nP * ln) * CBP + hi];
        xb[(size_t)ln * RL + sx] = v;
    }
}

template <int P, typename S, int CBP, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_solve_x(LaunchTable L) {
    __shared__ __align__(16) char smem[solve_x_lds<P, typename Prec<S>::C, CBP>()];
    pi_solve_x_body<P, S, CBP, MULTI>(L, blockIdx.x, gridDim.x, smem);
}

// The same solves and in-tile x-combine with one wavefront per tile of
// CW = floor(64 / (2p-1)) patches along x (12 at p = 3, 21 at p = 2) and
// four independent tiles per workgroup.  Lane (pc, q) holds plane z = q of
// patch pc (all y, x) and applies the x and y contractions in registers; one
// transpose through LDS gives it the y-line q (all z, x) for the z
// contractions and the eigenvalue scaling, a second one brings the planes
// back for y and x backward.  The patch thus passes through LDS twice
// instead of four times, with no workgroup barrier.  The x-overlap of the
// left neighbour comes from the lane to the left by a cross-lane read.  (A
// variant staging the tile's runs through LDS for coalesced loads and
// stores measured slower.)  The contractions, the scaling and the overlap
// sums are those of k_pi_solve_x term by term; the buffer layout is the
// same with CBP = CW.
template <int P> constexpr int solve_w_tile() { return 64 / (2 * P - 1); }
template <int P, typename C> constexpr int solve_w_lds() {
    return 4 * solve_w_tile<P>() * (2 * P - 1) * (2 * P - 1) * (2 * P - 1) * (int)sizeof(C);
}

template <int P, typename S, bool MULTI>
__device__ __forceinline__ void pi_solve_w_body(const LaunchTable& L, int item, int items, char* smem) {
    using C = typename Prec<S>::C;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    constexpr int REC = fd_record(P);
    constexpr int CW = solve_w_tile<P>();
    constexpr int SPAN = CW * P + P - 1;               // x-nodes of a full tile
    constexpr int NLO = P > 1 ? P - 1 : 1;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int lane = threadIdx.x % 64;
    const int tile = xcd_tile(item, items) * 4 + wave;
    if (tile >= L.total_tiles) return;                 // per wavefront: no workgroup barrier follows
    C* sv = reinterpret_cast<C*>(smem) + wave * (CW * nP3);
    const int pc = lane % CW, q = lane / CW;           // q == nP: lane without a patch line
    const bool act = q < nP;
    const int qq = act ? q : 0;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int t = tile - pe.tile_begin;
    const int npx = pe.n[0] - 1, npy = pe.n[1] - 1;
    const int tpr = (npx + CW - 1) / CW;
    const int row = t / tpr, xt = t % tpr;
    const int vj = 1 + row % npy, vk = 1 + row / npy;
    const int vi0 = 1 + xt * CW;
    const int nvalid = min(CW, npx - vi0 + 1);
    const bool valid = act && pc < nvalid;
    const int pcc = min(pc, nvalid - 1);               // lanes past the row end work on its last patch
    const C* fx = static_cast<const C*>(pe.fd[0]) + (size_t)(vi0 + pcc - 1) * REC;
    const C* fy = static_cast<const C*>(pe.fd[1]) + (size_t)(vj - 1) * REC;
    const C* fz = static_cast<const C*>(pe.fd[2]) + (size_t)(vk - 1) * REC;
    C* const pl = sv + pc * nP3;                       // this lane's patch in LDS, [z][y][x]
    C v[nP][nP];                                       // plane z = q: [y][x]
    {
        const C* g = static_cast<const C*>(pe.e);
        const size_t G0 = (size_t)pe.n[0] * P + 1, G1 = (size_t)pe.n[1] * P + 1;
        const C* src = g + (size_t)(vi0 + pcc - 1) * P + 1 +
                       G0 * (((size_t)(vj - 1) * P + 1) + G1 * ((size_t)(vk - 1) * P + 1 + qq));
#pragma unroll
        for (int y = 0; y < nP; ++y)
#pragma unroll
            for (int x = 0; x < nP; ++x) v[y][x] = src[G0 * y + x];
    }
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = fx[i];
#pragma unroll
        for (int y = 0; y < nP; ++y) {                              // x forward
            C u[nP];
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[y][i];
                u[j] = s;
            }
#pragma unroll
            for (int j = 0; j < nP; ++j) v[y][j] = u[j];
        }
    }
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = fy[i];
#pragma unroll
        for (int x = 0; x < nP; ++x) {                              // y forward
            C u[nP];
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i][x];
                u[j] = s;
            }
#pragma unroll
            for (int j = 0; j < nP; ++j) v[j][x] = u[j];
        }
    }
    if (act) {                                                      // plane q out
#pragma unroll
        for (int y = 0; y < nP; ++y)
#pragma unroll
            for (int x = 0; x < nP; ++x) pl[qq * nP2 + y * nP + x] = v[y][x];
    }
    wave_sync();
    {
        // y-line q in: v[z][x]; z forward, scaling, z backward
#pragma unroll
        for (int z = 0; z < nP; ++z)
#pragma unroll
            for (int x = 0; x < nP; ++x) v[z][x] = pl[z * nP2 + qq * nP + x];
        C Sm[nP2], lz[nP];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = fz[i];
#pragma unroll
        for (int i = 0; i < nP; ++i) lz[i] = fz[nP2 + i];
        const C ly = fy[nP2 + qq];
#pragma unroll
        for (int x = 0; x < nP; ++x) {
            const C lxy = fx[nP2 + x] + ly;
            C w[nP];
#pragma unroll
            for (int j = 0; j < nP; ++j) {
                C s = 0;
#pragma unroll
                for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i][x];
                w[j] = s * recip(lxy + lz[j]);
            }
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * w[j];
                v[i][x] = s;
            }
        }
        if (act) {
#pragma unroll
            for (int z = 0; z < nP; ++z)
#pragma unroll
                for (int x = 0; x < nP; ++x) pl[z * nP2 + qq * nP + x] = v[z][x];
        }
    }
    wave_sync();
#pragma unroll
    for (int y = 0; y < nP; ++y)                                    // plane q back
#pragma unroll
        for (int x = 0; x < nP; ++x) v[y][x] = pl[qq * nP2 + y * nP + x];
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = fy[i];
#pragma unroll
        for (int x = 0; x < nP; ++x) {                              // y backward
            C u[nP];
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * v[j][x];
                u[i] = s;
            }
#pragma unroll
            for (int i = 0; i < nP; ++i) v[i][x] = u[i];
        }
    }
    {
        C Sm[nP2];
#pragma unroll
        for (int i = 0; i < nP2; ++i) Sm[i] = fx[i];
#pragma unroll
        for (int y = 0; y < nP; ++y) {                              // x backward
            C u[nP];
#pragma unroll
            for (int i = 0; i < nP; ++i) {
                C s = 0;
#pragma unroll
                for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * v[y][j];
                u[i] = s;
            }
#pragma unroll
            for (int i = 0; i < nP; ++i) v[y][i] = u[i];
        }
    }
    // x-combine: tile node s = pc p + a (a < p) is the left patch's value at
    // x = a + p (a <= p - 2) plus this patch's at x = a; the last valid
    // patch also writes its x = p ... 2p - 2 alone.
    const int RL = xrow_len(npx, tpr, P);
    C* xb = static_cast<C*>(pe.d) + ((size_t)row * nP2) * RL + (size_t)xt * SPAN;
#pragma unroll
    for (int y = 0; y < nP; ++y) {
        C lo[NLO];
#pragma unroll
        for (int a = 0; a < P - 1; ++a) lo[a] = __shfl_up(v[y][a + P], 1, 64);
        if (valid) {
            C* dst = xb + (size_t)(y + nP * qq) * RL + pc * P;
#pragma unroll
            for (int a = 0; a < P; ++a) {
                C o = 0;
                if (a <= P - 2 && pc >= 1) o = lo[a < P - 1 ? a : 0];
                o = o + v[y][a];
                dst[a] = o;
            }
            if (pc == nvalid - 1) {
#pragma unroll
                for (int a = 0; a < P - 1; ++a) dst[P + a] = v[y][a + P];
            }
        }
    }
}

template <int P, typename S, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_solve_w(LaunchTable L) {
    __shared__ __align__(16) char smem[solve_w_lds<P, typename Prec<S>::C>()];
    pi_solve_w_body<P, S, MULTI>(L, blockIdx.x, gridDim.x, smem);
}

// Combine of the x-combined buffer (p <= 3): one wavefront per global node
// row (Y, Z) with lane i on cell column i.  Per node X of the row the terms
// are the z-patches (ascending vk), within each the y-patches (ascending vj),
// within each the overlapping tiles (ascending); the sum goes to every cell
// copy of the node (a vertex-plane node also into the left neighbour's last
// slot).  The first wavefront of a problem zeroes the padding cells of its
// last storage block.  pe: d = x-combined buffer, c = z (S), alpha = damping.
template <int P, typename S, int CBP, int ACC, bool MULTI>
__device__ __forceinline__ void pi_combine_x_body(const LaunchTable& L, int item, int items) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP;
    constexpr int SPAN = CBP * P + P - 1;
    const int tile = item;
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int npx = n0 - 1, npy = n1 - 1;
    const int G1 = n1 * P + 1, G2 = n2 * P + 1;
    const int row = (tile - pe.tile_begin) * 4 + (int)(threadIdx.x / 64);
    if (row >= G1 * G2) return;
    const int lane = threadIdx.x % 64;
    const int ntx = (npx + CBP - 1) / CBP;
    const int RL = xrow_len(npx, ntx, P);
    const C* xb = static_cast<const C*>(pe.d);
    S* z = static_cast<S*>(pe.c);
    const C alpha = (C)pe.alpha;
    if (row == 0) {
#pragma unroll 1
        for (int l = 0; l < NN; ++l) {
            const int e = (pe.nblk - 1) * kLanes + lane;
            if (e >= pe.ncells) store_from(z + cell_offset(e, l, NN), (C)0);
        }
    }
    const int Y = row % G1, Z = row / G1;
    // patch rows containing the node row along y and z (ascending vertex),
    // with the patch-local index, and the cell copies of the row
    int vyp[2], qyp[2], nyp = 0, vzp[2], qzp[2], nzp = 0;
    int cyc[2], byc[2], nyc = 0, czc[2], bzc[2], nzc = 0;
    {
        const int qy = Y / P, ry = Y - qy * P;
        if (ry == 0) {
            if (qy >= 1 && qy <= npy) { vyp[nyp] = qy; qyp[nyp] = P - 1; ++nyp; }
            if (qy >= 1) { cyc[nyc] = qy - 1; byc[nyc] = P; ++nyc; }
            if (qy <= n1 - 1) { cyc[nyc] = qy; byc[nyc] = 0; ++nyc; }
        } else {
            if (qy >= 1) { vyp[nyp] = qy; qyp[nyp] = ry + P - 1; ++nyp; }
            if (qy + 1 <= npy) { vyp[nyp] = qy + 1; qyp[nyp] = ry - 1; ++nyp; }
            cyc[nyc] = qy; byc[nyc] = ry; ++nyc;
        }
        const int qz = Z / P, rz = Z - qz * P;
        if (rz == 0) {
            if (qz >= 1 && qz <= n2 - 1) { vzp[nzp] = qz; qzp[nzp] = P - 1; ++nzp; }
            if (qz >= 1) { czc[nzc] = qz - 1; bzc[nzc] = P; ++nzc; }
            if (qz <= n2 - 1) { czc[nzc] = qz; bzc[nzc] = 0; ++nzc; }
        } else {
            if (qz >= 1) { vzp[nzp] = qz; qzp[nzp] = rz + P - 1; ++nzp; }
            if (qz + 1 <= n2 - 1) { vzp[nzp] = qz + 1; qzp[nzp] = rz - 1; ++nzp; }
            czc[nzc] = qz; bzc[nzc] = rz; ++nzc;
        }
    }
    // run of the x-combined buffer for each (z, y) patch pair (uniform)
    size_t rbase[2][2];
#pragma unroll
    for (int tz = 0; tz < 2; ++tz)
#pragma unroll
        for (int ty = 0; ty < 2; ++ty) {
            const bool ok = tz < nzp && ty < nyp;
            const int prow = ok ? (vyp[ty] - 1) + npy * (vzp[tz] - 1) : 0;
            const int ln = ok ? qyp[ty] + nP * qzp[tz] : 0;
            rbase[tz][ty] = ((size_t)prow * nP2 + ln) * RL;
        }
    for (int i0 = 0; i0 < n0; i0 += 64) {
        const int i = i0 + lane;
        const bool in = i < n0;
#pragma unroll
        for (int a = 0; a < P; ++a) {                      // node X = i P + a
            const int X = i * P + a;
            // tiles holding X: the last one starting at or before X, and its
            // predecessor when X is in their overlap (ascending order)
            int thi = X >= 1 ? (X - 1) / (CBP * P) : 0;
            thi = thi < ntx - 1 ? thi : ntx - 1;
            thi = thi > 0 ? thi : 0;
            const int shi = X - (thi * CBP * P + 1);
            const bool two = thi >= 1 && shi <= P - 2;
            // X is strictly inside the range of some patch (none when npx = 0)
            const bool xin = in && npx >= 1 && X >= 1 && X <= npx * P + P - 1;
            const size_t ohi = (size_t)thi * SPAN + shi;
            const size_t olo = (size_t)(thi - 1) * SPAN + (shi + CBP * P);
            C sum = 0;
#pragma unroll
            for (int tz = 0; tz < 2; ++tz) {
#pragma unroll
                for (int ty = 0; ty < 2; ++ty) {
                    const bool ok = xin && tz < nzp && ty < nyp;
                    const C vlo = xb[ok && two ? rbase[tz][ty] + olo : 0];
                    const C vhi = xb[ok ? rbase[tz][ty] + ohi : 0];
                    sum = ok && two ? sum + vlo : sum;
                    sum = ok ? sum + vhi : sum;
                }
            }
            if (!in) continue;
#pragma unroll
            for (int cz = 0; cz < 2; ++cz) {
                if (cz >= nzc) break;
#pragma unroll
                for (int cy = 0; cy < 2; ++cy) {
                    if (cy >= nyc) break;
                    const int e = i + n0 * (cyc[cy] + n1 * czc[cz]);
                    const int lyz = N * (byc[cy] + N * bzc[cz]);
                    S* d0 = z + cell_offset(e, a + lyz, NN);
                    C o0 = alpha * sum;
                    if (ACC) o0 = load_as<C>(d0) + o0;
                    store_stream(d0, o0);
                    if (a == 0 && i >= 1) {                    // the left cell's copy of the node
                        S* d1 = z + cell_offset(e - 1, P + lyz, NN);
                        C o1 = alpha * sum;
                        if (ACC) o1 = load_as<C>(d1) + o1;
                        store_stream(d1, o1);
                    }
                    if (i == n0 - 1) {                         // the row's last node: no patch
                        S* d2 = z + cell_offset(e, P + lyz, NN);
                        C o2 = alpha * (C)0;
                        if (ACC) o2 = load_as<C>(d2) + o2;
                        store_stream(d2, o2);
                    }
                }
            }
        }
    }
}

template <int P, typename S, int CBP, int ACC, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_combine_x(LaunchTable L) {
    pi_combine_x_body<P, S, CBP, ACC, MULTI>(L, blockIdx.x, gridDim.x);
}

// Assembly into the global-node array: one wavefront per node row (Y, Z),
// its lanes walking X, so writes are contiguous and the row's y/z copy
// structure is uniform over the wavefront.  Each node sums its copies in
// ascending cell order along z, y, x, the same order for every node.
// pe: a = r (S), e = global array (C); ntiles = ceil(rows / 4).
template <int P, typename S, typename C, bool MULTI>
__device__ __forceinline__ void assemble_nodes_body(const LaunchTable& L, int item, int items) {
    constexpr int N = P + 1, NN = N * N * N;
    const int tile = item;
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int G0 = n0 * P + 1, G1 = n1 * P + 1, G2 = n2 * P + 1;
    const int row = (tile - pe.tile_begin) * 4 + (int)(threadIdx.x / 64);
    if (row >= G1 * G2) return;
    const int lane = threadIdx.x % 64;
    const int J = row % G1, K = row / G1;
    // copies along y and z (uniform): lower cell first
    const int qy = J / P, ry = J - qy * P, qz = K / P, rz = K - qz * P;
    const int ny = (ry == 0 && qy >= 1 && qy <= n1 - 1) ? 2 : 1;
    const int nz = (rz == 0 && qz >= 1 && qz <= n2 - 1) ? 2 : 1;
    const int cy0 = (ry == 0 && qy >= 1) ? qy - 1 : qy, by0 = (ry == 0 && qy >= 1) ? P : ry;
    const int cz0 = (rz == 0 && qz >= 1) ? qz - 1 : qz, bz0 = (rz == 0 && qz >= 1) ? P : rz;
    const S* v = static_cast<const S*>(pe.a);
    C* out = static_cast<C*>(pe.e) + (size_t)row * G0;
    for (int I = lane; I < G0; I += 64) {
        const int qx = I / P, rx = I - qx * P;
        const bool two = rx == 0 && qx >= 1 && qx <= n0 - 1;        // a second copy along x
        const int cx0 = (rx == 0 && qx >= 1) ? qx - 1 : qx, ax0 = (rx == 0 && qx >= 1) ? P : rx;
        // copies along y/z in uniform branches, the x pair loaded together
        // (the second from the first's address when absent) and selected
        double val[2][2][2];
#pragma unroll
        for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                val[z][y][0] = val[z][y][1] = 0.0;
                if (z < nz && y < ny) {
                    const int e = cx0 + n0 * ((cy0 + y) + n1 * (cz0 + z));
                    const int lyz = N * ((y ? 0 : by0) + N * (z ? 0 : bz0));
                    val[z][y][0] = load_as<double>(v + cell_offset(e, ax0 + lyz, NN));
                    val[z][y][1] = load_as<double>(v + (two ? cell_offset(e + 1, lyz, NN) : cell_offset(e, ax0 + lyz, NN)));
                }
            }
        double s = 0.0;
#pragma unroll
        for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                if (z >= nz || y >= ny) continue;
                s += val[z][y][0];
                s = two ? s + val[z][y][1] : s;
            }
        out[I] = (C)s;
    }
}

template <int P, typename S, typename C, bool MULTI>
__global__ void __launch_bounds__(256) k_assemble_nodes(LaunchTable L) {
    assemble_nodes_body<P, S, C, MULTI>(L, blockIdx.x, gridDim.x);
}

// The same assembly for long rows: one wavefront per node row (Y, Z) with
// lane i on cell column i (64 cells per pass along x).  For each of the
// row's y/z copies (uniform over the wavefront) a lane loads its cell's p+1
// nodes along x, so every load is a run of consecutive cells of a storage
// block; the node a cell shares with its left neighbour takes the
// neighbour's last node through a lane shuffle.  Terms are added in the same
// order as k_assemble_nodes (ascending cell order along z, y, x), so the two
// kernels give identical results.
template <int P, typename S, typename C, bool MULTI>
__device__ __forceinline__ void assemble_cells_body(const LaunchTable& L, int item, int items) {
    constexpr int N = P + 1, NN = N * N * N;
    const int tile = item;
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int G0 = n0 * P + 1, G1 = n1 * P + 1, G2 = n2 * P + 1;
    const int row = (tile - pe.tile_begin) * 4 + (int)(threadIdx.x / 64);
    if (row >= G1 * G2) return;
    const int lane = threadIdx.x % 64;
    const int J = row % G1, K = row / G1;
    const int qy = J / P, ry = J - qy * P, qz = K / P, rz = K - qz * P;
    const int ny = (ry == 0 && qy >= 1 && qy <= n1 - 1) ? 2 : 1;
    const int nz = (rz == 0 && qz >= 1 && qz <= n2 - 1) ? 2 : 1;
    const int cy0 = (ry == 0 && qy >= 1) ? qy - 1 : qy, by0 = (ry == 0 && qy >= 1) ? P : ry;
    const int cz0 = (rz == 0 && qz >= 1) ? qz - 1 : qz, bz0 = (rz == 0 && qz >= 1) ? P : rz;
    const S* v = static_cast<const S*>(pe.a);
    C* out = static_cast<C*>(pe.e) + (size_t)row * G0;
    for (int i0 = 0; i0 < n0; i0 += 64) {
        const int i = i0 + lane;
        const bool in = i < n0;
        double val[2][2][N], left[2][2];
#pragma unroll
        for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
#pragma unroll
                for (int a = 0; a < N; ++a) val[z][y][a] = 0.0;
                left[z][y] = 0.0;
                if (z < nz && y < ny) {                        // uniform
                    const int e = i + n0 * ((cy0 + y) + n1 * (cz0 + z));
                    const int lyz = N * ((y ? 0 : by0) + N * (z ? 0 : bz0));
                    if (in) {
#pragma unroll
                        for (int a = 0; a < N; ++a) val[z][y][a] = load_stream<double>(v + cell_offset(e, a + lyz, NN));
                    }
                    left[z][y] = __shfl_up(val[z][y][P], 1, 64);
                    if (lane == 0 && i0 > 0) left[z][y] = load_as<double>(v + cell_offset(e - 1, P + lyz, NN));
                }
            }
        if (in) {
#pragma unroll
            for (int a = 0; a < P; ++a) {
                double s = 0.0;
#pragma unroll
                for (int z = 0; z < 2; ++z)
#pragma unroll
                    for (int y = 0; y < 2; ++y) {
                        if (z >= nz || y >= ny) continue;
                        if (a == 0 && i >= 1) s += left[z][y];    // lower cell first
                        s += val[z][y][a];
                    }
                out[i * P + a] = (C)s;
            }
            if (i == n0 - 1) {
                double s = 0.0;
#pragma unroll
                for (int z = 0; z < 2; ++z)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        if (z < nz && y < ny) s += val[z][y][P];
                out[n0 * P] = (C)s;
            }
        }
    }
}

template <int P, typename S, typename C, bool MULTI>
__global__ void __launch_bounds__(256) k_assemble_cells(LaunchTable L) {
    assemble_cells_body<P, S, C, MULTI>(L, blockIdx.x, gridDim.x);
}

// Fused sweep from the assembled residual (p <= 3): like k_pi_sweep, but the
// patch values are read from a ring of global-node z-planes instead of being
// summed from cell copies, so the restriction is a plain copy folded into the
// first transform.  A workgroup owns TX x TY cell columns and a chunk of cell
// layers and walks the vertex layers in order; per vertex layer it solves the
// (TX+1) x (TY+1) patches around its columns (work items are (patch, line)
// pairs) and combines them into the cells: cell layer vk-1 is finished and
// written, cell layer vk starts a partial sum.  Terms enter every node in
// ascending vertex order along z, y, x, so copies stay bitwise equal, also
// across workgroups (border patches are solved by both neighbours).
// pe: e = assembled residual (C), c = z (S), alpha = damping.
template <int P, typename S, int TX, int TY, int ACC, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_sweep_g(LaunchTable L) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    constexpr int REC = fd_record(P);
    constexpr int NPL = (TX + 1) * (TY + 1);       // patches per vertex layer
    constexpr int NTASK = NPL * nP2;               // (patch, line) pairs per pass
    constexpr int WX = (TX + 2) * P - 1, WY = (TY + 2) * P - 1;   // node window
    constexpr int WXY = WX * WY;
    constexpr int NZ = 2 * P - 1;                  // planes in the ring
    constexpr int NLOAD = P * WXY;                 // new planes per vertex layer
    constexpr int PF = (NLOAD + 255) / 256;
    __shared__ C ring[NZ * WXY];
    __shared__ C pv[nP3 * NPL];                    // current patch layer [q][patch]
    __shared__ C part[TX * TY * NN];               // partial sums of the open cell layer
    __shared__ C sSx[TX + 1][nP2 + 1];
    __shared__ C sSy[TY + 1][nP2 + 1];
    __shared__ C sSz[nP2];
    __shared__ C sLx[TX + 1][nP];
    __shared__ C sLy[TY + 1][nP];
    __shared__ C sLz[nP];

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int G0 = n0 * P + 1, G1 = n1 * P + 1;
    const int ntx = (n0 + TX - 1) / TX, nty = (n1 + TY - 1) / TY;
    int t = tile - pe.tile_begin;
    const int tx = t % ntx;
    t /= ntx;
    const int ty = t % nty;
    const int kc = t / nty;
    const int i0 = tx * TX, j0 = ty * TY;
    const int k0 = kc * pe.zchunk;
    const int k1 = min(k0 + pe.zchunk, n2);
    const int X0 = (i0 - 1) * P + 1, Y0 = (j0 - 1) * P + 1;
    const int tid = threadIdx.x;
    const C* g = static_cast<const C*>(pe.e);
    S* zout = static_cast<S*>(pe.c);
    const C alpha = (C)pe.alpha;

    for (int w = tid; w < (TX + 1) * (nP2 + nP); w += 256) {
        const int col = w / (nP2 + nP), o = w % (nP2 + nP);
        const int line = max(0, min(i0 + col, n0 - 1) - 1);
        const C v = static_cast<const C*>(pe.fd[0])[(size_t)line * REC + o];
        if (o < nP2) sSx[col][o] = v; else sLx[col][o - nP2] = v;
    }
    for (int w = tid; w < (TY + 1) * (nP2 + nP); w += 256) {
        const int col = w / (nP2 + nP), o = w % (nP2 + nP);
        const int line = max(0, min(j0 + col, n1 - 1) - 1);
        const C v = static_cast<const C*>(pe.fd[1])[(size_t)line * REC + o];
        if (o < nP2) sSy[col][o] = v; else sLy[col][o - nP2] = v;
    }

    // planes Z0 .. Z0+P-1 of the window (zero outside the mesh); ring slot Z mod NZ
    auto fetch = [&](int Z0, int nplanes, C* regs) {
#pragma unroll
        for (int m = 0; m < PF; ++m) {
            const int item = tid + 256 * m;
            C v = 0;
            if (item < nplanes * WXY) {
                const int wx = item % WX, wy = (item / WX) % WY, dz = item / WXY;
                const int X = X0 + wx, Y = Y0 + wy, Z = Z0 + dz;
                if (X >= 0 && X < G0 && Y >= 0 && Y < G1 && Z >= 0 && Z <= n2 * P)
                    v = g[(size_t)X + (size_t)G0 * ((size_t)Y + (size_t)G1 * Z)];
            }
            regs[m] = v;
        }
    };
    auto stash = [&](int Z0, int nplanes, const C* regs) {
#pragma unroll
        for (int m = 0; m < PF; ++m) {
            const int item = tid + 256 * m;
            if (item < nplanes * WXY) {
                const int dz = item / WXY;
                const int slot = ((Z0 + dz) % NZ + NZ) % NZ;
                ring[slot * WXY + item % WXY] = regs[m];
            }
        }
    };
    {
        // vertex layer k0 needs planes (k0-1)P+1 .. (k0+1)P-1
        C reg[PF];
        fetch((k0 - 1) * P + 1, P, reg);
        stash((k0 - 1) * P + 1, P, reg);
        if (P > 1) {
            fetch(k0 * P + 1, P - 1, reg);
            stash(k0 * P + 1, P - 1, reg);
        }
    }
    __syncthreads();

    for (int vk = k0; vk <= k1; ++vk) {
        C nxt[PF];
        // planes of the next layer not yet in the ring: (vk+1)P .. (vk+2)P-1
        fetch((vk + 1) * P, P, nxt);
        const bool layer_ok = vk >= 1 && vk <= n2 - 1;   // uniform over the workgroup
        if (layer_ok) {
            for (int w = tid; w < nP2 + nP; w += 256) {
                const C v = static_cast<const C*>(pe.fd[2])[(size_t)(vk - 1) * REC + w];
                if (w < nP2) sSz[w] = v; else sLz[w - nP2] = v;
            }
            __syncthreads();
            {
                C Sm[nP2];
#pragma unroll
                for (int i = 0; i < nP2; ++i) Sm[i] = sSz[i];
                const int Zb = (vk - 1) * P + 1;
                for (int task = tid; task < NTASK; task += 256) {     // forward z from the ring
                    const int ps = task % NPL, ln = task / NPL;
                    const int pxo = ps % (TX + 1), pyo = ps / (TX + 1);
                    const int wxy = (pxo * P + ln % nP) + WX * (pyo * P + ln / nP);
                    C v[nP];
#pragma unroll
                    for (int i = 0; i < nP; ++i) v[i] = ring[((Zb + i) % NZ) * WXY + wxy];
#pragma unroll
                    for (int j = 0; j < nP; ++j) {
                        C s = 0;
#pragma unroll
                        for (int i = 0; i < nP; ++i) s += Sm[i * nP + j] * v[i];
                        pv[(ln + nP2 * j) * NPL + ps] = s;
                    }
                }
            }
            __syncthreads();
            for (int task = tid; task < NTASK; task += 256) {         // forward y
                const int ps = task % NPL, ln = task / NPL;
                const int pyo = ps / (TX + 1);
                const int qx = ln % nP, qz = ln / nP;
                C v[nP];
#pragma unroll
                for (int i = 0; i < nP; ++i) v[i] = pv[(qx + nP * i + nP2 * qz) * NPL + ps];
#pragma unroll
                for (int j = 0; j < nP; ++j) {
                    C s = 0;
#pragma unroll
                    for (int i = 0; i < nP; ++i) s += sSy[pyo][i * nP + j] * v[i];
                    pv[(qx + nP * j + nP2 * qz) * NPL + ps] = s;
                }
            }
            __syncthreads();
            for (int task = tid; task < NTASK; task += 256) {         // x: forward, scale, back
                const int ps = task % NPL, ln = task / NPL;
                const int pxo = ps % (TX + 1), pyo = ps / (TX + 1);
                const int qy = ln % nP, qz = ln / nP;
                C v[nP], w[nP];
#pragma unroll
                for (int i = 0; i < nP; ++i) v[i] = pv[(i + nP * ln) * NPL + ps];
                const C lyz = sLy[pyo][qy] + sLz[qz];
#pragma unroll
                for (int j = 0; j < nP; ++j) {
                    C s = 0;
#pragma unroll
                    for (int i = 0; i < nP; ++i) s += sSx[pxo][i * nP + j] * v[i];
                    w[j] = s * recip(sLx[pxo][j] + lyz);
                }
#pragma unroll
                for (int i = 0; i < nP; ++i) {
                    C s = 0;
#pragma unroll
                    for (int j = 0; j < nP; ++j) s += sSx[pxo][i * nP + j] * w[j];
                    pv[(i + nP * ln) * NPL + ps] = s;
                }
            }
            __syncthreads();
            for (int task = tid; task < NTASK; task += 256) {         // backward y
                const int ps = task % NPL, ln = task / NPL;
                const int pyo = ps / (TX + 1);
                const int qx = ln % nP, qz = ln / nP;
                C v[nP];
#pragma unroll
                for (int j = 0; j < nP; ++j) v[j] = pv[(qx + nP * j + nP2 * qz) * NPL + ps];
#pragma unroll
                for (int i = 0; i < nP; ++i) {
                    C s = 0;
#pragma unroll
                    for (int j = 0; j < nP; ++j) s += sSy[pyo][i * nP + j] * v[j];
                    pv[(qx + nP * i + nP2 * qz) * NPL + ps] = s;
                }
            }
            __syncthreads();
            {
                C Sm[nP2];
#pragma unroll
                for (int i = 0; i < nP2; ++i) Sm[i] = sSz[i];
                for (int task = tid; task < NTASK; task += 256) {     // backward z
                    const int ps = task % NPL, ln = task / NPL;
                    C v[nP];
#pragma unroll
                    for (int j = 0; j < nP; ++j) v[j] = pv[(ln + nP2 * j) * NPL + ps];
#pragma unroll
                    for (int i = 0; i < nP; ++i) {
                        C s = 0;
#pragma unroll
                        for (int j = 0; j < nP; ++j) s += Sm[i * nP + j] * v[j];
                        pv[(ln + nP2 * i) * NPL + ps] = s;
                    }
                }
            }
            __syncthreads();
        }
        // finish cell layer vk-1, open cell layer vk
        for (int item = tid; item < TX * TY * NN; item += 256) {
            const int cx = item % TX;
            const int cy = (item / TX) % TY;
            const int l = item / (TX * TY);
            const int i = i0 + cx, j = j0 + cy;
            const int a = l % N, b = (l / N) % N, c = l / N2;
            auto terms = [&](int sz, C acc) -> C {
#pragma unroll
                for (int sy = 0; sy < 2; ++sy) {
                    if ((sy == 0 && b == P) || (sy == 1 && b == 0)) continue;
                    const int vy = j + sy;
                    if (vy < 1 || vy > n1 - 1) continue;
                    const int qy = sy == 0 ? P - 1 + b : b - 1;
#pragma unroll
                    for (int sx = 0; sx < 2; ++sx) {
                        if ((sx == 0 && a == P) || (sx == 1 && a == 0)) continue;
                        const int vx = i + sx;
                        if (vx < 1 || vx > n0 - 1) continue;
                        const int qx = sx == 0 ? P - 1 + a : a - 1;
                        const int qz = sz == 0 ? P - 1 + c : c - 1;
                        acc += pv[(qx + nP * (qy + nP * qz)) * NPL + (vx - i0) + (TX + 1) * (vy - j0)];
                    }
                }
                return acc;
            };
            if (i >= n0 || j >= n1) continue;
            if (vk > k0) {
                C sum = part[item];
                if (layer_ok && c >= 1) sum = terms(1, sum);
                const int e = i + n0 * (j + n1 * (vk - 1));
                S* dst = zout + cell_offset(e, l, NN);
                C out = alpha * sum;
                if (ACC) out = load_as<C>(dst) + out;
                store_from(dst, out);
            }
            if (vk < k1) part[item] = (layer_ok && c <= P - 1) ? terms(0, (C)0) : (C)0;
        }
        // the ring planes of layer vk below layer vk+1 are retired: the prefetched planes take their slots
        stash((vk + 1) * P, P, nxt);
        __syncthreads();
    }
}

template <int P, typename S>
static hipError_t launch_assemble_nodes(ProbEntry* ents, int nprob, TableStager* d_tab, hipStream_t s) {
    using C = typename Prec<S>::C;
    int tiles = 0;
    for (int i = 0; i < nprob; ++i) {
        const int rows = (ents[i].n[1] * P + 1) * (ents[i].n[2] * P + 1);
        ents[i].tile_begin = tiles;
        ents[i].ntiles = (rows + 3) / 4;
        tiles += ents[i].ntiles;
    }
    LaunchTable L{};
    L.nprob = nprob;
    L.total_tiles = tiles;
    hipError_t err = stage_table(L, ents, nprob, d_tab, s);
    if (err != hipSuccess || tiles == 0) return err;
    TraceSpan ts("pi_assemble", P, Prec<S>::id, s);
    // lanes over cells when every row is long (coalesced loads, no idle
    // tail pass), lanes over nodes otherwise; identical results either way
    bool long_rows = true;
    for (int i = 0; i < nprob; ++i) long_rows = long_rows && ents[i].n[0] >= 48;
    if (long_rows) {
        if (nprob > 1) hipLaunchKernelGGL((k_assemble_cells<P, S, C, true>), dim3(tiles), dim3(256), 0, s, L);
        else hipLaunchKernelGGL((k_assemble_cells<P, S, C, false>), dim3(tiles), dim3(256), 0, s, L);
    } else {
        if (nprob > 1) hipLaunchKernelGGL((k_assemble_nodes<P, S, C, true>), dim3(tiles), dim3(256), 0, s, L);
        else hipLaunchKernelGGL((k_assemble_nodes<P, S, C, false>), dim3(tiles), dim3(256), 0, s, L);
    }
    return hipGetLastError();
}

template <int P, typename S> struct SweepGShape;
template <typename S> struct SweepGShape<1, S> { static constexpr int TX = 16, TY = 4; };
template <typename S> struct SweepGShape<2, S> { static constexpr int TX = 16, TY = 4; };
template <> struct SweepGShape<2, double> { static constexpr int TX = 16, TY = 2; };
template <> struct SweepGShape<3, double> { static constexpr int TX = 8, TY = 2; };
template <typename S> struct SweepGShape<3, S> { static constexpr int TX = 8, TY = 4; };

// Fused patch inverse from the assembled residual: assembly, then one sweep.
template <int P, typename S>
static hipError_t launch_pi_sweep_g(int accumulate, ProbEntry* ents, int nprob, TableStager* d_tab, hipStream_t s) {
    constexpr int TX = SweepGShape<P, S>::TX, TY = SweepGShape<P, S>::TY;
    hipError_t err = launch_assemble_nodes<P, S>(ents, nprob, d_tab, s);
    if (err != hipSuccess) return err;
    LaunchTable L{};
    int tiles = 0;
    for (int i = 0; i < nprob; ++i) {
        const int ntx = (ents[i].n[0] + TX - 1) / TX, nty = (ents[i].n[1] + TY - 1) / TY;
        const int n2 = ents[i].n[2];
        int nkc = (2048 + ntx * nty - 1) / (ntx * nty);
        nkc = std::max(1, std::min(nkc, (n2 + 3) / 4));
        ents[i].zchunk = (n2 + nkc - 1) / nkc;
        nkc = (n2 + ents[i].zchunk - 1) / ents[i].zchunk;
        ents[i].tile_begin = tiles;
        ents[i].ntiles = ntx * nty * nkc;
        tiles += ents[i].ntiles;
    }
    L.nprob = nprob;
    L.total_tiles = tiles;
    err = stage_table(L, ents, nprob, d_tab, s);
    if (err != hipSuccess) return err;
    const int grid = (tiles + 7) / 8 * 8;
    {
        TraceSpan ts("pi_sweep", P, Prec<S>::id, s);
        if (nprob > 1) {
            if (accumulate) hipLaunchKernelGGL((k_pi_sweep_g<P, S, TX, TY, 1, true>), dim3(grid), dim3(256), 0, s, L);
            else hipLaunchKernelGGL((k_pi_sweep_g<P, S, TX, TY, 0, true>), dim3(grid), dim3(256), 0, s, L);
        } else {
            if (accumulate) hipLaunchKernelGGL((k_pi_sweep_g<P, S, TX, TY, 1, false>), dim3(grid), dim3(256), 0, s, L);
            else hipLaunchKernelGGL((k_pi_sweep_g<P, S, TX, TY, 0, false>), dim3(grid), dim3(256), 0, s, L);
        }
    }
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    for (int i = 0; i < nprob; ++i) {
        if (ents[i].ncells % kLanes == 0) continue;
        constexpr int NN = (P + 1) * (P + 1) * (P + 1);
        hipLaunchKernelGGL((k_zero_padding<S>), dim3(NN < 64 ? NN : 64), dim3(64), 0, s,
                           static_cast<S*>(ents[i].c), ents[i].ncells, ents[i].nblk, NN);
    }
    return hipGetLastError();
}

template <int P, typename S>
static hipError_t launch_pi_sweep(int accumulate, ProbEntry* ents, int nprob, TableStager* d_tab, hipStream_t s) {
    using Sh = SweepShape<P, S>;
    constexpr int TX = Sh::TX, TY = Sh::TY, NS = Sh::NS;
    LaunchTable L{};
    int tiles = 0;
    for (int i = 0; i < nprob; ++i) {
        const int ntx = (ents[i].n[0] + TX - 1) / TX, nty = (ents[i].n[1] + TY - 1) / TY;
        const int n2 = ents[i].n[2];
        // z-chunks: enough workgroups to fill the chip, at least 4 layers each
        int nkc = (2048 + ntx * nty - 1) / (ntx * nty);
        nkc = std::max(1, std::min(nkc, (n2 + 3) / 4));
        ents[i].zchunk = (n2 + nkc - 1) / nkc;
        nkc = (n2 + ents[i].zchunk - 1) / ents[i].zchunk;
        ents[i].tile_begin = tiles;
        ents[i].ntiles = ntx * nty * nkc;
        tiles += ents[i].ntiles;
    }
    L.nprob = nprob;
    L.total_tiles = tiles;
    hipError_t err = stage_table(L, ents, nprob, d_tab, s);
    if (err != hipSuccess) return err;
    const int grid = (tiles + 7) / 8 * 8;
    TraceSpan ts("pi_sweep", P, Prec<S>::id, s);
    if (nprob > 1) {
        if (accumulate) hipLaunchKernelGGL((k_pi_sweep<P, S, TX, TY, NS, 1, true>), dim3(grid), dim3(256), 0, s, L);
        else hipLaunchKernelGGL((k_pi_sweep<P, S, TX, TY, NS, 0, true>), dim3(grid), dim3(256), 0, s, L);
    } else {
        if (accumulate) hipLaunchKernelGGL((k_pi_sweep<P, S, TX, TY, NS, 1, false>), dim3(grid), dim3(256), 0, s, L);
        else hipLaunchKernelGGL((k_pi_sweep<P, S, TX, TY, NS, 0, false>), dim3(grid), dim3(256), 0, s, L);
    }
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    for (int i = 0; i < nprob; ++i) {
        if (ents[i].ncells % kLanes == 0) continue;
        constexpr int NN = (P + 1) * (P + 1) * (P + 1);
        hipLaunchKernelGGL((k_zero_padding<S>), dim3(NN < 64 ? NN : 64), dim3(64), 0, s,
                           static_cast<S*>(ents[i].c), ents[i].ncells, ents[i].nblk, NN);
    }
    return hipGetLastError();
}

// One thread per cell and z-plane, any degree: a wavefront takes the 64
// cells of a storage block at one plane c of their nodes (tile = block * N +
// c), so even small meshes give N times as many wavefronts as blocks; the
// eight corner-patch addresses are formed once per cell, (a, b) loops are
// unrolled.
template <int P> constexpr int combine_brows() { return P <= 3 ? P + 1 : 2; }

template <int P, typename S, int ACC, bool MULTI>
__device__ __forceinline__ void pi_combine_planes_body(const LaunchTable& L, int item, int items) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    constexpr int BS = combine_brows<P>();          // b rows per wavefront
    constexpr int NBG = (N + BS - 1) / BS;          // row groups per plane
    const int lane = threadIdx.x & 63;
    // consecutive storage blocks (cell rows that read the same patch rows)
    // on one XCD, so its L2 serves the shared patch values
    const int tile = xcd_tile(item, items) * 4 + (threadIdx.x >> 6);
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int blk = (tile - pe.tile_begin) / (N * NBG);
    const int c = ((tile - pe.tile_begin) / NBG) % N;
    const int b0 = ((tile - pe.tile_begin) % NBG) * BS;
    const int e = blk * kLanes + lane;
    S* z = static_cast<S*>(pe.c) + (size_t)blk * NN * kLanes + (size_t)c * N2 * kLanes + lane;
    if (e >= pe.ncells) {
#pragma unroll
        for (int bb = 0; bb < BS; ++bb)
#pragma unroll
            for (int a = 0; a < N; ++a)
                if (b0 + bb < N) store_from(z + (a + N * (b0 + bb)) * kLanes, (C)0);
        return;
    }
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int npx = n0 - 1, npy = n1 - 1;
    const int i = e % n0, j = (e / n0) % n1, k = e / (n0 * n1);
    const C* pbuf = static_cast<const C*>(pe.d);
    const C alpha = (C)pe.alpha;
    // the z-plane c selects the vertex layers (and their patch-local qz)
    int nz = 0, szs[2], qzs[2];
    if (c != P) { szs[nz] = 0; qzs[nz] = P - 1 + c; ++nz; }
    if (c != 0) { szs[nz] = 1; qzs[nz] = c - 1; ++nz; }
    // corner patches: a missing one (boundary vertex, or no second vertex
    // layer) reads element 0 of the buffer and its term is dropped by a
    // select, so every load of the wavefront can be in flight at once
    const C* corner[2][2][2];
    bool cok[2][2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int sy = 0; sy < 2; ++sy)
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
                const int vx = i + sx, vy = j + sy, vz = k + szs[t < nz ? t : 0];
                const bool ok = t < nz && vx >= 1 && vx <= npx && vy >= 1 && vy <= npy && vz >= 1 && vz <= n2 - 1;
                const int pidx = ok ? (vx - 1) + npx * ((vy - 1) + npy * (vz - 1)) : 0;
                cok[t][sy][sx] = ok;
                corner[t][sy][sx] = ok ? pbuf + (size_t)(pidx / kLanes) * nP3 * kLanes + (pidx % kLanes) +
                                             (size_t)nP2 * qzs[t] * kLanes
                                       : pbuf;     // element 0 exists even when the mesh has no patch
            }
#pragma unroll
    for (int bb = 0; bb < BS; ++bb)
#pragma unroll
        for (int a = 0; a < N; ++a) {
            const int b = b0 + bb;
            if (b >= N) break;
            C sum = 0;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
#pragma unroll
                for (int sy = 0; sy < 2; ++sy) {
                    if ((sy == 0 && b == P) || (sy == 1 && b == 0)) continue;
                    const int qy = sy == 0 ? P - 1 + b : b - 1;
#pragma unroll
                    for (int sx = 0; sx < 2; ++sx) {
                        if ((sx == 0 && a == P) || (sx == 1 && a == 0)) continue;
                        const int qx = sx == 0 ? P - 1 + a : a - 1;
                        const bool ok = cok[t][sy][sx];
                        const C v = corner[t][sy][sx][ok ? (size_t)(qx + nP * qy) * kLanes : 0];
                        sum = ok ? sum + v : sum;
                    }
                }
            }
            const int l = a + N * b;
            C out = alpha * sum;
            if (ACC) out = load_as<C>(z + l * kLanes) + out;
            store_from(z + l * kLanes, out);
        }
}

template <int P, typename S, int ACC, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_combine_planes(LaunchTable L) {
    pi_combine_planes_body<P, S, ACC, MULTI>(L, blockIdx.x, gridDim.x);
}

// Combine by global node rows, for long rows (p <= 3): one wavefront per
// node row (Y, Z) with lane i on cell column i.  Every patch value belongs to
// exactly one global node, so each node's terms are read once, and the sum
// goes to every cell copy of the node (a vertex-plane node also into the
// left neighbour's last slot).  The terms enter in ascending vertex order
// along z, y, x, as in k_pi_combine_planes, so the two kernels give
// identical results.  The first wavefront of a problem also zeroes the
// padding cells of its last storage block.
template <int P, typename S, int ACC, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_combine_rows(LaunchTable L) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    const int tile = blockIdx.x;
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int npx = n0 - 1, npy = n1 - 1;
    const int G1 = n1 * P + 1, G2 = n2 * P + 1;
    const int row = (tile - pe.tile_begin) * 4 + (int)(threadIdx.x / 64);
    if (row >= G1 * G2) return;
    const int lane = threadIdx.x % 64;
    const C* pbuf = static_cast<const C*>(pe.d);
    S* z = static_cast<S*>(pe.c);
    const C alpha = (C)pe.alpha;
    if (row == 0) {
#pragma unroll 1
        for (int l = 0; l < NN; ++l) {
            const int e = (pe.nblk - 1) * kLanes + lane;
            if (e >= pe.ncells) store_from(z + cell_offset(e, l, NN), (C)0);
        }
    }
    const int Y = row % G1, Z = row / G1;
    // patches containing the row's nodes along y and z (ascending vertex)
    // and the cell copies of the row along y and z
    int vyp[2], qyp[2], nyp = 0, vzp[2], qzp[2], nzp = 0;
    int cyc[2], byc[2], nyc = 0, czc[2], bzc[2], nzc = 0;
    {
        const int qy = Y / P, ry = Y - qy * P;
        if (ry == 0) {
            if (qy >= 1 && qy <= npy) { vyp[nyp] = qy; qyp[nyp] = P - 1; ++nyp; }
            if (qy >= 1) { cyc[nyc] = qy - 1; byc[nyc] = P; ++nyc; }
            if (qy <= n1 - 1) { cyc[nyc] = qy; byc[nyc] = 0; ++nyc; }
        } else {
            if (qy >= 1) { vyp[nyp] = qy; qyp[nyp] = ry + P - 1; ++nyp; }
            if (qy + 1 <= npy) { vyp[nyp] = qy + 1; qyp[nyp] = ry - 1; ++nyp; }
            cyc[nyc] = qy; byc[nyc] = ry; ++nyc;
        }
        const int qz = Z / P, rz = Z - qz * P;
        if (rz == 0) {
            if (qz >= 1 && qz <= n2 - 1) { vzp[nzp] = qz; qzp[nzp] = P - 1; ++nzp; }
            if (qz >= 1) { czc[nzc] = qz - 1; bzc[nzc] = P; ++nzc; }
            if (qz <= n2 - 1) { czc[nzc] = qz; bzc[nzc] = 0; ++nzc; }
        } else {
            if (qz >= 1) { vzp[nzp] = qz; qzp[nzp] = rz + P - 1; ++nzp; }
            if (qz + 1 <= n2 - 1) { vzp[nzp] = qz + 1; qzp[nzp] = rz - 1; ++nzp; }
            czc[nzc] = qz; bzc[nzc] = rz; ++nzc;
        }
    }
    for (int i0 = 0; i0 < n0; i0 += 64) {
        const int i = i0 + lane;
        const bool in = i < n0;
#pragma unroll
        for (int a = 0; a < P; ++a) {                      // node X = i P + a
            C sum = 0;
#pragma unroll
            for (int tz = 0; tz < 2; ++tz) {
#pragma unroll
                for (int ty = 0; ty < 2; ++ty) {
#pragma unroll
                    for (int sx = 0; sx < 2; ++sx) {
                        const int vx = i + sx;
                        const bool ok = in && tz < nzp && ty < nyp && !(sx == 1 && a == 0) && vx >= 1 && vx <= npx;
                        const int qx = sx == 0 ? P - 1 + a : a - 1;
                        size_t off = 0;
                        if (ok) {
                            const int pidx = (vx - 1) + npx * ((vyp[ty] - 1) + npy * (vzp[tz] - 1));
                            off = (size_t)(pidx / kLanes) * nP3 * kLanes + (pidx % kLanes) +
                                  (size_t)(qx + nP * (qyp[ty] + nP * qzp[tz])) * kLanes;
                        }
                        const C v = pbuf[off];
                        sum = ok ? sum + v : sum;
                    }
                }
            }
            if (!in) continue;
#pragma unroll
            for (int cz = 0; cz < 2; ++cz) {
                if (cz >= nzc) break;
#pragma unroll
                for (int cy = 0; cy < 2; ++cy) {
                    if (cy >= nyc) break;
                    const int e = i + n0 * (cyc[cy] + n1 * czc[cz]);
                    const int lyz = N * (byc[cy] + N * bzc[cz]);
                    S* d0 = z + cell_offset(e, a + lyz, NN);
                    C o0 = alpha * sum;
                    if (ACC) o0 = load_as<C>(d0) + o0;
                    store_from(d0, o0);
                    if (a == 0 && i >= 1) {                    // the left cell's copy of the node
                        S* d1 = z + cell_offset(e - 1, P + lyz, NN);
                        C o1 = alpha * sum;
                        if (ACC) o1 = load_as<C>(d1) + o1;
                        store_from(d1, o1);
                    }
                    if (i == n0 - 1) {                         // the row's last node: no patch
                        S* d2 = z + cell_offset(e, P + lyz, NN);
                        C o2 = alpha * (C)0;
                        if (ACC) o2 = load_as<C>(d2) + o2;
                        store_from(d2, o2);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// High-degree variant (4 <= p <= 7): the six 1D contractions of a patch are
// dense products of a (2p-1)x(2p-1) eigenbasis with the (2p-1) x (2p-1)^2
// matrix of the patch's lines, so they run on the matrix cores: 16x16x4
// MFMA tiles (FP64 or FP32), the basis zero-padded to 16x16 as the register
// A operand and 16 patch lines per tile as the B operand read from LDS.
// One or two wavefronts own one patch (mfma_waves_per_patch); the residual
// is first assembled into a global-node array (k_assemble_nodes), so a patch
// reads its (2p-1)^3 box without summing copies, and the results go to a
// patch-major buffer (one contiguous run per patch) for k_pi_combine_pm.
// out(j, line) = sum_i Op(j, i) v(i, line) in place over all lines of the
// patch; Op's 16x4 slices for the four k-steps are in `a`.  The patch's WPP
// wavefronts (sub = this one's index) take every WPP-th 16-line tile.
// Branch-free: the B operand of k >= 2p-1 is read from the clamped index
// (the A slice is zero there, so it adds exact zeros), the tail lines of the
// last tile read the last line, and every result row that is not part of the
// patch is stored to the wavefront's dump slot instead.
template <typename C, int nP, int DIR, int WPP>
__device__ __forceinline__ void mfma_pass(C* pv, C* dump, const C (&a)[4], int lane, int sub) {
    using M = Mfma<C>;
    constexpr int NL = nP * nP, NT = (NL + 15) / 16;
    // element (i, line) of the pass's lines sits at base(line) + STRIDE * i
    constexpr int STRIDE = DIR == 2 ? NL : DIR == 1 ? nP : 1;
    const int col = lane % 16, g = lane / 16;
    int koff[4], joff[4];
    bool jok[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) koff[ks] = STRIDE * min(4 * ks + g, nP - 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int j = M::row(lane, r);
        jok[r] = j < nP;
        joff[r] = STRIDE * (jok[r] ? j : 0);
    }
    for (int t = sub; t < NT; t += WPP) {
        const int line = 16 * t + col;
        const bool lok = line < NL;
        const int lc = lok ? line : NL - 1;
        const int base = DIR == 2 ? lc : DIR == 1 ? (lc % nP) + NL * (lc / nP) : nP * lc;
        typename M::V acc = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc = M::mma(a[ks], pv[base + koff[ks]], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) *((lok && jok[r]) ? pv + base + joff[r] : dump + lane) = acc[r];
    }
    if (WPP == 1) wave_sync();
    else __syncthreads();
}

// Combine from a patch-major buffer (p >= 4): a workgroup takes one storage
// block (64 cells) at one node plane c.  Each wavefront walks 16 of the
// cells; its lanes are the (a, b) nodes of the plane, so the reads of a
// corner patch are rows of contiguous values.  The sums go through LDS
// (padded rows) and leave as coalesced cell-wise stores.  Terms are added in
// ascending vertex order along z, y, x for every copy of a node.
template <typename C> constexpr int pm_cells() { return sizeof(C) >= 8 ? kLanes / 2 : kLanes; }
template <int P, typename C> constexpr int pm_lds() { return (P + 1) * (P + 1) * (pm_cells<C>() + 1) * (int)sizeof(C); }

template <int P, typename S, int ACC, bool MULTI>
__device__ __forceinline__ void pi_combine_pm_body(const LaunchTable& L, int item, int items, char* smem) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    // cells per LDS pass: half a block for 8-byte values keeps the LDS at
    // about 16 KB per workgroup
    constexpr int CH = pm_cells<C>();
    constexpr int RS = CH + 1;                      // padded LDS row
    C* sz = reinterpret_cast<C*>(smem);
    const int tile = xcd_tile(item, items);      // neighbouring blocks on one XCD
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int blk = (tile - pe.tile_begin) / N;
    const int c = (tile - pe.tile_begin) % N;
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int npx = n0 - 1, npy = n1 - 1;
    const C* pbuf = static_cast<const C*>(pe.d);
    const C alpha = (C)pe.alpha;
    const int ab = threadIdx.x % 64, wv = threadIdx.x / 64;
    const int a = ab % N, b = ab / N;
    // the z-plane c selects the vertex layers (and their patch-local qz)
    int nz = 0, szs[2], qzs[2];
    if (c != P) { szs[nz] = 0; qzs[nz] = P - 1 + c; ++nz; }
    if (c != 0) { szs[nz] = 1; qzs[nz] = c - 1; ++nz; }
    S* z = static_cast<S*>(pe.c) + (size_t)blk * NN * kLanes + (size_t)c * N2 * kLanes;
    for (int h = 0; h < kLanes; h += CH) {
        if (ab < N2) {
            for (int cl = wv; cl < CH; cl += 4) {
                const int e = blk * kLanes + h + cl;
                // every corner term is loaded (a missing one from element 0
                // of the buffer) and dropped by a select, so the loads of all
                // corners are in flight together; terms enter in ascending
                // vertex order along z, y, x
                C sum = 0;
                const bool cell_ok = e < pe.ncells;
                const int i = e % n0, j = (e / n0) % n1, k = e / (n0 * n1);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int vz = k + szs[t < nz ? t : 0];
                    const bool zok = cell_ok && t < nz && vz >= 1 && vz <= n2 - 1;
#pragma unroll
                    for (int sy = 0; sy < 2; ++sy) {
                        const int vy = j + sy;
                        const bool yok = zok && !((sy == 0 && b == P) || (sy == 1 && b == 0)) && vy >= 1 && vy <= npy;
                        const int qy = sy == 0 ? P - 1 + b : b - 1;
#pragma unroll
                        for (int sx = 0; sx < 2; ++sx) {
                            const int vx = i + sx;
                            const bool ok = yok && !((sx == 0 && a == P) || (sx == 1 && a == 0)) && vx >= 1 && vx <= npx;
                            const int qx = sx == 0 ? P - 1 + a : a - 1;
                            const size_t off = ok ? (size_t)((vx - 1) + npx * ((vy - 1) + npy * (vz - 1))) * nP3 +
                                                        qx + nP * qy + nP2 * qzs[t < nz ? t : 0]
                                                  : 0;
                            const C v = pbuf[off];
                            sum = ok ? sum + v : sum;
                        }
                    }
                }
                sz[ab * RS + cl] = sum;
            }
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < N2 * CH; idx += 256) {
            const int l = idx / CH, cl = idx % CH;
            const int e = blk * kLanes + h + cl;
            S* dst = z + (size_t)l * kLanes + h + cl;
            C out = e < pe.ncells ? alpha * sz[l * RS + cl] : (C)0;
            if (ACC && e < pe.ncells) out = load_as<C>(dst) + out;
            store_from(dst, out);
        }
        __syncthreads();
    }
}

template <int P, typename S, int ACC, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_combine_pm(LaunchTable L) {
    __shared__ __align__(16) char smem[pm_lds<P, typename Prec<S>::C>()];
    pi_combine_pm_body<P, S, ACC, MULTI>(L, blockIdx.x, gridDim.x, smem);
}

// The same combine by global node rows (p >= 4): a workgroup takes one node
// row (Y, Z) in chunks of 32 cells along x.  Thread t first sums node
// X = 32 i0 p + t of the chunk over the patches containing it (z, then y,
// then x patches in ascending vertex order, as k_pi_combine_pm), reading
// runs of consecutive x-nodes of each patch line, so every patch value is
// read once; the sums go through LDS and leave with threads on (node a,
// cell), a store covering up to 32 consecutive cells of a storage block.
// Bitwise equal to k_pi_combine_pm.  The first row of a problem zeroes the
// padding cells of its last storage block.
constexpr int kNrCells = 32;
// default p >= 4 combine by precision only: node rows for FP64 (measured
// faster there), per (block, plane) for 4- and 2-byte values
template <typename S> constexpr bool pm_rows_default() { return Prec<S>::id == FEM_F64; }
template <int P, typename C> constexpr int nr_lds() { return (kNrCells * P + 1) * (int)sizeof(C); }

template <int P, typename S, int ACC, bool MULTI>
__device__ __forceinline__ void pi_combine_nr_body(const LaunchTable& L, int item, int items, char* smem) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    constexpr int CC = kNrCells;
    static_assert(CC * P + 1 <= 256 && N * CC <= 256, "one chunk per workgroup pass");
    C* sx = reinterpret_cast<C*>(smem);
    const int tile = xcd_tile(item, items);      // neighbouring rows on one XCD
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int npx = n0 - 1, npy = n1 - 1;
    const int G1 = n1 * P + 1;
    const int row = tile - pe.tile_begin;
    const C* pbuf = static_cast<const C*>(pe.d);
    S* z = static_cast<S*>(pe.c);
    const C alpha = (C)pe.alpha;
    const int tid = threadIdx.x;
    if (row == 0) {
        for (int w = tid; w < NN * kLanes; w += 256) {
            const int e = (pe.nblk - 1) * kLanes + w % kLanes;
            if (e >= pe.ncells) store_from(z + cell_offset(e, w / kLanes, NN), (C)0);
        }
    }
    const int Y = row % G1, Z = row / G1;
    // patches containing the row along y and z (ascending vertex, with the
    // patch-local index), and the row's cell copies
    int vyp[2], qyp[2], nyp = 0, vzp[2], qzp[2], nzp = 0;
    int cyc[2], byc[2], nyc = 0, czc[2], bzc[2], nzc = 0;
    {
        const int qy = Y / P, ry = Y - qy * P;
        if (ry == 0) {
            if (qy >= 1 && qy <= npy) { vyp[nyp] = qy; qyp[nyp] = P - 1; ++nyp; }
            if (qy >= 1) { cyc[nyc] = qy - 1; byc[nyc] = P; ++nyc; }
            if (qy <= n1 - 1) { cyc[nyc] = qy; byc[nyc] = 0; ++nyc; }
        } else {
            if (qy >= 1) { vyp[nyp] = qy; qyp[nyp] = ry + P - 1; ++nyp; }
            if (qy + 1 <= npy) { vyp[nyp] = qy + 1; qyp[nyp] = ry - 1; ++nyp; }
            cyc[nyc] = qy; byc[nyc] = ry; ++nyc;
        }
        const int qz = Z / P, rz = Z - qz * P;
        if (rz == 0) {
            if (qz >= 1 && qz <= n2 - 1) { vzp[nzp] = qz; qzp[nzp] = P - 1; ++nzp; }
            if (qz >= 1) { czc[nzc] = qz - 1; bzc[nzc] = P; ++nzc; }
            if (qz <= n2 - 1) { czc[nzc] = qz; bzc[nzc] = 0; ++nzc; }
        } else {
            if (qz >= 1) { vzp[nzp] = qz; qzp[nzp] = rz + P - 1; ++nzp; }
            if (qz + 1 <= n2 - 1) { vzp[nzp] = qz + 1; qzp[nzp] = rz - 1; ++nzp; }
            czc[nzc] = qz; bzc[nzc] = rz; ++nzc;
        }
    }
    for (int i0 = 0; i0 < n0; i0 += CC) {
        const int nc = min(CC, n0 - i0);
        if (tid <= nc * P) {
            const int X = i0 * P + tid;
            const int qx = X / P, rx = X - qx * P;
            int vxp[2], qxp[2], nxp = 0;
            if (rx == 0) {
                if (qx >= 1 && qx <= npx) { vxp[nxp] = qx; qxp[nxp] = P - 1; ++nxp; }
            } else {
                if (qx >= 1) { vxp[nxp] = qx; qxp[nxp] = rx + P - 1; ++nxp; }
                if (qx + 1 <= npx) { vxp[nxp] = qx + 1; qxp[nxp] = rx - 1; ++nxp; }
            }
            // every term is loaded (a missing one from element 0) and dropped
            // by a select, so the loads are in flight together
            C sum = 0;
#pragma unroll
            for (int tz = 0; tz < 2; ++tz)
#pragma unroll
                for (int ty = 0; ty < 2; ++ty)
#pragma unroll
                    for (int tx = 0; tx < 2; ++tx) {
                        const bool ok = tz < nzp && ty < nyp && tx < nxp;
                        const size_t off =
                            ok ? (size_t)((vxp[tx] - 1) + npx * ((vyp[ty] - 1) + npy * (vzp[tz] - 1))) * nP3 + qxp[tx] +
                                     nP * qyp[ty] + nP2 * qzp[tz]
                               : 0;
                        const C v = pbuf[off];
                        sum = ok ? sum + v : sum;
                    }
            sx[tid] = sum;
        }
        __syncthreads();
        {
            const int a = tid / CC, c = tid % CC;
            if (a < N && c < nc) {
                const C v = sx[c * P + a];
#pragma unroll
                for (int cz = 0; cz < 2; ++cz) {
                    if (cz >= nzc) break;
#pragma unroll
                    for (int cy = 0; cy < 2; ++cy) {
                        if (cy >= nyc) break;
                        const int e = i0 + c + n0 * (cyc[cy] + n1 * czc[cz]);
                        S* d = z + cell_offset(e, a + N * (byc[cy] + N * bzc[cz]), NN);
                        C out = alpha * v;
                        if (ACC) out = load_as<C>(d) + out;
                        store_from(d, out);
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <int P, typename S, int ACC, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_combine_nr(LaunchTable L) {
    __shared__ __align__(16) char smem[nr_lds<P, typename Prec<S>::C>()];
    pi_combine_nr_body<P, S, ACC, MULTI>(L, blockIdx.x, gridDim.x, smem);
}

// The x pair (forward product, scaling by 1/(lambda_x+lambda_y+lambda_z),
// backward product) of every 16-line tile chained in registers: the
// forward product's accumulators are the backward product's B operand.  A
// lane holds accumulator rows row(lane, 0..3), so the backward k-steps take
// k = row(lane, ks) for lane group g = lane/16; `ab` holds the backward
// basis slices in that order (A[m][row(16 g + m, ks)]).  Branch-free as
// mfma_pass; a lane's four lambda_x values are loaded once.
template <typename C, int nP, int WPP>
__device__ __forceinline__ void mfma_pass_x2(C* pv, C* dump, const C (&af)[4], const C (&ab)[4], int lane, int sub,
                                             const C* lx, const C* ly, const C* lz) {
    using M = Mfma<C>;
    constexpr int NL = nP * nP, NT = (NL + 15) / 16;
    const int col = lane % 16, g = lane / 16;
    int koff[4], jr[4];
    bool jok[4];
    C lxr[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) koff[ks] = min(4 * ks + g, nP - 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int j = M::row(lane, r);
        jok[r] = j < nP;
        jr[r] = jok[r] ? j : 0;
        lxr[r] = lx[jr[r]];
    }
    for (int t = sub; t < NT; t += WPP) {
        const int line = 16 * t + col;
        const bool lok = line < NL;
        const int lc = lok ? line : NL - 1;
        const int qy = lc % nP, qz = lc / nP;
        const C* src = pv + nP * lc;
        typename M::V acc = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc = M::mma(af[ks], src[koff[ks]], acc);
        const C lyz = ly[qy] + lz[qz];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = jok[r] ? acc[r] * recip(lxr[r] + lyz) : (C)0;
        typename M::V out = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) out = M::mma(ab[ks], acc[ks], out);
#pragma unroll
        for (int r = 0; r < 4; ++r) *((lok && jok[r]) ? pv + nP * lc + jr[r] : dump + lane) = out[r];
    }
    if (WPP == 1) wave_sync();
    else __syncthreads();
}

// Wavefronts that share one patch: the larger patches split their 16-line
// tiles over the whole workgroup for more waves in flight per LDS byte.
template <int P> constexpr int mfma_waves_per_patch() { return P >= 6 ? 2 : 1; }

template <int P, typename C> constexpr int mfma_lds() {
    return ((4 / mfma_waves_per_patch<P>()) * (2 * P - 1) * (2 * P - 1) * (2 * P - 1) + 4 * 64) * (int)sizeof(C);
}

// pe: e = assembled global residual (C), d = patch buffer (C), fd = FD data (C)
template <int P, typename S, typename C, bool MULTI>
__device__ __forceinline__ void pi_solve_mfma_body(const LaunchTable& L, int item, int items, char* smem) {
    constexpr int nP = 2 * P - 1, nP2 = nP * nP, nP3 = nP2 * nP;
    constexpr int REC = fd_record(P);
    constexpr int WPP = mfma_waves_per_patch<P>();   // wavefronts per patch
    constexpr int PPW = 4 / WPP;                      // patches per workgroup
    static_assert(nP <= 16, "one MFMA tile per contraction");
    C (*spv)[nP3] = reinterpret_cast<C (*)[nP3]>(smem);
    C (*sdump)[64] = reinterpret_cast<C (*)[64]>(smem + sizeof(C) * PPW * nP3);   // per-wavefront sink for rows outside the patch
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int slot = wv / WPP, sub = wv % WPP;
    // a workgroup's patches are consecutive tiles.  A slot past the last
    // patch (the tail of an odd patch count) solves the last patch again in
    // its own LDS slot and stores nothing, so every wavefront of the
    // workgroup reaches every barrier
    const int tile_raw = item * PPW + slot;
    const bool active = tile_raw < L.total_tiles;
    const int tile = active ? tile_raw : L.total_tiles - 1;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int pidx = tile - pe.tile_begin;
    const int npx = pe.n[0] - 1, npy = pe.n[1] - 1;
    const int vi = 1 + pidx % npx, vj = 1 + (pidx / npx) % npy, vk = 1 + pidx / (npx * npy);
    const C* fx = static_cast<const C*>(pe.fd[0]) + (size_t)(vi - 1) * REC;
    const C* fy = static_cast<const C*>(pe.fd[1]) + (size_t)(vj - 1) * REC;
    const C* fz = static_cast<const C*>(pe.fd[2]) + (size_t)(vk - 1) * REC;
    // A operands: forward uses S^T (A[j][i] = S[i][j]), backward uses S;
    // each pass's slices are loaded while the previous pass runs
    auto loadA = [&](const C* f, bool fwd, C (&a)[4]) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int rr = lane % 16, kk = 4 * ks + lane / 16;
            const bool ok = rr < nP && kk < nP;
            a[ks] = ok ? (fwd ? f[kk * nP + rr] : f[rr * nP + kk]) : (C)0;
        }
    };
    C a0[4], a1[4];
    loadA(fz, true, a0);
    C* pv = spv[slot];
    const int t64 = sub * 64 + lane;                  // thread index within the patch's wavefronts
    // restrict: the patch's box of the assembled residual
    {
        const size_t G0 = (size_t)pe.n[0] * P + 1, G1 = (size_t)pe.n[1] * P + 1;
        const size_t I0 = (size_t)(vi - 1) * P + 1, J0 = (size_t)(vj - 1) * P + 1, K0 = (size_t)(vk - 1) * P + 1;
        // the box origin is uniform over the patch's wavefronts; offsets
        // within the box stay below G0 G1 nP < 2^32 (checked at set-up)
        const C* g = static_cast<const C*>(pe.e) + (I0 + G0 * (J0 + G1 * K0));
        // element q = qx + nP qy + nP^2 qz; the thread's (qx, qy, qz) advance
        // by the fixed stride without divisions, and all loads are issued
        // before the first LDS store
        constexpr int STEP = 64 * WPP, NIT = (nP3 + STEP - 1) / STEP;
        constexpr int DX = STEP % nP, DY = (STEP / nP) % nP, DZ = STEP / nP2;
        int qx = t64 % nP, qy = (t64 / nP) % nP;
        const uint32_t g0 = (uint32_t)G0, g1 = (uint32_t)G1;
        uint32_t off = qx + g0 * (qy + g1 * (uint32_t)(t64 / nP2));
        const uint32_t dstep = DX + g0 * (DY + g1 * DZ);            // uniform node-offset steps
        const uint32_t cx = g0 - nP, cy = g0 * (g1 - nP);           // carries into y and z
        C vals[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            vals[it] = t64 + STEP * it < nP3 ? g[off] : (C)0;
            qx += DX;
            qy += DY;
            off += dstep;
            if (qx >= nP) { qx -= nP; ++qy; off += cx; }
            if (qy >= nP) { qy -= nP; off += cy; }
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it)
            if (t64 + STEP * it < nP3) pv[t64 + STEP * it] = vals[it];
    }
    if (WPP == 1) wave_sync();
    else __syncthreads();
    const C* lx = fx + nP2;
    const C* ly = fy + nP2;
    const C* lz = fz + nP2;
    C* dump = sdump[wv];
    loadA(fy, true, a1);
    mfma_pass<C, nP, 2, WPP>(pv, dump, a0, lane, sub);
    loadA(fx, true, a0);
    mfma_pass<C, nP, 1, WPP>(pv, dump, a1, lane, sub);
    {
        // backward x basis in the accumulator row order of the forward product
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int rr = lane % 16, kk = Mfma<C>::row(lane, ks);
            a1[ks] = (rr < nP && kk < nP) ? fx[rr * nP + kk] : (C)0;
        }
        mfma_pass_x2<C, nP, WPP>(pv, dump, a0, a1, lane, sub, lx, ly, lz);
    }
    loadA(fy, false, a0);
    loadA(fz, false, a1);
    mfma_pass<C, nP, 1, WPP>(pv, dump, a0, lane, sub);
    mfma_pass<C, nP, 2, WPP>(pv, dump, a1, lane, sub);
    // patch-major buffer: each patch's values are one contiguous run
    C* out = static_cast<C*>(pe.d) + (size_t)pidx * nP3;
    if (active)
        for (int q = t64; q < nP3; q += 64 * WPP) out[q] = pv[q];
}

template <int P, typename S, typename C, bool MULTI>
__global__ void __launch_bounds__(256) k_pi_solve_mfma(LaunchTable L) {
    __shared__ __align__(16) char smem[mfma_lds<P, C>()];
    pi_solve_mfma_body<P, S, C, MULTI>(L, blockIdx.x, gridDim.x, smem);
}

template <int P, typename S>
static hipError_t launch_assemble_nodes(ProbEntry* ents, int nprob, TableStager* d_tab, hipStream_t s);

template <int P, typename S>
static hipError_t launch_assemble(ProbEntry* ents, int nprob, TableStager* d_tab, hipStream_t s, int gcap) {
    (void)gcap;
    return launch_assemble_nodes<P, S>(ents, nprob, d_tab, s);
}


template <int P, typename S>
static hipError_t launch_pi_mfma(int accumulate, ProbEntry* ents, int nprob, TableStager* d_tab, hipStream_t s,
                                 int gcap) {
    using C = typename Prec<S>::C;
    // 1. assemble r into each problem's global-node array
    hipError_t err = launch_assemble<P, S>(ents, nprob, d_tab, s, gcap);
    if (err != hipSuccess) return err;
    int tiles = 0;
    // 2. one wavefront per patch
    for (int i = 0; i < nprob; ++i) {
        const int npx = ents[i].n[0] - 1, npy = ents[i].n[1] - 1, npz = ents[i].n[2] - 1;
        ents[i].tile_begin = tiles;
        ents[i].ntiles = (npx > 0 && npy > 0 && npz > 0) ? npx * npy * npz : 0;
        tiles += ents[i].ntiles;
    }
    LaunchTable L1{};
    L1.nprob = nprob;
    L1.total_tiles = tiles;
    err = stage_table(L1, ents, nprob, d_tab, s);
    if (err != hipSuccess) return err;
    if (tiles > 0) {
        constexpr int PPW = 4 / mfma_waves_per_patch<P>();
        const int grid = (tiles + PPW - 1) / PPW;
        TraceSpan ts("pi_solve", P, Prec<S>::id, s);
        if (nprob > 1) hipLaunchKernelGGL((k_pi_solve_mfma<P, S, C, true>), dim3(grid), dim3(256), 0, s, L1);
        else hipLaunchKernelGGL((k_pi_solve_mfma<P, S, C, false>), dim3(grid), dim3(256), 0, s, L1);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    // 3. combine into the cells: by global node rows, or per (storage
    //    block, node plane) with the per-cell switch
    const int cpc = g_combine_per_cell.load(std::memory_order_relaxed);
    const bool rows = cpc == 2 || (cpc == 0 && pm_rows_default<S>());
    int tiles2 = 0;
    for (int i = 0; i < nprob; ++i) {
        ents[i].tile_begin = tiles2;
        ents[i].ntiles = rows ? (ents[i].n[1] * P + 1) * (ents[i].n[2] * P + 1) : ents[i].nblk * (P + 1);
        tiles2 += ents[i].ntiles;
    }
    LaunchTable L2{};
    L2.nprob = nprob;
    L2.total_tiles = tiles2;
    err = stage_table(L2, ents, nprob, d_tab, s);
    if (err != hipSuccess) return err;
    const int grid2 = (tiles2 + 7) / 8 * 8;
    TraceSpan ts("pi_combine", P, Prec<S>::id, s);
    if (rows) {
        if (nprob > 1) {
            if (accumulate) hipLaunchKernelGGL((k_pi_combine_nr<P, S, 1, true>), dim3(grid2), dim3(256), 0, s, L2);
            else hipLaunchKernelGGL((k_pi_combine_nr<P, S, 0, true>), dim3(grid2), dim3(256), 0, s, L2);
        } else {
            if (accumulate) hipLaunchKernelGGL((k_pi_combine_nr<P, S, 1, false>), dim3(grid2), dim3(256), 0, s, L2);
            else hipLaunchKernelGGL((k_pi_combine_nr<P, S, 0, false>), dim3(grid2), dim3(256), 0, s, L2);
        }
        return hipGetLastError();
    }
    if (nprob > 1) {
        if (accumulate) hipLaunchKernelGGL((k_pi_combine_pm<P, S, 1, true>), dim3(grid2), dim3(256), 0, s, L2);
        else hipLaunchKernelGGL((k_pi_combine_pm<P, S, 0, true>), dim3(grid2), dim3(256), 0, s, L2);
    } else {
        if (accumulate) hipLaunchKernelGGL((k_pi_combine_pm<P, S, 1, false>), dim3(grid2), dim3(256), 0, s, L2);
        else hipLaunchKernelGGL((k_pi_combine_pm<P, S, 0, false>), dim3(grid2), dim3(256), 0, s, L2);
    }
    return hipGetLastError();
}

// Two-phase patch inverse of one problem in z-slabs of vertex layers: the
// solves of a slab are followed at once by the combine of every cell block
// whose patches are now all solved, so a slab's patch results are read back
// while they still sit in the Infinity Cache.  Same kernels and the same
// arithmetic as one launch of each (the results are identical); tiles are
// offset through the entry's tile_begin.
template <int P, typename S>
static hipError_t launch_pi_slabs(int accumulate, ProbEntry e, hipStream_t s, int nslab, int gcap) {
    constexpr int CBP = solve_g_tile<P>();
    constexpr int N = P + 1;
    hipError_t err = launch_assemble<P, S>(&e, 1, nullptr, s, gcap);
    if (err != hipSuccess) return err;
    const int npx = e.n[0] - 1, npy = e.n[1] - 1, npz = e.n[2] - 1;
    const int tpr = (npx + CBP - 1) / CBP;
    const long layer_cells = (long)e.n[0] * e.n[1];
    int kdone = 0, bdone = 0;                       // cell layers / blocks combined so far
    for (int c = 0; c < nslab; ++c) {
        const int va = 1 + (int)((long)npz * c / nslab), vb = (int)((long)npz * (c + 1) / nslab);
        if (vb >= va && npx > 0 && npy > 0) {
            LaunchTable L{};
            L.nprob = 1;
            const int t0 = (va - 1) * npy * tpr, t1 = vb * npy * tpr;
            L.one = e;
            L.one.tile_begin = -t0;
            L.total_tiles = t1 - t0;
            TraceSpan ts("pi_solve", P, Prec<S>::id, s);
            hipLaunchKernelGGL((k_pi_solve_g<P, S, CBP, false>), dim3((t1 - t0 + 7) / 8 * 8), dim3(256), 0, s, L);
        }
        // cell layers whose covering vertex layers (k and k+1 within 1..npz) are solved
        const int kb = (c == nslab - 1) ? e.n[2] : vb;       // layers [kdone, kb) are complete
        int bb = (c == nslab - 1) ? e.nblk : (int)((kb * layer_cells) / kLanes);
        if (bb > bdone) {
            LaunchTable L{};
            L.nprob = 1;
            L.one = e;
            L.one.tile_begin = -bdone * N;
            L.total_tiles = (bb - bdone) * N;
            TraceSpan ts("pi_combine", P, Prec<S>::id, s);
            const int grid = ((L.total_tiles + 3) / 4 + 7) / 8 * 8;
            if (accumulate) hipLaunchKernelGGL((k_pi_combine_planes<P, S, 1, false>), dim3(grid), dim3(256), 0, s, L);
            else hipLaunchKernelGGL((k_pi_combine_planes<P, S, 0, false>), dim3(grid), dim3(256), 0, s, L);
            bdone = bb;
        }
        kdone = kb;
    }
    (void)kdone;
    return hipGetLastError();
}

// Patch inverse for p <= 3 through the x-combined buffer: assembly, the
// solves with the in-tile x-combine, the combine by global node rows.
template <int P, typename S, bool WAVE>
static hipError_t launch_pi_xcomb(int accumulate, ProbEntry* ents, int nprob, TableStager* d_tab, hipStream_t s,
                                  int gcap) {
    constexpr int CBP = WAVE ? solve_w_tile<P>() : solve_g_tile<P>();
    hipError_t err = launch_assemble<P, S>(ents, nprob, d_tab, s, gcap);
    if (err != hipSuccess) return err;
    int t1 = 0;
    for (int i = 0; i < nprob; ++i) {
        const int npx = ents[i].n[0] - 1, npy = ents[i].n[1] - 1, npz = ents[i].n[2] - 1;
        ents[i].tile_begin = t1;
        ents[i].ntiles = (npx > 0 && npy > 0 && npz > 0) ? ((npx + CBP - 1) / CBP) * npy * npz : 0;
        t1 += ents[i].ntiles;
    }
    if (t1 > 0) {
        LaunchTable Lg{};
        Lg.nprob = nprob;
        Lg.total_tiles = t1;
        err = stage_table(Lg, ents, nprob, d_tab, s);
        if (err != hipSuccess) return err;
        TraceSpan ts("pi_solve", P, Prec<S>::id, s);
        if constexpr (WAVE) {
            const int grid = ((t1 + 3) / 4 + 7) / 8 * 8;             // four tiles per workgroup
            if (nprob > 1) hipLaunchKernelGGL((k_pi_solve_w<P, S, true>), dim3(grid), dim3(256), 0, s, Lg);
            else hipLaunchKernelGGL((k_pi_solve_w<P, S, false>), dim3(grid), dim3(256), 0, s, Lg);
        } else {
            const int grid = (t1 + 7) / 8 * 8;
            if (nprob > 1) hipLaunchKernelGGL((k_pi_solve_x<P, S, CBP, true>), dim3(grid), dim3(256), 0, s, Lg);
            else hipLaunchKernelGGL((k_pi_solve_x<P, S, CBP, false>), dim3(grid), dim3(256), 0, s, Lg);
        }
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    int t4 = 0;
    for (int i = 0; i < nprob; ++i) {
        const int rows = (ents[i].n[1] * P + 1) * (ents[i].n[2] * P + 1);
        ents[i].tile_begin = t4;
        ents[i].ntiles = (rows + 3) / 4;
        t4 += ents[i].ntiles;
    }
    LaunchTable L4{};
    L4.nprob = nprob;
    L4.total_tiles = t4;
    err = stage_table(L4, ents, nprob, d_tab, s);
    if (err != hipSuccess) return err;
    TraceSpan ts("pi_combine", P, Prec<S>::id, s);
    if (nprob > 1) {
        if (accumulate) hipLaunchKernelGGL((k_pi_combine_x<P, S, CBP, 1, true>), dim3(t4), dim3(256), 0, s, L4);
        else hipLaunchKernelGGL((k_pi_combine_x<P, S, CBP, 0, true>), dim3(t4), dim3(256), 0, s, L4);
    } else {
        if (accumulate) hipLaunchKernelGGL((k_pi_combine_x<P, S, CBP, 1, false>), dim3(t4), dim3(256), 0, s, L4);
        else hipLaunchKernelGGL((k_pi_combine_x<P, S, CBP, 0, false>), dim3(t4), dim3(256), 0, s, L4);
    }
    return hipGetLastError();
}

// Default patch-inverse variant for p <= 3 (by degree and precision only):
// p = 2 in every precision, the wavefront-tiled solves with the in-tile
// x-combine; p = 3 in FP64, the workgroup-tiled ones; otherwise the two
// launches through the patch buffer.
template <int P, typename S> constexpr bool pi_wave_default() { return P == 2; }
template <int P, typename S> constexpr bool pi_xcomb_default() {
    return pi_wave_default<P, S>() || (P == 3 && Prec<S>::id == FEM_F64);
}
template <int P, typename S> constexpr int pi_xcomb_tile() {
    return pi_wave_default<P, S>() ? solve_w_tile<P>() : solve_g_tile<P>();
}

template <int P, typename S>
static hipError_t launch_pi_t(int accumulate, ProbEntry* ents, int nprob, TableStager* d_tab, hipStream_t s,
                              const LaunchCfg& cfg) {
    if constexpr (P <= 3) {
        // default by degree and precision only (never by size or launch mix, so
        // a problem gets the same variant alone and batched): the solves with
        // the in-tile x-combine where they measured faster (p = 2: one
        // wavefront per tile, in every precision; p = 3 in FP64: one
        // workgroup per tile), the two launches through the patch buffer
        // otherwise
        const int dflt = pi_wave_default<P, S>() ? 4 : pi_xcomb_default<P, S>() ? 3 : 0;
        const int gf = g_pi_fused.load(std::memory_order_relaxed);
        const int fused = cfg.pi_fused >= 0 ? cfg.pi_fused : gf >= 0 ? gf : dflt;
        if (fused == 3 || fused == 4) {
            const int gc = cfg.grid_cap > 0 ? cfg.grid_cap : kMaxGrid;
            return fused == 4 ? launch_pi_xcomb<P, S, true>(accumulate, ents, nprob, d_tab, s, gc)
                              : launch_pi_xcomb<P, S, false>(accumulate, ents, nprob, d_tab, s, gc);
        }
        if (fused == 2) return launch_pi_sweep_g<P, S>(accumulate, ents, nprob, d_tab, s);
        if (fused) return launch_pi_sweep<P, S>(accumulate, ents, nprob, d_tab, s);
    }
    const int gcap = cfg.grid_cap > 0 ? cfg.grid_cap : kMaxGrid;
    if constexpr (P >= 4) {
        const int gf = g_pi_fused.load(std::memory_order_relaxed);
        const int mode = cfg.pi_fused >= 0 ? cfg.pi_fused : gf >= 0 ? gf : 0;
        if (mode != 2) return launch_pi_mfma<P, S>(accumulate, ents, nprob, d_tab, s, gcap);
    }
    using C = typename Prec<S>::C;
    constexpr int CBP = pi_patches_per_tile<P, C>();
    if constexpr (P <= 3) {
        if (nprob == 1 && !g_restrict_from_cells && g_combine_per_cell != 1) {
            // slabs of at most ~pi_slab_bytes of patch results (one slab: plain two launches)
            const size_t pbytes = (size_t)(ents[0].n[0] - 1) * (ents[0].n[1] - 1) * (ents[0].n[2] - 1) *
                                  (2 * P - 1) * (2 * P - 1) * (2 * P - 1) * sizeof(C);
            const size_t slab_mb = (size_t)g_pi_slab_mb.load(std::memory_order_relaxed);
            int nslab = slab_mb > 0 ? (int)((pbytes + (slab_mb << 20) - 1) / (slab_mb << 20)) : 1;
            nslab = std::max(1, std::min(nslab, std::max(1, ents[0].n[2] - 1)));
            if (nslab > 1) return launch_pi_slabs<P, S>(accumulate, ents[0], s, nslab, gcap);
        }
    }
    LaunchTable L{};
    int tiles = 0;
    for (int i = 0; i < nprob; ++i) {
        const int npx = ents[i].n[0] - 1, npy = ents[i].n[1] - 1, npz = ents[i].n[2] - 1;
        ents[i].tile_begin = tiles;
        ents[i].ntiles = (npx > 0 && npy > 0 && npz > 0) ? ((npx + CBP - 1) / CBP) * npy * npz : 0;
        tiles += ents[i].ntiles;
    }
    L.nprob = nprob;
    L.total_tiles = tiles;
    // the default p <= 3 path stages its own tables (assembly, solves)
    const bool own_tables = (P <= 3) && !g_restrict_from_cells;
    hipError_t err = own_tables ? hipSuccess : stage_table(L, ents, nprob, d_tab, s);
    if (err != hipSuccess) return err;
    if (tiles > 0) {
        if constexpr (P <= 3) {
            const int grid = (tiles + 7) / 8 * 8;
            if (g_restrict_from_cells) {
                TraceSpan ts("pi_solve", P, Prec<S>::id, s);
                if (nprob > 1) hipLaunchKernelGGL((k_pi_solve_r<P, S, CBP, true>), dim3(grid), dim3(256), 0, s, L);
                else hipLaunchKernelGGL((k_pi_solve_r<P, S, CBP, false>), dim3(grid), dim3(256), 0, s, L);
            } else {
                err = launch_assemble<P, S>(ents, nprob, d_tab, s, gcap);
                if (err != hipSuccess) return err;
                int t1 = 0;
                for (int i = 0; i < nprob; ++i) {
                    const int npx = ents[i].n[0] - 1, npy = ents[i].n[1] - 1, npz = ents[i].n[2] - 1;
                    ents[i].tile_begin = t1;
                    constexpr int TG = solve_g_tile<P>();
                    ents[i].ntiles = (npx > 0 && npy > 0 && npz > 0) ? ((npx + TG - 1) / TG) * npy * npz : 0;
                    t1 += ents[i].ntiles;
                }
                LaunchTable Lg{};
                Lg.nprob = nprob;
                Lg.total_tiles = t1;
                err = stage_table(Lg, ents, nprob, d_tab, s);
                if (err != hipSuccess) return err;
                TraceSpan ts("pi_solve", P, Prec<S>::id, s);
                constexpr int TG = solve_g_tile<P>();
                const int grid_g = (t1 + 7) / 8 * 8;
                if (nprob > 1) hipLaunchKernelGGL((k_pi_solve_g<P, S, TG, true>), dim3(grid_g), dim3(256), 0, s, Lg);
                else hipLaunchKernelGGL((k_pi_solve_g<P, S, TG, false>), dim3(grid_g), dim3(256), 0, s, Lg);
            }
        } else if constexpr (P == 4) {
            const int grid = (tiles + 7) / 8 * 8;
            TraceSpan ts("pi_solve", P, Prec<S>::id, s);
            if (nprob > 1) hipLaunchKernelGGL((k_pi_solve_r<P, S, CBP, true>), dim3(grid), dim3(256), 0, s, L);
            else hipLaunchKernelGGL((k_pi_solve_r<P, S, CBP, false>), dim3(grid), dim3(256), 0, s, L);
        } else {
            const int grid = tiles < gcap ? tiles : gcap;
            TraceSpan ts("pi_solve", P, Prec<S>::id, s);
            if (nprob > 1) hipLaunchKernelGGL((k_pi_solve<P, S, CBP, true>), dim3(grid), dim3(256), 0, s, L);
            else hipLaunchKernelGGL((k_pi_solve<P, S, CBP, false>), dim3(grid), dim3(256), 0, s, L);
        }
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    // phase 2 over storage blocks (separate table: tile ranges differ)
    int tiles2 = 0;
    for (int i = 0; i < nprob; ++i) {
        ents[i].tile_begin = tiles2;
        ents[i].ntiles = ents[i].nblk;
        tiles2 += ents[i].nblk;
    }
    LaunchTable L2{};
    L2.nprob = nprob;
    L2.total_tiles = tiles2;
    err = stage_table(L2, ents, nprob, d_tab, s);
    if (err != hipSuccess) return err;
    if constexpr (P <= 3) {
        if (g_combine_per_cell == 1) {
            const int grid = (tiles2 + 3) / 4;
            TraceSpan ts("pi_combine", P, Prec<S>::id, s);
            if (nprob > 1) {
                if (accumulate) hipLaunchKernelGGL((k_pi_combine_cell<P, S, 1, true>), dim3(grid), dim3(256), 0, s, L2);
                else hipLaunchKernelGGL((k_pi_combine_cell<P, S, 0, true>), dim3(grid), dim3(256), 0, s, L2);
            } else {
                if (accumulate) hipLaunchKernelGGL((k_pi_combine_cell<P, S, 1, false>), dim3(grid), dim3(256), 0, s, L2);
                else hipLaunchKernelGGL((k_pi_combine_cell<P, S, 0, false>), dim3(grid), dim3(256), 0, s, L2);
            }
            return hipGetLastError();
        }
        // FP64 on long rows: one wavefront per global node row, each patch
        // value read once (identical results to the per-plane combine below,
        // which is the faster one for 4-byte values)
        bool long_rows = Prec<S>::id == FEM_F64;
        for (int i = 0; i < nprob; ++i) long_rows = long_rows && ents[i].n[0] >= 48;
        if (long_rows) {
            int t4 = 0;
            for (int i = 0; i < nprob; ++i) {
                const int rows = (ents[i].n[1] * P + 1) * (ents[i].n[2] * P + 1);
                ents[i].tile_begin = t4;
                ents[i].ntiles = (rows + 3) / 4;
                t4 += ents[i].ntiles;
            }
            LaunchTable L4{};
            L4.nprob = nprob;
            L4.total_tiles = t4;
            err = stage_table(L4, ents, nprob, d_tab, s);
            if (err != hipSuccess) return err;
            TraceSpan ts("pi_combine", P, Prec<S>::id, s);
            if (nprob > 1) {
                if (accumulate) hipLaunchKernelGGL((k_pi_combine_rows<P, S, 1, true>), dim3(t4), dim3(256), 0, s, L4);
                else hipLaunchKernelGGL((k_pi_combine_rows<P, S, 0, true>), dim3(t4), dim3(256), 0, s, L4);
            } else {
                if (accumulate) hipLaunchKernelGGL((k_pi_combine_rows<P, S, 1, false>), dim3(t4), dim3(256), 0, s, L4);
                else hipLaunchKernelGGL((k_pi_combine_rows<P, S, 0, false>), dim3(t4), dim3(256), 0, s, L4);
            }
            return hipGetLastError();
        }
        // one wavefront per (block, plane)
        int t3 = 0;
        for (int i = 0; i < nprob; ++i) {
            ents[i].tile_begin = t3;
            ents[i].ntiles = ents[i].nblk * (P + 1) * ((P + 1 + combine_brows<P>() - 1) / combine_brows<P>());
            t3 += ents[i].ntiles;
        }
        LaunchTable L3{};
        L3.nprob = nprob;
        L3.total_tiles = t3;
        err = stage_table(L3, ents, nprob, d_tab, s);
        if (err != hipSuccess) return err;
        const int grid = ((t3 + 3) / 4 + 7) / 8 * 8;
        TraceSpan ts("pi_combine", P, Prec<S>::id, s);
        if (nprob > 1) {
            if (accumulate) hipLaunchKernelGGL((k_pi_combine_planes<P, S, 1, true>), dim3(grid), dim3(256), 0, s, L3);
            else hipLaunchKernelGGL((k_pi_combine_planes<P, S, 0, true>), dim3(grid), dim3(256), 0, s, L3);
        } else {
            if (accumulate) hipLaunchKernelGGL((k_pi_combine_planes<P, S, 1, false>), dim3(grid), dim3(256), 0, s, L3);
            else hipLaunchKernelGGL((k_pi_combine_planes<P, S, 0, false>), dim3(grid), dim3(256), 0, s, L3);
        }
        return hipGetLastError();
    }
    const int grid2 = tiles2 < gcap ? tiles2 : gcap;
    TraceSpan ts("pi_combine", P, Prec<S>::id, s);
    if (nprob > 1) {
        if (accumulate) hipLaunchKernelGGL((k_pi_combine<P, S, 1, true>), dim3(grid2), dim3(256), 0, s, L2);
        else hipLaunchKernelGGL((k_pi_combine<P, S, 0, true>), dim3(grid2), dim3(256), 0, s, L2);
    } else {
        if (accumulate) hipLaunchKernelGGL((k_pi_combine<P, S, 1, false>), dim3(grid2), dim3(256), 0, s, L2);
        else hipLaunchKernelGGL((k_pi_combine<P, S, 0, false>), dim3(grid2), dim3(256), 0, s, L2);
    }
    return hipGetLastError();
}

template <int P>
static hipError_t launch_pi_p(int prec, int acc, ProbEntry* e, int n, TableStager* t, hipStream_t s,
                              const LaunchCfg& cfg) {
    switch (prec) {
        case FEM_F64: return launch_pi_t<P, double>(acc, e, n, t, s, cfg);
        case FEM_F32: return launch_pi_t<P, float>(acc, e, n, t, s, cfg);
        case FEM_F16: return launch_pi_t<P, f16_t>(acc, e, n, t, s, cfg);
        default: return launch_pi_t<P, bf16_t>(acc, e, n, t, s, cfg);
    }
}

// ---------------------------------------------------------------------------
// Mixed-degree patch inverse: every degree's default variant (p = 2, 3:
// solves with the in-tile x-combine in FP64, solves through the patch buffer
// in FP32/BF16; p = 7: MFMA solves), each of its three phases (assembly,
// solves, combine) one persistent launch over all degrees.
// (the assembly with lanes over nodes: the same sums as the long-row variant
// with lanes over cells, whose registers would bound the whole launch)
template <int P, typename S>
struct AssembleBody {
    using Arg = NoArg;
    static constexpr int kLds = 0;
    __device__ static __forceinline__ void run(const LaunchTable& L, const NoArg&, int item, int items, char*) {
        assemble_nodes_body<P, S, typename Prec<S>::C, true>(L, item, items);
    }
};

template <int P, typename S>
struct SolveBody {
    using C = typename Prec<S>::C;
    using Arg = NoArg;
    static constexpr int CBP = solve_g_tile<P>();
    static constexpr int kLds = P >= 4 ? mfma_lds<P, C>()
                              : pi_wave_default<P, S>() ? solve_w_lds<P, C>()
                              : pi_xcomb_default<P, S>() ? solve_x_lds<P, C, CBP>() : solve_g_lds<P, C, CBP>();
    __device__ static __forceinline__ void run(const LaunchTable& L, const NoArg&, int item, int items, char* smem) {
        if constexpr (P >= 4) pi_solve_mfma_body<P, S, C, true>(L, item, items, smem);
        else if constexpr (pi_wave_default<P, S>()) pi_solve_w_body<P, S, true>(L, item, items, smem);
        else if constexpr (pi_xcomb_default<P, S>()) pi_solve_x_body<P, S, CBP, true>(L, item, items, smem);
        else pi_solve_g_body<P, S, CBP, true>(L, item, items, smem);
    }
};

template <int P, typename S, int ACC>
struct CombineBody {
    using C = typename Prec<S>::C;
    using Arg = NoArg;
    static constexpr int kLds = P >= 4 ? (pm_rows_default<S>() ? nr_lds<P, C>() : pm_lds<P, C>()) : 0;
    __device__ static __forceinline__ void run(const LaunchTable& L, const NoArg&, int item, int items, char* smem) {
        if constexpr (P >= 4 && pm_rows_default<S>()) pi_combine_nr_body<P, S, ACC, true>(L, item, items, smem);
        else if constexpr (P >= 4) pi_combine_pm_body<P, S, ACC, true>(L, item, items, smem);
        else if constexpr (pi_xcomb_default<P, S>()) pi_combine_x_body<P, S, pi_xcomb_tile<P, S>(), ACC, true>(L, item, items);
        else pi_combine_planes_body<P, S, ACC, true>(L, item, items);
    }
};

// Tiles and items of each phase, as the single-degree launches count them.
template <int P, typename S> static int pi_solve_tiles(const ProbEntry& e) {
    const int npx = e.n[0] - 1, npy = e.n[1] - 1, npz = e.n[2] - 1;
    if (npx <= 0 || npy <= 0 || npz <= 0) return 0;
    if constexpr (P >= 4) return npx * npy * npz;
    else if constexpr (pi_wave_default<P, S>()) return ((npx + solve_w_tile<P>() - 1) / solve_w_tile<P>()) * npy * npz;
    else return ((npx + solve_g_tile<P>() - 1) / solve_g_tile<P>()) * npy * npz;
}
template <int P, typename S> static int pi_solve_items(int t) {
    if constexpr (P >= 4) return (t + 4 / mfma_waves_per_patch<P>() - 1) / (4 / mfma_waves_per_patch<P>());
    else if constexpr (pi_wave_default<P, S>()) return (t + 3) / 4;     // four tiles per workgroup
    else return t;
}
template <int P, typename S> static int pi_combine_tiles(const ProbEntry& e) {
    if constexpr (P >= 4 && pm_rows_default<S>()) return (e.n[1] * P + 1) * (e.n[2] * P + 1);
    else if constexpr (P >= 4) return e.nblk * (P + 1);
    else if constexpr (pi_xcomb_default<P, S>()) return ((e.n[1] * P + 1) * (e.n[2] * P + 1) + 3) / 4;
    else return e.nblk * (P + 1) * ((P + 1 + combine_brows<P>() - 1) / combine_brows<P>());
}
template <int P, typename S> static int pi_combine_items(int t) {
    if constexpr (P >= 4 || pi_xcomb_default<P, S>()) return t;
    else return (t + 3) / 4;
}

template <typename S, int ACC>
static hipError_t launch_pi_mixed_t(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    static_assert(mix_degree(0) == 7 && mix_degree(1) == 3 && mix_degree(2) == 2, "segment degrees");
    MixTable T{};
    int grid = 0;
    // 1. assembly into each problem's global-node array
    auto rows4 = [](int p, const ProbEntry& e) { return ((e.n[1] * p + 1) * (e.n[2] * p + 1) + 3) / 4; };
    auto same = [](int, int t) { return t; };
    hipError_t err = mix_build(ents, nprob, st, s, rows4, same, T, grid);
    if (err != hipSuccess) return err;
    if (grid > 0) {
        TraceSpan ts("pi_assemble", 0, Prec<S>::id, s);
        hipLaunchKernelGGL((k_mixed<AssembleBody<7, S>, AssembleBody<3, S>, AssembleBody<2, S>>), dim3(grid),
                           dim3(256), 0, s, T, NoArg{}, NoArg{}, NoArg{});
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    // 2. patch solves
    auto stiles = [](int p, const ProbEntry& e) {
        return p == 7 ? pi_solve_tiles<7, S>(e) : p == 3 ? pi_solve_tiles<3, S>(e) : pi_solve_tiles<2, S>(e);
    };
    auto sitems = [](int p, int t) {
        return p == 7 ? pi_solve_items<7, S>(t) : p == 3 ? pi_solve_items<3, S>(t) : pi_solve_items<2, S>(t);
    };
    err = mix_build(ents, nprob, st, s, stiles, sitems, T, grid);
    if (err != hipSuccess) return err;
    if (grid > 0) {
        TraceSpan ts("pi_solve", 0, Prec<S>::id, s);
        hipLaunchKernelGGL((k_mixed<SolveBody<7, S>, SolveBody<3, S>, SolveBody<2, S>>), dim3(grid), dim3(256), 0, s,
                           T, NoArg{}, NoArg{}, NoArg{});
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    // 3. combine into the cells
    auto ctiles = [](int p, const ProbEntry& e) {
        return p == 7 ? pi_combine_tiles<7, S>(e) : p == 3 ? pi_combine_tiles<3, S>(e) : pi_combine_tiles<2, S>(e);
    };
    auto citems = [](int p, int t) {
        return p == 7 ? pi_combine_items<7, S>(t) : p == 3 ? pi_combine_items<3, S>(t) : pi_combine_items<2, S>(t);
    };
    err = mix_build(ents, nprob, st, s, ctiles, citems, T, grid);
    if (err != hipSuccess || grid == 0) return err;
    TraceSpan ts("pi_combine", 0, Prec<S>::id, s);
    hipLaunchKernelGGL((k_mixed<CombineBody<7, S, ACC>, CombineBody<3, S, ACC>, CombineBody<2, S, ACC>>), dim3(grid),
                       dim3(256), 0, s, T, NoArg{}, NoArg{}, NoArg{});
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_pi_mixed_a(int accumulate, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    return accumulate ? launch_pi_mixed_t<S, 1>(ents, nprob, st, s) : launch_pi_mixed_t<S, 0>(ents, nprob, st, s);
}

hipError_t launch_patch_inverse_any(int prec, int accumulate, ProbEntry* ents, int nprob, TableStager* st,
                                    hipStream_t s, bool mix) {
    if (nprob <= 0) return hipSuccess;
    // the mixed bodies are the default variants: no process-wide override
    if (mix && g_pi_fused < 0 && !g_restrict_from_cells && !g_combine_per_cell && mix_degrees(ents, nprob) >= 2) {
        switch (prec) {
            case FEM_F64: return launch_pi_mixed_a<double>(accumulate, ents, nprob, st, s);
            case FEM_F32: return launch_pi_mixed_a<float>(accumulate, ents, nprob, st, s);
            case FEM_F16: return launch_pi_mixed_a<f16_t>(accumulate, ents, nprob, st, s);
            default: return launch_pi_mixed_a<bf16_t>(accumulate, ents, nprob, st, s);
        }
    }
    std::vector<ProbEntry> g;
    for (int p = 1; p <= kMaxP; ++p) {
        g.clear();
        for (int i = 0; i < nprob; ++i)
            if (ents[i].p == p) g.push_back(ents[i]);
        if (g.empty()) continue;
        hipError_t err = launch_patch_inverse(p, prec, accumulate, g.data(), (int)g.size(), st, s);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_patch_inverse(int p, int prec, int accumulate, ProbEntry* ents, int nprob,
                                TableStager* d_tab, hipStream_t s, const LaunchCfg& cfg) {
    switch (p) {
        case 1: return launch_pi_p<1>(prec, accumulate, ents, nprob, d_tab, s, cfg);
        case 2: return launch_pi_p<2>(prec, accumulate, ents, nprob, d_tab, s, cfg);
        case 3: return launch_pi_p<3>(prec, accumulate, ents, nprob, d_tab, s, cfg);
        case 4: return launch_pi_p<4>(prec, accumulate, ents, nprob, d_tab, s, cfg);
        case 5: return launch_pi_p<5>(prec, accumulate, ents, nprob, d_tab, s, cfg);
        case 6: return launch_pi_p<6>(prec, accumulate, ents, nprob, d_tab, s, cfg);
        case 7: return launch_pi_p<7>(prec, accumulate, ents, nprob, d_tab, s, cfg);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fem
