// Sum-factorised local operator apply on cell-wise storage.
//
// Laplace (Eq. "Laplace operator", Section 2.3) on a box cell of widths
// (hx, hy, hz) with 1D reference mass M and stiffness K on [0,1]:
//
//   y = cx (K x M x M) u + cy (M x K x M) u + cz (M x M x K) u,
//   cx = hy hz / hx,  cy = hx hz / hy,  cz = hx hy / hz,
//
// (the first factor acts along x).  Evaluated as seven 1D contractions:
//   A = Mz u,  Bz = Kz u,  C = cy Ky A + cz My Bz,  D = My A,
//   y = Mx C + cx Kx D.
// Mass (Eq. "mass operator"):  y = hx hy hz (M x M x M) u, three contractions.
// With Dirichlet conditions the Laplacian is P_I A P_I (boundary copies read
// and written as zero) while the mass apply is P_I M (input read in full), so
// that P_I M f is the load vector of nodal source values f.
//
// Two kernel shapes:
//  * k_apply_reg (p <= 3): one thread per cell.  The cell's (p+1)^3 values
//    are loaded into registers (one coalesced 64-cell segment per node), and
//    the output is produced one z-plane at a time, so the live state is the
//    input cell plus a few planes.
//  * k_apply_lds (any p): a workgroup owns CB cells staged in LDS and walks
//    the three directions with one thread per 1D line.
#include <atomic>

#include "fem_internal.h"
#include "launch.h"
#include "mfma.h"
#include "mixed.h"
#include "trace.h"

namespace fem {

// Process-wide switch for comparisons (FEM_OPT_APPLY_PLANES_P7; atomic: any
// thread may set it): 1 runs the p = 7 FP64 Laplace and residual applies on
// the plane-streamed VALU kernel.
std::atomic<int> g_apply_planes_p7{0};

enum ApplyMode { kApplyLaplace = 0, kApplyResidual = 1, kApplyMass = 2 };

template <typename C>
struct CellGeom {
    C cx, cy, cz, vol;
    bool xlo, xhi, ylo, yhi, zlo, zhi;
};

template <typename C>
__device__ __forceinline__ CellGeom<C> cell_geom(const ProbEntry& pe, int e) {
    const int n0 = pe.n[0], n1 = pe.n[1];
    const int i = e % n0, j = (e / n0) % n1, k = e / (n0 * n1);
    const double hx = pe.h[0][i], hy = pe.h[1][j], hz = pe.h[2][k];
    CellGeom<C> g;
    g.cx = (C)(hy * hz / hx);
    g.cy = (C)(hx * hz / hy);
    g.cz = (C)(hx * hy / hz);
    g.vol = (C)(hx * hy * hz);
    const bool d = pe.dirichlet != 0;
    g.xlo = d && i == 0;
    g.xhi = d && i == n0 - 1;
    g.ylo = d && j == 0;
    g.yhi = d && j == n1 - 1;
    g.zlo = d && k == 0;
    g.zhi = d && k == pe.n[2] - 1;
    return g;
}

template <int P, typename C>
__device__ __forceinline__ bool on_boundary(const CellGeom<C>& g, int a, int b, int c) {
    return (a == 0 && g.xlo) || (a == P && g.xhi) || (b == 0 && g.ylo) || (b == P && g.yhi) ||
           (c == 0 && g.zlo) || (c == P && g.zhi);
}

// ---------------------------------------------------------------------------
// One thread per cell, register resident.  Tile = one storage block (64
// cells) per wavefront.
// The kernel body takes the workgroup index and the grid size as arguments
// (here and below), so that a mixed-degree launch can run it on its items.
template <int P, typename S, int MODE, bool MULTI>
__device__ __forceinline__ void apply_reg_body(const LaunchTable& L, const RefMats<P, typename Prec<S>::C>& R,
                                               int item, int items) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    for (int tile = item * 4 + wv; tile < L.total_tiles; tile += items * 4) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int blk = tile - pe.tile_begin;
        const int e = blk * kLanes + lane;
        const size_t base = (size_t)blk * NN * kLanes + lane;
        const S* __restrict__ x = static_cast<const S*>(pe.a) + base;
        S* __restrict__ y = static_cast<S*>(pe.c) + base;
        if (e >= pe.ncells) {
            for (int l = 0; l < NN; ++l) store_from(y + l * kLanes, (C)0);
            continue;
        }
        const CellGeom<C> g = cell_geom<C>(pe, e);
        C u[NN];
#pragma unroll
        for (int l = 0; l < NN; ++l) u[l] = load_as<C>(x + l * kLanes);
        if (MODE != kApplyMass) {      // A_D = P_I A P_I; the mass apply is P_I M
#pragma unroll
            for (int c = 0; c < N; ++c)
#pragma unroll
                for (int b = 0; b < N; ++b)
#pragma unroll
                    for (int a = 0; a < N; ++a)
                        if (on_boundary<P>(g, a, b, c)) u[a + N * b + N2 * c] = (C)0;
        }

        const S* __restrict__ rres = (MODE == kApplyResidual)
            ? static_cast<const S*>(pe.b) + base : nullptr;

#pragma unroll
        for (int cz = 0; cz < N; ++cz) {
            C out[N2];
            if (MODE == kApplyMass) {
                C A[N2], Bp[N2];
#pragma unroll
                for (int ab = 0; ab < N2; ++ab) {
                    C s = 0;
#pragma unroll
                    for (int c = 0; c < N; ++c) s += R.M[cz * N + c] * u[ab + N2 * c];
                    A[ab] = s;
                }
#pragma unroll
                for (int a = 0; a < N; ++a)
#pragma unroll
                    for (int bb = 0; bb < N; ++bb) {
                        C s = 0;
#pragma unroll
                        for (int b = 0; b < N; ++b) s += R.M[bb * N + b] * A[a + N * b];
                        Bp[a + N * bb] = s;
                    }
#pragma unroll
                for (int b = 0; b < N; ++b)
#pragma unroll
                    for (int aa = 0; aa < N; ++aa) {
                        C s = 0;
#pragma unroll
                        for (int a = 0; a < N; ++a) s += R.M[aa * N + a] * Bp[a + N * b];
                        out[aa + N * b] = g.vol * s;
                    }
            } else {
                // z contraction onto output plane cz
                C A[N2], Bz[N2];
#pragma unroll
                for (int ab = 0; ab < N2; ++ab) {
                    C sm = 0, sk = 0;
#pragma unroll
                    for (int c = 0; c < N; ++c) {
                        sm += R.M[cz * N + c] * u[ab + N2 * c];
                        sk += R.K[cz * N + c] * u[ab + N2 * c];
                    }
                    A[ab] = sm;
                    Bz[ab] = sk;
                }
                // y contraction within the plane
                C Cc[N2], D[N2];
#pragma unroll
                for (int a = 0; a < N; ++a)
#pragma unroll
                    for (int bb = 0; bb < N; ++bb) {
                        C sky = 0, smb = 0, sma = 0;
#pragma unroll
                        for (int b = 0; b < N; ++b) {
                            sky += R.K[bb * N + b] * A[a + N * b];
                            smb += R.M[bb * N + b] * Bz[a + N * b];
                            sma += R.M[bb * N + b] * A[a + N * b];
                        }
                        Cc[a + N * bb] = g.cy * sky + g.cz * smb;
                        D[a + N * bb] = sma;
                    }
                // x contraction
#pragma unroll
                for (int b = 0; b < N; ++b)
#pragma unroll
                    for (int aa = 0; aa < N; ++aa) {
                        C sm = 0, sk = 0;
#pragma unroll
                        for (int a = 0; a < N; ++a) {
                            sm += R.M[aa * N + a] * Cc[a + N * b];
                            sk += R.K[aa * N + a] * D[a + N * b];
                        }
                        out[aa + N * b] = sm + g.cx * sk;
                    }
            }
#pragma unroll
            for (int b = 0; b < N; ++b)
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    const int l = a + N * b + N2 * cz;
                    C v = out[a + N * b];
                    if (MODE == kApplyResidual) v = load_as<C>(rres + l * kLanes) - v;
                    if (on_boundary<P>(g, a, b, cz)) v = (C)0;
                    store_from(y + l * kLanes, v);
                }
        }
    }
}

template <int P, typename S, int MODE, bool MULTI>
__global__ void __launch_bounds__(256)
k_apply_reg(LaunchTable L, RefMats<P, typename Prec<S>::C> R) {
    apply_reg_body<P, S, MODE, MULTI>(L, R, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// LDS line kernel.  Tile = CB consecutive cells of one storage block.
// LDS layout: value of local node l of tile cell c at [l * CB + c], so
// threads that differ in c touch consecutive words.
template <int P, typename S, int MODE, int CB, bool MULTI>
__global__ void __launch_bounds__(256)
k_apply_lds(LaunchTable L, RefMats<P, typename Prec<S>::C> R) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    constexpr int NT = 256;
    static_assert(NT % CB == 0, "tile cells must divide the workgroup");
    __shared__ C s0[NN * CB];
    __shared__ C s1[NN * CB];
    const int tid = threadIdx.x;
    const int c = tid % CB;            // the tile cell this thread serves in every loop
    for (int tile = blockIdx.x; tile < L.total_tiles; tile += gridDim.x) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        const int e0 = t * CB;                         // first cell of the tile
        const int blk = e0 / kLanes, lane0 = e0 % kLanes;
        const size_t base = (size_t)blk * NN * kLanes + lane0 + c;
        const S* __restrict__ x = static_cast<const S*>(pe.a) + base;
        S* __restrict__ y = static_cast<S*>(pe.c) + base;
        const S* __restrict__ rres = (MODE == kApplyResidual) ? static_cast<const S*>(pe.b) + base : nullptr;
        const int e = e0 + c;
        const bool valid = e < pe.ncells;
        CellGeom<C> g{};
        if (valid) g = cell_geom<C>(pe, e);
        // load (boundary copies of x read as zero)
        for (int l = tid / CB; l < NN; l += NT / CB) {
            C v = (C)0;
            if (valid && (MODE == kApplyMass || !on_boundary<P>(g, l % N, (l / N) % N, l / N2)))
                v = load_as<C>(x + (size_t)l * kLanes);
            s0[l * CB + c] = v;
        }
        __syncthreads();
        if (MODE == kApplyMass) {
            for (int ab = tid / CB; ab < N2; ab += NT / CB) {          // z lines
                C v[N];
#pragma unroll
                for (int k = 0; k < N; ++k) v[k] = s0[(ab + N2 * k) * CB + c];
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    C s = 0;
#pragma unroll
                    for (int m = 0; m < N; ++m) s += R.M[k * N + m] * v[m];
                    s0[(ab + N2 * k) * CB + c] = s;
                }
            }
            __syncthreads();
            for (int r = tid / CB; r < N2; r += NT / CB) {             // y lines, r = a + N k
                const int a = r % N, k = r / N;
                C v[N];
#pragma unroll
                for (int b = 0; b < N; ++b) v[b] = s0[(a + N * b + N2 * k) * CB + c];
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    C s = 0;
#pragma unroll
                    for (int m = 0; m < N; ++m) s += R.M[b * N + m] * v[m];
                    s0[(a + N * b + N2 * k) * CB + c] = s;
                }
            }
            __syncthreads();
            for (int r = tid / CB; r < N2; r += NT / CB) {             // x lines, r = b + N k
                C v[N];
#pragma unroll
                for (int a = 0; a < N; ++a) v[a] = s0[(a + N * r) * CB + c];
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    C s = 0;
#pragma unroll
                    for (int m = 0; m < N; ++m) s += R.M[a * N + m] * v[m];
                    s *= g.vol;
                    if (!valid || on_boundary<P>(g, a, r % N, r / N)) s = (C)0;
                    store_from(y + (size_t)(a + N * r) * kLanes, s);
                }
            }
            __syncthreads();
            continue;
        }
        // z pass: s0 <- A = Mz u, s1 <- Bz = Kz u
        for (int ab = tid / CB; ab < N2; ab += NT / CB) {
            C v[N];
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = s0[(ab + N2 * k) * CB + c];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                C sm = 0, sk = 0;
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    sm += R.M[k * N + m] * v[m];
                    sk += R.K[k * N + m] * v[m];
                }
                s0[(ab + N2 * k) * CB + c] = sm;
                s1[(ab + N2 * k) * CB + c] = sk;
            }
        }
        __syncthreads();
        // y pass: s1 <- C = cy Ky A + cz My Bz, s0 <- D = My A
        for (int r = tid / CB; r < N2; r += NT / CB) {
            const int a = r % N, k = r / N;
            C va[N], vb[N];
#pragma unroll
            for (int b = 0; b < N; ++b) {
                va[b] = s0[(a + N * b + N2 * k) * CB + c];
                vb[b] = s1[(a + N * b + N2 * k) * CB + c];
            }
#pragma unroll
            for (int b = 0; b < N; ++b) {
                C sky = 0, smb = 0, sma = 0;
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    sky += R.K[b * N + m] * va[m];
                    smb += R.M[b * N + m] * vb[m];
                    sma += R.M[b * N + m] * va[m];
                }
                s1[(a + N * b + N2 * k) * CB + c] = g.cy * sky + g.cz * smb;
                s0[(a + N * b + N2 * k) * CB + c] = sma;
            }
        }
        __syncthreads();
        // x pass: y = Mx C + cx Kx D, store
        for (int r = tid / CB; r < N2; r += NT / CB) {                 // r = b + N k
            C vc[N], vd[N];
#pragma unroll
            for (int a = 0; a < N; ++a) {
                vc[a] = s1[(a + N * r) * CB + c];
                vd[a] = s0[(a + N * r) * CB + c];
            }
#pragma unroll
            for (int a = 0; a < N; ++a) {
                C sm = 0, sk = 0;
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    sm += R.M[a * N + m] * vc[m];
                    sk += R.K[a * N + m] * vd[m];
                }
                C v = sm + g.cx * sk;
                const size_t off = (size_t)(a + N * r) * kLanes;
                if (MODE == kApplyResidual) v = load_as<C>(rres + off) - v;
                if (!valid || on_boundary<P>(g, a, r % N, r / N)) v = (C)0;
                store_from(y + off, v);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Launch selection.
template <int P, typename C>
static RefMats<P, C> ref_mats() {
    RefMats<P, C> R;
    const double* M = ref_mass(P);
    const double* K = ref_stiff(P);
    for (int i = 0; i < (P + 1) * (P + 1); ++i) {
        R.M[i] = (C)M[i];
        R.K[i] = (C)K[i];
    }
    return R;
}

// ---------------------------------------------------------------------------
// Plane-streamed apply for p >= 4.  A workgroup owns 16 consecutive cells of
// a storage block (so every load and store is a 128-byte run of one node
// plane) and walks the z node planes two at a time.  Per pair of planes the
// x and y contractions run in LDS with one thread per 1D line:
//     T1 = Kx u, T2 = Mx u                         (x lines)
//     P1 = cx My T1 + cy Ky T2,  P2 = My T2        (y lines, in place)
// and every (cell, a, b) z line accumulates y(k') += Mz(k',k) P1_k +
// cz Kz(k',k) P2_k in registers, so only two plane pairs of two arrays sit in
// LDS.  The mass apply keeps the T2/P2 chain: y = vol Mz (My Mx u).
// Workgroup shape of the plane-streamed apply (threads, z planes per step).
// A 512-thread, four-plane shape for 8-byte values measured slower.
template <int P, typename C> struct PlanesShape {
    static constexpr int NT = 256, KP = 2;
    static constexpr int CB = 16;                                   // cells per workgroup
    static constexpr int SL = KP * (P + 1) * (P + 1) * CB;          // values per LDS array
    static constexpr int kLds = (2 * SL + 2 * (P + 1) * (P + 1)) * (int)sizeof(C);
};

template <int P, typename S, int MODE, bool MULTI>
__device__ __forceinline__ void apply_planes_body(const LaunchTable& L, const RefMats<P, typename Prec<S>::C>& R,
                                                  int item, int items, char* smem) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    constexpr int NT = PlanesShape<P, C>::NT;
    constexpr int CB = PlanesShape<P, C>::CB;
    constexpr int KP = PlanesShape<P, C>::KP;   // z planes per step
    constexpr int NSTEP = (N + KP - 1) / KP;
    constexpr int SL = PlanesShape<P, C>::SL;
    constexpr int ZL = N2 * CB;            // z lines per workgroup
    constexpr int ZPT = (ZL + NT - 1) / NT;  // z lines per thread
    C* s1 = reinterpret_cast<C*>(smem);    // u -> T1 -> P1
    C* s2 = s1 + SL;                       // T2 -> P2
    // the 1D matrices (2 (p+1)^2 values) do not fit the scalar registers for
    // p = 7, so they are read as LDS broadcasts instead of being spilled
    C* sM = s2 + SL;
    C* sK = sM + N2;
    static_assert(NT % CB == 0 && kLanes % CB == 0, "cells per workgroup must divide the block");
    const int tid = threadIdx.x;
    for (int i = tid; i < N2; i += NT) {
        sM[i] = R.M[i];
        sK[i] = R.K[i];
    }
    __syncthreads();
    const int cl = tid % CB;               // the cell this thread serves in line passes
    for (int tile = item; tile < L.total_tiles; tile += items) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        const int blk = t / (kLanes / CB), lane0 = (t % (kLanes / CB)) * CB;
        const size_t base = (size_t)blk * NN * kLanes + lane0;
        const S* __restrict__ x = static_cast<const S*>(pe.a) + base;
        S* __restrict__ y = static_cast<S*>(pe.c) + base;
        const int e = blk * kLanes + lane0 + cl;
        const bool valid = e < pe.ncells;
        CellGeom<C> g{};
        if (valid) g = cell_geom<C>(pe, e);
        C acc[ZPT][N];
#pragma unroll
        for (int q = 0; q < ZPT; ++q)
#pragma unroll
            for (int k = 0; k < N; ++k) acc[q][k] = (C)0;

        for (int st = 0; st < NSTEP; ++st) {
            const int k0 = st * KP;
            // load planes k0, k0+1: item = cell + CB * (ab + N2 * kk)
            for (int item = tid; item < SL; item += NT) {
                const int kk = item / (N2 * CB), ab = (item / CB) % N2;
                const int k = k0 + kk;
                C v = (C)0;
                if (k < N && valid) {
                    const int l = ab + N2 * k;
                    if (MODE == kApplyMass || !on_boundary<P>(g, ab % N, ab / N, k))
                        v = load_as<C>(x + (size_t)l * kLanes + cl);
                }
                s1[item] = v;
            }
            __syncthreads();
            // x lines: task = cell + CB * (b + N * kk)
            for (int task = tid; task < CB * N * KP; task += NT) {
                const int r = task / CB;                   // b + N kk
                C v[N];
#pragma unroll
                for (int a = 0; a < N; ++a) v[a] = s1[(a + N * r) * CB + cl];
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    C sm = 0, sk = 0;
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        sm += sM[a * N + m] * v[m];
                        if (MODE != kApplyMass) sk += sK[a * N + m] * v[m];
                    }
                    s2[(a + N * r) * CB + cl] = sm;
                    if (MODE != kApplyMass) s1[(a + N * r) * CB + cl] = sk;
                }
            }
            __syncthreads();
            // y lines (in place): task = cell + CB * (a + N * kk)
            for (int task = tid; task < CB * N * KP; task += NT) {
                const int r = task / CB;
                const int a = r % N, kk = r / N;
                C v1[N], v2[N];
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    v2[b] = s2[(a + N * b + N2 * kk) * CB + cl];
                    if (MODE != kApplyMass) v1[b] = s1[(a + N * b + N2 * kk) * CB + cl];
                }
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    C m1 = 0, k2 = 0, m2 = 0;
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        m2 += sM[b * N + m] * v2[m];
                        if (MODE != kApplyMass) {
                            m1 += sM[b * N + m] * v1[m];
                            k2 += sK[b * N + m] * v2[m];
                        }
                    }
                    s2[(a + N * b + N2 * kk) * CB + cl] = m2;
                    if (MODE != kApplyMass) s1[(a + N * b + N2 * kk) * CB + cl] = g.cx * m1 + g.cy * k2;
                }
            }
            __syncthreads();
            // z accumulation: z line q of this thread = (cell, ab)
#pragma unroll
            for (int q = 0; q < ZPT; ++q) {
                const int zl = tid + NT * q;
                if (zl >= ZL) break;
                const int ab = zl / CB;               // the cell is cl: CB divides NT
#pragma unroll
                for (int kk = 0; kk < KP; ++kk) {
                    const int k = k0 + kk;
                    if (k >= N) break;
                    const C p2 = s2[(ab + N2 * kk) * CB + cl];
                    const C p1 = MODE != kApplyMass ? s1[(ab + N2 * kk) * CB + cl] : (C)0;
#pragma unroll
                    for (int kp = 0; kp < N; ++kp) {
                        if (MODE == kApplyMass) acc[q][kp] += sM[kp * N + k] * p2;
                        else acc[q][kp] += sM[kp * N + k] * p1 + g.cz * sK[kp * N + k] * p2;
                    }
                }
            }
            __syncthreads();
        }
        // store: z line (cell, ab) writes its N planes
        const S* __restrict__ rres = (MODE == kApplyResidual) ? static_cast<const S*>(pe.b) + base : nullptr;
#pragma unroll
        for (int q = 0; q < ZPT; ++q) {
            const int zl = tid + NT * q;
            if (zl >= ZL) break;
            const int ab = zl / CB;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const size_t off = (size_t)(ab + N2 * k) * kLanes + cl;
                C v = acc[q][k];
                if (MODE == kApplyMass) v *= g.vol;
                if (MODE == kApplyResidual) v = load_as<C>(rres + off) - v;
                if (!valid || on_boundary<P>(g, ab % N, ab / N, k)) v = (C)0;
                store_from(y + off, v);
            }
        }
    }
}

template <int P, typename S, int MODE, bool MULTI>
__global__ void __launch_bounds__((PlanesShape<P, typename Prec<S>::C>::NT))
k_apply_planes(LaunchTable L, RefMats<P, typename Prec<S>::C> R) {
    __shared__ __align__(16) char smem[PlanesShape<P, typename Prec<S>::C>::kLds];
    apply_planes_body<P, S, MODE, MULTI>(L, R, blockIdx.x, gridDim.x, smem);
}

// The matrix-core apply serves p = 7 in the Laplace and residual modes in
// FP64; with 4-byte values the plane-streamed kernel measured faster.
template <int P, int MODE, typename C> constexpr bool apply_mfma_default() {
    return P == 7 && MODE != kApplyMass && sizeof(C) == 8;
}

// ---------------------------------------------------------------------------
// Matrix-core apply for p = 7 (Laplace and residual modes).  Each 1D
// contraction of a cell is a dense 16x16 product on the MFMA units, one cell
// per wavefront, with the cell's 64 lines of a direction in four 16-line
// tiles (the B operand, from LDS) and the 1D matrices stacked into a 16-row
// A operand held in registers:
//   z: [Mz; Kz] (16 x 8) u                     -> A = Mz u, Bz = Kz u
//   y: [[My, 0], [cy Ky, cz My]] [A; Bz]        -> D = My A, C
//   x: [[Mx, cx Kx], [0, 0]] [C; D]             -> y (rows 0..7)
// so a cell takes 8 + 16 + 16 products, the cell's geometry entering only
// through the A operands.  Between passes the tiles go through the cell's
// LDS region (a 16-row matrix, rows padded to an odd stride) to the next
// direction's line order.  A workgroup stages 8 consecutive cells of a
// storage block (64-byte runs of every node in FP64) in LDS, each of its
// four wavefronts computes two of them, and the results leave through the
// same region as coalesced stores.
template <typename C> struct ApplyMfmaShape {
    static constexpr int CB = 8;                 // cells per workgroup tile
    static constexpr int KS = 65;                // row stride of the 16-row intermediates
    static constexpr int RG = 16 * KS + 24;      // per-cell region (8 mod 32: staged cells on distinct banks)
    static constexpr int kLds = CB * RG * (int)sizeof(C);
};

// node l of the cell's input / output (rows of 8 padded to 9)
__device__ __forceinline__ int mfma_node(int l) { return l + (l >> 3); }

template <int P, typename S, int MODE, bool MULTI>
__device__ __forceinline__ void apply_mfma_body(const LaunchTable& L, const RefMats<P, typename Prec<S>::C>& R,
                                                int item, int items, char* smem) {
    using C = typename Prec<S>::C;
    using M = Mfma<C>;
    static_assert(P == 7, "the matrix-core apply is written for 8 nodes per direction");
    constexpr int N = P + 1, NN = N * N * N;
    constexpr int CB = ApplyMfmaShape<C>::CB, KS = ApplyMfmaShape<C>::KS, RG = ApplyMfmaShape<C>::RG;
    static_assert(256 % CB == 0 && kLanes % CB == 0 && (NN * CB) % 256 == 0, "staging shape");
    constexpr int LPT = NN * CB / 256;               // staged values per thread
    C* reg = reinterpret_cast<C*>(smem);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = lane >> 4, col = lane & 15;
    // cell-independent A operands (lane: row col, k = 4 ks + g)
    C az[2], ayb[4], axb[4];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        const int k = 4 * ks + g;
        az[ks] = col < N ? R.M[col * N + k] : R.K[(col - N) * N + k];
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const int k = 4 * ks + g, kk = k % N;
        if (ks < 2) ayb[ks] = col < N ? R.M[col * N + kk] : R.K[(col - N) * N + kk];
        else ayb[ks] = col < N ? (C)0 : R.M[(col - N) * N + kk];
        axb[ks] = col < N ? (ks < 2 ? R.M[col * N + kk] : R.K[col * N + kk]) : (C)0;
    }
    // staging: thread tid moves cell scell's nodes l = l0 + 32 i (i < 16),
    // i.e. a = l0 % 8 (fixed), b = wv + 4 (i % 2), c = i / 2
    static_assert(CB == 8 && LPT == 16, "staging map");
    const int scell = tid % CB, l0 = tid / CB, sa = l0 % N;
    C pre[LPT];                                      // the next tile's staged values
    // boundary copies of the staged cell (Dirichlet), as masks over i
    auto stage_mask = [&](const ProbEntry& pe, int e) -> uint32_t {
        if (e >= pe.ncells) return 0xffffu;
        const CellGeom<C> gs = cell_geom<C>(pe, e);
        const bool xm = (sa == 0 && gs.xlo) || (sa == P && gs.xhi);
        uint32_t m = 0;
#pragma unroll
        for (int i = 0; i < LPT; ++i) {
            const int b = wv + 4 * (i % 2), c = i / 2;
            const bool bm = xm || (b == 0 && gs.ylo) || (b == P && gs.yhi) || (c == 0 && gs.zlo) || (c == P && gs.zhi);
            m |= (bm ? 1u : 0u) << i;
        }
        return m;
    };
    auto fetch = [&](int tile) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        const int blk = t / (kLanes / CB), lane0 = (t % (kLanes / CB)) * CB;
        const S* __restrict__ x = static_cast<const S*>(pe.a) + (size_t)blk * NN * kLanes + lane0 + scell +
                                  (size_t)l0 * kLanes;
        const uint32_t m = stage_mask(pe, blk * kLanes + lane0 + scell);
#pragma unroll
        for (int i = 0; i < LPT; ++i)
            pre[i] = ((m >> i) & 1u) ? (C)0 : load_as<C>(x + (size_t)(32 * i) * kLanes);
    };
    if (item < L.total_tiles) fetch(item);
    for (int tile = item; tile < L.total_tiles; tile += items) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        const int blk = t / (kLanes / CB), lane0 = (t % (kLanes / CB)) * CB;
        const size_t base = (size_t)blk * NN * kLanes + lane0;
        S* __restrict__ y = static_cast<S*>(pe.c) + base;
        const uint32_t smask = stage_mask(pe, blk * kLanes + lane0 + scell);
#pragma unroll
        for (int i = 0; i < LPT; ++i) reg[scell * RG + mfma_node(l0 + 32 * i)] = pre[i];
        __syncthreads();
        // the next tile's loads are in flight while this one computes
        if (tile + items < L.total_tiles) fetch(tile + items);
#pragma unroll 1
        for (int cc = wv; cc < CB; cc += 4) {
            const int e = blk * kLanes + lane0 + cc;
            if (e >= pe.ncells) continue;                // uniform over the wavefront
            const CellGeom<C> gc = cell_geom<C>(pe, e);
            C* rg = reg + cc * RG;
            typename M::V acc[4];
            // z: lines (a, b) = (col % 8, 2 t + col / 8), k = c
            {
                C bz[4][2];
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                    for (int ks = 0; ks < 2; ++ks) bz[tt][ks] = rg[mfma_node(col + 16 * tt + 64 * (4 * ks + g))];
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
                    acc[tt] = typename M::V{0, 0, 0, 0};
#pragma unroll
                    for (int ks = 0; ks < 2; ++ks) acc[tt] = M::mma(az[ks], bz[tt][ks], acc[tt]);
                }
                wave_sync();
                // row j < 8: A at c' = j, else Bz at c' = j - 8; stored as the y
                // pass's rows k = b (A) and 8 + b (Bz), lines (a, c')
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = M::row(lane, r), a = col % N, b = 2 * tt + col / N;
                        const int k = j < N ? b : N + b;
                        rg[k * KS + (j % N) * N + a] = acc[tt][r];
                    }
                wave_sync();
            }
            // y: lines (a, c') = (col % 8, 2 t + col / 8), k over [A; Bz]
            {
                C ay[4], by[4][4];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) ay[ks] = col < N ? ayb[ks] : ayb[ks] * (ks < 2 ? gc.cy : gc.cz);
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) by[tt][ks] = rg[(4 * ks + g) * KS + 16 * tt + col];
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
                    acc[tt] = typename M::V{0, 0, 0, 0};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) acc[tt] = M::mma(ay[ks], by[tt][ks], acc[tt]);
                }
                wave_sync();
                // row j < 8: D at b' = j, else C at b' = j - 8; stored as the x
                // pass's rows k = a (C) and 8 + a (D), lines (b', c')
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = M::row(lane, r), a = col % N, c = 2 * tt + col / N;
                        const int k = j < N ? N + a : a;
                        rg[k * KS + c * N + (j % N)] = acc[tt][r];
                    }
                wave_sync();
            }
            // x: lines (b', c') = (col % 8, 2 t + col / 8), k over [C; D]
            {
                C ax[4], bx[4][4];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) ax[ks] = ks < 2 ? axb[ks] : axb[ks] * gc.cx;
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) bx[tt][ks] = rg[(4 * ks + g) * KS + 16 * tt + col];
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
                    acc[tt] = typename M::V{0, 0, 0, 0};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) acc[tt] = M::mma(ax[ks], bx[tt][ks], acc[tt]);
                }
                wave_sync();
                // rows 0..7: y at a = j, node j + 8 b' + 64 c'
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = M::row(lane, r);
                        if (j < N) rg[mfma_node(j + N * (col % N) + N * N * (2 * tt + col / N))] = acc[tt][r];
                    }
            }
        }
        __syncthreads();
        // store: node l0 + 32 i of cell scell
        const S* __restrict__ rres = (MODE == kApplyResidual) ? static_cast<const S*>(pe.b) + base : nullptr;
#pragma unroll
        for (int i = 0; i < LPT; ++i) {
            const int l = l0 + 32 * i;
            const size_t off = (size_t)l * kLanes + scell;
            C v = reg[scell * RG + mfma_node(l)];
            if (MODE == kApplyResidual) v = load_as<C>(rres + off) - v;
            if ((smask >> i) & 1u) v = (C)0;
            store_from(y + off, v);
        }
        __syncthreads();
    }
}

template <int P, typename S, int MODE, bool MULTI>
__global__ void __launch_bounds__(256) k_apply_mfma(LaunchTable L, RefMats<P, typename Prec<S>::C> R) {
    __shared__ __align__(16) char smem[ApplyMfmaShape<typename Prec<S>::C>::kLds];
    apply_mfma_body<P, S, MODE, MULTI>(L, R, blockIdx.x, gridDim.x, smem);
}

template <int P> constexpr int lds_cells(int bytes) {
    // largest power of two <= 64 with two LDS arrays within 64 KiB
    int cb = 64;
    while (cb > 1 && 2 * cb * (P + 1) * (P + 1) * (P + 1) * bytes > 65536) cb >>= 1;
    return cb;
}

template <int P, typename S, int MODE>
static hipError_t launch_apply_t(ProbEntry* ents, int nprob, TableStager* d_tab, hipStream_t s,
                                 const LaunchCfg& cfg) {
    const int force_lds = cfg.apply_lds;
    const int gcap = cfg.grid_cap > 0 ? cfg.grid_cap : kMaxGrid;
    using C = typename Prec<S>::C;
    const RefMats<P, C> R = ref_mats<P, C>();
    const bool use_reg = (P <= 3) && !force_lds;
    // p = 7 (Laplace, residual): the matrix-core apply unless the plane-streamed
    // one is asked for (apply_lds = 2, or the process-wide option)
    const bool use_mfma = apply_mfma_default<P, MODE, C>() && !force_lds && g_apply_planes_p7 == 0;
    const bool use_planes = (P >= 4) && !use_mfma && (force_lds == 0 || force_lds == 2);
    constexpr int CB = lds_cells<P>((int)sizeof(C));
    constexpr int MCB = ApplyMfmaShape<C>::CB;
    LaunchTable L{};
    int tiles = 0;
    for (int i = 0; i < nprob; ++i) {
        ents[i].tile_begin = tiles;
        ents[i].ntiles = use_reg ? ents[i].nblk
                       : use_mfma ? ents[i].nblk * (kLanes / MCB)
                       : use_planes ? ents[i].nblk * (kLanes / 16) : ents[i].nblk * (kLanes / CB);
        tiles += ents[i].ntiles;
    }
    L.nprob = nprob;
    L.total_tiles = tiles;
    if (tiles == 0) return hipSuccess;
    hipError_t err = stage_table(L, ents, nprob, d_tab, s);
    if (err != hipSuccess) return err;
    TraceSpan ts(MODE == kApplyLaplace ? "apply" : MODE == kApplyResidual ? "apply_residual" : "mass_apply", P,
                 Prec<S>::id, s);
    if constexpr (P <= 3) {
        if (use_reg) {
            const int grid = (tiles + 3) / 4 < gcap ? (tiles + 3) / 4 : gcap;
            if (nprob > 1) hipLaunchKernelGGL((k_apply_reg<P, S, MODE, true>), dim3(grid), dim3(256), 0, s, L, R);
            else hipLaunchKernelGGL((k_apply_reg<P, S, MODE, false>), dim3(grid), dim3(256), 0, s, L, R);
            return hipGetLastError();
        }
    }
    if constexpr (apply_mfma_default<P, MODE, C>()) {
        if (use_mfma) {
            const int grid = tiles < gcap ? tiles : gcap;
            if (nprob > 1) hipLaunchKernelGGL((k_apply_mfma<P, S, MODE, true>), dim3(grid), dim3(256), 0, s, L, R);
            else hipLaunchKernelGGL((k_apply_mfma<P, S, MODE, false>), dim3(grid), dim3(256), 0, s, L, R);
            return hipGetLastError();
        }
    }
    if constexpr (P >= 4) {
        if (use_planes) {
            const int grid = tiles < gcap ? tiles : gcap;
            constexpr int NT = PlanesShape<P, C>::NT;
            if (nprob > 1) hipLaunchKernelGGL((k_apply_planes<P, S, MODE, true>), dim3(grid), dim3(NT), 0, s, L, R);
            else hipLaunchKernelGGL((k_apply_planes<P, S, MODE, false>), dim3(grid), dim3(NT), 0, s, L, R);
            return hipGetLastError();
        }
    }
    {
        const int grid = tiles < gcap ? tiles : gcap;
        if (nprob > 1) hipLaunchKernelGGL((k_apply_lds<P, S, MODE, CB, true>), dim3(grid), dim3(256), 0, s, L, R);
        else hipLaunchKernelGGL((k_apply_lds<P, S, MODE, CB, false>), dim3(grid), dim3(256), 0, s, L, R);
    }
    return hipGetLastError();
}

template <int P, typename S>
static hipError_t launch_apply_m(int mode, ProbEntry* e, int n, TableStager* t, hipStream_t s, const LaunchCfg& fl) {
    switch (mode) {
        case kApplyLaplace: return launch_apply_t<P, S, kApplyLaplace>(e, n, t, s, fl);
        case kApplyResidual: return launch_apply_t<P, S, kApplyResidual>(e, n, t, s, fl);
        default: return launch_apply_t<P, S, kApplyMass>(e, n, t, s, fl);
    }
}

template <int P>
static hipError_t launch_apply_p(int prec, int mode, ProbEntry* e, int n, TableStager* t, hipStream_t s, const LaunchCfg& fl) {
    switch (prec) {
        case FEM_F64: return launch_apply_m<P, double>(mode, e, n, t, s, fl);
        case FEM_F32: return launch_apply_m<P, float>(mode, e, n, t, s, fl);
        case FEM_F16: return launch_apply_m<P, f16_t>(mode, e, n, t, s, fl);
        default: return launch_apply_m<P, bf16_t>(mode, e, n, t, s, fl);
    }
}

// ---------------------------------------------------------------------------
// Mixed-degree apply: the register body for p = 2, 3 (four storage blocks
// per item, one per wavefront) and the plane-streamed body for p = 7 (16
// cells per item), in one persistent launch.
// (p = 7 takes the plane-streamed body: the mixed launch serves 4-byte
// values only when p = 7 is present, see launch_apply_any, and the
// matrix-core body's accumulator registers would bound the whole launch)
template <int P, typename S, int MODE>
struct ApplyBody {
    using C = typename Prec<S>::C;
    using Arg = RefMats<P, C>;
    static constexpr int kLds = P <= 3 ? 0 : PlanesShape<P, C>::kLds;
    __device__ static __forceinline__ void run(const LaunchTable& L, const Arg& R, int item, int items, char* smem) {
        if constexpr (P <= 3) apply_reg_body<P, S, MODE, true>(L, R, item, items);
        else apply_planes_body<P, S, MODE, true>(L, R, item, items, smem);
    }
};

template <typename S, int MODE>
static hipError_t launch_apply_mixed_t(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    using C = typename Prec<S>::C;
    static_assert(mix_degree(0) == 7 && mix_degree(1) == 3 && mix_degree(2) == 2, "segment degrees");
    MixTable T{};
    int grid = 0;
    auto tiles = [](int p, const ProbEntry& e) { return p <= 3 ? e.nblk : e.nblk * (kLanes / 16); };
    auto items = [](int p, int t) { return p <= 3 ? (t + 3) / 4 : t; };
    hipError_t err = mix_build(ents, nprob, st, s, tiles, items, T, grid);
    if (err != hipSuccess || grid == 0) return err;
    TraceSpan ts(MODE == kApplyLaplace ? "apply" : MODE == kApplyResidual ? "apply_residual" : "mass_apply", 0,
                 Prec<S>::id, s);
    hipLaunchKernelGGL((k_mixed<ApplyBody<7, S, MODE>, ApplyBody<3, S, MODE>, ApplyBody<2, S, MODE>>), dim3(grid),
                       dim3(256), 0, s, T, ref_mats<7, C>(), ref_mats<3, C>(), ref_mats<2, C>());
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_apply_mixed_m(int mode, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    switch (mode) {
        case kApplyLaplace: return launch_apply_mixed_t<S, kApplyLaplace>(ents, nprob, st, s);
        case kApplyResidual: return launch_apply_mixed_t<S, kApplyResidual>(ents, nprob, st, s);
        default: return launch_apply_mixed_t<S, kApplyMass>(ents, nprob, st, s);
    }
}

hipError_t launch_apply_any(int prec, int mode, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s,
                            bool mix) {
    if (nprob <= 0) return hipSuccess;
    // the mixed p = 7 body is the plane-streamed one, the default for 4-byte
    // values and the mass apply; FP64 Laplace and residual applies with p = 7
    // present take one launch per degree (p = 7 on the matrix cores)
    bool p7_mfma = false;
    for (int i = 0; i < nprob; ++i) p7_mfma = p7_mfma || (ents[i].p == 7 && prec == FEM_F64 && mode != kApplyMass);
    if (mix && mix_degrees(ents, nprob) >= 2 && (!p7_mfma || g_apply_planes_p7 != 0)) {
        switch (prec) {
            case FEM_F64: return launch_apply_mixed_m<double>(mode, ents, nprob, st, s);
            case FEM_F32: return launch_apply_mixed_m<float>(mode, ents, nprob, st, s);
            case FEM_F16: return launch_apply_mixed_m<f16_t>(mode, ents, nprob, st, s);
            default: return launch_apply_mixed_m<bf16_t>(mode, ents, nprob, st, s);
        }
    }
    std::vector<ProbEntry> g;
    for (int p = 1; p <= kMaxP; ++p) {
        g.clear();
        for (int i = 0; i < nprob; ++i)
            if (ents[i].p == p) g.push_back(ents[i]);
        if (g.empty()) continue;
        hipError_t err = launch_apply(p, prec, mode, g.data(), (int)g.size(), st, s);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_apply(int p, int prec, int mode, ProbEntry* ents, int nprob, TableStager* d_tab,
                        hipStream_t s, const LaunchCfg& force_lds) {
    switch (p) {
        case 1: return launch_apply_p<1>(prec, mode, ents, nprob, d_tab, s, force_lds);
        case 2: return launch_apply_p<2>(prec, mode, ents, nprob, d_tab, s, force_lds);
        case 3: return launch_apply_p<3>(prec, mode, ents, nprob, d_tab, s, force_lds);
        case 4: return launch_apply_p<4>(prec, mode, ents, nprob, d_tab, s, force_lds);
        case 5: return launch_apply_p<5>(prec, mode, ents, nprob, d_tab, s, force_lds);
        case 6: return launch_apply_p<6>(prec, mode, ents, nprob, d_tab, s, force_lds);
        case 7: return launch_apply_p<7>(prec, mode, ents, nprob, d_tab, s, force_lds);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fem
