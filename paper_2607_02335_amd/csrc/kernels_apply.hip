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
#include "fem_internal.h"
#include "launch.h"
#include "mixed.h"
#include "trace.h"

namespace fem {

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
    const bool use_planes = (P >= 4) && !force_lds;
    constexpr int CB = lds_cells<P>((int)sizeof(C));
    LaunchTable L{};
    int tiles = 0;
    for (int i = 0; i < nprob; ++i) {
        ents[i].tile_begin = tiles;
        ents[i].ntiles = use_reg ? ents[i].nblk : use_planes ? ents[i].nblk * (kLanes / 16) : ents[i].nblk * (kLanes / CB);
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
        default: return launch_apply_m<P, bf16_t>(mode, e, n, t, s, fl);
    }
}

// ---------------------------------------------------------------------------
// Mixed-degree apply: the register body for p = 2, 3 (four storage blocks
// per item, one per wavefront) and the plane-streamed body for p = 7 (16
// cells per item), in one persistent launch.
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
    if (mix && mix_degrees(ents, nprob) >= 2) {
        switch (prec) {
            case FEM_F64: return launch_apply_mixed_m<double>(mode, ents, nprob, st, s);
            case FEM_F32: return launch_apply_mixed_m<float>(mode, ents, nprob, st, s);
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
