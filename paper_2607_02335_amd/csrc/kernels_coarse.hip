// Coarse level of the two-level preconditioner: the trilinear (Q1)
// functions on the interior vertices of the same mesh, solved exactly by
// fast diagonalisation in FP64.
//
// Transfers, per cell K with local nodes (a, b, c) at reference coordinates
// (xi_a, xi_b, xi_c) (the GLL nodes) and 1D hats h0(xi) = 1 - xi,
// h1(xi) = xi:
//   restriction   c_v = sum_K sum_(a,b,c) t_K(a,b,c) h_sx(xi_a) h_sy(xi_b) h_sz(xi_c)
//                 over the cells K having v as corner (sx, sy, sz): the Q1 basis
//                 functions tested against the dual residual, which depends on
//                 t only through its assembly G^T t;
//   prolongation  z_K(a,b,c) += sum_corners e_v h_sx(xi_a) h_sy(xi_b) h_sz(xi_c)
//                 (trilinear interpolation; boundary vertices carry 0).
// The coarse operator of the nested spaces is the Q1 Laplacian of the mesh,
// a Kronecker sum of 1D matrices, so A_0^{-1} = (Sx (x) Sy (x) Sz)
// diag(1/(lx + ly + lz)) (Sx (x) Sy (x) Sz)^T with the 1D generalised
// eigenvectors S (S^T M S = I) of the interior vertices.
#include <mutex>
#include <vector>

#include "fem_internal.h"
#include "host_api.h"
#include "launch.h"
#include "mixed.h"
#include "trace.h"

namespace fem {

// The GLL nodes of each degree, computed once per process.
static const std::vector<double>& gll_cached(int p) {
    static std::once_flag once[kMaxP + 1];
    static std::vector<double> nodes[kMaxP + 1];
    std::call_once(once[p], [p]() { nodes[p] = host_gll_nodes(p); });
    return nodes[p];
}

struct GllNodes {
    double xi[kMaxP + 1];
};

// Operands of every coarse kernel, per problem entry: a = t (dual, the
// storage precision S), c = z (primal, S), d = corner sums
// ([8][nblk * 64] doubles), e = two coarse vectors (2 x (n0-1)(n1-1)(n2-1)
// doubles), fd[0..2] = per direction the coarse S ((n-1) x (n-1)) followed by
// lambda (n-1).  Tiles are 256 cells (restriction and prolongation) or 256
// coarse values (vertex sums and solve passes) of one problem.
__device__ __forceinline__ int coarse_m(const ProbEntry& pe, int d) { return pe.n[d] > 1 ? pe.n[d] - 1 : 0; }

// Cell -> its 8 corner sums, one thread per cell (lanes on the cells of a
// storage block, so every load is a contiguous run); sums in FP64, streamed
// over the z node planes.  corner[(sx + 2 sy + 4 sz) * nblk * 64 + e].
template <int P, typename S, bool MULTI>
__device__ __forceinline__ void restrict_cells_body(const LaunchTable& L, const GllNodes& g, int item, int items) {
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    const int tile = item;
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int stride = pe.nblk * kLanes;
    const int e = (tile - pe.tile_begin) * 256 + threadIdx.x;
    if (e >= stride) return;
    double out[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) out[i] = 0.0;
    if (e < pe.ncells) {
        const S* v = static_cast<const S*>(pe.a) + (size_t)(e / kLanes) * NN * kLanes + (e % kLanes);
        for (int c = 0; c < N; ++c) {
            double ux[2][N];
#pragma unroll
            for (int b = 0; b < N; ++b) {
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    const double x = load_as<double>(v + (size_t)(a + N * b + N2 * c) * kLanes);
                    s0 += x * (1.0 - g.xi[a]);
                    s1 += x * g.xi[a];
                }
                ux[0][b] = s0;
                ux[1][b] = s1;
            }
            const double wz[2] = {1.0 - g.xi[c], g.xi[c]};
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
                double y0 = 0.0, y1 = 0.0;
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    y0 += ux[sx][b] * (1.0 - g.xi[b]);
                    y1 += ux[sx][b] * g.xi[b];
                }
#pragma unroll
                for (int sz = 0; sz < 2; ++sz) {
                    out[sx + 4 * sz] += y0 * wz[sz];
                    out[sx + 2 + 4 * sz] += y1 * wz[sz];
                }
            }
        }
    }
    double* corner = static_cast<double*>(pe.d);
#pragma unroll
    for (int i = 0; i < 8; ++i) corner[(size_t)i * stride + e] = out[i];
}

template <int P, typename S, bool MULTI>
__global__ void __launch_bounds__(256) k_restrict_cells(LaunchTable L, GllNodes g) {
    restrict_cells_body<P, S, MULTI>(L, g, blockIdx.x, gridDim.x);
}

// Corner sums -> coarse right-hand side at the interior vertices (the first
// coarse vector), one thread per vertex, the eight cells added in ascending
// cell order.
template <bool MULTI>
__global__ void __launch_bounds__(256) k_restrict_vertices(LaunchTable L) {
    const int tile = blockIdx.x;
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int m0 = coarse_m(pe, 0), m1 = coarse_m(pe, 1), m2 = coarse_m(pe, 2);
    const long v = (long)(tile - pe.tile_begin) * 256 + threadIdx.x;
    if (v >= (long)m0 * m1 * m2) return;
    const int vi = 1 + (int)(v % m0), vj = 1 + (int)((v / m0) % m1), vk = 1 + (int)(v / ((long)m0 * m1));
    const int n0 = pe.n[0], n1 = pe.n[1];
    const int stride = pe.nblk * kLanes;
    const double* corner = static_cast<const double*>(pe.d);
    double s = 0.0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                // cell (vi-1+dx, ...) has this vertex as its corner (1-dx, 1-dy, 1-dz)
                const int e = (vi - 1 + dx) + n0 * ((vj - 1 + dy) + n1 * (vk - 1 + dz));
                s += corner[(size_t)((1 - dx) + 2 * (1 - dy) + 4 * (1 - dz)) * stride + e];
            }
    static_cast<double*>(pe.e)[v] = s;
}

// One 1D pass of the coarse fast-diagonalisation solve along `axis` (0 = x)
// from coarse vector `src` (0 or 1) to the other: forward (fwd = 1)
// out(j) = sum_i S(i, j) x(i) (S^T), backward out(i) = sum_j S(i, j) x(j).
// With `scale` the result is divided by lx + ly + lz (the last forward pass).
template <bool MULTI>
__global__ void __launch_bounds__(256) k_coarse_pass(LaunchTable L, int axis, int fwd, int src_half, int scale) {
    const int tile = blockIdx.x;
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int m0 = coarse_m(pe, 0), m1 = coarse_m(pe, 1), m2 = coarse_m(pe, 2);
    const long tot = (long)m0 * m1 * m2;
    const long id = (long)(tile - pe.tile_begin) * 256 + threadIdx.x;
    if (id >= tot) return;
    const int i0 = (int)(id % m0), i1 = (int)((id / m0) % m1), i2 = (int)(id / ((long)m0 * m1));
    const int m = axis == 0 ? m0 : axis == 1 ? m1 : m2;
    const int o = axis == 0 ? i0 : axis == 1 ? i1 : i2;
    const long stride = axis == 0 ? 1 : axis == 1 ? m0 : (long)m0 * m1;
    double* cv = static_cast<double*>(pe.e);
    const double* x = cv + (src_half ? tot : 0) + (id - (long)o * stride);
    double* dst = cv + (src_half ? 0 : tot);
    const double* Sd = static_cast<const double*>(pe.fd[axis]);
    double s = 0.0;
    if (fwd) {
        for (int i = 0; i < m; ++i) s += Sd[(size_t)i * m + o] * x[(long)i * stride];
    } else {
        for (int j = 0; j < m; ++j) s += Sd[(size_t)o * m + j] * x[(long)j * stride];
    }
    if (scale) {
        const double* lx = static_cast<const double*>(pe.fd[0]) + (size_t)m0 * m0;
        const double* ly = static_cast<const double*>(pe.fd[1]) + (size_t)m1 * m1;
        const double* lz = static_cast<const double*>(pe.fd[2]) + (size_t)m2 * m2;
        s /= lx[i0] + ly[i1] + lz[i2];
    }
    dst[id] = s;
}

// z += P_0 e: trilinear interpolation of the coarse correction (the first
// coarse vector) at the cell nodes, one thread per cell.  Only corners with
// a nonzero weight at a node are summed, in (sz, sy, sx) order, so the
// copies of a node shared by several cells add the same terms in the same
// order (bitwise continuous).
template <int P, typename S, bool MULTI>
__device__ __forceinline__ void prolong_add_body(const LaunchTable& L, const GllNodes& g, int item, int items) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    const int tile = item;
    if (tile >= L.total_tiles) return;
    const ProbEntry& pe = entry<MULTI>(L, tile);
    const int e = (tile - pe.tile_begin) * 256 + threadIdx.x;
    if (e >= pe.ncells) return;
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int m0 = coarse_m(pe, 0), m1 = coarse_m(pe, 1);
    const int i = e % n0, j = (e / n0) % n1, k = e / (n0 * n1);
    const double* ev = static_cast<const double*>(pe.e);
    double cv[8];
#pragma unroll
    for (int sz = 0; sz < 2; ++sz)
#pragma unroll
        for (int sy = 0; sy < 2; ++sy)
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
                const int vi = i + sx, vj = j + sy, vk = k + sz;
                const bool in = vi >= 1 && vi <= n0 - 1 && vj >= 1 && vj <= n1 - 1 && vk >= 1 && vk <= n2 - 1;
                cv[sx + 2 * sy + 4 * sz] = in ? ev[(vi - 1) + (long)m0 * ((vj - 1) + (long)m1 * (vk - 1))] : 0.0;
            }
    S* out = static_cast<S*>(pe.c) + (size_t)(e / kLanes) * NN * kLanes + (e % kLanes);
    for (int c = 0; c < N; ++c) {
        const double wz[2] = {1.0 - g.xi[c], g.xi[c]};
        for (int b = 0; b < N; ++b) {
            const double wy[2] = {1.0 - g.xi[b], g.xi[b]};
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const double wx[2] = {1.0 - g.xi[a], g.xi[a]};
                double s = 0.0;
#pragma unroll
                for (int sz = 0; sz < 2; ++sz) {
                    if (wz[sz] == 0.0) continue;
#pragma unroll
                    for (int sy = 0; sy < 2; ++sy) {
                        if (wy[sy] == 0.0) continue;
#pragma unroll
                        for (int sx = 0; sx < 2; ++sx) {
                            if (wx[sx] == 0.0) continue;
                            s += cv[sx + 2 * sy + 4 * sz] * (wx[sx] * wy[sy] * wz[sz]);
                        }
                    }
                }
                S* dst = out + (size_t)(a + N * b + N2 * c) * kLanes;
                store_from(dst, (C)(load_as<double>(dst) + s));
            }
        }
    }
}

template <int P, typename S, bool MULTI>
__global__ void __launch_bounds__(256) k_prolong_add(LaunchTable L, GllNodes g) {
    prolong_add_body<P, S, MULTI>(L, g, blockIdx.x, gridDim.x);
}

template <typename F>
static hipError_t by_prec(int prec, F&& f) {
    switch (prec) {
        case FEM_F64: return f(double{});
        case FEM_F32: return f(float{});
        case FEM_F16: return f(f16_t{});
        default: return f(bf16_t{});
    }
}

// Tiles of the cell kernels (256 cells each); a problem without interior
// vertices has no coarse space and takes no correction.
static int coarse_cell_tiles(const ProbEntry& e) {
    const bool any = e.n[0] > 1 && e.n[1] > 1 && e.n[2] > 1;
    return any ? (e.nblk * kLanes + 255) / 256 : 0;
}

template <int P>
static hipError_t coarse_p(int prec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    GllNodes g{};
    const std::vector<double>& xi = gll_cached(P);
    for (int a = 0; a <= P; ++a) g.xi[a] = xi[a];
    const bool multi = nprob > 1;
    // cell-based tables (restriction, prolongation)
    LaunchTable Lc{};
    int tc = 0;
    for (int i = 0; i < nprob; ++i) {
        ents[i].tile_begin = tc;
        ents[i].ntiles = coarse_cell_tiles(ents[i]);
        tc += ents[i].ntiles;
    }
    Lc.nprob = nprob;
    Lc.total_tiles = tc;
    hipError_t err = stage_table(Lc, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    // coarse-value tables (vertex sums, solve passes)
    LaunchTable Lv{};
    int tv = 0;
    for (int i = 0; i < nprob; ++i) {
        long nv = 1;
        for (int d = 0; d < 3; ++d) nv *= ents[i].n[d] > 1 ? ents[i].n[d] - 1 : 0;
        ents[i].tile_begin = tv;
        ents[i].ntiles = (int)((nv + 255) / 256);
        tv += ents[i].ntiles;
    }
    Lv.nprob = nprob;
    Lv.total_tiles = tv;
    if (tv == 0) return hipSuccess;                 // no interior vertex anywhere: no coarse space
    err = stage_table(Lv, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    return by_prec(prec, [&](auto tag) {
        using S = decltype(tag);
        TraceSpan ts("coarse_correction", P, Prec<S>::id, s);
        if (multi) hipLaunchKernelGGL((k_restrict_cells<P, S, true>), dim3(tc), dim3(256), 0, s, Lc, g);
        else hipLaunchKernelGGL((k_restrict_cells<P, S, false>), dim3(tc), dim3(256), 0, s, Lc, g);
        if (multi) hipLaunchKernelGGL(k_restrict_vertices<true>, dim3(tv), dim3(256), 0, s, Lv);
        else hipLaunchKernelGGL(k_restrict_vertices<false>, dim3(tv), dim3(256), 0, s, Lv);
        // x, y, z forward (then the eigenvalue scaling), z, y, x backward;
        // vector 0 -> 1 -> 0 -> 1 -> 0 -> 1 -> 0
        const int axis[6] = {0, 1, 2, 2, 1, 0}, fwd[6] = {1, 1, 1, 0, 0, 0};
        for (int k = 0; k < 6; ++k) {
            if (multi) hipLaunchKernelGGL(k_coarse_pass<true>, dim3(tv), dim3(256), 0, s, Lv, axis[k], fwd[k], k % 2, k == 2 ? 1 : 0);
            else hipLaunchKernelGGL(k_coarse_pass<false>, dim3(tv), dim3(256), 0, s, Lv, axis[k], fwd[k], k % 2, k == 2 ? 1 : 0);
        }
        if (multi) hipLaunchKernelGGL((k_prolong_add<P, S, true>), dim3(tc), dim3(256), 0, s, Lc, g);
        else hipLaunchKernelGGL((k_prolong_add<P, S, false>), dim3(tc), dim3(256), 0, s, Lc, g);
        return hipGetLastError();
    });
}

// Mixed-degree coarse correction: restriction and prolongation as mixed
// launches (cell tiles of the degrees 7, 3, 2), the vertex sums and the six
// solve passes (the same for every degree) over all problems at once.
template <int P, typename S>
struct RestrictBody {
    using Arg = GllNodes;
    static constexpr int kLds = 0;
    __device__ static __forceinline__ void run(const LaunchTable& L, const GllNodes& g, int item, int items, char*) {
        restrict_cells_body<P, S, true>(L, g, item, items);
    }
};

template <int P, typename S>
struct ProlongBody {
    using Arg = GllNodes;
    static constexpr int kLds = 0;
    __device__ static __forceinline__ void run(const LaunchTable& L, const GllNodes& g, int item, int items, char*) {
        prolong_add_body<P, S, true>(L, g, item, items);
    }
};

static GllNodes gll_arg(int p) {
    GllNodes g{};
    const std::vector<double>& xi = gll_cached(p);
    for (int a = 0; a <= p; ++a) g.xi[a] = xi[a];
    return g;
}

static hipError_t coarse_mixed(int prec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    static_assert(mix_degree(0) == 7 && mix_degree(1) == 3 && mix_degree(2) == 2, "segment degrees");
    // coarse-value tables (vertex sums, solve passes) over all problems
    LaunchTable Lv{};
    int tv = 0;
    for (int i = 0; i < nprob; ++i) {
        long nv = 1;
        for (int d = 0; d < 3; ++d) nv *= ents[i].n[d] > 1 ? ents[i].n[d] - 1 : 0;
        ents[i].tile_begin = tv;
        ents[i].ntiles = (int)((nv + 255) / 256);
        tv += ents[i].ntiles;
    }
    Lv.nprob = nprob;
    Lv.total_tiles = tv;
    if (tv == 0) return hipSuccess;                 // no interior vertex anywhere: no coarse space
    hipError_t err = stage_table(Lv, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    MixTable T{};
    int grid = 0;
    auto tiles = [](int, const ProbEntry& e) { return coarse_cell_tiles(e); };
    auto items = [](int, int t) { return t; };
    err = mix_build(ents, nprob, st, s, tiles, items, T, grid);
    if (err != hipSuccess) return err;
    const GllNodes g7 = gll_arg(7), g3 = gll_arg(3), g2 = gll_arg(2);
    const bool multi = nprob > 1;
    return by_prec(prec, [&](auto tag) {
        using S = decltype(tag);
        TraceSpan ts("coarse_correction", 0, Prec<S>::id, s);
        if (grid > 0)
            hipLaunchKernelGGL((k_mixed<RestrictBody<7, S>, RestrictBody<3, S>, RestrictBody<2, S>>), dim3(grid),
                               dim3(256), 0, s, T, g7, g3, g2);
        if (multi) hipLaunchKernelGGL(k_restrict_vertices<true>, dim3(tv), dim3(256), 0, s, Lv);
        else hipLaunchKernelGGL(k_restrict_vertices<false>, dim3(tv), dim3(256), 0, s, Lv);
        const int axis[6] = {0, 1, 2, 2, 1, 0}, fwd[6] = {1, 1, 1, 0, 0, 0};
        for (int k = 0; k < 6; ++k) {
            if (multi) hipLaunchKernelGGL(k_coarse_pass<true>, dim3(tv), dim3(256), 0, s, Lv, axis[k], fwd[k], k % 2, k == 2 ? 1 : 0);
            else hipLaunchKernelGGL(k_coarse_pass<false>, dim3(tv), dim3(256), 0, s, Lv, axis[k], fwd[k], k % 2, k == 2 ? 1 : 0);
        }
        if (grid > 0)
            hipLaunchKernelGGL((k_mixed<ProlongBody<7, S>, ProlongBody<3, S>, ProlongBody<2, S>>), dim3(grid),
                               dim3(256), 0, s, T, g7, g3, g2);
        return hipGetLastError();
    });
}

hipError_t launch_coarse_any(int prec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, bool mix) {
    if (nprob <= 0) return hipSuccess;
    if (mix && mix_degrees(ents, nprob) >= 2) return coarse_mixed(prec, ents, nprob, st, s);
    std::vector<ProbEntry> g;
    for (int p = 1; p <= kMaxP; ++p) {
        g.clear();
        for (int i = 0; i < nprob; ++i)
            if (ents[i].p == p) g.push_back(ents[i]);
        if (g.empty()) continue;
        hipError_t err = launch_coarse_correction(p, prec, g.data(), (int)g.size(), st, s);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

// Entry of a problem for the coarse kernels: a = t, c = z.
ProbEntry coarse_entry(fem_problem* P, const void* t, void* z) {
    ProbEntry e = entry_of(P);
    e.a = t;
    e.c = z;
    e.d = P->d_corner;
    e.e = P->d_cvec;
    for (int k = 0; k < 3; ++k) e.fd[k] = P->d_cfd + P->cfd_off[k];
    return e;
}

hipError_t launch_coarse_correction(int p, int prec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    switch (p) {
        case 1: return coarse_p<1>(prec, ents, nprob, st, s);
        case 2: return coarse_p<2>(prec, ents, nprob, st, s);
        case 3: return coarse_p<3>(prec, ents, nprob, st, s);
        case 4: return coarse_p<4>(prec, ents, nprob, st, s);
        case 5: return coarse_p<5>(prec, ents, nprob, st, s);
        case 6: return coarse_p<6>(prec, ents, nprob, st, s);
        case 7: return coarse_p<7>(prec, ents, nprob, st, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t run_coarse_correction(fem_problem* P, const void* t, void* z, int prec) {
    ProbEntry e = coarse_entry(P, t, z);
    return launch_coarse_correction(P->p, prec, &e, 1, nullptr, P->stream);
}

}  // namespace fem
