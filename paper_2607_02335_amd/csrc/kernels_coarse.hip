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

// Cell -> its 8 corner sums, one thread per cell (lanes on the cells of a
// storage block, so every load is a contiguous run); sums in FP64, streamed
// over the z node planes.  corner[(sx + 2 sy + 4 sz) * stride + e].
template <int P, typename S>
__global__ void __launch_bounds__(256) k_restrict_cells(ProbEntry pe, const S* __restrict__ t,
                                                        double* __restrict__ corner, int stride, GllNodes g) {
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= stride) return;
    double out[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) out[i] = 0.0;
    if (e < pe.ncells) {
        const S* v = t + (size_t)(e / kLanes) * NN * kLanes + (e % kLanes);
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
#pragma unroll
    for (int i = 0; i < 8; ++i) corner[(size_t)i * stride + e] = out[i];
}

// Corner sums -> coarse right-hand side at the interior vertices, one thread
// per vertex, the (up to) eight cells added in ascending cell order.
__global__ void __launch_bounds__(256) k_restrict_vertices(ProbEntry pe, const double* __restrict__ corner, int stride,
                                                           double* __restrict__ c, int m0, int m1, int m2) {
    const long v = (long)blockIdx.x * 256 + threadIdx.x;
    if (v >= (long)m0 * m1 * m2) return;
    const int vi = 1 + (int)(v % m0), vj = 1 + (int)((v / m0) % m1), vk = 1 + (int)(v / ((long)m0 * m1));
    const int n0 = pe.n[0], n1 = pe.n[1];
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
    c[v] = s;
}

// One 1D pass of the coarse fast-diagonalisation solve along `axis` (0 = x):
// forward (fwd = 1) out(j) = sum_i S(i, j) x(i) (S^T), backward out(i) =
// sum_j S(i, j) x(j).  With `scale`, the forward result is divided by
// lx + ly + lz (the last forward pass).
__global__ void __launch_bounds__(256) k_coarse_pass(const double* __restrict__ src, double* __restrict__ dst,
                                                     const double* __restrict__ Sd, int m0, int m1, int m2,
                                                     int axis, int fwd, const double* __restrict__ lx,
                                                     const double* __restrict__ ly, const double* __restrict__ lz) {
    const long id = (long)blockIdx.x * 256 + threadIdx.x;
    const long tot = (long)m0 * m1 * m2;
    if (id >= tot) return;
    const int i0 = (int)(id % m0), i1 = (int)((id / m0) % m1), i2 = (int)(id / ((long)m0 * m1));
    const int m = axis == 0 ? m0 : axis == 1 ? m1 : m2;
    const int o = axis == 0 ? i0 : axis == 1 ? i1 : i2;
    const long stride = axis == 0 ? 1 : axis == 1 ? m0 : (long)m0 * m1;
    const double* x = src + (id - (long)o * stride);
    double s = 0.0;
    if (fwd) {
        for (int i = 0; i < m; ++i) s += Sd[(size_t)i * m + o] * x[(long)i * stride];
    } else {
        for (int j = 0; j < m; ++j) s += Sd[(size_t)o * m + j] * x[(long)j * stride];
    }
    if (lx) s /= lx[i0] + ly[i1] + lz[i2];
    dst[id] = s;
}

// z += P_0 e: trilinear interpolation of the coarse correction at the cell
// nodes, one thread per cell.  Only corners with a nonzero weight at a node
// are summed, in (sz, sy, sx) order, so the copies of a node shared by
// several cells add the same terms in the same order (bitwise continuous).
template <int P, typename S>
__global__ void __launch_bounds__(256) k_prolong_add(ProbEntry pe, const double* __restrict__ ev, S* __restrict__ z,
                                                     int m0, int m1, GllNodes g) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= pe.ncells) return;
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const int i = e % n0, j = (e / n0) % n1, k = e / (n0 * n1);
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
    S* out = z + (size_t)(e / kLanes) * NN * kLanes + (e % kLanes);
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

template <typename F>
static hipError_t by_prec(int prec, F&& f) {
    switch (prec) {
        case FEM_F64: return f(double{});
        case FEM_F32: return f(float{});
        default: return f(bf16_t{});
    }
}

template <int P>
static hipError_t coarse_transfers_p(fem_problem* P_, int prec, const void* t, void* z, bool restrict_, GllNodes g) {
    const ProbEntry pe = entry_of(P_);
    const int stride = P_->nblk * kLanes;
    hipStream_t s = P_->stream;
    return by_prec(prec, [&](auto tag) {
        using S = decltype(tag);
        if (restrict_) {
            TraceSpan ts("coarse_restrict", P, Prec<S>::id, s);
            hipLaunchKernelGGL((k_restrict_cells<P, S>), dim3((stride + 255) / 256), dim3(256), 0, s, pe,
                               static_cast<const S*>(t), P_->d_corner, stride, g);
            const long nv = (long)P_->cm[0] * P_->cm[1] * P_->cm[2];
            hipLaunchKernelGGL(k_restrict_vertices, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, pe,
                               P_->d_corner, stride, P_->d_cvec, P_->cm[0], P_->cm[1], P_->cm[2]);
        } else {
            TraceSpan ts("coarse_prolong", P, Prec<S>::id, s);
            hipLaunchKernelGGL((k_prolong_add<P, S>), dim3((P_->ncells + 255) / 256), dim3(256), 0, s, pe,
                               P_->d_cvec, static_cast<S*>(z), P_->cm[0], P_->cm[1], g);
        }
        return hipGetLastError();
    });
}

static hipError_t coarse_transfers(fem_problem* P, int prec, const void* t, void* z, bool restrict_) {
    GllNodes g{};
    const std::vector<double>& xi = gll_cached(P->p);
    for (int a = 0; a <= P->p; ++a) g.xi[a] = xi[a];
    switch (P->p) {
        case 1: return coarse_transfers_p<1>(P, prec, t, z, restrict_, g);
        case 2: return coarse_transfers_p<2>(P, prec, t, z, restrict_, g);
        case 3: return coarse_transfers_p<3>(P, prec, t, z, restrict_, g);
        case 4: return coarse_transfers_p<4>(P, prec, t, z, restrict_, g);
        case 5: return coarse_transfers_p<5>(P, prec, t, z, restrict_, g);
        case 6: return coarse_transfers_p<6>(P, prec, t, z, restrict_, g);
        case 7: return coarse_transfers_p<7>(P, prec, t, z, restrict_, g);
        default: return hipErrorInvalidValue;
    }
}

hipError_t run_coarse_correction(fem_problem* P, const void* t, void* z, int prec) {
    const int m0 = P->cm[0], m1 = P->cm[1], m2 = P->cm[2];
    const long nv = (long)m0 * m1 * m2;
    if (nv == 0) return hipSuccess;                     // no interior vertex: no coarse space
    hipError_t err = coarse_transfers(P, prec, t, z, true);
    if (err != hipSuccess) return err;
    double* c = P->d_cvec;
    double* w = P->d_cvec + nv;
    const double* Sx = P->d_cfd + P->cfd_off[0];
    const double* Sy = P->d_cfd + P->cfd_off[1];
    const double* Sz = P->d_cfd + P->cfd_off[2];
    const double* lx = Sx + (size_t)m0 * m0;
    const double* ly = Sy + (size_t)m1 * m1;
    const double* lz = Sz + (size_t)m2 * m2;
    const dim3 grid((unsigned)((nv + 255) / 256)), blk(256);
    hipStream_t s = P->stream;
    {
        TraceSpan ts("coarse_solve", P->p, FEM_F64, s);
        hipLaunchKernelGGL(k_coarse_pass, grid, blk, 0, s, c, w, Sx, m0, m1, m2, 0, 1, nullptr, nullptr, nullptr);
        hipLaunchKernelGGL(k_coarse_pass, grid, blk, 0, s, w, c, Sy, m0, m1, m2, 1, 1, nullptr, nullptr, nullptr);
        hipLaunchKernelGGL(k_coarse_pass, grid, blk, 0, s, c, w, Sz, m0, m1, m2, 2, 1, lx, ly, lz);
        hipLaunchKernelGGL(k_coarse_pass, grid, blk, 0, s, w, c, Sz, m0, m1, m2, 2, 0, nullptr, nullptr, nullptr);
        hipLaunchKernelGGL(k_coarse_pass, grid, blk, 0, s, c, w, Sy, m0, m1, m2, 1, 0, nullptr, nullptr, nullptr);
        hipLaunchKernelGGL(k_coarse_pass, grid, blk, 0, s, w, c, Sx, m0, m1, m2, 0, 0, nullptr, nullptr, nullptr);
    }
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    return coarse_transfers(P, prec, nullptr, z, false);
}

}  // namespace fem
