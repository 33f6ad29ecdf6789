// Cell-wise vector kernels: layout converters, deterministic reductions, the
// assembled residual norm, the DSS axis pass and the fused (F)PCG updates.
//
// Every pairing in the solver is a plain local dot product over all cell-wise
// entries: for a dual f and a primal u, <f, u> = <G^T f, u_global> (Lemma
// "Duality Pairing Identity", Section 3.1), so no assembly is needed.
// Reductions are deterministic: a problem's vector is cut into a fixed number
// of tiles (independent of anything else in the launch), each tile is summed
// in a fixed order (thread-strided sums, a fixed shuffle tree, four wave
// partials), and a final kernel adds the tile partials in index order.
#include <cstring>

#include "fem_internal.h"
#include "launch.h"
#include "mixed.h"
#include "trace.h"

namespace fem {

__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------- dots
// partial[group][t] = sum over tile t of a[i] * b[i]
template <typename SA, typename SB, bool MULTI>
__global__ void __launch_bounds__(256) k_dot(LaunchTable L, int group) {
    __shared__ double sh[4];
    for (int tile = blockIdx.x; tile < L.total_tiles; tile += gridDim.x) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        size_t lo, hi;
        red_range(pe, t, lo, hi);
        const SA* a = static_cast<const SA*>(pe.a);
        const SB* b = static_cast<const SB*>(pe.b);
        double acc = 0.0;
        for (size_t i = lo + threadIdx.x; i < hi; i += 256)
            acc += (double)load_as<double>(a + i) * (double)load_as<double>(b + i);
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) pe.red[group * kRedParts + t] = s;
    }
}

// slots[slot] = sum of the group's tile partials (one workgroup per problem)
template <bool MULTI>
__global__ void __launch_bounds__(256) k_red_final(LaunchTable L, int group, int slot) {
    __shared__ double sh[4];
    const int i = blockIdx.x;
    const ProbEntry& pe = entry_at<MULTI>(L, i);
    double acc = 0.0;
    for (int t = threadIdx.x; t < pe.ntiles_red; t += 256) acc += pe.red[group * kRedParts + t];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) red_slots(pe.red)[slot] = s;
}

// -------------------------------------------------- assembled norm ||G^T r||^2
// Each global node is owned by its copy in the lowest-numbered cell along
// every direction; the owner sums all copies (fixed order) and squares.
template <int P, typename S, bool MULTI>
__device__ __forceinline__ void anorm_body(const LaunchTable& L, int group, int item, int items, char* smem) {
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    double* sh = reinterpret_cast<double*>(smem);
    const int lane = threadIdx.x % kLanes, lq = threadIdx.x / kLanes;
    for (int tile = item; tile < L.total_tiles; tile += items) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        size_t lo, hi;
        red_range(pe, t, lo, hi);
        const S* v = static_cast<const S*>(pe.a);
        const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
        double acc = 0.0;
        // walk the range block by block: a thread keeps its cell (lane) within a block
        for (size_t base = lo - lo % ((size_t)NN * kLanes); base < hi; base += (size_t)NN * kLanes) {
            const int blk = (int)(base / ((size_t)NN * kLanes));
            const int e = blk * kLanes + lane;
            if (e >= pe.ncells) continue;
            const int lb = base < lo ? (int)((lo - base) / kLanes) : 0;
            const int le = base + (size_t)NN * kLanes > hi ? (int)((hi - base) / kLanes) : NN;
            const int i = e % n0, j = (e / n0) % n1, k = e / (n0 * n1);
            for (int l = lb + lq; l < le; l += 4) {
                const int a = l % N, b = (l / N) % N, c = l / N2;
                if ((a == P && i < n0 - 1) || (b == P && j < n1 - 1) || (c == P && k < n2 - 1)) continue;
                const int cx = (a == 0 && i > 0) ? 2 : 1;
                const int cy = (b == 0 && j > 0) ? 2 : 1;
                const int cz = (c == 0 && k > 0) ? 2 : 1;
                double s = 0.0;
                for (int sz = 0; sz < cz; ++sz)
                    for (int sy = 0; sy < cy; ++sy)
                        for (int sx = 0; sx < cx; ++sx) {
                            const int ee = (i - sx) + n0 * ((j - sy) + n1 * (k - sz));
                            const int ll = (sx ? P : a) + N * ((sy ? P : b) + N * (sz ? P : c));
                            s += load_as<double>(v + cell_offset(ee, ll, NN));
                        }
                acc += s * s;
            }
        }
        const double r = block_sum(acc, sh);
        if (threadIdx.x == 0) pe.red[group * kRedParts + t] = r;
    }
}

template <int P, typename S, bool MULTI>
__global__ void __launch_bounds__(256) k_anorm(LaunchTable L, int group) {
    __shared__ __align__(16) char smem[4 * sizeof(double)];
    anorm_body<P, S, MULTI>(L, group, blockIdx.x, gridDim.x, smem);
}

// ------------------------------------- assembled residual for a demoted smoother
// rs(copy) = (G^T r)(node) / multiplicity(node), summed in FP64 over all copies
// in ascending cell order (the same order for every copy), then rounded to
// the smoother precision RS; owner copies add (G^T r)^2 to the norm partials.
// The unassembled dual residual of a converging solve carries per-copy
// values far larger than its assembly (they cancel across interfaces), so
// rounding copies before assembling would leave an absolute error of
// eps(RS) times those values in the smoother's input.
//
// The same pass serves the simple preconditioners of Section 3.3 (MODE):
//   kDistMean     rs = G^T r / multiplicity (above),
//   kDistDss      z = S r = G G^T r: every copy gets the assembled value
//                 (Eq. "dss_operator"), zero on a Dirichlet boundary,
//   kDistJacobi   z = D_cell^{-1} S r: the assembled value divided by the
//                 diagonal of the assembled operator at the node, which is
//                 summed from the cells' element diagonals in the same loop
//                 (diag A_K at local (a,b,c) = cx Kaa Mbb Mcc + cy Maa Kbb Mcc
//                 + cz Maa Mbb Kcc), zero on a Dirichlet boundary.
// Every copy of a node computes the same terms in the same order, so the
// output is continuous bit for bit.
enum { kDistMean = 0, kDistDss = 1, kDistJacobi = 2 };

struct Diag1D {
    double k[kMaxP + 1];    // diagonal of the 1D reference stiffness
    double m[kMaxP + 1];    // diagonal of the 1D reference mass
};

// FP16 copies of a solver's residual are stored scaled by a power of two
// (exact), chosen so that the residual's root-mean-square node value lands
// in [2^-10, 2^-9): late in a solve the values are far below FP16's normal
// range, while the patch inverse multiplies them by up to 1/lambda_min of a
// patch operator (about 2.5e3 for p = 7 on 48^3 cells, more on graded
// cells), and the smoother stores that result in FP16 too, whose largest
// value is 65504.  Entries more than 16 times below the mean are subnormal;
// their absolute spacing 2^-24 stays under the rounding of a typical entry.
// The scale comes from the problem's residual norm slot (the current or the
// previous ||G^T r||^2, which the solver keeps there).  Every preconditioner
// here is linear, and the (F)PCG iterates do not change when z is scaled by
// a positive factor (alpha and beta absorb it), so the solver uses the
// scaled z as it is.  Entries with alpha = 0 (the public conversion calls)
// are not scaled.
__device__ __forceinline__ double f16_residual_scale(const ProbEntry& pe) {
    const double rn = red_slots(pe.red)[kSlotRN];
    if (pe.alpha == 0.0 || !(rn > 0.0) || !__builtin_isfinite(rn)) return 1.0;
    const double nodes = ((double)pe.n[0] * pe.p + 1) * ((double)pe.n[1] * pe.p + 1) * ((double)pe.n[2] * pe.p + 1);
    int ex;
    frexp(sqrt(rn / nodes), &ex);
    return ldexp(1.0, -9 - ex);
}

template <int P, typename RS, int MODE, bool MULTI>
__device__ __forceinline__ void distribute_body(const LaunchTable& L, int group, const Diag1D& dg, int item, int items,
                                                char* smem) {
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    double* sh = reinterpret_cast<double*>(smem);
    const int lane = threadIdx.x % kLanes, lq = threadIdx.x / kLanes;
    for (int tile = item; tile < L.total_tiles; tile += items) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        size_t lo, hi;
        red_range(pe, t, lo, hi);
        const double* v = static_cast<const double*>(pe.a);
        RS* out = static_cast<RS*>(pe.c);
        const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
        double os = 1.0;                     // scale of the stored copies
        if constexpr (Prec<RS>::id == FEM_F16) os = f16_residual_scale(pe);
        double acc = 0.0;
        for (size_t base = lo - lo % ((size_t)NN * kLanes); base < hi; base += (size_t)NN * kLanes) {
            const int blk = (int)(base / ((size_t)NN * kLanes));
            const int e = blk * kLanes + lane;
            const int lb = base < lo ? (int)((lo - base) / kLanes) : 0;
            const int le = base + (size_t)NN * kLanes > hi ? (int)((hi - base) / kLanes) : NN;
            if (e >= pe.ncells) {
                for (int l = lb + lq; l < le; l += 4) store_from(out + base + (size_t)l * kLanes + lane, (typename Prec<RS>::C)0);
                continue;
            }
            const int i = e % n0, j = (e / n0) % n1, k = e / (n0 * n1);
            for (int l = lb + lq; l < le; l += 4) {
                const int a = l % N, b = (l / N) % N, c = l / N2;
                // sharing cells per direction: (cell, local index), ascending cell
                int ci[2], ai[2], nx, cj[2], bj[2], ny, ck[2], ck_l[2], nz;
                if (a == 0 && i > 0) { ci[0] = i - 1; ai[0] = P; ci[1] = i; ai[1] = 0; nx = 2; }
                else if (a == P && i < n0 - 1) { ci[0] = i; ai[0] = P; ci[1] = i + 1; ai[1] = 0; nx = 2; }
                else { ci[0] = i; ai[0] = a; nx = 1; }
                if (b == 0 && j > 0) { cj[0] = j - 1; bj[0] = P; cj[1] = j; bj[1] = 0; ny = 2; }
                else if (b == P && j < n1 - 1) { cj[0] = j; bj[0] = P; cj[1] = j + 1; bj[1] = 0; ny = 2; }
                else { cj[0] = j; bj[0] = b; ny = 1; }
                if (c == 0 && k > 0) { ck[0] = k - 1; ck_l[0] = P; ck[1] = k; ck_l[1] = 0; nz = 2; }
                else if (c == P && k < n2 - 1) { ck[0] = k; ck_l[0] = P; ck[1] = k + 1; ck_l[1] = 0; nz = 2; }
                else { ck[0] = k; ck_l[0] = c; nz = 1; }
                double s = 0.0, d = 0.0;
                for (int z = 0; z < nz; ++z)
                    for (int y = 0; y < ny; ++y)
                        for (int x = 0; x < nx; ++x) {
                            const int ee = ci[x] + n0 * (cj[y] + n1 * ck[z]);
                            const int ll = ai[x] + N * (bj[y] + N * ck_l[z]);
                            s += v[cell_offset(ee, ll, NN)];
                            if (MODE == kDistJacobi) {
                                const double hx = pe.h[0][ci[x]], hy = pe.h[1][cj[y]], hz = pe.h[2][ck[z]];
                                const int ax = ai[x], by = bj[y], cz = ck_l[z];
                                d += (hy * hz / hx) * dg.k[ax] * dg.m[by] * dg.m[cz] +
                                     (hx * hz / hy) * dg.m[ax] * dg.k[by] * dg.m[cz] +
                                     (hx * hy / hz) * dg.m[ax] * dg.m[by] * dg.k[cz];
                            }
                        }
                double o;
                if (MODE == kDistMean) {
                    o = s / (double)(nx * ny * nz);
                } else {
                    const bool bnd = pe.dirichlet && ((a == 0 && i == 0) || (a == P && i == n0 - 1) ||
                                                      (b == 0 && j == 0) || (b == P && j == n1 - 1) ||
                                                      (c == 0 && k == 0) || (c == P && k == n2 - 1));
                    o = bnd ? 0.0 : (MODE == kDistJacobi ? s / d : s);
                }
                if constexpr (Prec<RS>::id == FEM_F16) o *= os;
                store_from(out + base + (size_t)l * kLanes + lane, (typename Prec<RS>::C)o);
                // owner copy: lowest cell along every direction
                if (ci[0] == i && cj[0] == j && ck[0] == k) acc += s * s;
            }
        }
        const double r = block_sum(acc, sh);
        if (threadIdx.x == 0) pe.red[group * kRedParts + t] = r;
    }
}

template <int P, typename RS, int MODE, bool MULTI>
__global__ void __launch_bounds__(256) k_distribute(LaunchTable L, int group, Diag1D dg) {
    __shared__ __align__(16) char smem[4 * sizeof(double)];
    distribute_body<P, RS, MODE, MULTI>(L, group, dg, blockIdx.x, gridDim.x, smem);
}

// ------------------------------------------------------------ DSS axis pass
// One thread per (interface, face node): both coincident copies receive their
// sum (Algorithm "Dimensionally-Split Structured Summation").
template <int P, typename S>
__global__ void __launch_bounds__(256) k_dss_axis(ProbEntry pe, int axis, long total) {
    using C = typename Prec<S>::C;
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int n0 = pe.n[0], n1 = pe.n[1];
    int eL, lL, eR, lR;
    if (axis == 0) {
        const int ii = t % (n0 - 1);
        long r = t / (n0 - 1);
        const int fn = r % N2;
        r /= N2;
        const int j = r % n1, k = r / n1;
        const int b = fn % N, c = fn / N;
        eL = ii + n0 * (j + n1 * k);
        eR = eL + 1;
        lL = P + N * (b + N * c);
        lR = 0 + N * (b + N * c);
    } else if (axis == 1) {
        const int i = t % n0;
        long r = t / n0;
        const int jj = r % (n1 - 1);
        r /= (n1 - 1);
        const int fn = r % N2;
        const int k = r / N2;
        const int a = fn % N, c = fn / N;
        eL = i + n0 * (jj + n1 * k);
        eR = eL + n0;
        lL = a + N * (P + N * c);
        lR = a + N * (0 + N * c);
    } else {
        const int i = t % n0;
        long r = t / n0;
        const int j = r % n1;
        r /= n1;
        const int kk = r % (pe.n[2] - 1);
        const int fn = r / (pe.n[2] - 1);
        const int a = fn % N, b = fn / N;
        eL = i + n0 * (j + n1 * kk);
        eR = eL + n0 * n1;
        lL = a + N * (b + N * P);
        lR = a + N * (b + N * 0);
    }
    S* v = static_cast<S*>(pe.c);
    S* pL = v + cell_offset(eL, lL, NN);
    S* pR = v + cell_offset(eR, lR, NN);
    const C s = load_as<C>(pL) + load_as<C>(pR);
    store_from(pL, s);
    store_from(pR, s);
}

// ------------------------------------------------------------ converters
template <typename S>
__global__ void __launch_bounds__(256) k_gather(ProbEntry pe, const double* __restrict__ xg) {
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= pe.len) return;
    const int p = pe.p, N = p + 1, NN = N * N * N;
    const int blk = t / ((size_t)NN * kLanes);
    const int rem = t % ((size_t)NN * kLanes);
    const int l = rem / kLanes, lane = rem % kLanes;
    const int e = blk * kLanes + lane;
    double v = 0.0;
    if (e < pe.ncells) {
        const int n0 = pe.n[0], n1 = pe.n[1];
        const int i = e % n0, j = (e / n0) % n1, k = e / (n0 * n1);
        const int a = l % N, b = (l / N) % N, c = l / (N * N);
        const size_t G0 = (size_t)n0 * p + 1, G1 = (size_t)n1 * p + 1;
        v = xg[(size_t)(i * p + a) + G0 * ((size_t)(j * p + b) + G1 * (size_t)(k * p + c))];
    }
    store_from(static_cast<S*>(pe.c) + t, v);
}

// mode 0: sum all copies (G^T); mode 1: copy of the lowest-numbered cell
template <typename S>
__global__ void __launch_bounds__(256) k_to_global(ProbEntry pe, double* __restrict__ yg, int mode) {
    const int p = pe.p, N = p + 1, NN = N * N * N;
    const int n0 = pe.n[0], n1 = pe.n[1], n2 = pe.n[2];
    const size_t G0 = (size_t)n0 * p + 1, G1 = (size_t)n1 * p + 1, G2 = (size_t)n2 * p + 1;
    const size_t g = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= G0 * G1 * G2) return;
    const int I = g % G0, J = (g / G0) % G1, K = g / (G0 * G1);
    int ci[3][2], li[3][2], cnt[3];
    const int idx[3] = {I, J, K};
    const int nn[3] = {n0, n1, n2};
    for (int d = 0; d < 3; ++d) {
        cnt[d] = 0;
        const int q = idx[d] / p, r = idx[d] % p;
        if (r == 0 && q >= 1) { ci[d][cnt[d]] = q - 1; li[d][cnt[d]] = p; ++cnt[d]; }
        if (q <= nn[d] - 1) { ci[d][cnt[d]] = q; li[d][cnt[d]] = r; ++cnt[d]; }
        if (mode == 1) cnt[d] = 1;
    }
    const S* v = static_cast<const S*>(pe.a);
    double s = 0.0;
    for (int z = 0; z < cnt[2]; ++z)
        for (int y = 0; y < cnt[1]; ++y)
            for (int x = 0; x < cnt[0]; ++x) {
                const int e = ci[0][x] + n0 * (ci[1][y] + n1 * ci[2][z]);
                const int l = li[0][x] + N * (li[1][y] + N * li[2][z]);
                s += load_as<double>(v + cell_offset(e, l, NN));
            }
    yg[g] = s;
}

template <typename S>
__global__ void __launch_bounds__(256) k_pack(ProbEntry pe, const double* __restrict__ canon,
                                              double* __restrict__ out_canon, int unpack) {
    const int N = pe.p + 1, NN = N * N * N;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)pe.ncells * NN) return;
    const int e = t / NN, l = t % NN;
    const size_t off = cell_offset(e, l, NN);
    if (unpack) out_canon[t] = load_as<double>(static_cast<const S*>(pe.a) + off);
    else store_from(static_cast<S*>(pe.c) + off, canon[t]);
}

template <typename SA, typename SB>
__global__ void __launch_bounds__(256) k_convert(const SA* __restrict__ a, SB* __restrict__ b, size_t n) {
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) store_from(b + t, load_as<typename Prec<SB>::C>(a + t));
}

template <typename S>
__global__ void __launch_bounds__(256) k_fill_zero(S* __restrict__ a, size_t n) {
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) store_from(a + t, (typename Prec<S>::C)0);
}

// --------------------------------------------------------- (F)PCG updates
// r -= alpha q with alpha = <r,z>/<q,p> from the slots; alpha is saved in a
// slot and u += alpha p happens in the next p update (which reads p anyway),
// or in k_cg_u when the iteration stops.  The smoother's copy of r
// (precision RS) is written in the same pass when requested.
template <typename RS, bool MULTI>
__global__ void __launch_bounds__(256) k_cg_ur(LaunchTable L) {
    for (int tile = blockIdx.x; tile < L.total_tiles; tile += gridDim.x) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        double* sl = red_slots(pe.red);
        if (sl[kSlotState] != 0.0) continue;       // finished: r and alpha stay
        // a breakdown (<q,p> not positive, or a non-finite step) leaves r and
        // u where they are: the host sees <q,p> and stops the solve, and a
        // zero right-hand side (r = z = p = 0) takes no step at all
        double alpha = sl[kSlotRZ] / sl[kSlotQP];
        if (!(sl[kSlotQP] > 0.0) || !__builtin_isfinite(alpha)) alpha = 0.0;
        if (t == 0 && threadIdx.x == 0) sl[kSlotAlpha] = alpha;
        size_t lo, hi;
        red_range(pe, t, lo, hi);
        const double* q = static_cast<const double*>(pe.b);
        double* r = static_cast<double*>(pe.d);
        RS* rs = static_cast<RS*>(pe.e);
        for (size_t i = lo + threadIdx.x; i < hi; i += 256) {
            const double rn = r[i] - alpha * q[i];
            r[i] = rn;
            if (rs) store_from(rs + i, (typename Prec<RS>::C)rn);
        }
    }
}

// u += alpha p with the saved alpha; then p = z + beta p with
// beta = <r',z'>/<r,z> (PCG) or -<q,z'>/<q,p> (FCG).  pe: a = z, c = p, d = u.
template <typename SZ, bool MULTI>
__global__ void __launch_bounds__(256) k_cg_p(LaunchTable L, int variant) {
    for (int tile = blockIdx.x; tile < L.total_tiles; tile += gridDim.x) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        const double* sl = red_slots(pe.red);
        if (sl[kSlotState] == 2.0) continue;       // frozen: u and p stay
        const double beta = variant == FEM_CG_PCG ? sl[kSlotRZ] / sl[kSlotRZOld] : -sl[kSlotQZ] / sl[kSlotQP];
        const double alpha = sl[kSlotAlpha];
        size_t lo, hi;
        red_range(pe, t, lo, hi);
        const SZ* z = static_cast<const SZ*>(pe.a);
        double* p = static_cast<double*>(pe.c);
        double* u = static_cast<double*>(pe.d);
        // a zero step (breakdown, zero right-hand side) leaves u untouched
        const bool step = alpha != 0.0;
        for (size_t i = lo + threadIdx.x; i < hi; i += 256) {
            const double pi = p[i];
            if (step) u[i] = u[i] + alpha * pi;
            p[i] = load_as<double>(z + i) + beta * pi;
        }
    }
}

// u += alpha p with the saved alpha (the iteration's last step)
template <bool MULTI>
__global__ void __launch_bounds__(256) k_cg_u(LaunchTable L) {
    for (int tile = blockIdx.x; tile < L.total_tiles; tile += gridDim.x) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        const double alpha = red_slots(pe.red)[kSlotAlpha];
        size_t lo, hi;
        red_range(pe, t, lo, hi);
        const double* p = static_cast<const double*>(pe.a);
        double* u = static_cast<double*>(pe.c);
        for (size_t i = lo + threadIdx.x; i < hi; i += 256) u[i] = u[i] + alpha * p[i];
    }
}

// partials of <q, z> (group 0) and <r, z> (group 3) in one pass.
// pe: a = q, d = r (FP64), b = z (SZ).
template <typename SZ, bool MULTI>
__global__ void __launch_bounds__(256) k_dot_qz_rz(LaunchTable L) {
    __shared__ double sh[4];
    for (int tile = blockIdx.x; tile < L.total_tiles; tile += gridDim.x) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        size_t lo, hi;
        red_range(pe, t, lo, hi);
        const double* q = static_cast<const double*>(pe.a);
        const double* r = static_cast<const double*>(pe.d);
        const SZ* z = static_cast<const SZ*>(pe.b);
        double aq = 0.0, ar = 0.0;
        for (size_t i = lo + threadIdx.x; i < hi; i += 256) {
            const double zi = load_as<double>(z + i);
            aq += q[i] * zi;
            ar += r[i] * zi;
        }
        const double sq = block_sum(aq, sh);
        const double sr = block_sum(ar, sh);
        if (threadIdx.x == 0) {
            pe.red[0 * kRedParts + t] = sq;
            pe.red[3 * kRedParts + t] = sr;
        }
    }
}

// elementwise a (SA) -> c (SB) over whole cell vectors of several problems
template <typename SA, typename SB, bool MULTI>
__global__ void __launch_bounds__(256) k_convert_multi(LaunchTable L) {
    for (int tile = blockIdx.x; tile < L.total_tiles; tile += gridDim.x) {
        const ProbEntry& pe = entry<MULTI>(L, tile);
        const int t = tile - pe.tile_begin;
        size_t lo, hi;
        red_range(pe, t, lo, hi);
        const SA* a = static_cast<const SA*>(pe.a);
        SB* c = static_cast<SB*>(pe.c);
        for (size_t i = lo + threadIdx.x; i < hi; i += 256) store_from(c + i, load_as<typename Prec<SB>::C>(a + i));
    }
}

// out[2i] = slot sa, out[2i+1] = slot sb of problem i
template <bool MULTI>
__global__ void k_collect_slots(LaunchTable L, int sa, int sb, double* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.nprob) return;
    const ProbEntry& pe = entry_at<MULTI>(L, i);
    const double* sl = red_slots(pe.red);
    out[2 * i] = sl[sa];
    out[2 * i + 1] = sl[sb];
}

// device-side convergence state (see launch_cg_check)
template <bool MULTI>
__global__ void k_solve_init(LaunchTable L) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.nprob) return;
    const ProbEntry& pe = entry_at<MULTI>(L, i);
    double* sl = red_slots(pe.red);
    sl[kSlotState] = 0.0;
    sl[kSlotIters] = 0.0;
    sl[kSlotRel] = 1.0;
    sl[kSlotStatus] = (double)FEM_OK;
    sl[kSlotRtol] = pe.alpha;
    sl[kSlotMaxit] = (double)pe.zchunk;
}

template <bool MULTI>
__global__ void k_cg_check(LaunchTable L) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.nprob) return;
    const ProbEntry& pe = entry_at<MULTI>(L, i);
    double* sl = red_slots(pe.red);
    if (sl[kSlotState] == 1.0) {
        sl[kSlotState] = 2.0;
        return;
    }
    if (sl[kSlotState] != 0.0) return;
    const double it = sl[kSlotIters] + 1.0;
    sl[kSlotIters] = it;
    const double b2 = sl[kSlotB2], rn = sl[kSlotRN], qp = sl[kSlotQP];
    const double rel = b2 > 0.0 ? sqrt(rn / b2) : 0.0;
    sl[kSlotRel] = rel;
    int status = -1;
    if (b2 == 0.0) {
        status = FEM_OK;                 // zero right-hand side: u = 0, no iteration counted
        sl[kSlotIters] = 0.0;
    } else if (!(qp > 0.0) || !__builtin_isfinite(qp) || !__builtin_isfinite(rel)) {
        status = FEM_EBREAKDOWN;
    } else if (rel <= sl[kSlotRtol]) {
        status = FEM_OK;
    } else if (it >= sl[kSlotMaxit]) {
        status = FEM_ENOTCONV;
    }
    if (status >= 0) {
        sl[kSlotStatus] = (double)status;
        sl[kSlotState] = 1.0;
    }
}

// p = z (initial direction), z in precision SZ
template <bool MULTI>
__global__ void k_slot_copy(LaunchTable L, int dst, int src) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.nprob) return;
    const ProbEntry& pe = entry_at<MULTI>(L, i);
    double* sl = red_slots(pe.red);
    sl[dst] = sl[src];
}

// =========================================================================
// Host launchers
static inline int grid_for(size_t n) { return (int)((n + 255) / 256); }

ProbEntry entry_of(const fem_problem* P) {
    ProbEntry e{};
    e.n[0] = P->n[0];
    e.n[1] = P->n[1];
    e.n[2] = P->n[2];
    e.p = P->p;
    e.len = P->cell_len;
    e.ncells = P->ncells;
    e.nblk = P->nblk;
    e.dirichlet = P->bc == FEM_BC_DIRICHLET;
    e.h[0] = P->d_h;
    e.h[1] = P->d_h + P->n[0];
    e.h[2] = P->d_h + P->n[0] + P->n[1];
    e.red = P->d_red;
    // tiles of about 8192 elements (a few per thread of a 256-thread
    // workgroup), at most kRedParts; fixed by the problem's own sizes
    constexpr size_t kTileElems = 8192;
    const int nn = (P->p + 1) * (P->p + 1) * (P->p + 1);
    size_t want = (P->cell_len + kTileElems - 1) / kTileElems;
    if (want < 1) want = 1;
    if (want > (size_t)kRedParts) want = kRedParts;
    if ((int)want <= P->nblk) {
        e.blocks_per_red = (int)((P->nblk + want - 1) / want);
        e.red_lsplit = 1;
        e.ntiles_red = (P->nblk + e.blocks_per_red - 1) / e.blocks_per_red;
    } else {
        e.blocks_per_red = 1;
        int split = (int)((want + P->nblk - 1) / P->nblk);
        if (split > kRedParts / P->nblk) split = kRedParts / P->nblk;   // nblk * split <= kRedParts
        if (split > (nn + 3) / 4) split = (nn + 3) / 4;        // at least 4 node planes per tile
        if (split < 1) split = 1;
        const int lchunk = (nn + split - 1) / split;
        e.red_lsplit = (nn + lchunk - 1) / lchunk;
        e.ntiles_red = P->nblk * e.red_lsplit;
    }
    return e;
}

template <typename F>
static hipError_t dispatch_prec(int prec, F&& f) {
    switch (prec) {
        case FEM_F64: return f(double{});
        case FEM_F32: return f(float{});
        case FEM_BF16: return f(bf16_t{});
        case FEM_F16: return f(f16_t{});
        default: return hipErrorInvalidValue;
    }
}

hipError_t run_fill_zero(fem_problem* P, void* v, int prec) {
    return dispatch_prec(prec, [&](auto tag) {
        using S = decltype(tag);
        hipLaunchKernelGGL((k_fill_zero<S>), dim3(grid_for(P->cell_len)), dim3(256), 0, P->stream,
                           static_cast<S*>(v), P->cell_len);
        return hipGetLastError();
    });
}

hipError_t run_convert(fem_problem* P, const void* src, int sp, void* dst, int dp) {
    return dispatch_prec(sp, [&](auto ta) {
        using SA = decltype(ta);
        return dispatch_prec(dp, [&](auto tb) {
            using SB = decltype(tb);
            hipLaunchKernelGGL((k_convert<SA, SB>), dim3(grid_for(P->cell_len)), dim3(256), 0, P->stream,
                               static_cast<const SA*>(src), static_cast<SB*>(dst), P->cell_len);
            return hipGetLastError();
        });
    });
}

hipError_t run_gather(fem_problem* P, const double* xg, void* xc, int prec) {
    ProbEntry e = entry_of(P);
    e.c = xc;
    return dispatch_prec(prec, [&](auto tag) {
        using S = decltype(tag);
        hipLaunchKernelGGL((k_gather<S>), dim3(grid_for(P->cell_len)), dim3(256), 0, P->stream, e, xg);
        return hipGetLastError();
    });
}

static hipError_t run_to_global(fem_problem* P, const void* yc, double* yg, int prec, int mode) {
    ProbEntry e = entry_of(P);
    e.a = yc;
    return dispatch_prec(prec, [&](auto tag) {
        using S = decltype(tag);
        hipLaunchKernelGGL((k_to_global<S>), dim3(grid_for(P->global_len)), dim3(256), 0, P->stream, e, yg, mode);
        return hipGetLastError();
    });
}
hipError_t run_scatter(fem_problem* P, const void* yc, double* yg, int prec) {
    return run_to_global(P, yc, yg, prec, 0);
}
hipError_t run_extract(fem_problem* P, const void* uc, double* ug, int prec) {
    return run_to_global(P, uc, ug, prec, 1);
}

hipError_t run_pack_entry(ProbEntry e, const double* canon, void* vc, int prec, int unpack, hipStream_t st) {
    const int N = e.p + 1;
    const size_t n = (size_t)e.ncells * N * N * N;
    if (unpack) e.a = vc; else e.c = vc;
    return dispatch_prec(prec, [&](auto tag) {
        using S = decltype(tag);
        hipError_t err = hipSuccess;
        if (!unpack) {      // padding entries must be zero
            hipLaunchKernelGGL((k_fill_zero<S>), dim3(grid_for(e.len)), dim3(256), 0, st, static_cast<S*>(vc), e.len);
            err = hipGetLastError();
            if (err != hipSuccess) return err;
        }
        if (n == 0) return hipSuccess;
        hipLaunchKernelGGL((k_pack<S>), dim3(grid_for(n)), dim3(256), 0, st, e, canon, const_cast<double*>(canon),
                           unpack);
        return hipGetLastError();
    });
}

hipError_t run_pack(fem_problem* P, const double* canon, void* vc, int prec, int unpack) {
    return run_pack_entry(entry_of(P), canon, vc, prec, unpack, P->stream);
}

template <int P_, typename S>
static void launch_dss_axis(const ProbEntry& e, int axis, long total, hipStream_t s) {
    TraceSpan ts("dss_axis", P_, Prec<S>::id, s);
    hipLaunchKernelGGL((k_dss_axis<P_, S>), dim3((total + 255) / 256), dim3(256), 0, s, e, axis, total);
}

hipError_t run_dss_axis_entry(int p, const ProbEntry& e, int axis, int prec, hipStream_t st) {
    const int N = p + 1;
    long total;
    if (axis == 0) total = (long)(e.n[0] - 1) * e.n[1] * e.n[2] * N * N;
    else if (axis == 1) total = (long)e.n[0] * (e.n[1] - 1) * e.n[2] * N * N;
    else total = (long)e.n[0] * e.n[1] * (e.n[2] - 1) * N * N;
    if (total <= 0) return hipSuccess;
    return dispatch_prec(prec, [&](auto tag) {
        using S = decltype(tag);
        switch (p) {
            case 1: launch_dss_axis<1, S>(e, axis, total, st); break;
            case 2: launch_dss_axis<2, S>(e, axis, total, st); break;
            case 3: launch_dss_axis<3, S>(e, axis, total, st); break;
            case 4: launch_dss_axis<4, S>(e, axis, total, st); break;
            case 5: launch_dss_axis<5, S>(e, axis, total, st); break;
            case 6: launch_dss_axis<6, S>(e, axis, total, st); break;
            case 7: launch_dss_axis<7, S>(e, axis, total, st); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    });
}

hipError_t run_dss_axis(fem_problem* P, void* v, int axis, int prec) {
    ProbEntry e = entry_of(P);
    e.c = v;
    return run_dss_axis_entry(P->p, e, axis, prec, P->stream);
}

static hipError_t finish_reduction(fem_problem* P, const ProbEntry& e, int group, int slot) {
    LaunchTable L{};
    L.nprob = 1;
    L.one = e;
    hipLaunchKernelGGL(k_red_final<false>, dim3(1), dim3(256), 0, P->stream, L, group, slot);
    return hipGetLastError();
}

hipError_t run_dot(fem_problem* P, const void* a, int pa, const void* b, int pb, int slot) {
    ProbEntry e = entry_of(P);
    e.a = a;
    e.b = b;
    e.tile_begin = 0;
    LaunchTable L{};
    L.nprob = 1;
    L.total_tiles = e.ntiles_red;
    L.one = e;
    hipError_t err = dispatch_prec(pa, [&](auto ta) {
        using SA = decltype(ta);
        return dispatch_prec(pb, [&](auto tb) {
            using SB = decltype(tb);
            TraceSpan ts("dot", P->p, Prec<SA>::id, P->stream);
            hipLaunchKernelGGL((k_dot<SA, SB, false>), dim3(L.total_tiles), dim3(256), 0, P->stream, L, 0);
            return hipGetLastError();
        });
    });
    if (err != hipSuccess) return err;
    return finish_reduction(P, e, 0, slot);
}

hipError_t run_assembled_norm2(fem_problem* P, const void* r, int prec, int slot) {
    ProbEntry e = entry_of(P);
    e.a = r;
    e.tile_begin = 0;
    LaunchTable L{};
    L.nprob = 1;
    L.total_tiles = e.ntiles_red;
    L.one = e;
    hipError_t err = dispatch_prec(prec, [&](auto tag) {
        using S = decltype(tag);
        dim3 g(L.total_tiles), b(256);
        TraceSpan ts("assembled_norm", P->p, Prec<S>::id, P->stream);
        switch (P->p) {
            case 1: hipLaunchKernelGGL((k_anorm<1, S, false>), g, b, 0, P->stream, L, 1); break;
            case 2: hipLaunchKernelGGL((k_anorm<2, S, false>), g, b, 0, P->stream, L, 1); break;
            case 3: hipLaunchKernelGGL((k_anorm<3, S, false>), g, b, 0, P->stream, L, 1); break;
            case 4: hipLaunchKernelGGL((k_anorm<4, S, false>), g, b, 0, P->stream, L, 1); break;
            case 5: hipLaunchKernelGGL((k_anorm<5, S, false>), g, b, 0, P->stream, L, 1); break;
            case 6: hipLaunchKernelGGL((k_anorm<6, S, false>), g, b, 0, P->stream, L, 1); break;
            case 7: hipLaunchKernelGGL((k_anorm<7, S, false>), g, b, 0, P->stream, L, 1); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    });
    if (err != hipSuccess) return err;
    return finish_reduction(P, e, 1, slot);
}

static Diag1D diag_1d(int p) {
    Diag1D dg{};
    const double* M = ref_mass(p);
    const double* K = ref_stiff(p);
    for (int a = 0; a <= p; ++a) {
        dg.m[a] = M[a * (p + 1) + a];
        dg.k[a] = K[a * (p + 1) + a];
    }
    return dg;
}

template <int P, typename S, int MODE>
static void launch_distribute_one(LaunchTable& L, hipStream_t s, const Diag1D& dg) {
    hipLaunchKernelGGL((k_distribute<P, S, MODE, false>), dim3(L.total_tiles), dim3(256), 0, s, L, 2, dg);
}

template <int MODE>
static hipError_t run_distribute_mode(fem_problem* P, const double* r, void* out, int prec, int slot,
                                      const char* label, bool solver) {
    ProbEntry e = entry_of(P);
    e.a = r;
    e.c = out;
    e.alpha = solver ? 1.0 : 0.0;            // FP16 residual scaling (solver copies only)
    e.tile_begin = 0;
    LaunchTable L{};
    L.nprob = 1;
    L.total_tiles = e.ntiles_red;
    L.one = e;
    const Diag1D dg = MODE == kDistJacobi ? diag_1d(P->p) : Diag1D{};
    hipError_t err = dispatch_prec(prec, [&](auto tag) {
        using S = decltype(tag);
        TraceSpan ts(label, P->p, Prec<S>::id, P->stream);
        switch (P->p) {
            case 1: launch_distribute_one<1, S, MODE>(L, P->stream, dg); break;
            case 2: launch_distribute_one<2, S, MODE>(L, P->stream, dg); break;
            case 3: launch_distribute_one<3, S, MODE>(L, P->stream, dg); break;
            case 4: launch_distribute_one<4, S, MODE>(L, P->stream, dg); break;
            case 5: launch_distribute_one<5, S, MODE>(L, P->stream, dg); break;
            case 6: launch_distribute_one<6, S, MODE>(L, P->stream, dg); break;
            case 7: launch_distribute_one<7, S, MODE>(L, P->stream, dg); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    });
    if (err != hipSuccess) return err;
    return finish_reduction(P, e, 2, slot);
}

hipError_t run_distribute(fem_problem* P, const double* r, void* out, int prec, int slot, bool solver) {
    return run_distribute_mode<kDistMean>(P, r, out, prec, slot, "distribute", solver);
}

hipError_t run_simple_precond(fem_problem* P, int kind, const double* r, void* z, int prec, int slot, bool solver) {
    if (kind == FEM_PC_DSS) return run_distribute_mode<kDistDss>(P, r, z, prec, slot, "precond_dss", solver);
    if (kind == FEM_PC_JACOBI)
        return run_distribute_mode<kDistJacobi>(P, r, z, prec, slot, "precond_jacobi", solver);
    return hipErrorInvalidValue;
}

hipError_t run_cg_update_r(fem_problem* P, double* r, const double* q, void* rs, int rs_prec) {
    ProbEntry e = entry_of(P);
    e.b = q;
    e.d = r;
    e.e = rs;
    e.tile_begin = 0;
    LaunchTable L{};
    L.nprob = 1;
    L.total_tiles = e.ntiles_red;
    L.one = e;
    const int grid = e.ntiles_red < kMaxGrid ? e.ntiles_red : kMaxGrid;
    return dispatch_prec(rs ? rs_prec : FEM_F64, [&](auto tag) {
        using S = decltype(tag);
        TraceSpan ts("cg_update_ur", P->p, Prec<S>::id, P->stream);
        hipLaunchKernelGGL((k_cg_ur<S, false>), dim3(grid), dim3(256), 0, P->stream, L);
        return hipGetLastError();
    });
}

hipError_t run_cg_update_p(fem_problem* P, double* p, double* u, const void* z, int zprec, int variant) {
    ProbEntry e = entry_of(P);
    e.a = z;
    e.c = p;
    e.d = u;
    e.tile_begin = 0;
    LaunchTable L{};
    L.nprob = 1;
    L.total_tiles = e.ntiles_red;
    L.one = e;
    const int grid = e.ntiles_red < kMaxGrid ? e.ntiles_red : kMaxGrid;
    return dispatch_prec(zprec, [&](auto tag) {
        using S = decltype(tag);
        TraceSpan ts("cg_update_p", P->p, Prec<S>::id, P->stream);
        hipLaunchKernelGGL((k_cg_p<S, false>), dim3(grid), dim3(256), 0, P->stream, L, variant);
        return hipGetLastError();
    });
}

hipError_t run_cg_update_u(fem_problem* P, double* u, const double* p) {
    ProbEntry e = entry_of(P);
    e.a = p;
    e.c = u;
    e.tile_begin = 0;
    LaunchTable L{};
    L.nprob = 1;
    L.total_tiles = e.ntiles_red;
    L.one = e;
    const int grid = e.ntiles_red < kMaxGrid ? e.ntiles_red : kMaxGrid;
    TraceSpan ts("cg_update_u", P->p, FEM_F64, P->stream);
    hipLaunchKernelGGL(k_cg_u<false>, dim3(grid), dim3(256), 0, P->stream, L);
    return hipGetLastError();
}

hipError_t run_dot_qz_rz(fem_problem* P, const double* q, const double* r, const void* z, int zprec) {
    ProbEntry e = entry_of(P);
    e.a = q;
    e.d = const_cast<double*>(r);
    e.b = z;
    e.tile_begin = 0;
    LaunchTable L{};
    L.nprob = 1;
    L.total_tiles = e.ntiles_red;
    L.one = e;
    hipError_t err = dispatch_prec(zprec, [&](auto tag) {
        using S = decltype(tag);
        TraceSpan ts("dot", P->p, Prec<S>::id, P->stream);
        hipLaunchKernelGGL((k_dot_qz_rz<S, false>), dim3(L.total_tiles), dim3(256), 0, P->stream, L);
        return hipGetLastError();
    });
    if (err != hipSuccess) return err;
    err = finish_reduction(P, e, 0, kSlotQZ);
    if (err != hipSuccess) return err;
    return finish_reduction(P, e, 3, kSlotRZ);
}

hipError_t run_slot_copy(fem_problem* P, int dst, int src) {
    LaunchTable L{};
    L.nprob = 1;
    L.one = entry_of(P);
    hipLaunchKernelGGL(k_slot_copy<false>, dim3(1), dim3(64), 0, P->stream, L, dst, src);
    return hipGetLastError();
}

// =========================================================================
// Multi-problem launchers
static int tiles_red(ProbEntry* ents, int nprob) {
    int t = 0;
    for (int i = 0; i < nprob; ++i) {
        ents[i].tile_begin = t;
        t += ents[i].ntiles_red;
    }
    return t;
}

static hipError_t final_multi(LaunchTable& L, hipStream_t s, int group, int slot) {
    if (L.nprob > 1) hipLaunchKernelGGL(k_red_final<true>, dim3(L.nprob), dim3(256), 0, s, L, group, slot);
    else hipLaunchKernelGGL(k_red_final<false>, dim3(1), dim3(256), 0, s, L, group, slot);
    return hipGetLastError();
}

hipError_t launch_dot(int pa, int pb, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, int slot) {
    if (nprob <= 0) return hipSuccess;
    LaunchTable L{};
    L.nprob = nprob;
    L.total_tiles = tiles_red(ents, nprob);
    hipError_t err = stage_table(L, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    const int grid = L.total_tiles < kMaxGrid ? L.total_tiles : kMaxGrid;
    err = dispatch_prec(pa, [&](auto ta) {
        using SA = decltype(ta);
        return dispatch_prec(pb, [&](auto tb) {
            using SB = decltype(tb);
            if (nprob > 1) hipLaunchKernelGGL((k_dot<SA, SB, true>), dim3(grid), dim3(256), 0, s, L, 0);
            else hipLaunchKernelGGL((k_dot<SA, SB, false>), dim3(grid), dim3(256), 0, s, L, 0);
            return hipGetLastError();
        });
    });
    if (err != hipSuccess) return err;
    return final_multi(L, s, 0, slot);
}

template <int P, typename S>
static void launch_distribute_pt(LaunchTable& L, int grid, hipStream_t s) {
    const Diag1D dg{};
    if (L.nprob > 1) hipLaunchKernelGGL((k_distribute<P, S, kDistMean, true>), dim3(grid), dim3(256), 0, s, L, 2, dg);
    else hipLaunchKernelGGL((k_distribute<P, S, kDistMean, false>), dim3(grid), dim3(256), 0, s, L, 2, dg);
}

hipError_t launch_distribute(int p, int prec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, int slot) {
    if (nprob <= 0) return hipSuccess;
    LaunchTable L{};
    L.nprob = nprob;
    L.total_tiles = tiles_red(ents, nprob);
    hipError_t err = stage_table(L, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    const int grid = L.total_tiles < kMaxGrid ? L.total_tiles : kMaxGrid;
    err = dispatch_prec(prec, [&](auto tag) {
        using S = decltype(tag);
        switch (p) {
            case 1: launch_distribute_pt<1, S>(L, grid, s); break;
            case 2: launch_distribute_pt<2, S>(L, grid, s); break;
            case 3: launch_distribute_pt<3, S>(L, grid, s); break;
            case 4: launch_distribute_pt<4, S>(L, grid, s); break;
            case 5: launch_distribute_pt<5, S>(L, grid, s); break;
            case 6: launch_distribute_pt<6, S>(L, grid, s); break;
            case 7: launch_distribute_pt<7, S>(L, grid, s); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    });
    if (err != hipSuccess) return err;
    return final_multi(L, s, 2, slot);
}

// Mixed-degree norm passes (the FP64 assembled norm, or the norm with the
// smoother's copy of the residual): one item per reduction tile; the
// per-problem finals run over the whole table.
template <int P, typename S>
struct AnormBody {
    using Arg = NoArg;
    static constexpr int kLds = 4 * sizeof(double);
    __device__ static __forceinline__ void run(const LaunchTable& L, const NoArg&, int item, int items, char* smem) {
        anorm_body<P, S, true>(L, 1, item, items, smem);
    }
};

template <int P, typename RS>
struct DistributeBody {
    using Arg = NoArg;
    static constexpr int kLds = 4 * sizeof(double);
    __device__ static __forceinline__ void run(const LaunchTable& L, const NoArg&, int item, int items, char* smem) {
        distribute_body<P, RS, kDistMean, true>(L, 2, Diag1D{}, item, items, smem);
    }
};

static hipError_t launch_norm_mixed(int kind, int prec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s,
                                    int slot) {
    static_assert(mix_degree(0) == 7 && mix_degree(1) == 3 && mix_degree(2) == 2, "segment degrees");
    MixTable T{};
    int grid = 0;
    auto tiles = [](int, const ProbEntry& e) { return e.ntiles_red; };
    auto items = [](int, int t) { return t; };
    hipError_t err = mix_build(ents, nprob, st, s, tiles, items, T, grid);
    if (err != hipSuccess) return err;
    if (grid > 0) {
        if (kind == 1) {
            TraceSpan ts("anorm", 0, FEM_F64, s);
            hipLaunchKernelGGL((k_mixed<AnormBody<7, double>, AnormBody<3, double>, AnormBody<2, double>>), dim3(grid),
                               dim3(256), 0, s, T, NoArg{}, NoArg{}, NoArg{});
        } else {
            err = dispatch_prec(prec, [&](auto tag) {
                using S = decltype(tag);
                TraceSpan ts("distribute", 0, Prec<S>::id, s);
                hipLaunchKernelGGL((k_mixed<DistributeBody<7, S>, DistributeBody<3, S>, DistributeBody<2, S>>),
                                   dim3(grid), dim3(256), 0, s, T, NoArg{}, NoArg{}, NoArg{});
                return hipGetLastError();
            });
        }
        if (err == hipSuccess) err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    // the whole table (segment 0 starts it) for the per-problem finals
    LaunchTable Lall{};
    Lall.nprob = nprob;
    Lall.tab = T.seg[0].L.tab;
    return final_multi(Lall, s, kind, slot);
}

hipError_t launch_norm_any(int smoother_prec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, int slot,
                           bool mix) {
    if (nprob <= 0) return hipSuccess;
    const int kind = smoother_prec == FEM_F64 ? 1 : 2;
    if (mix && mix_degrees(ents, nprob) >= 2) return launch_norm_mixed(kind, smoother_prec, ents, nprob, st, s, slot);
    std::vector<ProbEntry> g;
    for (int p = 1; p <= kMaxP; ++p) {
        g.clear();
        for (int i = 0; i < nprob; ++i)
            if (ents[i].p == p) g.push_back(ents[i]);
        if (g.empty()) continue;
        hipError_t err = kind == 1 ? launch_anorm(p, g.data(), (int)g.size(), st, s, slot)
                                   : launch_distribute(p, smoother_prec, g.data(), (int)g.size(), st, s, slot);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

template <int P>
static void launch_anorm_p(LaunchTable& L, int grid, hipStream_t s) {
    if (L.nprob > 1) hipLaunchKernelGGL((k_anorm<P, double, true>), dim3(grid), dim3(256), 0, s, L, 1);
    else hipLaunchKernelGGL((k_anorm<P, double, false>), dim3(grid), dim3(256), 0, s, L, 1);
}

hipError_t launch_anorm(int p, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, int slot) {
    if (nprob <= 0) return hipSuccess;
    LaunchTable L{};
    L.nprob = nprob;
    L.total_tiles = tiles_red(ents, nprob);
    hipError_t err = stage_table(L, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    const int grid = L.total_tiles < kMaxGrid ? L.total_tiles : kMaxGrid;
    switch (p) {
        case 1: launch_anorm_p<1>(L, grid, s); break;
        case 2: launch_anorm_p<2>(L, grid, s); break;
        case 3: launch_anorm_p<3>(L, grid, s); break;
        case 4: launch_anorm_p<4>(L, grid, s); break;
        case 5: launch_anorm_p<5>(L, grid, s); break;
        case 6: launch_anorm_p<6>(L, grid, s); break;
        case 7: launch_anorm_p<7>(L, grid, s); break;
        default: return hipErrorInvalidValue;
    }
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    return final_multi(L, s, 1, slot);
}

hipError_t launch_cg_ur(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    LaunchTable L{};
    L.nprob = nprob;
    L.total_tiles = tiles_red(ents, nprob);
    hipError_t err = stage_table(L, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    const int grid = L.total_tiles < kMaxGrid ? L.total_tiles : kMaxGrid;
    if (nprob > 1) hipLaunchKernelGGL((k_cg_ur<double, true>), dim3(grid), dim3(256), 0, s, L);
    else hipLaunchKernelGGL((k_cg_ur<double, false>), dim3(grid), dim3(256), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_cg_p(int zprec, int variant, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    LaunchTable L{};
    L.nprob = nprob;
    L.total_tiles = tiles_red(ents, nprob);
    hipError_t err = stage_table(L, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    const int grid = L.total_tiles < kMaxGrid ? L.total_tiles : kMaxGrid;
    return dispatch_prec(zprec, [&](auto tag) {
        using S = decltype(tag);
        if (nprob > 1) hipLaunchKernelGGL((k_cg_p<S, true>), dim3(grid), dim3(256), 0, s, L, variant);
        else hipLaunchKernelGGL((k_cg_p<S, false>), dim3(grid), dim3(256), 0, s, L, variant);
        return hipGetLastError();
    });
}

hipError_t launch_dot_qz_rz(int zprec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    LaunchTable L{};
    L.nprob = nprob;
    L.total_tiles = tiles_red(ents, nprob);
    hipError_t err = stage_table(L, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    const int grid = L.total_tiles < kMaxGrid ? L.total_tiles : kMaxGrid;
    err = dispatch_prec(zprec, [&](auto tag) {
        using S = decltype(tag);
        if (nprob > 1) hipLaunchKernelGGL((k_dot_qz_rz<S, true>), dim3(grid), dim3(256), 0, s, L);
        else hipLaunchKernelGGL((k_dot_qz_rz<S, false>), dim3(grid), dim3(256), 0, s, L);
        return hipGetLastError();
    });
    if (err != hipSuccess) return err;
    err = final_multi(L, s, 0, kSlotQZ);
    if (err != hipSuccess) return err;
    return final_multi(L, s, 3, kSlotRZ);
}

hipError_t launch_slot_copy(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, int dst, int src) {
    if (nprob <= 0) return hipSuccess;
    LaunchTable L{};
    L.nprob = nprob;
    hipError_t err = stage_table(L, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    const int grid = (nprob + 63) / 64;
    if (nprob > 1) hipLaunchKernelGGL(k_slot_copy<true>, dim3(grid), dim3(64), 0, s, L, dst, src);
    else hipLaunchKernelGGL(k_slot_copy<false>, dim3(grid), dim3(64), 0, s, L, dst, src);
    return hipGetLastError();
}

hipError_t launch_solve_init(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    LaunchTable L{};
    L.nprob = nprob;
    hipError_t err = stage_table(L, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    const int grid = (nprob + 63) / 64;
    if (nprob > 1) hipLaunchKernelGGL(k_solve_init<true>, dim3(grid), dim3(64), 0, s, L);
    else hipLaunchKernelGGL(k_solve_init<false>, dim3(grid), dim3(64), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_cg_check(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    LaunchTable L{};
    L.nprob = nprob;
    hipError_t err = stage_table(L, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    const int grid = (nprob + 63) / 64;
    if (nprob > 1) hipLaunchKernelGGL(k_cg_check<true>, dim3(grid), dim3(64), 0, s, L);
    else hipLaunchKernelGGL(k_cg_check<false>, dim3(grid), dim3(64), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_collect_slots(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, int sa, int sb,
                                double* out) {
    if (nprob <= 0) return hipSuccess;
    LaunchTable L{};
    L.nprob = nprob;
    hipError_t err = stage_table(L, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    const int grid = (nprob + 63) / 64;
    if (nprob > 1) hipLaunchKernelGGL(k_collect_slots<true>, dim3(grid), dim3(64), 0, s, L, sa, sb, out);
    else hipLaunchKernelGGL(k_collect_slots<false>, dim3(grid), dim3(64), 0, s, L, sa, sb, out);
    return hipGetLastError();
}

hipError_t launch_convert(int sp, int dp, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    LaunchTable L{};
    L.nprob = nprob;
    L.total_tiles = tiles_red(ents, nprob);
    hipError_t err = stage_table(L, ents, nprob, st, s);
    if (err != hipSuccess) return err;
    const int grid = L.total_tiles < kMaxGrid ? L.total_tiles : kMaxGrid;
    return dispatch_prec(sp, [&](auto ta) {
        using SA = decltype(ta);
        return dispatch_prec(dp, [&](auto tb) {
            using SB = decltype(tb);
            if (nprob > 1) hipLaunchKernelGGL((k_convert_multi<SA, SB, true>), dim3(grid), dim3(256), 0, s, L);
            else hipLaunchKernelGGL((k_convert_multi<SA, SB, false>), dim3(grid), dim3(256), 0, s, L);
            return hipGetLastError();
        });
    });
}

// ------------------------------------------------------------- stager
hipError_t TableStager::init(int cap_entries) {
    cap = cap_entries;
    const size_t slot = sizeof(ProbEntry) * cap;
    hipError_t e = hipHostMalloc((void**)&host_block, slot * kSlots, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    e = hipMalloc((void**)&dev_block, slot * kSlots);
    if (e != hipSuccess) return e;
    for (int i = 0; i < kSlots; ++i) {
        host[i] = host_block + (size_t)i * cap;
        dev[i] = dev_block + (size_t)i * cap;
        e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
        if (e != hipSuccess) return e;
        used[i] = false;
    }
    return hipSuccess;
}

void TableStager::destroy() {
    for (int i = 0; i < kSlots; ++i) {
        if (used[i]) hipEventSynchronize(ev[i]);
        if (ev[i]) hipEventDestroy(ev[i]);
        host[i] = nullptr;
        dev[i] = nullptr;
        ev[i] = nullptr;
        used[i] = false;
    }
    if (host_block) hipHostFree(host_block);
    if (dev_block) hipFree(dev_block);
    host_block = nullptr;
    dev_block = nullptr;
}

hipError_t TableStager::upload(const ProbEntry* ents, int n, hipStream_t s, const ProbEntry** out) {
    if (n > cap) return hipErrorInvalidValue;
    const int k = next;
    next = (next + 1) % kSlots;
    if (used[k]) {
        hipError_t e = hipEventSynchronize(ev[k]);
        if (e != hipSuccess) return e;
    }
    std::memcpy(host[k], ents, sizeof(ProbEntry) * n);
    hipError_t e = hipMemcpyAsync(dev[k], host[k], sizeof(ProbEntry) * n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipEventRecord(ev[k], s);
    used[k] = true;
    *out = dev[k];
    return e;
}

}  // namespace fem
