// Layout study: the storage block size B of the blocked element-fastest
// layout (Section 5.1, "BXYZE"), swept for the two kinds of kernel it trades
// off against each other (Section 6.1, "Layout study"): the volumetric mass
// apply, which streams whole cells, and the structured DSS, whose face
// exchanges are coalesced only when many cells of a block sit side by side.
//
// A vector of the layout with block size B stores cell e's local node l at
//     offset_B(e, l) = (e / B) (p+1)^3 B + l B + e % B
// (the library's own vectors are B = 64).  These kernels serve the study
// only: FP64, a uniform cube mesh of n[0] x n[1] x n[2] cells of width h per
// direction, no boundary conditions (the plain mass operator M and the plain
// S = G G^T), degrees 2..5.
#include "fem_internal.h"
#include "host_api.h"
#include "launch.h"
#include "trace.h"

namespace fem {
namespace {

template <int B>
__host__ __device__ __forceinline__ size_t lay_off(long e, int l, int nn) {
    return (size_t)(e / B) * nn * B + (size_t)l * B + (size_t)(e % B);
}

template <int P>
struct LayMass {
    double M[(P + 1) * (P + 1)];
};

// y = vol (M (x) M (x) M) x per cell: CB cells per workgroup tile staged in
// LDS, one thread per 1D line in each of the three passes
template <int P, int B, int CB>
__global__ void __launch_bounds__(256) k_lay_mass(const double* __restrict__ x, double* __restrict__ y, long ncells,
                                                  double vol, LayMass<P> R) {
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    constexpr int NT = 256;
    __shared__ double s0[NN * CB];
    const int tid = threadIdx.x;
    const int c = tid % CB;
    const long ntiles = (ncells + CB - 1) / CB;
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long e = tile * CB + c;
        const bool valid = e < ncells;
        for (int l = tid / CB; l < NN; l += NT / CB) s0[l * CB + c] = valid ? x[lay_off<B>(e, l, NN)] : 0.0;
        __syncthreads();
        for (int ab = tid / CB; ab < N2; ab += NT / CB) {          // z lines
            double v[N];
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = s0[(ab + N2 * k) * CB + c];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                double s = 0;
#pragma unroll
                for (int m = 0; m < N; ++m) s += R.M[k * N + m] * v[m];
                s0[(ab + N2 * k) * CB + c] = s;
            }
        }
        __syncthreads();
        for (int r = tid / CB; r < N2; r += NT / CB) {             // y lines, r = a + N k
            const int a = r % N, k = r / N;
            double v[N];
#pragma unroll
            for (int b = 0; b < N; ++b) v[b] = s0[(a + N * b + N2 * k) * CB + c];
#pragma unroll
            for (int b = 0; b < N; ++b) {
                double s = 0;
#pragma unroll
                for (int m = 0; m < N; ++m) s += R.M[b * N + m] * v[m];
                s0[(a + N * b + N2 * k) * CB + c] = s;
            }
        }
        __syncthreads();
        for (int r = tid / CB; r < N2; r += NT / CB) {             // x lines, r = b + N k
            double v[N];
#pragma unroll
            for (int a = 0; a < N; ++a) v[a] = s0[(a + N * r) * CB + c];
#pragma unroll
            for (int a = 0; a < N; ++a) {
                double s = 0;
#pragma unroll
                for (int m = 0; m < N; ++m) s += R.M[a * N + m] * v[m];
                if (valid) y[lay_off<B>(e, a + N * r, NN)] = vol * s;
            }
        }
        __syncthreads();
    }
}

// one structured axis pass: each face pair across an interface normal to
// `axis` is replaced by its sum on both sides (lanes along x)
template <int P, int B>
__global__ void __launch_bounds__(256) k_lay_dss_axis(double* v, int n0, int n1, int n2, int axis, long total) {
    constexpr int N = P + 1, N2 = N * N, NN = N2 * N;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    long eL, eR;
    int lL, lR;
    if (axis == 0) {
        const int ii = t % (n0 - 1);
        long r = t / (n0 - 1);
        const int fn = r % N2;
        r /= N2;
        const int j = r % n1, k = r / n1;
        eL = ii + (long)n0 * (j + (long)n1 * k);
        eR = eL + 1;
        lL = P + N * fn;
        lR = N * fn;
    } else if (axis == 1) {
        const int i = t % n0;
        long r = t / n0;
        const int jj = r % (n1 - 1);
        r /= (n1 - 1);
        const int fn = r % N2;
        const int k = r / N2;
        const int a = fn % N, c = fn / N;
        eL = i + (long)n0 * (jj + (long)n1 * k);
        eR = eL + n0;
        lL = a + N * (P + N * c);
        lR = a + N * (N * c);
    } else {
        const int i = t % n0;
        long r = t / n0;
        const int j = r % n1;
        r /= n1;
        const int kk = r % (n2 - 1);
        const int fn = r / (n2 - 1);
        eL = i + (long)n0 * (j + (long)n1 * kk);
        eR = eL + (long)n0 * n1;
        lL = fn + N2 * P;
        lR = fn;
    }
    double* pL = v + lay_off<B>(eL, lL, NN);
    double* pR = v + lay_off<B>(eR, lR, NN);
    const double s = *pL + *pR;
    *pL = s;
    *pR = s;
}

__global__ void __launch_bounds__(256) k_lay_zero(double* v, long n) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t < n) v[t] = 0.0;
}

template <int B>
__global__ void __launch_bounds__(256) k_lay_pack(const double* __restrict__ src, double* __restrict__ dst, long n,
                                                  int nn, int unpack) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    const long e = t / nn;
    const int l = (int)(t % nn);
    const size_t o = lay_off<B>(e, l, nn);
    if (unpack) dst[t] = src[o];
    else dst[o] = src[t];
}

template <typename F>
hipError_t by_block(int B, F&& f) {
    switch (B) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 8: return f(std::integral_constant<int, 8>{});
        case 16: return f(std::integral_constant<int, 16>{});
        case 32: return f(std::integral_constant<int, 32>{});
        case 64: return f(std::integral_constant<int, 64>{});
        case 128: return f(std::integral_constant<int, 128>{});
        default: return hipErrorInvalidValue;
    }
}

template <typename F>
hipError_t by_degree(int p, F&& f) {
    switch (p) {
        case 2: return f(std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, 3>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 5: return f(std::integral_constant<int, 5>{});
        default: return hipErrorInvalidValue;
    }
}

fem_status check_layout(int p, const int* n, int B) {
    if (p < 2 || p > 5) return set_error(FEM_EINVAL, "layout study: p in 2..5");
    if (!n || n[0] < 1 || n[1] < 1 || n[2] < 1) return set_error(FEM_EINVAL, "layout study: n >= 1");
    if (B < 1 || B > 128 || (B & (B - 1))) return set_error(FEM_EINVAL, "layout study: B a power of two <= 128");
    return FEM_OK;
}

}  // namespace
}  // namespace fem

using namespace fem;

extern "C" size_t fem_layout_len(int p, const int* n, int B) {
    if (check_layout(p, n, B) != FEM_OK) return 0;
    const size_t nc = (size_t)n[0] * n[1] * n[2];
    return (nc + B - 1) / B * B * (size_t)(p + 1) * (p + 1) * (p + 1);
}

extern "C" fem_status fem_layout_pack(int p, const int* n, int B, const double* src, double* dst, int unpack,
                                      void* stream) {
    fem_status st = check_layout(p, n, B);
    if (st != FEM_OK) return st;
    if (!src || !dst) return set_error(FEM_EINVAL, "fem_layout_pack: NULL vector");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nn = (p + 1) * (p + 1) * (p + 1);
    const long ncell = (long)n[0] * n[1] * n[2];
    const long tot = ncell * nn;
    if (!unpack) {      // padding cells of the last block are zero
        const long len = (long)fem_layout_len(p, n, B);
        hipLaunchKernelGGL(k_lay_zero, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, dst, len);
        FEM_HIP(hipGetLastError(), "fem_layout_pack");
    }
    FEM_HIP(by_block(B, [&](auto b) {
                hipLaunchKernelGGL((k_lay_pack<decltype(b)::value>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                                   s, src, dst, tot, nn, unpack);
                return hipGetLastError();
            }),
            "fem_layout_pack");
    return FEM_OK;
}

extern "C" fem_status fem_layout_mass(int p, const int* n, int B, int tile, const double* x, double* y,
                                      void* stream) {
    fem_status st = check_layout(p, n, B);
    if (st != FEM_OK) return st;
    if (!x || !y || x == y) return set_error(FEM_EINVAL, "fem_layout_mass: bad vectors");
    if (tile != 16 && tile != 32) return set_error(FEM_EINVAL, "fem_layout_mass: tile is 16 or 32 cells");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long ncell = (long)n[0] * n[1] * n[2];
    const double vol = 1.0 / ((double)n[0] * n[1] * n[2]);      // uniform cells of the unit cube
    FEM_HIP(by_degree(p, [&](auto pp) {
                constexpr int P = decltype(pp)::value;
                LayMass<P> R;
                const double* M = ref_mass(P);
                for (int i = 0; i < (P + 1) * (P + 1); ++i) R.M[i] = M[i];
                return by_block(B, [&](auto b) {
                    constexpr int BB = decltype(b)::value;
                    TraceSpan ts("layout_mass", P, FEM_F64, s);
                    const long tiles = (ncell + tile - 1) / tile;
                    const int grid = (int)(tiles < 2048 ? tiles : 2048);
                    if (tile == 16) hipLaunchKernelGGL((k_lay_mass<P, BB, 16>), dim3(grid), dim3(256), 0, s, x, y, ncell, vol, R);
                    else hipLaunchKernelGGL((k_lay_mass<P, BB, 32>), dim3(grid), dim3(256), 0, s, x, y, ncell, vol, R);
                    return hipGetLastError();
                });
            }),
            "fem_layout_mass");
    return FEM_OK;
}

extern "C" fem_status fem_layout_dss(int p, const int* n, int B, double* v, void* stream) {
    fem_status st = check_layout(p, n, B);
    if (st != FEM_OK) return st;
    if (!v) return set_error(FEM_EINVAL, "fem_layout_dss: NULL vector");
    hipStream_t s = static_cast<hipStream_t>(stream);
    FEM_HIP(by_degree(p, [&](auto pp) {
                constexpr int P = decltype(pp)::value;
                constexpr int N = P + 1;
                return by_block(B, [&](auto b) {
                    constexpr int BB = decltype(b)::value;
                    TraceSpan ts("layout_dss", P, FEM_F64, s);
                    for (int axis = 2; axis >= 0; --axis) {
                        long total = (long)n[0] * n[1] * n[2] / n[axis] * (n[axis] - 1) * N * N;
                        if (total <= 0) continue;
                        hipLaunchKernelGGL((k_lay_dss_axis<P, BB>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                                           s, v, n[0], n[1], n[2], axis, total);
                    }
                    return hipGetLastError();
                });
            }),
            "fem_layout_dss");
    return FEM_OK;
}
