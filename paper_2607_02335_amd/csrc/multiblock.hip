// Direct stiffness summation on multi-block meshes (Section 4.2, Algorithm
// "Unstructured Inter-Block Summation").
//
// A multi-block mesh is a set of blocks, each n[0] x n[1] x n[2] cells of
// degree p in its own local axes, glued along whole block faces in any
// relative orientation.  Its cell-wise vector is the blocks' cell-wise
// vectors one after another (each in the library's blocked layout).  The
// summation runs in two stages that touch disjoint sets of copies' sources:
//   1. the structured cascade inside every block (three axis passes);
//   2. the inter-block skeleton, split by the cell-level entity a node lies
//      in, each in its own launch writing disjoint copies:
//      faces    nodes interior to a cell face on a shared block face: exactly
//               one copy per side; the pair is summed and written back to
//               both, side b's index computed from side a's by the face's
//               orientation bits (axis swap, flips), no lookup;
//      lines    nodes interior to a cell edge on the skeleton, and
//      vertices cell corners on the skeleton: copies in several cells of
//               several blocks.  Stage 1 left every block's copies equal, so
//               one representative copy per block enters the sum, which is
//               then written to every copy (sharing lists padded to a fixed
//               width per launch).
// The sharing lists come from the block topology (corner vertex ids): the
// face orientations from the matching corner ids, the line and vertex
// classes from a union-find over the block faces' lattice nodes glued by
// those orientations.
#include <algorithm>
#include <array>
#include <map>
#include <new>
#include <numeric>
#include <vector>

#include "fem_internal.h"
#include "host_api.h"
#include "launch.h"
#include "trace.h"

using namespace fem;

namespace fem {
namespace {

// One shared block face: side a's face-local node (U, V) (U along the first,
// V along the second of the face's two block axes in increasing order) is
// side b's (U', V'):  swap ? (fu ? Nu' - V : V, fv ? Nv' - U : U)
//                          : (fu ? Nu' - U : U, fv ? Nv' - V : V).
struct MbFace {
    int ba, fa, bb, fb;      // blocks and faces (2 axis + side)
    int swap, fu, fv;        // orientation bits
    int cu, cv;              // cells of side a along U and V
    long long off_a, off_b;  // element offsets of the two blocks
    int na[3], nb[3];        // cells per direction of the two blocks
    int tile_begin;          // first thread of this face in the launch
};

__device__ __forceinline__ void face_axes(int f, int& ax, int& side, int& au, int& av) {
    ax = f >> 1;
    side = f & 1;
    au = ax == 0 ? 1 : 0;
    av = ax == 2 ? 1 : 2;
}

// element offset of block-lattice node (I, J, K) in the lowest cell holding it
template <int P>
__device__ __forceinline__ long long lattice_copy(long long off, const int* n, int I, int J, int K) {
    constexpr int N = P + 1, NN = N * N * N;
    const int L[3] = {I, J, K};
    int c[3], l[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c[d] = L[d] / P;
        if (c[d] == n[d]) c[d] -= 1;
        l[d] = L[d] - c[d] * P;
    }
    const int e = c[0] + n[0] * (c[1] + n[1] * c[2]);
    return off + (long long)cell_offset(e, l[0] + N * (l[1] + N * l[2]), NN);
}

template <int P, typename S>
__global__ void __launch_bounds__(256) k_mb_faces(const MbFace* __restrict__ faces, int nfaces, int total, S* v) {
    using C = typename Prec<S>::C;
    if constexpr (P == 1) return;      // p = 1: every shared node is a cell corner
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    int lo = 0, hi = nfaces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (faces[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const MbFace& F = faces[lo];
    int r = t - F.tile_begin;
    // (cell u, node u in 1..p-1, cell v, node v in 1..p-1), u fastest
    constexpr int PM = P > 1 ? P - 1 : 1;
    const int uu = 1 + r % PM;
    r /= PM;
    const int cu = r % F.cu;
    r /= F.cu;
    const int vv = 1 + r % PM;
    const int cv = r / PM;
    const int U = cu * P + uu, V = cv * P + vv;
    int ax, side, au, av;
    face_axes(F.fa, ax, side, au, av);
    int La[3];
    La[ax] = side ? F.na[ax] * P : 0;
    La[au] = U;
    La[av] = V;
    int bx, bside, bu, bv;
    face_axes(F.fb, bx, bside, bu, bv);
    const int Nu = F.nb[bu] * P, Nv = F.nb[bv] * P;
    const int Ub = F.swap ? (F.fu ? Nu - V : V) : (F.fu ? Nu - U : U);
    const int Vb = F.swap ? (F.fv ? Nv - U : U) : (F.fv ? Nv - V : V);
    int Lb[3];
    Lb[bx] = bside ? F.nb[bx] * P : 0;
    Lb[bu] = Ub;
    Lb[bv] = Vb;
    S* pa = v + lattice_copy<P>(F.off_a, F.na, La[0], La[1], La[2]);
    S* pb = v + lattice_copy<P>(F.off_b, F.nb, Lb[0], Lb[1], Lb[2]);
    const C s = load_as<C>(pa) + load_as<C>(pb);
    store_from(pa, s);
    store_from(pb, s);
}

// lines / vertices: entity k has nrep[k] representatives (one per block) at
// rep[k * WR + i] and ncopy[k] copies at copy[k * WC + i]
template <typename S>
__global__ void __launch_bounds__(256) k_mb_gather(int nent, const int* __restrict__ nrep,
                                                   const long long* __restrict__ rep, int WR,
                                                   const int* __restrict__ ncopy,
                                                   const long long* __restrict__ copy, int WC, S* v) {
    using C = typename Prec<S>::C;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= nent) return;
    C s = 0;
    for (int i = 0; i < WR; ++i)
        if (i < nrep[k]) s = s + load_as<C>(v + rep[(size_t)k * WR + i]);
    for (int i = 0; i < WC; ++i)
        if (i < ncopy[k]) store_from(v + copy[(size_t)k * WC + i], s);
}

struct UF {
    std::vector<long long> par;
    explicit UF(size_t n) : par(n) { std::iota(par.begin(), par.end(), 0LL); }
    long long find(long long x) {
        while (par[x] != x) {
            par[x] = par[par[x]];
            x = par[x];
        }
        return x;
    }
    void join(long long a, long long b) {
        a = find(a);
        b = find(b);
        if (a != b) par[std::max(a, b)] = std::min(a, b);
    }
};

}  // namespace
}  // namespace fem

struct fem_mb_plan {
    int p = 0, nb = 0;
    std::vector<std::array<int, 3>> n;
    std::vector<long long> off;          // element offset of each block
    long long cell_len = 0;
    hipStream_t stream = nullptr;
    std::vector<MbFace> faces;
    int face_threads = 0;
    MbFace* d_faces = nullptr;
    // line and vertex entities
    int nent[2] = {0, 0}, WR[2] = {0, 0}, WC[2] = {0, 0};
    int* d_nrep[2] = {nullptr, nullptr};
    int* d_ncopy[2] = {nullptr, nullptr};
    long long* d_rep[2] = {nullptr, nullptr};
    long long* d_copy[2] = {nullptr, nullptr};
};

static void mb_free(fem_mb_plan* M) {
    if (!M) return;
    hipFree(M->d_faces);
    for (int t = 0; t < 2; ++t) {
        hipFree(M->d_nrep[t]);
        hipFree(M->d_ncopy[t]);
        hipFree(M->d_rep[t]);
        hipFree(M->d_copy[t]);
    }
    delete M;
}

extern "C" fem_status fem_mb_create(int p, int nblocks, const int* block_n, const int* corners, void* stream,
                                    fem_mb_plan** out) {
    if (!out) return set_error(FEM_EINVAL, "fem_mb_create: out is NULL");
    *out = nullptr;
    if (p < 1 || p > kMaxP || nblocks < 1 || !block_n || !corners)
        return set_error(FEM_EINVAL, "fem_mb_create: p in 1..7, nblocks >= 1, arrays required");
    fem_mb_plan* M = new (std::nothrow) fem_mb_plan();
    if (!M) return set_error(FEM_ENOMEM, "host allocation failed");
    M->p = p;
    M->nb = nblocks;
    M->stream = static_cast<hipStream_t>(stream);
    const int NN = (p + 1) * (p + 1) * (p + 1);
    std::vector<long long> lat_off(nblocks + 1, 0);         // union-find ids of block lattices
    for (int b = 0; b < nblocks; ++b) {
        std::array<int, 3> nn{block_n[3 * b], block_n[3 * b + 1], block_n[3 * b + 2]};
        for (int d = 0; d < 3; ++d)
            if (nn[d] < 1) {
                mb_free(M);
                return set_error(FEM_EINVAL, "fem_mb_create: cells per direction must be >= 1");
            }
        M->n.push_back(nn);
        M->off.push_back(M->cell_len);
        const long long cells = (long long)nn[0] * nn[1] * nn[2];
        M->cell_len += (cells + kLanes - 1) / kLanes * kLanes * NN;
        lat_off[b + 1] = lat_off[b] + (long long)(nn[0] * p + 1) * (nn[1] * p + 1) * (nn[2] * p + 1);
    }
    auto corner_of = [&](int b, int f, int cu, int cv) {
        const int ax = f >> 1, side = f & 1;
        const int au = ax == 0 ? 1 : 0, av = ax == 2 ? 1 : 2;
        const int c = (side << ax) | (cu << au) | (cv << av);
        return corners[8 * b + c];
    };
    // shared faces: matched by their sorted corner ids
    std::map<std::array<int, 4>, std::vector<std::pair<int, int>>> fmap;
    for (int b = 0; b < nblocks; ++b)
        for (int f = 0; f < 6; ++f) {
            std::array<int, 4> key{corner_of(b, f, 0, 0), corner_of(b, f, 1, 0), corner_of(b, f, 0, 1),
                                   corner_of(b, f, 1, 1)};
            std::sort(key.begin(), key.end());
            fmap[key].emplace_back(b, f);
        }
    UF uf((size_t)lat_off[nblocks]);
    auto lat_id = [&](int b, int I, int J, int K) {
        const auto& nn = M->n[b];
        return lat_off[b] + I + (long long)(nn[0] * p + 1) * (J + (long long)(nn[1] * p + 1) * K);
    };
    for (auto& kv : fmap) {
        if (kv.second.size() == 1) continue;                  // domain boundary
        if (kv.second.size() > 2) {
            mb_free(M);
            return set_error(FEM_EINVAL, "fem_mb_create: a face is shared by more than two blocks");
        }
        const int ba = kv.second[0].first, fa = kv.second[0].second;
        const int bb = kv.second[1].first, fb = kv.second[1].second;
        // where side a's face corners (0,0), (1,0), (0,1) sit on side b
        int uv[3][2];
        const int cc[3][2] = {{0, 0}, {1, 0}, {0, 1}};
        for (int q = 0; q < 3; ++q) {
            const int id = corner_of(ba, fa, cc[q][0], cc[q][1]);
            uv[q][0] = uv[q][1] = -1;
            for (int cu = 0; cu < 2; ++cu)
                for (int cv = 0; cv < 2; ++cv)
                    if (corner_of(bb, fb, cu, cv) == id) {
                        uv[q][0] = cu;
                        uv[q][1] = cv;
                    }
        }
        MbFace F{};
        F.ba = ba; F.fa = fa; F.bb = bb; F.fb = fb;
        F.swap = uv[1][0] == uv[0][0];
        F.fu = uv[0][0] == 1;
        F.fv = uv[0][1] == 1;
        const int ax = fa >> 1, au = ax == 0 ? 1 : 0, av = ax == 2 ? 1 : 2;
        const int bx = fb >> 1, bu = bx == 0 ? 1 : 0, bv = bx == 2 ? 1 : 2;
        for (int d = 0; d < 3; ++d) {
            F.na[d] = M->n[ba][d];
            F.nb[d] = M->n[bb][d];
        }
        // side a's U axis meets side b's U (or V when swapped): lengths must agree
        const int la_u = F.na[au], la_v = F.na[av];
        const int lb_u = F.swap ? F.nb[bv] : F.nb[bu], lb_v = F.swap ? F.nb[bu] : F.nb[bv];
        if (la_u != lb_u || la_v != lb_v) {
            mb_free(M);
            return set_error(FEM_EINVAL, "fem_mb_create: glued faces have different cell counts");
        }
        F.cu = la_u;
        F.cv = la_v;
        F.off_a = M->off[ba];
        F.off_b = M->off[bb];
        F.tile_begin = M->face_threads;
        if (p >= 2) M->face_threads += F.cu * (p - 1) * F.cv * (p - 1);
        M->faces.push_back(F);
        // glue the whole face lattice (interior and boundary) in the union-find
        const int Nu = la_u * p, Nv = la_v * p, Nbu = F.nb[bu] * p, Nbv = F.nb[bv] * p;
        for (int V = 0; V <= Nv; ++V)
            for (int U = 0; U <= Nu; ++U) {
                int La[3], Lb[3];
                La[ax] = (fa & 1) ? F.na[ax] * p : 0;
                La[au] = U;
                La[av] = V;
                const int Ub = F.swap ? (F.fu ? Nbu - V : V) : (F.fu ? Nbu - U : U);
                const int Vb = F.swap ? (F.fv ? Nbv - U : U) : (F.fv ? Nbv - V : V);
                Lb[bx] = (fb & 1) ? F.nb[bx] * p : 0;
                Lb[bu] = Ub;
                Lb[bv] = Vb;
                uf.join(lat_id(ba, La[0], La[1], La[2]), lat_id(bb, Lb[0], Lb[1], Lb[2]));
            }
    }
    // classes of glued lattice nodes: cell-edge interior (lines) and cell
    // corners (vertices) get sharing lists
    std::map<long long, std::vector<std::array<int, 4>>> cls;   // root -> block lattice nodes
    for (int b = 0; b < nblocks; ++b) {
        const auto& nn = M->n[b];
        const int N0 = nn[0] * p, N1 = nn[1] * p, N2 = nn[2] * p;
        for (int K = 0; K <= N2; ++K)
            for (int J = 0; J <= N1; ++J)
                for (int I = 0; I <= N0; ++I) {
                    const bool bnd = I == 0 || I == N0 || J == 0 || J == N1 || K == 0 || K == N2;
                    if (!bnd) continue;
                    cls[uf.find(lat_id(b, I, J, K))].push_back({b, I, J, K});
                }
    }
    std::vector<int> nrep[2], ncopy[2];
    std::vector<std::vector<long long>> reps[2], copies[2];
    for (auto& kv : cls) {
        if (kv.second.size() < 2) continue;
        const auto& m0 = kv.second[0];
        int zeros = 0;
        for (int d = 0; d < 3; ++d) zeros += (m0[1 + d] % p) == 0;
        if (p == 1) zeros = 3;
        if (zeros == 1) continue;                       // cell-face interior: the face pass
        const int t = zeros == 2 ? 0 : 1;               // 0 lines, 1 vertices
        std::vector<long long> rl, cl;
        for (const auto& bn : kv.second) {
            const int b = bn[0];
            const auto& nn = M->n[b];
            const int L[3] = {bn[1], bn[2], bn[3]};
            // cells of the block holding this lattice node (ascending), and
            // the node's local index in each
            int cs[3][2], ls[3][2], nc[3];
            for (int d = 0; d < 3; ++d) {
                nc[d] = 0;
                const int q = L[d] / p, rr = L[d] - q * p;
                if (rr == 0) {
                    if (q >= 1) { cs[d][nc[d]] = q - 1; ls[d][nc[d]] = p; ++nc[d]; }
                    if (q <= nn[d] - 1) { cs[d][nc[d]] = q; ls[d][nc[d]] = 0; ++nc[d]; }
                } else {
                    cs[d][0] = q; ls[d][0] = rr; nc[d] = 1;
                }
            }
            bool first = true;
            for (int z = 0; z < nc[2]; ++z)
                for (int y = 0; y < nc[1]; ++y)
                    for (int x = 0; x < nc[0]; ++x) {
                        const int e = cs[0][x] + nn[0] * (cs[1][y] + nn[1] * cs[2][z]);
                        const int l = ls[0][x] + (p + 1) * (ls[1][y] + (p + 1) * ls[2][z]);
                        const long long o = M->off[b] + (long long)cell_offset(e, l, NN);
                        if (first) rl.push_back(o);
                        first = false;
                        cl.push_back(o);
                    }
        }
        nrep[t].push_back((int)rl.size());
        ncopy[t].push_back((int)cl.size());
        M->WR[t] = std::max(M->WR[t], (int)rl.size());
        M->WC[t] = std::max(M->WC[t], (int)cl.size());
        reps[t].push_back(std::move(rl));
        copies[t].push_back(std::move(cl));
    }
    hipError_t e = hipSuccess;
    if (!M->faces.empty()) {
        e = hipMalloc((void**)&M->d_faces, sizeof(MbFace) * M->faces.size());
        if (e == hipSuccess)
            e = hipMemcpy(M->d_faces, M->faces.data(), sizeof(MbFace) * M->faces.size(), hipMemcpyHostToDevice);
    }
    for (int t = 0; t < 2 && e == hipSuccess; ++t) {
        M->nent[t] = (int)nrep[t].size();
        if (M->nent[t] == 0) continue;
        std::vector<long long> R((size_t)M->nent[t] * M->WR[t], 0), Cp((size_t)M->nent[t] * M->WC[t], 0);
        for (int k = 0; k < M->nent[t]; ++k) {
            std::copy(reps[t][k].begin(), reps[t][k].end(), R.begin() + (size_t)k * M->WR[t]);
            std::copy(copies[t][k].begin(), copies[t][k].end(), Cp.begin() + (size_t)k * M->WC[t]);
        }
        e = hipMalloc((void**)&M->d_nrep[t], sizeof(int) * M->nent[t]);
        if (e == hipSuccess) e = hipMalloc((void**)&M->d_ncopy[t], sizeof(int) * M->nent[t]);
        if (e == hipSuccess) e = hipMalloc((void**)&M->d_rep[t], sizeof(long long) * R.size());
        if (e == hipSuccess) e = hipMalloc((void**)&M->d_copy[t], sizeof(long long) * Cp.size());
        if (e == hipSuccess) e = hipMemcpy(M->d_nrep[t], nrep[t].data(), sizeof(int) * M->nent[t], hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(M->d_ncopy[t], ncopy[t].data(), sizeof(int) * M->nent[t], hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(M->d_rep[t], R.data(), sizeof(long long) * R.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(M->d_copy[t], Cp.data(), sizeof(long long) * Cp.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        mb_free(M);
        return hip_error(e, "fem_mb_create upload");
    }
    *out = M;
    return FEM_OK;
}

extern "C" fem_status fem_mb_destroy(fem_mb_plan* M) {
    if (!M) return FEM_OK;
    hipStreamSynchronize(M->stream);
    mb_free(M);
    return FEM_OK;
}

extern "C" size_t fem_mb_cell_len(const fem_mb_plan* M) { return M ? (size_t)M->cell_len : 0; }

extern "C" size_t fem_mb_block_offset(const fem_mb_plan* M, int b) {
    return (M && b >= 0 && b < M->nb) ? (size_t)M->off[b] : 0;
}

extern "C" fem_status fem_mb_stats(const fem_mb_plan* M, int* out, int n) {
    if (!M || !out) return set_error(FEM_EINVAL, "fem_mb_stats: NULL argument");
    const int v[6] = {(int)M->faces.size(), M->face_threads, M->nent[0], M->WC[0], M->nent[1], M->WC[1]};
    for (int i = 0; i < n && i < 6; ++i) out[i] = v[i];
    return FEM_OK;
}

namespace {
template <int P, typename S>
hipError_t mb_launch(fem_mb_plan* M, S* v) {
    hipStream_t s = M->stream;
    if (M->face_threads > 0) {
        TraceSpan ts("mb_faces", P, Prec<S>::id, s);
        hipLaunchKernelGGL((k_mb_faces<P, S>), dim3((M->face_threads + 255) / 256), dim3(256), 0, s, M->d_faces,
                           (int)M->faces.size(), M->face_threads, v);
    }
    for (int t = 0; t < 2; ++t) {
        if (M->nent[t] == 0) continue;
        TraceSpan ts(t == 0 ? "mb_lines" : "mb_vertices", P, Prec<S>::id, s);
        hipLaunchKernelGGL((k_mb_gather<S>), dim3((M->nent[t] + 255) / 256), dim3(256), 0, s, M->nent[t],
                           M->d_nrep[t], M->d_rep[t], M->WR[t], M->d_ncopy[t], M->d_copy[t], M->WC[t], v);
    }
    return hipGetLastError();
}

template <typename S>
hipError_t mb_dispatch(fem_mb_plan* M, S* v) {
    switch (M->p) {
        case 1: return mb_launch<1, S>(M, v);
        case 2: return mb_launch<2, S>(M, v);
        case 3: return mb_launch<3, S>(M, v);
        case 4: return mb_launch<4, S>(M, v);
        case 5: return mb_launch<5, S>(M, v);
        case 6: return mb_launch<6, S>(M, v);
        case 7: return mb_launch<7, S>(M, v);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

static fem_status mb_pack(fem_mb_plan* M, const double* canon, void* v, int prec, int unpack) {
    const size_t es = prec == FEM_F64 ? 8 : prec == FEM_F32 ? 4 : 2;
    const int NN = (M->p + 1) * (M->p + 1) * (M->p + 1);
    size_t coff = 0;
    for (int b = 0; b < M->nb; ++b) {
        ProbEntry e{};
        for (int d = 0; d < 3; ++d) e.n[d] = M->n[b][d];
        e.p = M->p;
        e.ncells = M->n[b][0] * M->n[b][1] * M->n[b][2];
        e.nblk = (e.ncells + kLanes - 1) / kLanes;
        e.len = (size_t)e.nblk * NN * kLanes;
        FEM_HIP(run_pack_entry(e, canon + coff, static_cast<char*>(v) + (size_t)M->off[b] * es, prec, unpack,
                               M->stream),
                "fem_mb_pack");
        coff += (size_t)e.ncells * NN;
    }
    return FEM_OK;
}

extern "C" fem_status fem_mb_pack(fem_mb_plan* M, const double* canon, void* v, int prec) {
    if (!M || !canon || !v) return set_error(FEM_EINVAL, "fem_mb_pack: NULL argument");
    if (prec != FEM_F64 && prec != FEM_F32 && prec != FEM_BF16 && prec != FEM_F16)
        return set_error(FEM_EINVAL, "unknown precision");
    return mb_pack(M, canon, v, prec, 0);
}

extern "C" fem_status fem_mb_unpack(fem_mb_plan* M, const void* v, double* canon, int prec) {
    if (!M || !canon || !v) return set_error(FEM_EINVAL, "fem_mb_unpack: NULL argument");
    if (prec != FEM_F64 && prec != FEM_F32 && prec != FEM_BF16 && prec != FEM_F16)
        return set_error(FEM_EINVAL, "unknown precision");
    return mb_pack(M, canon, const_cast<void*>(v), prec, 1);
}

extern "C" fem_status fem_mb_dss(fem_mb_plan* M, void* v, int prec, int stages) {
    if (!M || !v) return set_error(FEM_EINVAL, "fem_mb_dss: NULL argument");
    if (prec != FEM_F64 && prec != FEM_F32 && prec != FEM_BF16 && prec != FEM_F16)
        return set_error(FEM_EINVAL, "unknown precision");
    if (stages < 1 || stages > 3) return set_error(FEM_EINVAL, "fem_mb_dss: stages is 1, 2 or 3");
    const size_t es = prec == FEM_F64 ? 8 : prec == FEM_F32 ? 4 : 2;
    if (stages & 1) {
        for (int b = 0; b < M->nb; ++b) {
            ProbEntry e{};
            for (int d = 0; d < 3; ++d) e.n[d] = M->n[b][d];
            e.p = M->p;
            e.c = static_cast<char*>(v) + (size_t)M->off[b] * es;
            for (int axis = 2; axis >= 0; --axis)
                FEM_HIP(run_dss_axis_entry(M->p, e, axis, prec, M->stream), "fem_mb_dss structured");
        }
    }
    if (stages & 2) {
        hipError_t err;
        if (prec == FEM_F64) err = mb_dispatch(M, static_cast<double*>(v));
        else if (prec == FEM_F32) err = mb_dispatch(M, static_cast<float*>(v));
        else if (prec == FEM_F16) err = mb_dispatch(M, static_cast<f16_t*>(v));
        else err = mb_dispatch(M, static_cast<bf16_t*>(v));
        FEM_HIP(err, "fem_mb_dss inter-block");
    }
    return FEM_OK;
}
