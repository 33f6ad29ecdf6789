// Host-side launch helpers shared by the kernel translation units.
#pragma once

#include "fem_internal.h"

namespace fem {

// Cap on persistent grids: kernels loop over their tiles, so a grid of a few
// workgroups per compute unit (256 CUs) keeps every CU busy.
constexpr int kMaxGrid = 256 * 8;
// Number of workgroup partial sums of one reduction (fixed, so the
// reduction order of a problem never depends on what else is launched).
constexpr int kRedParts = 2048;
// Scalar slots after the partials in a problem's reduction area.
enum RedSlot {
    kSlotRZ = 0,      // <r, z>
    kSlotQP = 1,      // <q, p>
    kSlotQZ = 2,      // <q, z>
    kSlotRN = 3,      // ||G^T r||^2
    kSlotRZOld = 4,   // previous <r, z>
    kSlotTmp = 5,     // generic dot result
    kSlotB2 = 6,      // ||G^T b||^2
    kSlotAlpha = 7,   // alpha of the last r update (u catches up in the next p update)
    // device-side convergence state of a solve (the server's batched
    // iterations decide convergence on the device, see launch_cg_check)
    kSlotState = 8,   // 0 running, 1 finished in the current iteration, 2 frozen
    kSlotIters = 9,   // iterations taken
    kSlotRel = 10,    // ||G^T r|| / ||G^T b|| after the last iteration
    kSlotStatus = 11, // fem_status once finished
    kSlotRtol = 12,   // stopping tolerance
    kSlotMaxit = 13,  // iteration limit
    kSlotCount = 16
};
constexpr int kRedStride = kRedParts * 4 + kSlotCount;   // 4 partial groups + slots
__host__ __device__ inline double* red_slots(double* red) { return red + kRedParts * 4; }

// Element range [lo, hi) of reduction (and elementwise) tile t of a problem:
// either blocks_per_red whole storage blocks, or, for problems with few
// blocks, one of red_lsplit contiguous slices of node planes of one block.
// Depends only on the problem's own sizes.
__host__ __device__ inline void red_range(const ProbEntry& pe, int t, size_t& lo, size_t& hi) {
    const size_t bs = pe.len / pe.nblk;
    if (pe.red_lsplit <= 1) {
        lo = (size_t)t * pe.blocks_per_red * bs;
        hi = lo + (size_t)pe.blocks_per_red * bs;
    } else {
        const int nn = (int)(bs / kLanes);
        const int lchunk = (nn + pe.red_lsplit - 1) / pe.red_lsplit;
        const int blk = t / pe.red_lsplit, part = t % pe.red_lsplit;
        const int l0 = part * lchunk, l1 = l0 + lchunk < nn ? l0 + lchunk : nn;
        lo = (size_t)blk * bs + (size_t)l0 * kLanes;
        hi = (size_t)blk * bs + (size_t)l1 * kLanes;
    }
    if (hi > pe.len) hi = pe.len;
    if (lo > hi) lo = hi;
}

// 1D reference matrices of degree p on [0,1] (row-major, (p+1)^2), built on
// the host once per process.
const double* ref_mass(int p);
const double* ref_stiff(int p);

// Device copies of multi-problem entry tables.  Each upload takes the next of
// kSlots pinned host / device slot pairs; the host side of a slot is reused
// only after the copy that read it has run (event), and the device side only
// by work later on the same stream.
struct TableStager {
    // enough slots for the uploads of many launches in flight (a server step
    // stages a table per launch), so the host seldom waits for a slot
    static constexpr int kSlots = 256;
    int cap = 0;
    ProbEntry* host_block = nullptr;   // kSlots * cap entries, pinned
    ProbEntry* dev_block = nullptr;    // kSlots * cap entries
    ProbEntry* host[kSlots] = {};
    ProbEntry* dev[kSlots] = {};
    hipEvent_t ev[kSlots] = {};
    bool used[kSlots] = {};
    int next = 0;
    hipError_t init(int cap_entries);
    void destroy();
    hipError_t upload(const ProbEntry* ents, int n, hipStream_t s, const ProbEntry** out);
};

// Kernel shape choices of one launch (picked by the batch autotuner).
struct LaunchCfg {
    int apply_lds = 0;      // 1: LDS line kernel even where the register kernel exists
    int pi_fused = -1;      // -1: process-wide default, 0: two-phase, 1: fused sweep
    int grid_cap = 0;       // cap on persistent grids (0: default)
};

// Put the entry table where the kernel reads it: by value for a single
// problem, else through the stager.
inline hipError_t stage_table(LaunchTable& L, const ProbEntry* ents, int nprob, TableStager* st,
                              hipStream_t s) {
    if (nprob == 1) {
        L.one = ents[0];
        L.tab = nullptr;
        return hipSuccess;
    }
    if (!st) return hipErrorInvalidValue;
    return st->upload(ents, nprob, s, &L.tab);
}

// Kernel launchers.  Each fills tile_begin/ntiles of the entries.
// apply: mode 0 y=Ax (a=x, c=y), 1 y=b-Ax (a=x, b=b, c=y), 2 y=Mx.
hipError_t launch_apply(int p, int prec, int mode, ProbEntry* ents, int nprob, TableStager* st,
                        hipStream_t s, const LaunchCfg& cfg = LaunchCfg());
// apply over problems of any degrees: with `mix`, one mixed-degree launch
// when the degrees are two or three of {2, 3, 7}, else one launch per degree
// (the same kernel bodies and results either way)
hipError_t launch_apply_any(int prec, int mode, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s,
                            bool mix = true);
// patch inverse: a = r (dual), c = z (primal), d = patch buffer,
// alpha = damping; accumulate: z = (acc ? z : 0) + alpha * P_AS r.
hipError_t launch_patch_inverse(int p, int prec, int accumulate, ProbEntry* ents, int nprob,
                                TableStager* st, hipStream_t s, const LaunchCfg& cfg = LaunchCfg());

// patch inverse over problems of any degrees (as launch_apply_any)
hipError_t launch_patch_inverse_any(int prec, int accumulate, ProbEntry* ents, int nprob, TableStager* st,
                                    hipStream_t s, bool mix = true);

// Multi-problem vector operations (all problems in `ents`, any degrees where
// noted).  Operands in the entries as for the single-problem versions.
// dot: a . b into slot (precisions pa, pb)
hipError_t launch_dot(int pa, int pb, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, int slot);
// distribute + norm (one degree p): a = r (FP64), c = out (prec); slot <- ||G^T r||^2
hipError_t launch_distribute(int p, int prec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s,
                             int slot);
// residual norm over problems of any degrees (as launch_apply_any): the
// assembled norm for an FP64 smoother, else distribute + norm
hipError_t launch_norm_any(int smoother_prec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, int slot,
                           bool mix = true);
// assembled norm (one degree p): a = r (FP64); slot <- ||G^T r||^2
hipError_t launch_anorm(int p, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, int slot);
// r -= alpha q with alpha = <r,z>/<q,p> (saved in kSlotAlpha); entries b = q,
// d = r.  u is updated later by launch_cg_p (or run_cg_update_u when the
// iteration stops)
hipError_t launch_cg_ur(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s);
// u += alpha p (saved alpha), then p = z + beta p; entries a = z (zprec),
// c = p, d = u
hipError_t launch_cg_p(int zprec, int variant, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s);
// <q, z> -> kSlotQZ and <r, z> -> kSlotRZ in one pass; entries a = q, d = r, b = z
hipError_t launch_dot_qz_rz(int zprec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s);
hipError_t launch_slot_copy(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, int dst, int src);
// Start of a solve's device-side convergence state: running, 0 iterations,
// rtol = entry alpha, maxit = entry zchunk.
hipError_t launch_solve_init(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s);
// After an iteration's residual norm: every running solve counts the
// iteration and finishes (state 1, status) on a zero right-hand side, a
// breakdown (<q,p> not positive or a non-finite residual), rtol or maxit, in
// that order, as pcg_solve decides on the host; a solve finished in the
// previous iteration is frozen (state 2).  The r update skips solves that are
// not running, and the p update (which also applies the last u step) skips
// frozen ones, so further iterations leave a finished solve's u unchanged.
hipError_t launch_cg_check(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s);
// out[2i] = slot a, out[2i+1] = slot b of problem i (device array)
hipError_t launch_collect_slots(ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, int sa, int sb,
                                double* out);
// elementwise convert a (sp) -> c (dp) over whole cell vectors
hipError_t launch_convert(int sp, int dp, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s);

// z += P_0 A_0^{-1} R_0 t: the exact Q1 coarse correction of the two-level
// preconditioner (t dual and z primal, both in `prec`; the coarse solve in
// FP64).  No-op when the mesh has no interior vertex.
hipError_t run_coarse_correction(fem_problem* P, const void* t, void* z, int prec);
// The same over several problems of degree p (entries from coarse_entry).
hipError_t launch_coarse_correction(int p, int prec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s);
// The same over problems of any degrees (as launch_apply_any).
hipError_t launch_coarse_any(int prec, ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, bool mix = true);
ProbEntry coarse_entry(fem_problem* P, const void* t, void* z);

// Single-problem helpers (problem handle in, stream of the handle).
ProbEntry entry_of(const fem_problem* P);
hipError_t run_dss_axis(fem_problem* P, void* v, int axis, int prec);
// The same axis pass on the mesh of an entry (e.n, e.c = vector).
hipError_t run_dss_axis_entry(int p, const ProbEntry& e, int axis, int prec, hipStream_t s);
hipError_t run_gather(fem_problem* P, const double* xg, void* xc, int prec);
hipError_t run_scatter(fem_problem* P, const void* yc, double* yg, int prec);
hipError_t run_extract(fem_problem* P, const void* uc, double* ug, int prec);
hipError_t run_pack(fem_problem* P, const double* canon, void* vc, int prec, int unpack);
// The same for the mesh of an entry (e.p, e.ncells, e.len).
hipError_t run_pack_entry(ProbEntry e, const double* canon, void* vc, int prec, int unpack, hipStream_t s);
hipError_t run_convert(fem_problem* P, const void* src, int sp, void* dst, int dp);
hipError_t run_fill_zero(fem_problem* P, void* v, int prec);
// Dot product of two cell vectors into slot `slot` of the problem's
// reduction area (device), deterministic order.
hipError_t run_dot(fem_problem* P, const void* a, int pa, const void* b, int pb, int slot);
// ||G^T r||^2 into slot `slot`.
hipError_t run_assembled_norm2(fem_problem* P, const void* r, int prec, int slot);
// out = G^T r / multiplicity per copy, assembled in FP64 and rounded to
// `prec`; ||G^T r||^2 into slot `slot` (same pass).  solver: out is a
// solver's copy of its residual (FP16 copies are then scaled by a power of
// two chosen from the residual norm slot, which must hold the current or the
// previous ||G^T r||^2).
hipError_t run_distribute(fem_problem* P, const double* r, void* out, int prec, int slot, bool solver = false);
// z = S r (kind FEM_PC_DSS) or z = D_cell^{-1} S r (FEM_PC_JACOBI), zero on a
// Dirichlet boundary, from the FP64 dual r; ||G^T r||^2 into slot `slot`;
// solver as for run_distribute.
hipError_t run_simple_precond(fem_problem* P, int kind, const double* r, void* z, int prec, int slot,
                              bool solver = false);
// (F)PCG vector updates, scalars read from the device slots.
// r -= alpha q (alpha saved for the next u update); optionally rs = r in the
// smoother precision.
hipError_t run_cg_update_r(fem_problem* P, double* r, const double* q, void* rs, int rs_prec);
// u += alpha p with the saved alpha (the step the last r update left out)
hipError_t run_cg_update_u(fem_problem* P, double* u, const double* p);
// <q, z> -> kSlotQZ and <r, z> -> kSlotRZ in one pass
hipError_t run_dot_qz_rz(fem_problem* P, const double* q, const double* r, const void* z, int zprec);
// u += alpha p, then p = z + beta p (beta from slots, variant 1 = PCG,
// 2 = FCG); z in zprec.
hipError_t run_cg_update_p(fem_problem* P, double* p, double* u, const void* z, int zprec, int variant);
// rz_old <- rz (slot copy), on device
hipError_t run_slot_copy(fem_problem* P, int dst, int src);

}  // namespace fem
