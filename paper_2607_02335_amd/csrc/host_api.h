// Internal host declarations shared by the C-ABI translation units.
#pragma once

#include <string>
#include <vector>

#include "fem_internal.h"

namespace fem {

fem_status set_error(fem_status st, const std::string& msg);
fem_status hip_error(hipError_t e, const char* what);

std::vector<double> host_gll_nodes(int p);
void host_gauss(int nq, std::vector<double>& x, std::vector<double>& w);
void host_ref_matrices(int p, double* M, double* K);
void host_patch_1d(int p, double h0, double h1, std::vector<double>& M, std::vector<double>& K);
int host_fd_1d(int p, double h0, double h1, double* S, double* lam);
// Generalised eigenproblem K S = M S diag(lam) with S^T M S = I (n x n).
int host_gen_eig(int n, const std::vector<double>& M, const std::vector<double>& K, double* S, double* lam);
// The coarse (Q1, interior vertices) 1D fast-diagonalisation data of a 1D
// mesh of n cells: S ((n-1) x (n-1), row-major, columns eigenvectors) and
// lam (n-1).  n < 2 writes nothing.
int host_coarse_1d(int n, const double* h, double* S, double* lam);
void host_q1_1d(int n, const double* h, std::vector<double>& M, std::vector<double>& K);

// Validate a description; on failure sets the error message.
fem_status check_desc(const fem_desc* d);
// Bytes of the handle workspace of a description (geometry, FD data,
// reductions, patch buffer, smoother scratch).
size_t workspace_bytes(const fem_desc* d);
// Bytes of pcg_solve's own vectors for a smoother precision.
size_t solve_vector_bytes(const fem_desc* d, int smoother_prec);
size_t desc_cell_len(const fem_desc* d);
// Create a problem; with mem, its workspace is carved from caller memory and
// its set-up data uploaded asynchronously from the caller's pinned staging.
fem_status create_problem(const fem_desc* d, hipStream_t stream, fem_problem** out, const ProblemMem* mem = nullptr);
// Pinned staging bytes create_problem needs with caller memory.
size_t problem_stage_bytes(const fem_desc* d);
// Free a problem without synchronising its stream (no queued work may use it).
void destroy_problem_nosync(fem_problem* P);

// Solver pieces reused by the server (all asynchronous on P->stream).
fem_status smoother_run(fem_problem* P, const void* r, void* z, int prec, int sweeps, double omega);
// The two-level preconditioner: `sweeps` smoothing sweeps from z = 0, the
// exact coarse correction, `sweeps` more smoothing sweeps.
fem_status two_level_run(fem_problem* P, const void* r, void* z, int prec, int sweeps, double omega);

#define FEM_HIP(call, what)                                   \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return ::fem::hip_error(e_, what); \
    } while (0)

}  // namespace fem
