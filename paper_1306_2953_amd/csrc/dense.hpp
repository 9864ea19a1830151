// Dense (N x N) stage of orthogonalisation and subspace diagonalisation.
#pragma once

#include <vector>

#include "internal.hpp"

namespace rs {

// Workspace of the point-summed contractions and small-matrix kernels,
// sized for max_states at creation (the field calls never allocate).
struct DenseWork {
    int max_states = 0;
    int max_chunks = 512;               // set by dense_work_init
    DevBuf partial;                    // double [max_chunks][N16][N16]
    DevBuf red;                        // double [16][N16][N16] group sums of the partials
    int blocks_n = 0;                  // N16 the block lists were built for
    DevBuf d_blocks_syrk, d_blocks_full;
    DevBuf mwork;                      // double [N][N] scratch
    DevBuf xth, xtm, xtl;              // bfloat16 [N16][N32] three-term split rotation matrix
    DevBuf sweeps;                     // int
    DevBuf diag;                       // double [N] Jacobi diagonal
    DevBuf rot;                        // double2 [30][M-1][M/2] Jacobi rotations
    bool jacobi_lds_set = false, chol_lds_set = false, rot_lds_set = false, rotbf_lds_set = false;
    int ncu = 0;                       // compute units of the device (persistent rotation)
};

rs_status dense_work_init(DenseWork &w, int64_t np, int max_states);
// Scratch of the point-summed products: chunk partials (partial_bytes),
// group sums red [16][N16][N16], and the 16 x 16 output block lists
// [(N16/16)^2] (full) and [(N16/16)(N16/16+1)/2] (symmetric).
constexpr int kGramRedGroups = 16;   // group sums of the chunk partials
struct GramScratch {
    double *partial;
    int64_t partial_bytes;
    double *red;
    int2 *blocks_full, *blocks_syrk;
    int max_chunks;
};
// gram on explicit scratch; make_lists: (re)build the block lists first.
rs_status gram_core(const GramScratch &w, bool make_lists, const void *X, const void *Y, int64_t np, int B,
                    int nblk, int dtype, int prec, double dv, double *S, int mode, hipStream_t st);
// S = dv X^T Y over points; mode 0 plain, 2 symmetrised (X == Y is computed
// as a symmetric rank-k product).
rs_status gram(DenseWork &w, const void *X, const void *Y, int64_t np, int B, int nblk, int dtype,
               int prec, double dv, double *S, int mode, hipStream_t st);
// psi <- psi X in place (skipped when *skip != 0, if skip is given).
// upper: X is upper triangular (exact zeros below the diagonal), which the
// FP64 kernel for N <= 128 uses to skip the zero blocks.
rs_status rotate(DenseWork &w, void *psi, const double *Xm, int64_t np, int B, int nblk, int dtype,
                 int prec, const int *skip, hipStream_t st, bool upper = false);
rs_status cholesky(DenseWork &w, const double *S, double *U, int N, int *info_dev, hipStream_t st);
rs_status trinv(const double *U, double *T, int N, const int *info_dev, hipStream_t st);
// Jacobi eigensolver for a symmetric A (overwritten); max_sweeps (at most
// 30) bounds the work (30 reaches full FP64 accuracy from any start).
rs_status eigh(DenseWork &w, double *A, double *V, double *evals, int N, hipStream_t st,
               int max_sweeps = 30);
// Complex overlap from the real one of interleaved columns: G is the
// 2N x 2N real product (column 2j = re of state j, 2j + 1 = im), S the
// N x N complex matrix (re, im interleaved) with
// S[j][k] = (G[2j][2k] + G[2j+1][2k+1]) + i (G[2j][2k+1] - G[2j+1][2k]).
rs_status complex_fold(const double *G, double *S, int N, hipStream_t st);
// Padded states n..N-1 (all zero): S[i][i] = 1 for i >= n.
rs_status pad_identity(double *S, int N, int n, hipStream_t st);
// Eigenpairs of the leading n x n block of A (N x N); V = diag(V_n, I),
// evals[n..N) = 0.  scratch_a, scratch_v: n*n doubles each.
rs_status eigh_leading(DenseWork &w, double *A, double *V, double *evals, int N, int n, double *scratch_a,
                       double *scratch_v, hipStream_t st, int max_sweeps);

}  // namespace rs
