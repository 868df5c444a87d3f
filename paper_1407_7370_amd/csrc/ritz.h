// Ritz values of the Lanczos tridiagonal T and their error bounds (Sec. 2
// eq. error_est): the host-side eigenvalue problems of the eigen modes and
// of the adjoint.  Plain C++, no device code.
#pragma once

#include <utility>
#include <vector>

namespace dlh {

// Eigenvalues and all eigenvectors (column l of v, row-major k x k) of the
// symmetric tridiagonal matrix with diagonal d and off-diagonal e[0..k-2]:
// implicit QR steps with Wilkinson shift (Golub & Van Loan, symmetric QR).
void tridiag_full(std::vector<double> d, std::vector<double> e, std::vector<double> &lam,
                  std::vector<double> &v);

// Eigenvalues of the same matrix in (lo, hi] (ascending, with multiplicity)
// and the last component of each unit eigenvector.  Values by bisection on
// Sturm counts to full relative precision, vectors by inverse iteration on
// the pivoted LU factors of T - theta I; eigenvalues closer than
// max(group, 1e-8 ||T||) are solved as one group whose vectors are kept
// orthogonal, so the sum of zlast^2 over a group of near-equal values is the
// weight of e_k on their invariant subspace.  O(k) work per value and
// iteration, against O(k^2) for a QR sweep over the whole spectrum.
void tridiag_window(const std::vector<double> &d, const std::vector<double> &e, double lo, double hi, double group,
                    std::vector<double> &lam, std::vector<double> &zlast);

// Ritz values of T (eigenvalues lam, last eigenvector components zl) in
// [e_lo, e_hi], grouped into clusters of neighbours closer than tol; a
// cluster with bound |beta_k| ||zl over the cluster|| <= tol is reported as its
// mean (at most n_wanted, ascending).  rep (optional) receives, per reported
// cluster, the index of its member with the smallest |zl|.  Returns the count.
int ritz_select(const std::vector<double> &lam, const std::vector<double> &zl, double beta_k, double e_lo,
                double e_hi, double tol, int n_wanted, double *evals, double *bounds, std::vector<int> *rep);

// Ritz values (and with V, all eigenvectors of T: column l of V, row-major
// k x k) of the tridiagonal T_k with diagonal alpha1[0..k) and off-diagonal
// beta1[0..k-1), bound factor beta1[k-1] = beta_k; selection as ritz_select.
// Without V only the window is solved (tridiag_window).
int ritz_chain(const double *alpha1, const double *beta1, int k, double e_lo, double e_hi, double tol, int n_wanted,
               double *evals, double *bounds, std::vector<int> *rep, std::vector<double> *V);

// The eigen mode computes the Ritz values every this many iterations and
// stops once n_wanted clusters have converged.
constexpr int kEigenCheckEvery = 64;

// Add converged clusters (values ev, bounds bd) to `found` (ascending by
// value): a value within tol of a found one is the same eigenvalue and keeps
// the smaller bound.  Once orthogonality is lost a converged Ritz value gets
// copies whose eigenvectors of T mix with its own, so its bound can grow
// again while the value stays within its earlier bound of an eigenvalue of H
// (Paige's analysis of the finite-precision recurrence).
void merge_converged(std::vector<std::pair<double, double>> &found, const double *ev, const double *bd, int n,
                     double tol);

// Host threads for the Ritz computations: the hardware's, at most 16.
int host_threads();

// The converged clusters of the leading blocks T_j, j = every, 2 every, ...
// and j = k, merged (merge_converged) into `found`.  The blocks are solved
// on up to `threads` host threads.
void converged_union(const double *alpha1, const double *beta1, int k, double e_lo, double e_hi, double tol,
                     int every, int threads, std::vector<std::pair<double, double>> &found);

}  // namespace dlh
