// Least squares of block FGMRES (host side, small dense arithmetic): the block
// Hessenberg matrix of one cycle reduced to upper triangular form by complex
// Givens rotations as its block columns arrive, the same rotations applied to
// the right-hand side block [S0; 0]; the residual norm of every right-hand
// side after each block column, and the coefficients Y of the update
// X += [Z_0 .. Z_{k-1}] Y by back substitution.
//
// Values are kept split into real and imaginary planes so that every inner
// loop runs over the s right-hand sides with unit stride; the loops are
// compiled for AVX-512 and AVX2 as well as the baseline instruction set and
// picked at load time.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace mx {

class BlockLsq {
 public:
  // s right-hand sides (1..32), at most m block columns; S0 upper triangular
  // s x s, row-major (the factor R of the first residual block)
  void reset(int s, int m, const std::vector<std::complex<double>>& S0);
  // block column k (0 <= k < m, in order): P row-major [(k+2)s][s] holding the
  // projections onto V_0..V_k and, in its last s rows, the upper triangular
  // factor R_{k+1} of the new basis block
  void add(int k, const std::vector<std::complex<double>>& P);
  // residual norm of right-hand side b after the last added block column
  double colres(int b) const;
  // Y [(k s) x s] row-major, interleaved complex, for the k added columns
  void solve(double* Y) const;
  int done() const { return kdone_; }

 private:
  int s_ = 0, m_ = 0, kdone_ = 0;
  int64_t ncol_ = 0;
  std::vector<double> hr_, hi_;    // rotated block Hessenberg [(m+1)s][ms]
  std::vector<double> gr_, gi_;    // rotated right-hand sides [(m+1)s][s]
  std::vector<double> pr_, pi_;    // block column being added [(m+1)s][s]
  std::vector<int32_t> ri_, rj_;   // rotation t acts on rows ri_[t], rj_[t]
  std::vector<double> rc_, rsr_, rsi_;  // its cosine and sine
};

}  // namespace mx
