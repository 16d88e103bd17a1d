// Internal (not part of the C ABI): a read-only view of a problem's fine-grid system on the
// device, for the coarse-grid (NLMC) builder.  The fine operator of the coupled scheme is
// M/tau + A with A = D + Q (+ the implicit wells on the fracture diagonal); the view gives
// its pieces as the problem's own setup kernels computed them.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/mcdec.h"

namespace mc {

struct FineView {
  int nx = 0, ny = 0, nz = 1, n_omega = 0, nf = 0, ncont = 0, scheme = 0;
  long ncell = 0;
  double h = 0, tau = 0;
  double s12 = 0;                 // Omega-Omega transfer sigma_omega h^2 (3C)
  double mtau[2] = {0, 0};        // grid storage over tau, c h^2 / tau
  double c[2] = {0, 0};           // grid storage coefficients
  double c_f = 0;                 // fracture storage coefficient
  int has_t[2] = {0, 0};          // per-face conductance arrays (else tconst)
  double tconst[2] = {0, 0};
  const double* diag[3] = {nullptr, nullptr, nullptr};  // M/tau + D + S (+ wells) diagonal
  const double* tx[2] = {nullptr, nullptr};             // east face conductance (0 at the side)
  const double* ty[2] = {nullptr, nullptr};             // north face conductance
  const double* F[3] = {nullptr, nullptr, nullptr};     // right-hand side F per continuum
  const double* state[3] = {nullptr, nullptr, nullptr}; // current layer p^n
  const double* mt = nullptr;     // fracture storage over tau
  const double* flen = nullptr;   // fracture cell lengths
  double aperture = 0;
  const int* rowptr = nullptr;    // fracture CSR (off-diagonal conductances in val)
  const int* col = nullptr;
  const double* val = nullptr;
  const int* host = nullptr;      // host cell of every fracture cell
  const int* hptr = nullptr;      // fracture cells hosted per grid cell (CSR, ascending)
  const int* hidx = nullptr;
  const double* sigma_f = nullptr;  // [n_omega * nf] transfer to the host cell
  hipStream_t stream = nullptr;
  int device = 0;
  // host copies of the integer structure
  std::vector<int> h_host, h_rowptr, h_col;
};

// Fills v from problem p (throws std::invalid_argument for a 3-D grid or the EX split).
void fine_view(const mc_problem* p, FineView& v);

// In place: the K x K SPD matrix S (column-major, device, leading dimension lda) -> S^-1
// (full, symmetric), by rocSOLVER potrf / potri.  Throws on failure.
void spd_inverse(double* S, int K, hipStream_t s, int lda);

}  // namespace mc
