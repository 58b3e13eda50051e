// Host-side plan of the planar exact (Kac-Ward) solver for bit-flip noise
// (paper Sec. 3.1.3, exact solutions on planar graphs; Sec. 3.1.1, eq.
// "rbim").
//
// Under bit-flip noise a coset partition function Z_l(s) is the partition
// function of a random-bond Ising model whose spins sit on the X-type checks
// and whose bonds are the qubits: qubit q couples its two X-type checks with
// K_q = ln((1 - p_q) / p_q) / 2 and sign eta_q = (-1)^(x-bit of the coset's
// reference error on q); a qubit in one X-type check couples it to a fixed +1
// spin.  The graph is planar.  The fixed spin is realised as two ghost spins
// (one beyond the left boundary, one beyond the right) joined by a bond of
// weight tanh = 1 that runs above the patch, so they take one common value.
// With t_q = tanh(eta_q K_q) = eta_q (1 - 2 p_q), the high-temperature
// expansion gives
//     Z_l(s) = 2^(m_X - n) * (sum over even subgraphs of prod t_e),
// and the Kac-Ward determinant gives that sum as sqrt(det(I - Lambda)), with
// Lambda indexed by directed edges: Lambda[a][b] = t_b exp(i phi_ab / 2) when
// b leaves the head of a and is not the reverse of a, phi_ab being the turning
// angle from the end of a to the start of b plus the turns inside b (boundary
// bonds bend at a point beyond the boundary, the ghost bond at two corners).
// The logical X coset flips eta on the column of the X representative
// (the last column, as in the boundary-MPS path); the Y and Z cosets are
// impossible under bit-flip noise.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace tnmld {

// Lambda[row][col] = t[edge] * (re + i im), row != col
struct KwEntry {
  int16_t row, col;
  int16_t edge;  // undirected edge of col: a qubit q < n, or n (the ghost bond, t = 1)
  int16_t pad;
  double re, im;
};
static_assert(sizeof(KwEntry) == 24, "KwEntry layout");

struct KwHeader {
  int32_t d, n, m, mx;   // distance, qubits, checks, X-type checks
  int32_t ne, N, ld;     // undirected edges (n + 1), directed edges N = 2 ne, row length (N rounded up to 16)
  int32_t nnz;           // entries of Lambda
  int32_t nz_ofs;        // KwEntry[nnz]
  int32_t zcheck_ofs;    // int8[m / 2][2]: Z-type check j (syndrome bit j): column and last row of its X string
  int32_t bytes;         // blob size
  int32_t pad;
  double log_pref;       // (m_X - n) ln 2
};

struct KwPlan {
  KwHeader h;
  std::vector<uint8_t> blob;  // header + tables, as uploaded
};

// Build the plan for distance d; returns an empty string on success.
std::string build_kw_plan(int d, KwPlan* out);

}  // namespace tnmld
