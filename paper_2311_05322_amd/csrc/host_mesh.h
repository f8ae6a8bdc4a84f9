// Host-side mesh topology, domain decomposition and point location.
//
// Integer definitions (they fix the unknown numbering and the subdomains):
//   * each tetrahedron's vertex ids are sorted ascending, so a local edge
//     (a<b) is oriented low -> high id, which is the global orientation;
//   * global edges are the distinct (vmin, vmax) pairs in lexicographic order;
//   * boundary faces are the sorted vertex triples owned by one tetrahedron,
//     in lexicographic order;
//   * subdomains come from recursive coordinate bisection of tetrahedron
//     centroids ((x0+x1)+x2)+x3)*0.25 (input vertex order), split along the
//     axis of largest extent (first axis on ties), ordered by (coordinate,
//     id), left part = first floor(m/2) tetrahedra;
//   * overlap: delta layers of tetrahedra sharing a vertex with the previous
//     layer; vertex weight omega(v) = delta - (first layer containing v),
//     edge weight w(e) = omega(a) + omega(b), D_i(e) = w_i(e) / sum_j w_j(e);
//   * colours: greedy in subdomain order, smallest colour unused by a
//     subdomain sharing a DOF.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace mx {

struct Topology {
  int32_t nv = 0, nt = 0;
  int64_t ne = 0, nnz = 0, nbf = 0, nfaces = 0;
  std::vector<double> xyz;        // [nv*3]
  std::vector<int32_t> tet_in;    // [nt*4] as given
  std::vector<int32_t> ts;        // [nt*4] sorted ids
  std::vector<int32_t> edges;     // [ne*2]
  std::vector<int32_t> t2e;       // [nt*6]
  std::vector<int32_t> nbr;       // [nt*4] tetrahedron across local face, -1 on the boundary
  std::vector<int32_t> bf_of;     // [nt*4] boundary-face index of a local face, -1 otherwise
  std::vector<int32_t> bf_tet, bf_lf;   // [nbf]
  std::vector<int64_t> row_ptr;   // [ne+1]
  std::vector<int32_t> col;       // [nnz]
  // contributions of the global matrix: source index into
  // [element blocks nt*36 | boundary-face blocks nbf*9]
  std::vector<int64_t> cptr;      // [nnz+1]
  std::vector<int32_t> csrc;
  std::vector<int64_t> e2t_ptr;   // [ne+1] edge -> tetrahedra (ascending)
  std::vector<int32_t> e2t;
  std::vector<int64_t> v2t_ptr;   // [nv+1] vertex -> tetrahedra (ascending)
  std::vector<int32_t> v2t;
};

// Builds the topology; returns an empty string or an error message.
std::string build_topology(int32_t nv, int32_t nt, const double* xyz, const int32_t* tet,
                           Topology& T);

struct Decomposition {
  int32_t nsub = 0, overlap = 0, ncolour = 0, nb = 64;
  std::vector<int32_t> part;          // [nt]
  std::vector<int64_t> dof_ptr;       // [nsub+1]
  std::vector<int32_t> dofs;          // [sum n_i]
  std::vector<int32_t> w;             // [sum n_i] integer PU weights
  std::vector<double> D;              // [sum n_i] w / sum_j w_j
  std::vector<int32_t> colour;        // [nsub]
  std::vector<int64_t> tet_ptr;       // [nsub+1] overlapping tetrahedra
  std::vector<int32_t> tets;
  std::vector<int64_t> nbr_ptr;       // [nsub+1] adjacent subdomains
  std::vector<int32_t> nbrs;
  // dense row of each local DOF: a reverse Cuthill-McKee order of the
  // subdomain's DOF graph (DOFs sharing a tetrahedron of the subdomain), so
  // that the dense local matrix is banded; dense_edge is the inverse map
  // (global edge of each dense row, -1 on the padding rows)
  std::vector<int32_t> lpos;          // [sum n_i]
  std::vector<int32_t> dense_edge;    // [sum N_i]
  // band0[i * band_np + p]: last 64-row tile holding a structural non-zero
  // of the columns of panel p of the dense matrix in that order (the matrix
  // pattern is symmetric, so it is also the last column tile of its rows);
  // band_np = max N_i / 64
  int32_t band_np = 0;
  std::vector<int32_t> band0;
  // padded dense sizes and offsets of the local matrices
  std::vector<int32_t> Npad;          // [nsub]
  std::vector<int64_t> mat_off;       // [nsub+1] offsets in entries
  std::vector<int64_t> vec_off;       // [nsub+1] padded row offsets (sum of Npad)
  // interface faces (unique (tet, local face) pairs on some artificial interface)
  std::vector<int32_t> if_tet, if_lf;
  // local assembly: local non-zero -> destination entry and contributions
  // (source index into [elements nt*36 | boundary faces nbf*9 | interface nif*9])
  std::vector<int64_t> ldest, lptr;
  std::vector<int32_t> lsrc;
  // prolongation entries grouped by colour: destination edge, source padded
  // row (vec_off[i] + lpos), weight
  std::vector<int64_t> pcol_ptr;      // [ncolour+1]
  std::vector<int32_t> p_edge;
  std::vector<int64_t> p_row;
  std::vector<double> p_w;
  // the same entries grouped by destination edge (pg_ptr [ne+1]), in colour
  // order within an edge: a gather gives every edge its sum in the order
  // the colour-by-colour accumulation would add it
  std::vector<int64_t> pg_ptr;
  std::vector<int64_t> pg_row;
  std::vector<double> pg_w;
};

std::string build_decomposition(const Topology& T, int32_t nsub, int32_t overlap, int32_t nb,
                                Decomposition& D);

// Column windows of the operator's rows for the LDS-staged product: the rows
// are cut, in order, into slices of at most max_rows consecutive rows whose
// non-zeros touch at most cap distinct columns (cap <= 256). ucol lists each
// slice's columns in ascending order and lcol gives, for every non-zero in
// CSR order, the position of its column in its slice's list.
struct ColWindows {
  int32_t cap = 0, max_rows = 0, umax = 0;
  std::vector<int32_t> row;     // [ns+1] first row of each slice
  std::vector<int32_t> cptr;    // [ns+1] offsets into ucol
  std::vector<int32_t> ucol;
  std::vector<uint8_t> lcol;    // [nnz]
};
// Returns false (and an empty W) when a single row has more than cap columns.
bool build_col_windows(const Topology& T, int32_t cap, int32_t max_rows, ColWindows& W);

// Point functional r[e] = p . N_e(x), averaged over all tetrahedra whose
// closure contains x (min barycentric >= -1e-12).  Output: sorted edges and
// complex values (re, im interleaved).  Returns false when x is outside.
bool point_functional(const Topology& T, const double x[3], const double p_re[3],
                      const double p_im[3], std::vector<int32_t>& edge,
                      std::vector<double>& val);

}  // namespace mx
