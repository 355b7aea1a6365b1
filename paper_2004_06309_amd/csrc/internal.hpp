// Internal types of libhelm (host side).
#pragma once

#include <complex>
#include <cstdint>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/helm.h"

namespace helm {

using cplx = std::complex<double>;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

// Complex CSR with 64-bit row pointers (rows may exceed 2^31 entries in total).
struct Csr {
  int64_t n = 0;  // rows
  int64_t m = 0;  // columns
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<cplx> val;
  int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

struct CsrReal {
  int64_t n = 0, m = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

// Mesh plus its P1/P2 dof numbering, boundary classification and the
// per-tet element matrices (unit coefficient) of the Helmholtz weak form.
struct Discretization {
  int order = 1;
  int nloc = 4;       // dofs per tet
  int nfloc = 3;      // dofs per face
  int64_t nv = 0, nt = 0, ne = 0, n = 0;
  std::vector<double> xyz;       // [nv][3]
  std::vector<int64_t> tets;     // [nt][4], positively oriented
  std::vector<int64_t> edges;    // [ne][2], sorted (min, max), lexicographic
  std::vector<int64_t> tet_dofs; // [nt][nloc]
  std::vector<double> vol;       // [nt]
  std::vector<double> Ke;        // [nt][nloc][nloc]  int grad phi_a . grad phi_b
  std::vector<double> Me;        // [nt][nloc][nloc]  int phi_a phi_b
  std::vector<cplx> k;           // wavenumber per tet
  double omega = 0;
  double ztop = 0;
  // boundary faces (faces of exactly one tet)
  std::vector<int64_t> bface;    // [nb][3] sorted vertex ids
  std::vector<int64_t> bowner;   // owning tet
  std::vector<uint8_t> bdir;     // 1 = Dirichlet (top), 0 = absorbing
  std::vector<uint8_t> dir_mask; // per dof
  // dof -> tets adjacency (CSR)
  std::vector<int64_t> d2t_ptr, d2t_idx;
  Csr A;

  int64_t edge_id(int64_t a, int64_t b) const;
  void face_dofs(const int64_t* f, int64_t* out) const;  // sorted triple -> nfloc dofs
  double face_area(const int64_t* f) const;
  void dof_coord(int64_t d, double* x) const;
};

struct ImpFace {
  int64_t v[3];  // sorted vertex ids
  int64_t owner; // tet whose k is used
};

// fem.cpp
void build_discretization(Discretization& D, const helm_mesh& mesh, const double* c_tet, double omega);
void face_matrix(int order, double area, double* B);  // nfloc x nfloc, int psi_a psi_b
// Assemble -K + M_{k^2} + i B_k over tet_list (+ impedance faces), restricted
// to the sorted dof list `dofs` (global ids), Dirichlet rows/cols replaced by
// identity.  Rows/cols of the result index into `dofs`.
void assemble_local(const Discretization& D, const std::vector<int64_t>& tet_list,
                    const std::vector<ImpFace>& faces, const std::vector<int64_t>& dofs, Csr& out);
// Locate a point: tet index (or -1) and barycentric coordinates.
int64_t locate_point(const std::vector<double>& xyz, const std::vector<int64_t>& tets, const double* p,
                     double* lam, const std::vector<int64_t>* candidates = nullptr);
void basis_values(int order, const double* lam, double* phi);

// ---------------------------------------------------------------------------
// Factorisation data (one "batch" = the fine subdomains, or the coarse matrix)
// ---------------------------------------------------------------------------

// Symbolic structure of one matrix (subdomain) after nested dissection.
struct Symbolic {
  int64_t n = 0;
  std::vector<int32_t> perm;      // new -> old local index
  std::vector<int32_t> iperm;     // old -> new
  int32_t nsn = 0;
  std::vector<int32_t> sn_c0, sn_w; // column range [c0, c0 + w) in new order
  std::vector<int32_t> sn_parent;   // -1 for roots
  std::vector<int64_t> sn_rptr;     // R_s = rows[sn_rptr[s] .. sn_rptr[s+1]) (new order)
  std::vector<int32_t> rows;
  std::vector<int32_t> height, depth;
  std::vector<int64_t> sn_fwd_off, sn_bwd_off;  // panel offsets (complex entries) of each supernode
  int64_t fwd_entries = 0, bwd_entries = 0;
  double flops = 0;
  int32_t max_front = 0;
  int32_t tile_rows = 64;  // rows per solve tile (16, 32 or 64)
};

// tile_rows: rows per solve tile of the panels (16, 32 or 64); shorter tiles
// give a level more workgroups at the cost of re-reading its input columns.
void nested_dissection(const Csr& A, const std::vector<double>& coords, int leaf, Symbolic& S,
                       int tile_rows = 64);

// Numeric factor of one matrix in the solve layout.
struct TileDesc {
  int64_t off;   // offset of the tile in the panel buffer (complex entries)
  int32_t sn;    // supernode (batch-global id)
  int32_t row0;  // first front row of the tile
  int32_t nrows; // rows in the tile (<= 64)
  int32_t col0;  // first input column
  int32_t ncols; // input columns
  int32_t pad;
};

constexpr int kTileRows = 64;

// Pivots of a factored matrix (the numeric factorisation runs on the
// device, device_factor.hip).
struct NumericOut {
  std::vector<int32_t> piv;  // per new-order row position: pivot permutation within the supernode
  int32_t n_perturbed = 0;
};
// Tile shapes of a supernode's panels (rows [row0, row0+nrows), input
// columns [col0, col0+ncols)), in storage order.
struct TileShape {
  int32_t row0, nrows, col0, ncols;
};
void tiles_fwd(int32_t w, int32_t r, int32_t tile_rows, std::vector<TileShape>& out);
void tiles_bwd(int32_t w, int32_t r, int32_t tile_rows, std::vector<TileShape>& out);

// Overlapping subdomain (host side).
struct SubdomainHost {
  std::vector<int64_t> tets;   // tets of Gamma_i, ascending
  std::vector<int64_t> dofs;   // global dofs, ascending (R_i)
  std::vector<int32_t> level;  // overlap layer l(j)
  std::vector<double> chi, D;  // partition of unity
  std::vector<double> coords;  // [n_i][3]
  Csr A;                       // impedance local matrix
};
void build_subdomains(const Discretization& D, const int32_t* part, int32_t n_sub, int32_t overlap,
                      std::vector<SubdomainHost>& subs);

// coarse.cpp
void coarse_interpolation(const Discretization& D, const helm_mesh& cm, CsrReal& Z, std::vector<double>& ccoords);
void transpose_real(const CsrReal& A, CsrReal& T);
void galerkin(const Csr& A, const CsrReal& Z, const CsrReal& ZT, Csr& E);

}  // namespace helm
