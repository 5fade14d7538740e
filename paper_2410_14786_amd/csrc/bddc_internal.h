// Internal declarations shared by the host planner, the kernels and the ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bddc.h"

namespace bddc {

constexpr int NB = 64;        // tile edge (rows and columns) of every dense factor
constexpr int MAX_NCI = 64;   // constraints per subdomain (one extra tile row)
constexpr int IFC_MAXC = 8;   // subdomains sharing one dof (2^dim at most for box partitions)

// Envelope storage of one tile row of a factor: its first stored column fc (the
// tiles left of it are zero) and rd = (its first stored tile, counted from the
// matrix's first tile) - fc, so that tile (i, j) is tile_off + rd + j.
struct EnvRow {
  int32_t fc;
  int32_t rd;
};

// Per-matrix descriptor used by the factorisation and the triangular solves.
// A "matrix" is a subdomain's equilibrated A_RR bordered by one extra tile row
// holding (D B)^T with B = [C_AR^T | A_RPi], or the coarse matrix A_c.
struct MatDesc {
  int64_t tile_off;   // first tile of this matrix in the tile array
  int64_t dinv_off;   // first inverse-diagonal tile
  int64_t vec_off;    // offset of this matrix's padded vectors (T*NB entries)
  int64_t loc_off;    // offset of its local dof arrays (n_i entries)
  int32_t T;          // factored tile rows: ceil(n_R / NB)
  int32_t Tx;         // stored tile rows: T + 1 with the border row, else T
  int32_t TI;         // tile rows covering the interior block: ceil(n_I / NB)
  int32_t n_R;        // rows of A_RR (interior + non-corner interface)
  int32_t n_I;        // interior rows (the leading block)
  int32_t n_i;        // all local dofs (n_R + corners)
  int32_t n_A;        // average constraints
  int32_t n_P;        // corner (primal point) constraints
  int32_t n_ci;       // n_A + n_P
  int32_t coarse_off; // offset into the per-subdomain coarse arrays
  int32_t box_lo[3];  // first element of the box along each axis
  int32_t box_len[3]; // box length in elements
  int32_t lmap_off;   // offset of the box-node -> local index table
  int32_t sym_row;    // global index of this matrix's first row of symmetric interface tiles
  int64_t xg_off;     // first tile of the inverse of the trailing block (tile rows n_I/NB .. T-1)
  int64_t sg_off;     // first tile of the symmetric interface matrices (sym_tile_rows tile rows)
  // Envelope storage of the factor: tile row i < T holds only its tiles env[i].fc
  // .. i (those left of the envelope are zero), tile (i, j) at tile_off +
  // env[i].rd + j; the border row T holds all tiles 0 .. T from tile_off + tb.
  // env points to this matrix's rows of the per-row table (the host copy in the
  // plan, the device copy in the uploaded descriptors); null: every row dense.
  const EnvRow* env;
  int64_t tb;
  int64_t ztile;      // the shared all-zero tile, read for any tile left of the envelope
};

// Host-side plan: everything bddc_setup derives from the mesh and partition
// before any device work.
struct Plan {
  int dim = 0;
  int64_t nel[3] = {1, 1, 1};
  int nsub[3] = {1, 1, 1};
  std::vector<int64_t> cuts[3];
  uint32_t constraints = 0;
  int64_t n_free = 0;
  int64_t n_el = 0;
  int nsubs = 0;

  // global CSR pattern (values come from the device assembly)
  std::vector<int32_t> rowptr;   // n_free + 1
  int64_t nnz = 0;
  std::vector<uint8_t> kappa;    // multiplicity of each free dof

  std::vector<MatDesc> subs;
  // concatenated local arrays (sum n_i): order [interior | interface R | corners]
  std::vector<int32_t> gmap;     // local dof -> global free dof
  std::vector<double> weight;    // 1/kappa
  std::vector<int32_t> avg_of;   // local average-constraint index, or -1
  std::vector<double> avg_coef;  // 1/(nodes in the class) for constrained dofs
  std::vector<int32_t> lmap;     // box node -> local index, -1 on the Dirichlet boundary

  // coarse space
  int n_coarse = 0;
  int n_corner_classes = 0, n_edge_classes = 0, n_face_classes = 0;
  std::vector<int32_t> rc;        // per subdomain local coarse index -> global (sum n_ci)
  std::vector<int32_t> cinv_ptr;  // global coarse dof -> slots in rc
  std::vector<int32_t> cinv;
  std::vector<int32_t> inv_ptr;   // global dof -> slots in the local arrays
  std::vector<int32_t> inv;

  // coarse matrix assembly: unique lower entries (p >= q) and their sources
  std::vector<int32_t> ac_row, ac_col;   // per unique entry
  std::vector<int32_t> ac_src_ptr;       // per unique entry -> sources
  std::vector<int32_t> ac_src;           // source = s * MAX_NCI*MAX_NCI + a*MAX_NCI + b
  std::vector<int32_t> ac_diag;          // entry index of (p, p)

  // envelope of each local factor (indexed vec_off/NB + tile row): fcol = first
  // tile column holding a nonzero of that tile row of L (tiles left of it are
  // zero: Cholesky fills no entry left of a row's first nonzero of A_RR), fcol_ii
  // the same over the interior rows only; lrow_rr / lrow_ii = last tile row j
  // (j < T with fcol[j] <= k, resp. j < TI with fcol_ii[j] <= k), the rows a
  // backward pass over column k reads
  std::vector<int32_t> fcol, fcol_ii, lrow_rr, lrow_ii;
  // per tile row (vec_off / NB + i): the envelope storage of that row
  std::vector<EnvRow> envrow;
  // per tile column k (vec_off / NB + k, one extra end entry): the rows j > k
  // of L_RR whose envelope reaches column k, in descending order, and the index
  // of tile (j, k) counted from the matrix's tile_off
  std::vector<int32_t> bptr, brows, btile;
  // the same for the interior block (tile columns k < TI, rows j <= lrow_ii[k]
  // with fcol_ii[j] <= k; empty for k >= TI): row, tile (j, k) and tile (j, k-1)
  // (-1 when left of row j's interior envelope), counted from tile_off
  std::vector<int32_t> iptr, irows, itile0, itile1;

  // ticket-ordered task lists of the triangular solves, (matrix, tile row)
  std::vector<int32_t> fwd_rr, bwd_rr, fwd_ii, bwd_ii;
  // ticket-ordered tile tasks of the persistent factorisation, (matrix, i, j)
  std::vector<int32_t> factor_tasks;
  // interface form: the symmetric interface matrices of all subdomains form one
  // stream of n_sg tiles (sg_off order) and n_symrows tile rows (sym_row order).
  // symfin = (matrix, ii) per row; tinfo per tile = (global row << 8) | (ii - jj);
  // padz / padf per local dof: its slot in the padded per-row input vectors
  // (64 per row) of the operator (interface and corner dofs) and of the
  // preconditioner (interface dofs), -1 elsewhere
  std::vector<int32_t> symfin, tinfo, padz, padf;
  // per tile, the rows the mat-vec reads and the tile's column jj:
  // h | z0 << 8 | z1 << 16 | jj << 24 (rows below h outside [z0, z1)); the
  // operator skips its zero average-constraint rows
  std::vector<int32_t> trows_op, trows_pc;
  int64_t n_symrows = 0;
  // floating-point operations of the batched tile Cholesky inside the envelope
  // (diagonal factor 64^3/3, panel solve 64^3, update 2*64^3, diagonal update 64^3)
  double factor_flops = 0.0;
  // interface dofs (kappa >= 2): global index and IFC_MAXC local copies each
  // (local dof, operator slot, preconditioner slot; -1 past the last copy)
  std::vector<int32_t> ifc_g, ifc_l, ifc_slotz, ifc_slotf;

  int maxT = 0, maxTx = 0, maxTI = 0;
  int64_t n_tiles = 0, n_dinv = 0, n_vec = 0, n_loc = 0, n_lmap = 0, n_xg = 0, n_sg = 0;
  int maxTG = 0, maxTS = 0;
  int max_nci = 0;
};

// Tile tasks (matrix, i, j) of the persistent left-looking factorisation in
// ticket order; fcol: per tile row (vec_off / NB + i) first envelope column, or
// null for dense matrices.  Checks that every tile a task reads comes earlier.
int make_factor_tasks(const std::vector<MatDesc>& mats, const std::vector<int32_t>* fcol, std::vector<int32_t>& out,
                      std::string& err);

// Validates and plans; returns a bddc_status, with a message in err.
int make_plan(const bddc_mesh* mesh, const bddc_partition* part, uint32_t constraints,
              Plan& plan, std::string& err);

#if defined(__HIPCC__)
#define BDDC_HD __host__ __device__
#else
#define BDDC_HD
#endif

// Tile index of tile (i, j), j <= i, inside a matrix's packed lower storage.
BDDC_HD inline int64_t tri_tile(int64_t i, int64_t j) { return i * (i + 1) / 2 + j; }

// Index of stored tile (i, j), j <= i, of a matrix's factor (see MatDesc).
BDDC_HD inline int64_t env_tile(const MatDesc& D, int i, int j) {
  if (i >= D.T) return D.tile_off + D.tb + j;
  if (D.env == nullptr) return D.tile_off + tri_tile(i, j);
  const EnvRow e = D.env[i];
  return j < e.fc ? D.ztile : D.tile_off + e.rd + j;
}

// Tile (i, j) of row i is row_origin(D, i) + j for every j inside the row's
// envelope (and the border row): one lookup per row for loops along a row.
BDDC_HD inline int64_t row_origin(const MatDesc& D, int i) {
  if (i >= D.T) return D.tile_off + D.tb;
  if (D.env == nullptr) return D.tile_off + tri_tile(i, 0);
  return D.tile_off + D.env[i].rd;
}

// Symmetric interface matrices of a subdomain: rows 0..n_G-1 are its interface
// rows (local dofs n_I..n_R-1), rows n_G..n_G+n_ci-1 its constraints; tile rows:
BDDC_HD inline int sym_tile_rows(const MatDesc& D) { return (D.n_R - D.n_I + D.n_ci + NB - 1) / NB; }

}  // namespace bddc
