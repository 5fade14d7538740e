// Launch wrappers of the HIP kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bddc_internal.h"

namespace bddc {

constexpr int MAX_PCG_IT = 8192;

struct MeshDevHost {
  int dim;
  int nel[3];
  double h[3];
};

enum {
  TRSV_FWD_RR = 0,  // L y = D W_i R_i r on the whole A_RR factor (+ border partials)
  TRSV_BWD_RR = 1,  // L^T x = y + W coef on the whole factor (-> weighted local output)
  TRSV_FWD_II = 2,  // interior block, rhs = D (r - A v12) on interior rows
  TRSV_BWD_II = 3   // interior block, z = v12 + D x on interior rows
};

struct TrsvArgs {
  const MatDesc* mats;
  const void* tiles;
  const void* dinv;
  const int32_t* tasks;
  int ntasks;
  unsigned* ticket;
  void* sol;             // published solution, sentinel-initialised
  const void* src;       // backward passes: the forward solution
  const int* done;       // optional early exit (converged PCG)
  const int32_t* gmap;
  const double* wd;      // weight * equilibration per local dof
  const double* dsc;     // equilibration per local dof
  const double* rin;     // forward input vector (global)
  const double* v12;     // FWD_II: subtract A v12 (may be null)
  const int32_t* rowptr;
  const int32_t* colind;
  const double* vals;
  double* part;          // FWD_RR border partial products
  const double* coef;    // BWD_RR per-matrix coefficients of the border columns
  double* ww;            // BWD_RR weighted local output
  double* zout;          // BWD_II output
  const double* base;    // BWD_II: added to the output (may be null)
  const int32_t* fcol;   // per tile row: first nonzero tile column (null: dense)
  const int32_t* lrow;   // backward passes, per tile column k: last tile row to read (null: dense)
  const int32_t* bptr;   // whole-space backward pass, per tile column k (vec_off / NB + k): its
  const int32_t* brows;  //   rows j > k inside the envelope, descending, brows[bptr[.]..bptr[.+1]) (null: range)
  const int32_t* btile;  //   and the tile (j, k) of each, counted from the matrix's tile_off
  const int32_t* iptr;   // interior backward pass, per tile column k: rows j inside the interior
  const int32_t* irows;  //   envelope, descending, and the tiles (j, k) and (j, k-1) (-1: zero),
  const int32_t* itile0; //   counted from the matrix's tile_off (null: the range k+1 .. lrow)
  const int32_t* itile1;
  int* werr;             // device status word: DEV_WAIT_GAVE_UP when a wait gives up
  int spin;              // polls of a published value before giving up (< 0: give up at once)
};

// bits of the device status word of a ctx (set by kernels, read and cleared by
// the host at the end of a solve or by bddc_sync)
constexpr int DEV_WAIT_GAVE_UP = 1;     // a triangular-solve task stopped waiting for a value
constexpr int DEV_COARSE_NOCONV = 2;    // the coarse CG stopped at its iteration limit or broke down


struct PcgScalars {
  double tol2;
  double bb;
  double rr0;
  int done;    // 0 running, 1 converged, 2 breakdown
  int iters;
  double rz[MAX_PCG_IT + 1];
  double pq[MAX_PCG_IT + 1];
  double rr[MAX_PCG_IT + 1];
  double alpha[MAX_PCG_IT + 1];
  double beta[MAX_PCG_IT + 1];
};

struct IfaceArgs {
  const MatDesc* mats;
  const void* m;            // symmetric interface matrices, one stream of ntiles tiles
  int m32;                  // their elements: 0 double, 1 float (applied with FP32 accumulation)
  const int32_t* tinfo;     // per tile: (global row << 8) | (ii - jj)
  const int32_t* trows;     // per tile: rows to read and column, h | z0 << 8 | z1 << 16 | jj << 24
                            //   (rows r < h outside [z0, z1))
  int64_t ntiles;
  int nwg;                  // workgroups of the mat-vec launch (its range split)
  const int32_t* tasks;     // finishers: (matrix, row ii)
  int ntasks;
  const PcgScalars* sc;
  const double* xpad;       // padded per-row input (64 per row): D^{-1} z + corners, or W D r
  int check_it;             // >= 0: first take the convergence decision of this CG iteration
  int* hdone;               // mapped pinned host word set to 1 when that decision ends the solve
  const double* part_rr;    // its partial sums of r.r
  int nparts_rr;            // their count
  double* part;             // column products, 64 per tile
  double* rowp;             // row products per row piece, 64 per piece start tile
  const double* dsc;
  const double* wd;
  const double* wgt;
  double* sploc;            // (S z) per local dof
  double* ww;               // weighted local preconditioner output
  const double* coef;       // coefficients of the coarse correction, MAX_NCI per subdomain
  int lds_cols;             // columns jj < lds_cols (<= SYM_LDS_COLS) have their products summed in LDS
  int row_pieces;           // row pieces (<= SYM_ROW_PIECES) a workgroup keeps in LDS until its end
};

template <typename T> void launch_fill(T* p, T v, int64_t n, hipStream_t st);
template <typename T> void launch_fill_sentinel(T* p, int64_t n, hipStream_t st);

void launch_check_theta(const double* theta, int64_t n, int* err, hipStream_t st);
void launch_assemble_csr(const MeshDevHost& m, const double* theta, const int32_t* rowptr, int32_t* col,
                         double* val, int64_t n, int* err, hipStream_t st);
// rho-scaling weights into wgt (per local dof); rho: scratch of n_loc doubles
void launch_rho_weights(const MeshDevHost& m, const double* theta, const MatDesc* mats, int nmats, int max_ni,
                        const int32_t* gmap, const int32_t* inv_ptr, const int32_t* inv, int64_t n_free,
                        double* rho, double* wgt, hipStream_t st);
void launch_local_assembly(const MeshDevHost& m, const double* theta, const MatDesc* mats, int nmats, int max_ni,
                           const int32_t* gmap, const int32_t* lmap, const double* wgt, double* dsc, double* wd,
                           const int32_t* avg_of, const double* avg_coef, void* tiles, bool fp32, double* app,
                           int* err, hipStream_t st);
void launch_pad_identity(const MatDesc* mats, int nmats, void* tiles, bool fp32, hipStream_t st);
// One persistent launch factors every matrix (left-looking, tile tasks in the
// order of make_factor_tasks); ready: nready ints of scratch, ticket: 1 counter.
// err bits: 2 non-positive pivot, 8 a dependency wait gave up.
void launch_factor_persistent(const MatDesc* mats, void* tiles, void* dinv, bool fp32, const int32_t* fcol,
                              const int32_t* tasks, int ntasks, unsigned* ticket, int* ready, int64_t nready,
                              int grid, int* err, hipStream_t st);
void launch_local_small(const MatDesc* mats, int nmats, const void* tiles, bool fp32, const double* app,
                        double* sainv, double* sainve, double* aci, double* cpp, int* err, hipStream_t st);
void launch_coarse_assembly(const int32_t* src_ptr, const int32_t* src, const int32_t* row, const int32_t* col,
                            const int32_t* diag, int nentries, int nc, const double* aci, double* val, double* dc,
                            double* tiles, int* err, hipStream_t st);
// t0 / t1: optional events recorded by the dispatch itself at kernel start / end
void launch_trsv(int mode, bool fp32, const TrsvArgs& a, int grid, hipStream_t st, hipEvent_t t0 = nullptr,
                 hipEvent_t t1 = nullptr);
// interior passes (TRSV_FWD_II, TRSV_BWD_II; launch_trsv routes them here): two
// tile rows per task, two workgroups per CU
void launch_trsv2(int mode, bool fp32, const TrsvArgs& a, int grid, hipStream_t st, hipEvent_t t0 = nullptr,
                  hipEvent_t t1 = nullptr);
void launch_coarse_prep(const MatDesc* mats, int nmats, const double* part, const double* sainv,
                        const double* sainve, const int32_t* gmap, const double* wgt, const double* r,
                        double* gbuf, double* mu, const int* done, const double* rowp, int64_t ntiles, int nwg,
                        hipStream_t st);
// (uc: nsplit partial vectors of nc values, summed in order)
void launch_coarse_coef(const MatDesc* mats, int nmats, const int32_t* rc, const double* uc, int nc, int nsplit,
                        const double* mu, const double* sainv, const double* sainve, const double* wgt,
                        double* coef, double* ww, const int* done, hipStream_t st);
void launch_gather_v12(const int32_t* inv_ptr, const int32_t* inv, const double* ww, const uint8_t* kappa,
                       double* v12, double* z, int64_t n, const int* done, hipStream_t st);
void launch_zero_interface(const uint8_t* kappa, double* x, int64_t n, hipStream_t st);
void launch_zero_interior(const uint8_t* kappa, double* x, int64_t n, hipStream_t st);
void launch_spmv(const int32_t* rowptr, const int32_t* col, const double* val, const double* x, double* y, int64_t n,
                 hipStream_t st);
void launch_residual(const int32_t* rowptr, const int32_t* col, const double* val, const double* x, const double* b,
                     double* r, double* part_rr, double* part_bb, int64_t n, hipStream_t st,
                     const uint8_t* iface_only = nullptr);
void launch_pcg_init(const double* part_rr, const double* part_bb, PcgScalars* sc, double rtol2, hipStream_t st);
void launch_pcg_dir(const int32_t* rowptr, const int32_t* col, const double* val, const double* z, double* p,
                    double* q, const double* part_rz, double* part_pq, PcgScalars* sc, int it, int fresh, int64_t n,
                    hipStream_t st);
void launch_pcg_update(double* x, double* r, const double* p, const double* q, const double* part_pq,
                       double* part_rr, PcgScalars* sc, int it, int64_t n, hipStream_t st);
// hdone: mapped pinned host word set to 1 when the solve ends (may be null)
void launch_pcg_check(const double* part_rr, PcgScalars* sc, int it, int* hdone, hipStream_t st);
// out: mapped pinned host memory of 5 + 3 n doubles
void launch_pack_readback(const PcgScalars* sc, const double* rr_true, const int* werr, int seg, int n,
                          double* out, hipStream_t st);
void launch_dot(const double* a, const double* b, double* part, int64_t n, const int* done, hipStream_t st);
void launch_finish_dot(const double* part, double* out, hipStream_t st);
void launch_elem_grad(const MeshDevHost& m, const double* lam, const double* u, double* g, int64_t nel,
                      hipStream_t st);

constexpr int VEC_GRID = 1024;   // partial-sum count of the vector kernels

// Before the triangular passes: sentinels into the published-solution buffers,
// tickets to zero, and (n > 0) zero_all[i] = 0 and zero_iface[i] = 0 where
// kappa[i] > 1 (either may be null).
void launch_reset(bool fp32, void* pub, int64_t n_pub, double* pubc, int64_t n_pubc, unsigned* tickets,
                  const int* done, hipStream_t st, const uint8_t* kappa = nullptr, double* zero_iface = nullptr,
                  double* zero_all = nullptr, int64_t n = 0);



// interface-form vector kernels over the interface dofs (IFC_MAXC copy slots each)
struct IfcArgs {
  const int32_t* g;         // global index of interface dof k
  const int32_t* l;         // local copies (-1 past the last)
  const int32_t* slotz;     // their slots in the operator's padded input
  const int32_t* slotf;     // their slots in the preconditioner's padded input
  const double* dsc;        // equilibration of each copy
  const double* wd;         // weight * equilibration of each copy
  int64_t n;
  PcgScalars* sc;
  int it;
  int fresh;
  const double* part_in;    // partial sums read (r.z or p.q)
  double* part_out;         // partial sums written
  const double* ww;         // weighted local preconditioner output
  const double* sploc;      // (S z) per local dof
  double* x;
  double* r;
  double* z;
  double* p;
  double* q;
  double* zpad;
  double* fpad;
};
void launch_ifc_setup(const int32_t* ifc_l, const double* dsc, const double* wd, double* ifc_dsc, double* ifc_wd,
                      int64_t n_ifc, hipStream_t st);
int ifc_blocks(int64_t n);
void launch_gather_z_ifc(const IfcArgs& a, hipStream_t st);
void launch_gather_sp_ifc(const IfcArgs& a, hipStream_t st);
void launch_pcg_update_ifc(const IfcArgs& a, hipStream_t st);
void launch_scatter_f_ifc(const IfcArgs& a, hipStream_t st);
enum { SYM_OP = 0, SYM_PC = 1 };
// out32: write the matrices as float (the preconditioner's only)
void launch_sym_build(int mode, const MatDesc* mats, int nmats, int maxTS, const double* tiles, const double* xg,
                      const double* cpp, void* out, bool out32, hipStream_t st);
void launch_sym_mv(const IfaceArgs& a, hipStream_t st, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
void launch_op_finish(const IfaceArgs& a, hipStream_t st);
void launch_pc_finish(const IfaceArgs& a, hipStream_t st);
constexpr int COARSE_SPLIT_COLS = 512;   // columns of A_c^{-1} per coarse GEMV block
constexpr int IFACE_MAX_TS = 255;        // interface form: tile rows of a symmetric interface matrix
constexpr int SYM_LDS_COLS = 64;         // interface mat-vec: columns whose products a workgroup sums in LDS
constexpr int SYM_ROW_PIECES = 28;       // interface mat-vec: row pieces a workgroup keeps in LDS until its end
void launch_coarse_inverse(const double* xg, const double* dc, int nc, double* ainv, hipStream_t st);
void launch_coarse_gemv(const double* ainv, int nc, int nsplit, const int32_t* cinv_ptr, const int32_t* cinv,
                        const double* gbuf, double* upart, const int* done, hipStream_t st);
// coarse problem by Jacobi-preconditioned CG in one workgroup (u = A_c^{-1} r_c to
// relative residual tol); work: 3 nc doubles
// full symmetric A_c in CSR for the coarse CG: fval[k] = val[fsrc[k]]
void launch_coarse_cg_matrix(const int32_t* fsrc, const double* val, double* fval, int nnz, hipStream_t st);
// (work: 7 nc doubles, and at least nc + 3 * 64 doubles + 2 words for the
// multi-workgroup variant used when A_c does not fit one workgroup's LDS; its
// grid barrier gives up after `spin` polls and records DEV_WAIT_GAVE_UP)
bool coarse_cg_grid_fits(int nc);
void launch_coarse_cg(const int32_t* rowptr, const int32_t* col, const double* fval, int nnz, const double* dc,
                      int nc, const int32_t* cinv_ptr, const int32_t* cinv, const double* gbuf, double* u,
                      double* work, double tol, int maxit, int spin, const int* done, int* werr,
                      hipStream_t st);
// Size of the fixed device workspace of the allocation-free apply, and its
// address on the current device (looked up once per device; 0 on success).
constexpr size_t STATIC_SCRATCH_BYTES = size_t(64) << 20;
int static_scratch_address(void** ptr);

void launch_trailing_inverse(const MatDesc* mats, int nmats, int maxTG, const double* tiles, const double* dinv,
                             double* xg, hipStream_t st);

}  // namespace bddc
