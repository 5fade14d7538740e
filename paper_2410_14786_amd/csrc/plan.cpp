// Host stage of bddc_setup: validation, dof numbering, multiplicities, interface
// classes, local orderings, coarse numbering, inverse maps and task lists.
//
// Paper Sec. 2 fixes what is computed: subdomain restrictions R_i, weights
// w = 1/kappa with kappa the number of subdomains sharing a dof, constraints
// that take full values at corners and averages over edges and faces, and the
// local-to-global coarse maps R_ci.  For a tensor-product box partition the
// set of subdomains sharing an interface node is fixed by which interior cut
// planes the node lies on, so a class is named by a position code per axis
// (inside box interval m, or on cut c) and its kind by how many axes are cut:
// all of them -> corner, dim-1 -> edge, one (3D) -> face.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "bddc_internal.h"

namespace bddc {

namespace {

struct AxisInfo {
  std::vector<int32_t> cut_of;   // node coordinate -> interior cut index (1..nsub-1) or -1
  std::vector<int32_t> box_of;   // node coordinate -> box interval m with cuts[m] <= x < cuts[m+1]
};

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

int make_plan(const bddc_mesh* mesh, const bddc_partition* part, uint32_t constraints,
              Plan& P, std::string& err) {
  if (!mesh || !part) { err = "mesh and partition must not be NULL"; return BDDC_EINVAL; }
  if (mesh->dim != 2 && mesh->dim != 3) { err = "dim must be 2 or 3"; return BDDC_EINVAL; }
  if (constraints & ~15u) { err = "unknown constraint bits"; return BDDC_EINVAL; }
  P = Plan();
  P.dim = mesh->dim;
  P.constraints = constraints;
  const int dim = P.dim;
  int64_t nfree = 1, nel_tot = 1;
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      if (mesh->nel[a] < 2 || mesh->nel[a] > (1 << 20)) { err = "nel must be in [2, 2^20]"; return BDDC_EINVAL; }
      P.nel[a] = mesh->nel[a];
      if (part->nsub[a] < 1 || part->nsub[a] > mesh->nel[a]) { err = "nsub out of range"; return BDDC_EINVAL; }
      if (!part->cuts[a]) { err = "cuts must not be NULL"; return BDDC_EINVAL; }
      P.nsub[a] = part->nsub[a];
      P.cuts[a].assign(part->cuts[a], part->cuts[a] + part->nsub[a] + 1);
      if (P.cuts[a].front() != 0 || P.cuts[a].back() != P.nel[a]) { err = "cuts must start at 0 and end at nel"; return BDDC_EINVAL; }
      for (int m = 0; m < P.nsub[a]; ++m)
        if (P.cuts[a][m + 1] - P.cuts[a][m] < 2) { err = "every box must be at least 2 elements long"; return BDDC_EINVAL; }
      nfree *= P.nel[a] - 1;
      nel_tot *= P.nel[a];
    } else {
      P.nel[a] = 1;
      P.nsub[a] = 1;
      P.cuts[a] = {0, 1};
    }
  }
  if (nfree >= (int64_t(1) << 31) - 1) { err = "too many dofs for 32-bit indices"; return BDDC_EINVAL; }
  P.n_free = nfree;
  P.n_el = nel_tot;
  P.nsubs = P.nsub[0] * P.nsub[1] * P.nsub[2];

  // per-axis node information (node coordinates 0..nel)
  AxisInfo ax[3];
  for (int a = 0; a < 3; ++a) {
    const int64_t n = (a < dim) ? P.nel[a] : 1;
    ax[a].cut_of.assign(n + 1, -1);
    ax[a].box_of.assign(n + 1, 0);
    for (int c = 1; c < P.nsub[a]; ++c) ax[a].cut_of[P.cuts[a][c]] = c;
    int m = 0;
    for (int64_t x = 0; x <= n; ++x) {
      while (m + 1 < P.nsub[a] && x >= P.cuts[a][m + 1]) ++m;
      ax[a].box_of[x] = m;
    }
  }
  const int64_t nx1 = P.nel[0] - 1, ny1 = P.nel[1] - 1;
  auto free_index = [&](const int64_t c[3]) -> int64_t {
    for (int a = 0; a < dim; ++a)
      if (c[a] < 1 || c[a] > P.nel[a] - 1) return -1;
    int64_t idx = c[0] - 1;
    if (dim >= 2) idx += nx1 * (c[1] - 1);
    if (dim >= 3) idx += nx1 * ny1 * (c[2] - 1);
    return idx;
  };
  // position code per axis: inside interval m -> 2m, on interior cut c -> 2c-1
  int64_t pcount[3];
  for (int a = 0; a < 3; ++a) pcount[a] = 2 * P.nsub[a] - 1;
  auto class_key = [&](const int64_t c[3], int& ncut) -> int64_t {
    int64_t key = 0, stride = 1;
    ncut = 0;
    for (int a = 0; a < dim; ++a) {
      int cc = ax[a].cut_of[c[a]];
      int64_t pc = cc >= 0 ? 2 * cc - 1 : 2 * ax[a].box_of[c[a]];
      if (cc >= 0) ++ncut;
      key += pc * stride;
      stride *= pcount[a];
    }
    return key;
  };
  auto kind_of = [&](int ncut) -> int {  // 1 corner, 2 edge, 4 face, 0 interior
    if (ncut == 0) return 0;
    if (ncut == dim) return 1;
    if (ncut == dim - 1) return 2;
    return 4;
  };
  const bool all_primal = constraints & BDDC_ALL_PRIMAL;
  auto active = [&](int kind) -> bool {
    if (all_primal) return kind != 0;
    return (kind == 1 && (constraints & BDDC_CORNERS)) || (kind == 2 && (constraints & BDDC_EDGES)) ||
           (kind == 4 && (constraints & BDDC_FACES));
  };

  // ---- global pass: multiplicity, class sizes, CSR pattern ----
  P.kappa.assign(nfree, 1);
  std::unordered_map<int64_t, int32_t> class_size;   // key -> number of nodes
  std::unordered_map<int64_t, int> class_kind;
  P.rowptr.assign(nfree + 1, 0);
  {
    int64_t c[3] = {1, 1, 1};
    const int64_t nz = dim == 3 ? P.nel[2] - 1 : 1;
    const int64_t ny = P.nel[1] - 1;
    int64_t g = 0;
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx1; ++x, ++g) {
          c[0] = x + 1; c[1] = y + 1; c[2] = dim == 3 ? z + 1 : 0;
          int ncut;
          int64_t key = class_key(c, ncut);
          P.kappa[g] = uint8_t(1 << ncut);
          if (ncut) {
            class_size[key] += 1;
            class_kind[key] = kind_of(ncut);
          }
          int64_t cnt = 1;
          for (int a = 0; a < dim; ++a) {
            int64_t k = 1 + (c[a] - 1 >= 1) + (c[a] + 1 <= P.nel[a] - 1);
            cnt *= k;
          }
          P.rowptr[g + 1] = int32_t(cnt);
        }
  }
  {
    int64_t acc = 0;
    for (int64_t g = 0; g < nfree; ++g) {
      acc += P.rowptr[g + 1];
      if (acc >= (int64_t(1) << 31)) { err = "too many nonzeros for 32-bit row pointers"; return BDDC_EINVAL; }
      P.rowptr[g + 1] = int32_t(acc);
    }
    P.nnz = acc;
  }
  // coarse numbering: active classes sorted by key (all-primal: one per node, by dof)
  std::unordered_map<int64_t, int32_t> coarse_of_class;
  std::vector<int64_t> keys;
  for (auto& kv : class_kind) {
    if (kv.second == 1) ++P.n_corner_classes;
    if (kv.second == 2) ++P.n_edge_classes;
    if (kv.second == 4) ++P.n_face_classes;
    if (active(kv.second)) keys.push_back(kv.first);
  }
  std::sort(keys.begin(), keys.end());
  std::vector<int32_t> coarse_of_dof;   // all-primal only
  if (all_primal) {
    coarse_of_dof.assign(nfree, -1);
    int32_t id = 0;
    for (int64_t g = 0; g < nfree; ++g)
      if (P.kappa[g] > 1) coarse_of_dof[g] = id++;
    P.n_coarse = id;
  } else {
    for (size_t i = 0; i < keys.size(); ++i) coarse_of_class[keys[i]] = int32_t(i);
    P.n_coarse = int(keys.size());
  }

  // ---- subdomains ----
  P.subs.resize(P.nsubs);
  int64_t loc_off = 0, lmap_off = 0, tile_off = 0, dinv_off = 0, vec_off = 0;
  int32_t coarse_off = 0;
  std::vector<int32_t> inv_count(nfree, 0);
  for (int s = 0; s < P.nsubs; ++s) {
    MatDesc& D = P.subs[s];
    std::memset(&D, 0, sizeof(D));
    int b[3] = {s % P.nsub[0], (s / P.nsub[0]) % P.nsub[1], s / (P.nsub[0] * P.nsub[1])};
    int64_t lo[3], len[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = P.cuts[a][b[a]];
      len[a] = P.cuts[a][b[a] + 1] - lo[a];
      if (a >= dim) { lo[a] = 0; len[a] = 0; }
      D.box_lo[a] = int32_t(lo[a]);
      D.box_len[a] = int32_t(len[a]);
    }
    const int64_t n1[3] = {len[0] + 1, len[1] + 1, dim == 3 ? len[2] + 1 : 1};
    const int64_t nbox = n1[0] * n1[1] * n1[2];
    std::vector<int64_t> interior, gamma;
    std::vector<std::pair<int32_t, int64_t>> corners;   // (coarse id, node)
    std::vector<std::pair<int32_t, int64_t>> avgs;      // (coarse id of average class) - unique
    std::vector<int32_t> node_coarse(nbox, -1);         // coarse id of an average class for Gamma_R nodes
    for (int64_t q = 0; q < nbox; ++q) {
      int64_t lc[3] = {q % n1[0], (q / n1[0]) % n1[1], q / (n1[0] * n1[1])};
      int64_t c[3] = {lo[0] + lc[0], lo[1] + lc[1], dim == 3 ? lo[2] + lc[2] : 0};
      int64_t g = free_index(c);
      if (g < 0) continue;
      bool inside = true;
      for (int a = 0; a < dim; ++a) inside &= (lc[a] > 0 && lc[a] < len[a]);
      if (inside) { interior.push_back(q); continue; }
      int ncut;
      int64_t key = class_key(c, ncut);
      int kind = kind_of(ncut);
      if (all_primal) {
        corners.push_back({coarse_of_dof[g], q});
      } else if (kind == 1 && active(kind)) {
        corners.push_back({coarse_of_class[key], q});
      } else {
        gamma.push_back(q);
        if (active(kind)) {
          int32_t cid = coarse_of_class[key];
          node_coarse[q] = cid;
          avgs.push_back({cid, key});
        }
      }
    }
    std::sort(corners.begin(), corners.end());
    std::sort(avgs.begin(), avgs.end());
    avgs.erase(std::unique(avgs.begin(), avgs.end()), avgs.end());
    D.n_I = int32_t(interior.size());
    D.n_R = int32_t(interior.size() + gamma.size());
    D.n_P = int32_t(corners.size());
    D.n_A = int32_t(avgs.size());
    D.n_ci = D.n_A + D.n_P;
    D.n_i = D.n_R + D.n_P;
    if (D.n_ci > MAX_NCI) {
      err = "a subdomain has more than 64 constraints";
      return BDDC_ENOTIMPL;
    }
    // A_RR is factored by Cholesky.  For a box that touches no Dirichlet
    // boundary (every face an interior cut) it is the Neumann matrix of the box
    // minus its corner nodes: singular when no corner is a primal constraint
    // (and SPD otherwise, or when any box node is a Dirichlet node)
    {
      bool floating = true;
      for (int a = 0; a < dim; ++a) floating = floating && lo[a] > 0 && lo[a] + len[a] < P.nel[a];
      if (floating && D.n_P == 0) {
        err = "subdomain " + std::to_string(s) + " touches no Dirichlet boundary and has no corner constraints, so "
              "its A_RR is singular (add BDDC_CORNERS)";
        return BDDC_ENOTSPD;
      }
    }
    P.max_nci = std::max(P.max_nci, int(D.n_ci));
    D.loc_off = loc_off;
    D.lmap_off = int32_t(lmap_off);
    D.coarse_off = coarse_off;
    D.T = int32_t(ceil_div(D.n_R, NB));
    D.Tx = D.T + (D.n_ci > 0 ? 1 : 0);
    D.TI = int32_t(ceil_div(D.n_I, NB));
    D.tile_off = tile_off;
    D.dinv_off = dinv_off;
    D.vec_off = vec_off;
    dinv_off += D.T;
    vec_off += int64_t(D.T) * NB;
    if (lmap_off + nbox >= (int64_t(1) << 31)) { err = "box tables too large"; return BDDC_EINVAL; }

    // local arrays in order [interior | Gamma_R | corners]
    P.lmap.resize(lmap_off + nbox, -1);
    std::unordered_map<int32_t, int32_t> avg_local;
    for (int a = 0; a < D.n_A; ++a) avg_local[avgs[a].first] = a;
    auto push_local = [&](int64_t q) {
      int64_t lc[3] = {q % n1[0], (q / n1[0]) % n1[1], q / (n1[0] * n1[1])};
      int64_t c[3] = {lo[0] + lc[0], lo[1] + lc[1], dim == 3 ? lo[2] + lc[2] : 0};
      int64_t g = free_index(c);
      int32_t l = int32_t(P.gmap.size() - loc_off);
      P.lmap[lmap_off + q] = l;
      P.gmap.push_back(int32_t(g));
      P.weight.push_back(1.0 / double(P.kappa[g]));
      int32_t cid = node_coarse[q];
      if (cid >= 0) {
        int ncut;
        int64_t key = class_key(c, ncut);
        P.avg_of.push_back(avg_local[cid]);
        P.avg_coef.push_back(1.0 / double(class_size[key]));
      } else {
        P.avg_of.push_back(-1);
        P.avg_coef.push_back(0.0);
      }
      inv_count[g] += 1;
    };
    for (int64_t q : interior) push_local(q);
    for (int64_t q : gamma) push_local(q);
    for (auto& cq : corners) push_local(cq.second);
    // envelope of A_RR by tile rows: a Q1 node couples with the nodes of the
    // elements around it, |offset| <= 1 per axis inside the box
    {
      std::vector<int32_t> fc(D.T), fi(D.T);   // all rows of A_RR, interior rows only
      for (int k = 0; k < D.T; ++k) fc[k] = fi[k] = k;
      for (int64_t q = 0; q < nbox; ++q) {
        const int32_t la = P.lmap[lmap_off + q];
        if (la < 0 || la >= D.n_R) continue;
        const int64_t lc[3] = {q % n1[0], (q / n1[0]) % n1[1], q / (n1[0] * n1[1])};
        int32_t fmin = la;
        for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int64_t x = lc[0] + dx, y = lc[1] + dy, z = lc[2] + dz;
              if (x < 0 || x >= n1[0] || y < 0 || y >= n1[1] || z < 0 || z >= n1[2]) continue;
              const int32_t lb = P.lmap[lmap_off + (z * n1[1] + y) * n1[0] + x];
              if (lb >= 0 && lb < D.n_R) fmin = std::min(fmin, lb);
            }
        fc[la / NB] = std::min(fc[la / NB], fmin / NB);
        if (la < D.n_I) fi[la / NB] = std::min(fi[la / NB], fmin / NB);
      }
      // envelope storage: row k keeps tiles fc[k] .. k, tile (k, j) at rd[k] + j
      // from the matrix's first tile, then the dense border row
      std::vector<int64_t> rd(D.T);
      int64_t off = 0;
      for (int k = 0; k < D.T; ++k) {
        rd[k] = off - fc[k];
        off += k - fc[k] + 1;
      }
      if (off >= (int64_t(1) << 31)) { err = "a local factor has too many tiles"; return BDDC_EINVAL; }
      for (int k = 0; k < D.T; ++k) P.envrow.push_back(EnvRow{fc[k], int32_t(rd[k])});
      D.tb = off;
      tile_off += off + (D.Tx > D.T ? D.T + 1 : 0);
      for (int k = 0; k < D.T; ++k) {
        int32_t lr = k, li = k;
        for (int j = k + 1; j < D.T; ++j) {
          if (fc[j] <= k) lr = j;
          if (j < D.TI && fi[j] <= k) li = j;
        }
        P.lrow_rr.push_back(lr);
        P.lrow_ii.push_back(li);
        P.bptr.push_back(int32_t(P.brows.size()));
        for (int j = D.T - 1; j > k; --j)
          if (fc[j] <= k) {
            P.brows.push_back(j);
            P.btile.push_back(int32_t(rd[j] + k));
          }
      }
      // the forward interior pass reads each interior tile row k from fi[k] on
      // along the stored row: inside the row's envelope (fi >= fc)
      for (int k = 0; k < D.TI; ++k)
        if (fi[k] < fc[k]) { err = "internal: interior envelope outside the factor envelope"; return BDDC_EINVAL; }
      for (int k = 0; k < D.T; ++k) {
        P.iptr.push_back(int32_t(P.irows.size()));
        if (k >= D.TI) continue;
        const int lr = P.lrow_ii[P.lrow_ii.size() - D.T + k];
        for (int j = lr; j > k; --j)
          if (fi[j] <= k) {
            P.irows.push_back(j);
            P.itile0.push_back(int32_t(rd[j] + k));
            P.itile1.push_back(k >= 1 && fi[j] <= k - 1 ? int32_t(rd[j] + k - 1) : -1);
          }
      }
      P.fcol.insert(P.fcol.end(), fc.begin(), fc.end());
      P.fcol_ii.insert(P.fcol_ii.end(), fi.begin(), fi.end());
      {
        // the tile operations the factorisation runs: tile (i, k) is zero when
        // k < fc[i] (the bordering row T, if any, is dense)
        // (per column k: a panel solve for every nonzero tile (i, k), a diagonal
        // update of (i, i) and an off-diagonal update of (i, j) for every nonzero
        // (j, k) with k < j < i, counted by a running total over i)
        const double b3 = double(NB) * NB * NB;
        auto nz = [&](int i, int k) { return i >= D.T || fc[i] <= k; };
        for (int k = 0; k < D.T; ++k) {
          P.factor_flops += b3 / 3.0;
          int64_t above = 0;   // nonzero tiles (j, k), k < j < i
          for (int i = k + 1; i < D.Tx; ++i) {
            if (!nz(i, k)) continue;
            P.factor_flops += b3 + b3 + 2.0 * b3 * double(above);
            ++above;
          }
        }
      }
    }
    // local coarse order [averages | corners]
    for (auto& a : avgs) P.rc.push_back(a.first);
    for (auto& cq : corners) P.rc.push_back(cq.first);
    loc_off += D.n_i;
    lmap_off += nbox;
    coarse_off += D.n_ci;
    P.maxT = std::max(P.maxT, int(D.T));
    P.maxTx = std::max(P.maxTx, int(D.Tx));
    P.maxTI = std::max(P.maxTI, int(D.TI));
  }
  {
    int64_t xg = 0, sg = 0, rows = 0;
    for (auto& D : P.subs) {
      const int TG = D.T - D.n_I / NB;
      D.xg_off = xg;
      D.sg_off = sg;
      const int TS = sym_tile_rows(D);
      D.sym_row = int32_t(rows);
      const int nG = D.n_R - D.n_I, m = nG + D.n_ci;
      auto clamp64 = [](int v) { return std::max(0, std::min(NB, v)); };
      for (int ii = 0; ii < TS; ++ii) {
        const int h = clamp64(m - ii * NB);
        const int z0 = clamp64(nG - ii * NB), z1 = clamp64(nG + D.n_A - ii * NB);
        for (int jj = 0; jj <= ii; ++jj) {
          P.tinfo.push_back(int32_t(((rows + ii) << 8) | (ii - jj)));
          const uint32_t col = uint32_t(jj & 255) << 24;   // the interface form has TS <= IFACE_MAX_TS
          P.trows_op.push_back(int32_t(uint32_t(h | (z0 << 8) | (z1 << 16)) | col));
          P.trows_pc.push_back(int32_t(uint32_t(h) | col));
        }
      }
      xg += tri_tile(TG, 0);
      sg += tri_tile(TS, 0);
      rows += TS;
      P.maxTG = std::max(P.maxTG, TG);
      P.maxTS = std::max(P.maxTS, TS);
    }
    P.n_xg = xg;
    P.n_sg = sg;
    P.n_symrows = rows;
    if (rows >= (int64_t(1) << 23)) { err = "too many interface tile rows"; return BDDC_EINVAL; }
    // padded input slots of the local dofs
    P.padz.assign(loc_off, -1);
    P.padf.assign(loc_off, -1);
    for (auto& D : P.subs) {
      const int nG = D.n_R - D.n_I;
      for (int r = 0; r < nG; ++r) {
        const int32_t slot = int32_t(int64_t(D.sym_row) * NB + r);
        P.padz[D.loc_off + D.n_I + r] = slot;
        P.padf[D.loc_off + D.n_I + r] = slot;
      }
      for (int c = 0; c < D.n_P; ++c)
        P.padz[D.loc_off + D.n_R + c] = int32_t(int64_t(D.sym_row) * NB + nG + D.n_A + c);
    }
  }
  // one all-zero tile after the last matrix: the tile read for any tile left of
  // a row's envelope
  P.n_tiles = tile_off + 1;
  P.iptr.push_back(int32_t(P.irows.size()));
  for (auto& D : P.subs) D.ztile = tile_off;
  P.bptr.push_back(int32_t(P.brows.size()));
  P.n_dinv = dinv_off;
  P.n_vec = vec_off;
  P.n_loc = loc_off;
  P.n_lmap = lmap_off;
  if (loc_off >= (int64_t(1) << 31)) { err = "too many local dofs"; return BDDC_EINVAL; }

  // ---- inverse maps ----
  P.inv_ptr.assign(nfree + 1, 0);
  for (int64_t g = 0; g < nfree; ++g) P.inv_ptr[g + 1] = P.inv_ptr[g] + inv_count[g];
  P.inv.assign(P.inv_ptr[nfree], 0);
  {
    std::vector<int32_t> fill(P.inv_ptr.begin(), P.inv_ptr.end() - 1);
    for (int64_t l = 0; l < loc_off; ++l) P.inv[fill[P.gmap[l]]++] = int32_t(l);
  }
  for (int64_t g = 0; g < nfree; ++g)
    if (P.inv_ptr[g + 1] - P.inv_ptr[g] != P.kappa[g]) { err = "internal: multiplicity mismatch"; return BDDC_EINVAL; }
  for (int64_t g = 0; g < nfree; ++g) {
    const int32_t b = P.inv_ptr[g], e = P.inv_ptr[g + 1];
    if (e - b < 2) continue;
    if (e - b > IFC_MAXC) { err = "internal: more than 8 subdomains share a dof"; return BDDC_EINVAL; }
    P.ifc_g.push_back(int32_t(g));
    for (int c = 0; c < IFC_MAXC; ++c) {
      const int32_t l = b + c < e ? P.inv[b + c] : -1;
      P.ifc_l.push_back(l);
      P.ifc_slotz.push_back(l >= 0 ? P.padz[l] : -1);
      P.ifc_slotf.push_back(l >= 0 ? P.padf[l] : -1);
    }
  }
  P.cinv_ptr.assign(P.n_coarse + 1, 0);
  for (int32_t p : P.rc) P.cinv_ptr[p + 1] += 1;
  for (int p = 0; p < P.n_coarse; ++p) P.cinv_ptr[p + 1] += P.cinv_ptr[p];
  P.cinv.assign(P.rc.size(), 0);
  {
    std::vector<int32_t> fill(P.cinv_ptr.begin(), P.cinv_ptr.end() - 1);
    for (size_t i = 0; i < P.rc.size(); ++i) P.cinv[fill[P.rc[i]]++] = int32_t(i);
  }

  // ---- coarse matrix assembly lists (lower triangle, p >= q) ----
  {
    struct Src { int32_t p, q, src; };
    std::vector<Src> all;
    for (int s = 0; s < P.nsubs; ++s) {
      const MatDesc& D = P.subs[s];
      for (int a = 0; a < D.n_ci; ++a)
        for (int c = 0; c < D.n_ci; ++c) {
          int32_t p = P.rc[D.coarse_off + a], q = P.rc[D.coarse_off + c];
          if (p >= q) all.push_back({p, q, s * MAX_NCI * MAX_NCI + a * MAX_NCI + c});
        }
    }
    std::stable_sort(all.begin(), all.end(), [](const Src& x, const Src& y) {
      return x.p != y.p ? x.p < y.p : x.q < y.q;
    });
    P.ac_diag.assign(P.n_coarse, -1);
    P.ac_src_ptr.push_back(0);
    for (size_t i = 0; i < all.size();) {
      size_t j = i;
      while (j < all.size() && all[j].p == all[i].p && all[j].q == all[i].q) {
        P.ac_src.push_back(all[j].src);
        ++j;
      }
      if (all[i].p == all[i].q) P.ac_diag[all[i].p] = int32_t(P.ac_row.size());
      P.ac_row.push_back(all[i].p);
      P.ac_col.push_back(all[i].q);
      P.ac_src_ptr.push_back(int32_t(P.ac_src.size()));
      i = j;
    }
    for (int p = 0; p < P.n_coarse; ++p)
      if (P.ac_diag[p] < 0) { err = "internal: coarse dof without diagonal"; return BDDC_EINVAL; }
  }

  // ---- task lists: forward passes by tile row, backward passes from the bottom ----
  // (interior passes: two tile rows per task, the task names the first).  The
  // chains of the subdomains are aligned at their ends: a chain of n tasks
  // enters n levels before the last level, so the longest chains (the critical
  // paths) start first, while the workgroups are shared by few chains and can
  // take their later tasks early.  Each chain keeps its own order, so tickets
  // stay in dependency order.
  auto make_tasks = [&](std::vector<int32_t>& out, bool interior_only, bool backward) {
    const int step = interior_only ? 2 : 1;
    std::vector<int> nt(P.nsubs);
    int maxN = 0;
    for (int s = 0; s < P.nsubs; ++s) {
      const int T = interior_only ? P.subs[s].TI : P.subs[s].T;
      nt[s] = (T + step - 1) / step;
      maxN = std::max(maxN, nt[s]);
    }
    for (int e = 0; e < maxN; ++e)
      for (int s = 0; s < P.nsubs; ++s) {
        const int i = e - (maxN - nt[s]);
        if (i < 0) continue;
        const int T = interior_only ? P.subs[s].TI : P.subs[s].T;
        const int d = i * step;
        out.push_back(s);
        out.push_back(backward ? T - 1 - d : d);
      }
  };
  make_tasks(P.fwd_rr, false, false);
  make_tasks(P.bwd_rr, false, true);
  make_tasks(P.fwd_ii, true, false);
  make_tasks(P.bwd_ii, true, true);
  // interface form
  {
    for (int s = 0; s < P.nsubs; ++s) {
      const int TS = sym_tile_rows(P.subs[s]);
      for (int ii = 0; ii < TS; ++ii) {
        P.symfin.push_back(s);
        P.symfin.push_back(ii);
      }
    }
  }
  if (int rc_ = make_factor_tasks(P.subs, &P.fcol, P.factor_tasks, err)) return rc_;
  for (auto& D : P.subs) {
    D.env = P.envrow.data() + D.vec_off / NB;
  }
  return BDDC_OK;
}

int make_factor_tasks(const std::vector<MatDesc>& mats, const std::vector<int32_t>* fcol, std::vector<int32_t>& out,
                      std::string& err) {
  // tile (i, k) of matrix m can be nonzero: border row, or inside the envelope
  auto nz = [&](const MatDesc& D, int i, int k) {
    return i >= D.T || fcol == nullptr || (*fcol)[D.vec_off / NB + i] <= k;
  };
  auto first_col = [&](const MatDesc& D, int r) {
    return (fcol == nullptr || r >= D.T) ? 0 : (*fcol)[D.vec_off / NB + r];
  };
  // per matrix: its tasks in step order (step s: the diagonal tile (s, s), the
  // tiles (i, s - 1) for i > s, then (s + 1, s), which the next diagonal tile waits for)
  std::vector<std::vector<std::vector<int32_t>>> steps(mats.size());
  int max_steps = 0;
  for (size_t m = 0; m < mats.size(); ++m) {
    const MatDesc& D = mats[m];
    steps[m].resize(D.Tx);
    max_steps = std::max(max_steps, int(D.Tx));
    for (int st = 0; st < D.Tx; ++st) {
      auto& v = steps[m][st];
      v.push_back(st);
      v.push_back(st);
      if (st >= 1)
        for (int i = st + 1; i < D.Tx; ++i)
          if (nz(D, i, st - 1)) {
            v.push_back(i);
            v.push_back(st - 1);
          }
      if (st < D.T && st + 1 < D.Tx && nz(D, st + 1, st)) {
        v.push_back(st + 1);
        v.push_back(st);
      }
    }
    // check the order: every tile a task reads (L_ik, L_jk for k in
    // [max(first_col(i), first_col(j)), j), and Dinv_j) comes earlier, and every
    // tile of the envelope appears exactly once
    std::vector<int32_t> pos(tri_tile(D.Tx, 0), -1);
    int32_t n = 0;
    for (auto& v : steps[m])
      for (size_t q = 0; q < v.size(); q += 2) {
        int32_t& p = pos[tri_tile(v[q], v[q + 1])];
        if (p >= 0) { err = "internal: factor task listed twice"; return BDDC_EINVAL; }
        p = n++;
      }
    for (int i = 0; i < D.Tx; ++i)
      for (int j = 0; j <= i; ++j) {
        const int32_t p = pos[tri_tile(i, j)];
        if ((p >= 0) != (i == j || nz(D, i, j))) { err = "internal: factor tasks do not cover the envelope"; return BDDC_EINVAL; }
        if (p < 0) continue;
        const int kf = std::max(first_col(D, i), first_col(D, j));
        for (int k = kf; k < j; ++k) {
          const int32_t a = pos[tri_tile(i, k)], b = pos[tri_tile(j, k)];
          if (a < 0 || b < 0 || a >= p || b >= p) { err = "internal: factor task order"; return BDDC_EINVAL; }
        }
        if (i != j && pos[tri_tile(j, j)] >= p) { err = "internal: factor task order"; return BDDC_EINVAL; }
      }
  }
  for (int st = 0; st < max_steps; ++st)
    for (size_t m = 0; m < mats.size(); ++m) {
      if (st >= mats[m].Tx) continue;
      const auto& v = steps[m][st];
      for (size_t q = 0; q < v.size(); q += 2) {
        out.push_back(int32_t(m));
        out.push_back(v[q]);
        out.push_back(v[q + 1]);
      }
    }
  return BDDC_OK;
}

}  // namespace bddc
