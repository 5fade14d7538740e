// HIP kernels for gfx950: assembly, batched tiled Cholesky on MFMA, persistent
// sync-free triangular solves, the coarse problem and the PCG vector kernels.
//
// Paper Sec. 2 defines what every kernel computes (eqs. (1)-(5)); the way it is
// computed here is this library's own:
//  * each subdomain's A_RR (interior first, then non-corner interface dofs) is
//    equilibrated to unit diagonal and stored as NB x NB lower tiles; one more
//    tile row holds (D B)^T with B = [C_AR^T | A_RPi], so the right-looking
//    factorisation also produces W = L^{-1} D B and, in the bordering diagonal
//    tile, -W^T W (the constraint Schur complement and its coupling blocks);
//  * the leading interior block of L is chol(A_II), reused for eq. (5);
//  * triangular solves are persistent kernels that take (matrix, tile row)
//    tasks from a ticket counter in dependency order; each published solution
//    value doubles as its own ready flag (a signalling-NaN sentinel until it
//    is written), read and written with device-scope atomics.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <map>
#include <mutex>

#include "bddc_internal.h"
#include "kernels.h"

namespace bddc {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Factor and interface-matrix tiles are read once per pass and not again
// before the whole stream has gone by: non-temporal loads, so that they do not
// displace the vectors and partial results that are reused from the caches.
template <typename V>
__device__ __forceinline__ V stream_load(const V* p) {
  return __builtin_nontemporal_load(p);
}

// Offset of element (r, c) inside an FP32 interface-matrix tile: four blocks of
// 16 columns, each 64 rows x 16 columns row-major (64 bytes per row).
__host__ __device__ __forceinline__ int sym_f32_off(int r, int c) { return (c >> 4) * (NB * 16) + r * 16 + (c & 15); }

// read-only data that is uniform per wave: scalar loads
typedef __attribute__((address_space(4))) const int32_t cint32_t;
// env_tile with the row's envelope entry (fc, rd) read by scalar loads (i uniform)
__device__ __forceinline__ int64_t env_tile_s(const MatDesc& D, int i, int j) {
  if (i >= D.T) return D.tile_off + D.tb + j;
  if (D.env == nullptr) return D.tile_off + tri_tile(i, j);
  static_assert(sizeof(EnvRow) == 2 * sizeof(int32_t), "EnvRow is (fc, rd)");
  const cint32_t* e = (const cint32_t*)(D.env + i);
  return j < e[0] ? D.ztile : D.tile_off + e[1] + j;
}

template <typename T> struct Traits;
template <> struct Traits<double> {
  using U = unsigned long long;
  using V = d2v;
  static constexpr int VEC = 2;
  static constexpr U SENT = 0x7FF4A5A5A5A5A5A5ull;   // signalling NaN, never produced by arithmetic
};
template <> struct Traits<float> {
  using U = unsigned int;
  using V = f4v;
  static constexpr int VEC = 4;
  static constexpr U SENT = 0x7F85A5A5u;
};

template <typename T>
__device__ __forceinline__ T load_published(const T* p) {
  using U = typename Traits<T>::U;
  U v = __hip_atomic_load(reinterpret_cast<const U*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(T, v);
}

template <typename T>
__device__ __forceinline__ bool is_sentinel(T v) {
  using U = typename Traits<T>::U;
  return __builtin_bit_cast(U, v) == Traits<T>::SENT;
}

// Wait for a published value; after `spin` polls (at once for spin < 0) give up,
// record DEV_WAIT_GAVE_UP in the status word and use 0, so that the kernel
// still finishes (the host then reports the failure).
template <typename T>
__device__ __forceinline__ T poll_published(const T* p, int spin, int* werr) {
  T v = spin < 0 ? T(0) : load_published(p);
  if (spin >= 0 && !is_sentinel(v)) return v;
  for (int n = 0; n < spin; ++n) {
    __builtin_amdgcn_s_sleep(2);
    v = load_published(p);
    if (!is_sentinel(v)) return v;
  }
  atomicOr(werr, DEV_WAIT_GAVE_UP);
  return T(0);
}

// A lane's N published values v[i] = p[base + i * stride] in two steps, so that
// their round trips overlap each other and the loads issued in between (the
// next tile): issue_published sends every load, resolve_published then tests
// them all and waits, one at a time, only for values still holding the
// sentinel (with poll_published's bound and give-up).
template <typename T, int N>
__device__ __forceinline__ void issue_published(T (&v)[N], const T* base, int stride) {
  for (int i = 0; i < N; ++i) v[i] = load_published(base + i * stride);
}
template <typename T, int N>
__device__ __forceinline__ void resolve_published(T (&v)[N], const T* base, int stride, int spin, int* werr) {
  bool miss = spin < 0;
  for (int i = 0; i < N; ++i) miss |= is_sentinel(v[i]);
  if (miss)
    for (int i = 0; i < N; ++i)
      if (spin < 0 || is_sentinel(v[i])) v[i] = poll_published(base + i * stride, spin, werr);
}

template <typename T>
__device__ __forceinline__ void store_published(T* p, T v) {
  using U = typename Traits<T>::U;
  __hip_atomic_store(reinterpret_cast<U*>(p), __builtin_bit_cast(U, v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Q1 element matrix entries (closed form of the tensor-product integrals)
// ---------------------------------------------------------------------------

struct MeshDev {
  int dim;
  int nel[3];
  double h[3];
};

// integral of grad N_a . grad N_b over one element; a, b are local node numbers
// (bit d = offset along axis d)
__device__ __forceinline__ double kref(const MeshDev& M, int a, int b) {
  double val = 0.0;
  for (int d = 0; d < M.dim; ++d) {
    double t = (((a >> d) & 1) == ((b >> d) & 1)) ? 1.0 / M.h[d] : -1.0 / M.h[d];
    for (int o = 0; o < M.dim; ++o)
      if (o != d) t *= M.h[o] * ((((a >> o) & 1) == ((b >> o) & 1)) ? 2.0 : 1.0) / 6.0;
    val += t;
  }
  return val;
}

// Stiffness entry between nodes n1 and n2 (integer coordinates), summed over the
// elements of the box [lo, lo+len) that contain both.
__device__ double stiff_entry(const MeshDev& M, const double* theta, const int n1[3], const int n2[3],
                              const int lo[3], const int len[3]) {
  int e0[3], e1[3];
  for (int d = 0; d < 3; ++d) {
    if (d >= M.dim) { e0[d] = 0; e1[d] = 0; continue; }
    int a = max(max(n1[d], n2[d]) - 1, lo[d]);
    int b = min(min(n1[d], n2[d]), lo[d] + len[d] - 1);
    e0[d] = a;
    e1[d] = b;
    if (a > b) return 0.0;
  }
  double v = 0.0;
  for (int ez = e0[2]; ez <= e1[2]; ++ez)
    for (int ey = e0[1]; ey <= e1[1]; ++ey)
      for (int ex = e0[0]; ex <= e1[0]; ++ex) {
        int e[3] = {ex, ey, ez};
        int la = 0, lb = 0;
        for (int d = 0; d < M.dim; ++d) {
          la |= (n1[d] - e[d]) << d;
          lb |= (n2[d] - e[d]) << d;
        }
        int64_t eid = ex + int64_t(M.nel[0]) * (ey + int64_t(M.nel[1]) * ez);
        v += theta[eid] * kref(M, la, lb);
      }
  return v;
}

__device__ __forceinline__ void free_coords(const MeshDev& M, int64_t g, int c[3]) {
  int nx1 = M.nel[0] - 1, ny1 = M.nel[1] - 1;
  c[0] = int(g % nx1) + 1;
  g /= nx1;
  if (M.dim == 3) {
    c[1] = int(g % ny1) + 1;
    c[2] = int(g / ny1) + 1;
  } else {
    c[1] = int(g) + 1;
    c[2] = 0;
  }
}

__device__ __forceinline__ int64_t free_of(const MeshDev& M, const int c[3]) {
  for (int d = 0; d < M.dim; ++d)
    if (c[d] < 1 || c[d] > M.nel[d] - 1) return -1;
  int64_t g = c[0] - 1;
  g += int64_t(M.nel[0] - 1) * (c[1] - 1);
  if (M.dim == 3) g += int64_t(M.nel[0] - 1) * (M.nel[1] - 1) * (c[2] - 1);
  return g;
}

// ---------------------------------------------------------------------------
// Simple fills
// ---------------------------------------------------------------------------

template <typename T>
__global__ void fill_kernel(T* p, T v, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

template <typename T>
__global__ void fill_bits_kernel(T* p, int64_t n) {
  using U = typename Traits<T>::U;
  U* q = reinterpret_cast<U*>(p);
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    q[i] = Traits<T>::SENT;
}

static int grid_for(int64_t n, int block = 256, int cap = 8192) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

template <typename T>
void launch_fill(T* p, T v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_for(n)), dim3(256), 0, st, p, v, n);
}
template void launch_fill<double>(double*, double, int64_t, hipStream_t);
template void launch_fill<float>(float*, float, int64_t, hipStream_t);
template void launch_fill<int>(int*, int, int64_t, hipStream_t);
template void launch_fill<unsigned>(unsigned*, unsigned, int64_t, hipStream_t);

template <typename T>
void launch_fill_sentinel(T* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_bits_kernel<T>, dim3(grid_for(n)), dim3(256), 0, st, p, n);
}
template void launch_fill_sentinel<double>(double*, int64_t, hipStream_t);
template void launch_fill_sentinel<float>(float*, int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// Global CSR assembly (paper Sec. 2: A from all elements)
// ---------------------------------------------------------------------------

__global__ void assemble_csr_kernel(MeshDev M, const double* theta, const int32_t* rowptr, int32_t* col,
                                    double* val, int64_t n, int* err) {
  int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (g >= n) return;
  int c[3];
  free_coords(M, g, c);
  int lo[3] = {0, 0, 0}, len[3] = {M.nel[0], M.nel[1], M.dim == 3 ? M.nel[2] : 1};
  int64_t j = rowptr[g];
  const int zr = M.dim == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int nb[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
        int64_t q = free_of(M, nb);
        if (q < 0) continue;
        col[j] = int32_t(q);
        val[j] = stiff_entry(M, theta, c, nb, lo, len);
        ++j;
      }
  if (j != rowptr[g + 1]) atomicOr(err, 4);
}

void launch_assemble_csr(const MeshDevHost& mh, const double* theta, const int32_t* rowptr, int32_t* col,
                         double* val, int64_t n, int* err, hipStream_t st) {
  MeshDev M{mh.dim, {mh.nel[0], mh.nel[1], mh.nel[2]}, {mh.h[0], mh.h[1], mh.h[2]}};
  hipLaunchKernelGGL(assemble_csr_kernel, dim3((n + 255) / 256), dim3(256), 0, st, M, theta, rowptr, col, val,
                     n, err);
}

__global__ void check_theta_kernel(const double* theta, int64_t n, int* err) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    if (!(theta[i] > 0.0) || !(theta[i] < 1e300)) atomicOr(err, 1);
}

void launch_check_theta(const double* theta, int64_t n, int* err, hipStream_t st) {
  hipLaunchKernelGGL(check_theta_kernel, dim3(grid_for(n)), dim3(256), 0, st, theta, n, err);
}

// ---------------------------------------------------------------------------
// Local (subdomain) assembly into equilibrated tiles
// ---------------------------------------------------------------------------

// Coefficient-aware weights (rho-scaling, an option beyond the paper's 1/kappa):
// rho_i(x) = the largest conductivity among subdomain i's elements that contain
// node x, w_i(x) = rho_i(x) / sum_j rho_j(x) over the subdomains sharing x.
__global__ void rho_local_kernel(MeshDev M, const double* theta, const MatDesc* mats, const int32_t* gmap,
                                 double* rho) {
  const MatDesc D = mats[blockIdx.y];
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= D.n_i) return;
  int c[3];
  free_coords(M, gmap[D.loc_off + a], c);
  int e0[3], e1[3];
  for (int d = 0; d < 3; ++d) {
    if (d >= M.dim) {
      e0[d] = e1[d] = 0;
      continue;
    }
    e0[d] = max(c[d] - 1, int(D.box_lo[d]));
    e1[d] = min(c[d], int(D.box_lo[d] + D.box_len[d]) - 1);
  }
  double r = 0.0;
  for (int ez = e0[2]; ez <= e1[2]; ++ez)
    for (int ey = e0[1]; ey <= e1[1]; ++ey)
      for (int ex = e0[0]; ex <= e1[0]; ++ex)
        r = fmax(r, theta[ex + int64_t(M.nel[0]) * (ey + int64_t(M.nel[1]) * ez)]);
  rho[D.loc_off + a] = r;
}

__global__ void rho_normalize_kernel(const int32_t* inv_ptr, const int32_t* inv, const double* rho, double* wgt,
                                     int64_t n) {
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < n; g += int64_t(gridDim.x) * blockDim.x) {
    double t = 0.0;
    for (int q = inv_ptr[g]; q < inv_ptr[g + 1]; ++q) t += rho[inv[q]];
    for (int q = inv_ptr[g]; q < inv_ptr[g + 1]; ++q) wgt[inv[q]] = rho[inv[q]] / t;
  }
}

// local dof a of matrix s -> box-local node coordinates
__device__ __forceinline__ void local_node(const MeshDev& M, const MatDesc& D, const int32_t* gmap, int a,
                                           int c[3]) {
  free_coords(M, gmap[D.loc_off + a], c);
}

// d_a = 1 / sqrt(A_aa) for a < n_R (diagonal of the box-restricted Neumann matrix)
__global__ void local_diag_kernel(MeshDev M, const double* theta, const MatDesc* mats, const int32_t* gmap,
                                  const double* wgt, double* dsc, double* wd, int* err) {
  const MatDesc D = mats[blockIdx.y];
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= D.n_i) return;
  if (a >= D.n_R) {
    dsc[D.loc_off + a] = 1.0;
    wd[D.loc_off + a] = wgt[D.loc_off + a];
    return;
  }
  int c[3];
  local_node(M, D, gmap, a, c);
  int lo[3] = {D.box_lo[0], D.box_lo[1], D.box_lo[2]};
  int len[3] = {D.box_len[0], D.box_len[1], M.dim == 3 ? D.box_len[2] : 1};
  double v = stiff_entry(M, theta, c, c, lo, len);
  if (!(v > 0.0)) { atomicOr(err, 1); v = 1.0; }
  const double d = 1.0 / sqrt(v);
  dsc[D.loc_off + a] = d;
  wd[D.loc_off + a] = wgt[D.loc_off + a] * d;
}

template <typename T>
__global__ void local_assemble_kernel(MeshDev M, const double* theta, const MatDesc* mats, const int32_t* gmap,
                                      const int32_t* lmap, const double* dsc, const int32_t* avg_of,
                                      const double* avg_coef, T* tiles, double* app) {
  const int s = blockIdx.y;
  const MatDesc D = mats[s];
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= D.n_i) return;
  int c[3];
  local_node(M, D, gmap, a, c);
  int lo[3] = {D.box_lo[0], D.box_lo[1], D.box_lo[2]};
  int len[3] = {D.box_len[0], D.box_len[1], M.dim == 3 ? D.box_len[2] : 1};
  const int n1x = D.box_len[0] + 1, n1y = D.box_len[1] + 1;
  const double da = dsc[D.loc_off + a];
  const int zr = M.dim == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int nb[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
        int bl[3] = {nb[0] - lo[0], nb[1] - lo[1], nb[2] - lo[2]};
        if (bl[0] < 0 || bl[0] > D.box_len[0] || bl[1] < 0 || bl[1] > D.box_len[1]) continue;
        if (M.dim == 3 && (bl[2] < 0 || bl[2] > D.box_len[2])) continue;
        int q = bl[0] + n1x * (bl[1] + n1y * (M.dim == 3 ? bl[2] : 0));
        int b = lmap[D.lmap_off + q];
        if (b < 0) continue;
        if (a < D.n_R && b < D.n_R) {
          if (b > a) continue;
          double v = stiff_entry(M, theta, c, nb, lo, len) * da * dsc[D.loc_off + b];
          const int64_t t = env_tile(D, a / NB, b / NB);   // inside the envelope by its definition
          tiles[t * NB * NB + (a % NB) * NB + (b % NB)] = T(v);
        } else if (a < D.n_R && b >= D.n_R) {
          // border row: (D A_R,Pi)^T, constraint row n_A + corner index
          double v = stiff_entry(M, theta, c, nb, lo, len) * da;
          int row = D.n_A + (b - D.n_R);
          const int64_t t = env_tile(D, D.T, a / NB);
          tiles[t * NB * NB + row * NB + (a % NB)] = T(v);
        } else if (a >= D.n_R && b >= D.n_R) {
          double v = stiff_entry(M, theta, c, nb, lo, len);
          app[int64_t(s) * MAX_NCI * MAX_NCI + (a - D.n_R) * MAX_NCI + (b - D.n_R)] = v;
        }
      }
  if (a < D.n_R) {
    int k = avg_of[D.loc_off + a];
    if (k >= 0) {
      const int64_t t = env_tile(D, D.T, a / NB);
      tiles[t * NB * NB + k * NB + (a % NB)] = T(avg_coef[D.loc_off + a] * da);
    }
  }
}

// identity on the padding rows of the last tile row
template <typename T>
__global__ void pad_identity_kernel(const MatDesc* mats, T* tiles) {
  const MatDesc D = mats[blockIdx.x];
  int r = D.n_R + threadIdx.x;
  if (D.T == 0 || r >= D.T * NB) return;
  const int64_t t = env_tile(D, D.T - 1, D.T - 1);
  tiles[t * NB * NB + (r % NB) * NB + (r % NB)] = T(1);
}

void launch_rho_weights(const MeshDevHost& m, const double* theta, const MatDesc* mats, int nmats, int max_ni,
                        const int32_t* gmap, const int32_t* inv_ptr, const int32_t* inv, int64_t n_free,
                        double* rho, double* wgt, hipStream_t st) {
  MeshDev M{m.dim, {m.nel[0], m.nel[1], m.nel[2]}, {m.h[0], m.h[1], m.h[2]}};
  hipLaunchKernelGGL(rho_local_kernel, dim3((max_ni + 255) / 256, nmats), dim3(256), 0, st, M, theta, mats, gmap,
                     rho);
  hipLaunchKernelGGL(rho_normalize_kernel, dim3(grid_for(n_free, 256, 4096)), dim3(256), 0, st, inv_ptr, inv, rho,
                     wgt, n_free);
}

void launch_local_assembly(const MeshDevHost& mh, const double* theta, const MatDesc* mats, int nmats,
                           int max_ni, const int32_t* gmap, const int32_t* lmap, const double* wgt, double* dsc,
                           double* wd, const int32_t* avg_of, const double* avg_coef, void* tiles, bool fp32,
                           double* app, int* err, hipStream_t st) {
  MeshDev M{mh.dim, {mh.nel[0], mh.nel[1], mh.nel[2]}, {mh.h[0], mh.h[1], mh.h[2]}};
  dim3 grid((max_ni + 127) / 128, nmats);
  hipLaunchKernelGGL(local_diag_kernel, grid, dim3(128), 0, st, M, theta, mats, gmap, wgt, dsc, wd, err);
  if (fp32) {
    hipLaunchKernelGGL(local_assemble_kernel<float>, grid, dim3(128), 0, st, M, theta, mats, gmap, lmap, dsc,
                       avg_of, avg_coef, (float*)tiles, app);
  } else {
    hipLaunchKernelGGL(local_assemble_kernel<double>, grid, dim3(128), 0, st, M, theta, mats, gmap, lmap, dsc,
                       avg_of, avg_coef, (double*)tiles, app);
  }
  launch_pad_identity(mats, nmats, tiles, fp32, st);
}

void launch_pad_identity(const MatDesc* mats, int nmats, void* tiles, bool fp32, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(pad_identity_kernel<float>, dim3(nmats), dim3(NB), 0, st, mats, (float*)tiles);
  else
    hipLaunchKernelGGL(pad_identity_kernel<double>, dim3(nmats), dim3(NB), 0, st, mats, (double*)tiles);
}

// ---------------------------------------------------------------------------
// Tile algebra on MFMA shared by the factorisation and the setup kernels
// ---------------------------------------------------------------------------

constexpr int LDT = NB + 1;   // padded LDS row stride

// MFMA 16x16x4 wrappers: a operand = A[row0 + lane%16][k + lane/16], b operand =
// B[col0 + lane%16][k + lane/16].  Accumulator item i of lane l holds column
// l%16 of the 16x16 block, row 4*i + l/16 for the FP64 instruction and row
// 4*(l/16) + i for the FP32 one (acc_row below).
__device__ __forceinline__ d4v mfma16(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mfma16(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct Acc4;
template <> struct Acc4<double> {
  using type = d4v;
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * i + (lane >> 4); }
};
template <> struct Acc4<float> {
  using type = f4v;
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// acc(64x64, distributed over 4 waves as 32x32 quadrants) = A * B^T with A, B
// 64x64 row-major tiles in LDS (stride LDT).
template <typename T>
__device__ __forceinline__ void gemm_nt_tile(const T* A, const T* B, typename Acc4<T>::type acc[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
  for (int kk = 0; kk < NB; kk += 4) {
    T a0 = A[(r0 + li) * LDT + kk + lk];
    T a1 = A[(r0 + 16 + li) * LDT + kk + lk];
    T b0 = B[(c0 + li) * LDT + kk + lk];
    T b1 = B[(c0 + 16 + li) * LDT + kk + lk];
    acc[0][0] = mfma16(a0, b0, acc[0][0]);
    acc[0][1] = mfma16(a0, b1, acc[0][1]);
    acc[1][0] = mfma16(a1, b0, acc[1][0]);
    acc[1][1] = mfma16(a1, b1, acc[1][1]);
  }
}

// ---------------------------------------------------------------------------
// Persistent left-looking tile Cholesky: one launch for all matrices
// ---------------------------------------------------------------------------
// A task is one tile (i, j), j <= i, of one matrix inside its envelope.  It sums
// P = sum_k L_ik L_jk^T over the columns k < j where both tiles can be nonzero
// (k >= max(fcol_i, fcol_j)), keeping P in MFMA accumulators, and then
//   i == j < T : factors A_jj - P = L_jj L_jj^T and inverts L_jj (Dinv_j);
//   i == j == T: stores A_TT - P (the bordering tile, -W^T W);
//   i > j      : L_ij = (A_ij - P) Dinv_j^T.
// Tasks are taken from one ticket counter in an order where every tile a task
// reads belongs to an earlier ticket (host: make_factor_tasks), so a task only
// waits for tasks already taken by running workgroups: no deadlock for any
// grid size.  A finished tile is announced by a per-tile ready word; tile values
// that other tasks read (off-diagonal L, Dinv) are written and read with
// device-scope (agent) atomic accesses, which are coherent across the XCDs'
// L2 caches, and the ready word is stored after every value has landed.

// Bounded wait for a ready word; gives up after about a second and records
// FACTOR_ERR_WAIT so that a broken dependency order cannot hang the GPU.
constexpr int FACTOR_ERR_PIVOT = 2;
constexpr int FACTOR_ERR_WAIT = 8;
__device__ __forceinline__ void wait_ready(const int* flag, int* err) {
  if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  for (long n = 0; n < (1L << 24); ++n) {
    __builtin_amdgcn_s_sleep(4);
    if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  }
  atomicOr(err, FACTOR_ERR_WAIT);
}

template <typename T>
__device__ __forceinline__ T load_agent(const T* p) {
  using U = typename Traits<T>::U;
  return __builtin_bit_cast(T, __hip_atomic_load(reinterpret_cast<const U*>(p), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT));
}
template <typename T>
__device__ __forceinline__ void store_agent(T* p, T v) {
  using U = typename Traits<T>::U;
  __hip_atomic_store(reinterpret_cast<U*>(p), __builtin_bit_cast(U, v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cholesky factor and inverse of the 64 x 64 SPD tile in a (LDS, stride LDT):
// on return a = L (upper part zero) and x = L^{-1}.  Thread t holds the 4 x 4
// block of rows 4 (t & 15).., columns 4 (t >> 4).. in registers; the 16 threads
// that own a column block form one wave's quarter, so the pivot reaches them by
// a lane shuffle.  Right-looking, one barrier per column for the factor and one
// per row for the inverse (column / row broadcast through double-buffered LDS).
// Returns false on a non-positive or non-finite pivot (replaced by 1).
template <typename T>
__device__ bool tile_potrf_inv(T* a, T* x, T* bc /* 2 x NB */, T* dg /* NB */) {
  const int t = threadIdx.x;
  const int r0 = 4 * (t & 15), c0 = 4 * (t >> 4);
  T v[4][4];
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) v[p][q] = a[(r0 + p) * LDT + c0 + q];
  bool ok = true;
  for (int jb = 0; jb < NB / 4; ++jb) {
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int j = 4 * jb + jj;
      T* col = bc + (j & 1) * NB;
      if ((t >> 4) == jb) {
        // the pivot sits with the thread of row block jb in this column block
        const int src = (16 * jb + jb) & 63;
        T d = __shfl(v[jj][jj], src);
        if (!(d > T(0)) || !(d < T(3e38))) {
          ok = false;
          d = T(1);
        }
        const T ljj = sqrt(d);
        const T rinv = T(1) / ljj;
        for (int p = 0; p < 4; ++p) {
          const int r = r0 + p;
          const T l = r > j ? v[p][jj] * rinv : (r == j ? ljj : T(0));
          v[p][jj] = l;
          col[r] = l;
        }
        if ((t & 15) == jb) dg[j] = rinv;
      }
      __syncthreads();
      if (c0 + 3 > j) {
        T lc[4], lr[4];
        for (int q = 0; q < 4; ++q) lc[q] = col[c0 + q];
        for (int p = 0; p < 4; ++p) lr[p] = col[r0 + p];
        for (int p = 0; p < 4; ++p)
          for (int q = 0; q < 4; ++q)
            if (c0 + q > j) v[p][q] -= lr[p] * lc[q];
      }
    }
  }
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) a[(r0 + p) * LDT + c0 + q] = v[p][q];
  // X = L^{-1} by elimination on [L | I], row j at step j: x_j /= l_jj, then
  // x_r -= l_rj x_j for r > j
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) v[p][q] = (r0 + p == c0 + q) ? T(1) : T(0);
  __syncthreads();
  for (int jb = 0; jb < NB / 4; ++jb) {
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int j = 4 * jb + jj;
      T* row = bc + (j & 1) * NB;
      if ((t & 15) == jb) {
        const T s = dg[j];
        for (int q = 0; q < 4; ++q) {
          v[jj][q] *= s;
          row[c0 + q] = v[jj][q];
        }
      }
      __syncthreads();
      if (r0 + 3 > j) {
        T lr[4], xc[4];
        for (int p = 0; p < 4; ++p) lr[p] = a[(r0 + p) * LDT + j];
        for (int q = 0; q < 4; ++q) xc[q] = row[c0 + q];
        for (int p = 0; p < 4; ++p)
          if (r0 + p > j)
            for (int q = 0; q < 4; ++q) v[p][q] -= lr[p] * xc[q];
      }
    }
  }
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) x[(r0 + p) * LDT + c0 + q] = v[p][q];
  return ok;
}

struct FactorArgs {
  const MatDesc* mats;
  void* tiles;
  void* dinv;
  const int32_t* fcol;    // per tile row (vec_off / NB + i): first envelope column; null: dense
  const int32_t* tasks;   // (matrix, i, j) per ticket
  int ntasks;
  unsigned* ticket;
  int* ready;             // per stored tile (env_tile(D, i, j)), zero before the launch
  int* err;
};

template <typename T>
__global__ __launch_bounds__(256, 2) void factor_persistent_kernel(FactorArgs F) {
  __shared__ T sa[NB * LDT];
  __shared__ T sb[NB * LDT];
  __shared__ T bc[2 * NB];
  __shared__ T dg[NB];
  __shared__ int s_task;
  T* tiles = static_cast<T*>(F.tiles);
  T* dinv = static_cast<T*>(F.dinv);
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int qr0 = 32 * (w >> 1), qc0 = 32 * (w & 1);
  using AccT = typename Acc4<T>::type;
  for (;;) {
    if (tid == 0) s_task = int(atomicAdd(F.ticket, 1u));
    __syncthreads();
    // the same value in every lane: read it as a scalar so that the compiler
    // keeps the loop (and the barriers in it) uniform across the workgroup
    const int task = __builtin_amdgcn_readfirstlane(s_task);
    __syncthreads();
    if (task >= F.ntasks) return;
    const int m = F.tasks[3 * task], i = F.tasks[3 * task + 1], j = F.tasks[3 * task + 2];
    const MatDesc D = F.mats[m];
    const int64_t rbase = D.vec_off / NB;
    auto first_col = [&](int r) { return (F.fcol == nullptr || r >= D.T) ? 0 : F.fcol[rbase + r]; };
    const int kf = max(first_col(i), first_col(j));
    // tiles (i, k) and (j, k), k >= kf, lie inside both rows' envelopes
    const int64_t oi = row_origin(D, i), oj = row_origin(D, j);
    AccT acc[2][2];
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 2; ++q) acc[p][q] = AccT(0);
    // L_ik and L_jk of the next column are loaded into registers while the
    // product of the current column runs from LDS; every lane checks the
    // ready words itself (one request per wave), so no barrier sits between the
    // wait and the loads
    constexpr int PER = NB * NB / 256;
    T ra[PER], rb[PER];
    auto fetch = [&](int k) {
      wait_ready(F.ready + oi + k, F.err);
      if (i != j) wait_ready(F.ready + oj + k, F.err);
      const T* pa = tiles + (oi + k) * int64_t(NB * NB);
      const T* pb = tiles + (oj + k) * int64_t(NB * NB);
      for (int q = 0; q < PER; ++q) ra[q] = load_agent(pa + tid + 256 * q);
      if (i != j)
        for (int q = 0; q < PER; ++q) rb[q] = load_agent(pb + tid + 256 * q);
    };
    if (kf < j) fetch(kf);
    for (int k = kf; k < j; ++k) {
      // LDS is free: the previous product ended with a barrier
      for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        sa[(e / NB) * LDT + (e % NB)] = ra[q];
        if (i != j) sb[(e / NB) * LDT + (e % NB)] = rb[q];
      }
      __syncthreads();
      if (k + 1 < j) fetch(k + 1);
      gemm_nt_tile<T>(sa, i != j ? sb : sa, acc);
      __syncthreads();
    }
    // R = A_ij - P into LDS (sa)
    T* tij = tiles + (oi + j) * int64_t(NB * NB);
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 2; ++q)
        for (int it = 0; it < 4; ++it) {
          const int r = qr0 + 16 * p + Acc4<T>::row(lane, it), c = qc0 + 16 * q + (lane & 15);
          sa[r * LDT + c] = tij[r * NB + c] - acc[p][q][it];
        }
    if (i == j && i < D.T) {
      __syncthreads();
      const bool ok = tile_potrf_inv<T>(sa, sb, bc, dg);
      __syncthreads();
      T* dt = dinv + (D.dinv_off + j) * int64_t(NB * NB);
      for (int e = tid; e < NB * NB; e += 256) {
        const int r = e / NB, c = e % NB;
        tij[e] = sa[r * LDT + c];
        store_agent(dt + e, sb[r * LDT + c]);
      }
      if (!ok && tid == 0) atomicOr(F.err, FACTOR_ERR_PIVOT);
    } else if (i == j) {
      __syncthreads();
      for (int e = tid; e < NB * NB; e += 256) tij[e] = sa[(e / NB) * LDT + (e % NB)];
    } else {
      wait_ready(F.ready + oj + j, F.err);
      const T* dj = dinv + (D.dinv_off + j) * int64_t(NB * NB);
      for (int q = 0; q < PER; ++q) rb[q] = load_agent(dj + tid + 256 * q);
      for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        sb[(e / NB) * LDT + (e % NB)] = rb[q];
      }
      __syncthreads();
      for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) acc[p][q] = AccT(0);
      gemm_nt_tile<T>(sa, sb, acc);
      for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q)
          for (int it = 0; it < 4; ++it) {
            const int r = qr0 + 16 * p + Acc4<T>::row(lane, it), c = qc0 + 16 * q + (lane & 15);
            store_agent(tij + r * NB + c, acc[p][q][it]);
          }
    }
    // every value of this tile has landed before its ready word is set
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) __hip_atomic_store(F.ready + oi + j, 1, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    // end the body with a barrier: the thread-0 regions at the end of one task
    // and at the start of the next must not be merged into one region that
    // the other lanes loop around (they would re-run the task without a ticket)
    __syncthreads();
  }
}

void launch_factor_persistent(const MatDesc* mats, void* tiles, void* dinv, bool fp32, const int32_t* fcol,
                              const int32_t* tasks, int ntasks, unsigned* ticket, int* ready, int64_t nready,
                              int grid, int* err, hipStream_t st) {
  launch_fill<int>(ready, 0, nready, st);
  launch_fill<unsigned>(ticket, 0u, 1, st);
  FactorArgs F{mats, tiles, dinv, fcol, tasks, ntasks, ticket, ready, err};
  grid = std::max(1, std::min(grid, ntasks));
  if (fp32)
    hipLaunchKernelGGL(factor_persistent_kernel<float>, dim3(grid), dim3(256), 0, st, F);
  else
    hipLaunchKernelGGL(factor_persistent_kernel<double>, dim3(grid), dim3(256), 0, st, F);
}

// ---------------------------------------------------------------------------
// Per-subdomain small dense algebra after the factorisation
// ---------------------------------------------------------------------------
// The bordering diagonal tile holds -G with G = W^T W, W = L^{-1} D [C_AR^T | A_RPi]
// (constraint order: averages then corners).  With S_A = G_AA and E = G_A,Pi:
//   A_ci = [[S_A^{-1}, S_A^{-1} E], [E^T S_A^{-1}, A_PiPi - G_PiPi + E^T S_A^{-1} E]]
// which equals Phi_i^T A_i Phi_i = -Lambda_i of eq. (1).
template <typename T>
__global__ __launch_bounds__(256) void local_small_kernel(const MatDesc* mats, const T* tiles,
                                                          const double* app, double* sainv, double* sainve,
                                                          double* aci, double* cpp, int* err) {
  const int s = blockIdx.x;
  const MatDesc D = mats[s];
  const int nA = D.n_A, nP = D.n_P, nc = D.n_ci;
  if (nc == 0) return;
  __shared__ double G[MAX_NCI * MAX_NCI];
  __shared__ double L[MAX_NCI * MAX_NCI];
  __shared__ double X[MAX_NCI * MAX_NCI];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const T* bt = tiles + env_tile(D, D.T, D.T) * int64_t(NB * NB);
  for (int i = tid; i < MAX_NCI * MAX_NCI; i += 256) {
    int r = i / MAX_NCI, c = i % MAX_NCI;
    // the tile holds the lower triangle reliably; symmetrise from it
    double v = (r < nc && c < nc) ? -double(r >= c ? bt[r * NB + c] : bt[c * NB + r]) : 0.0;
    G[i] = v;
    L[i] = 0.0;
    X[i] = 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  // Cholesky of S_A (one thread, n_A <= 64)
  if (tid == 0 && nA > 0) {
    for (int j = 0; j < nA; ++j) {
      double sdiag = G[j * MAX_NCI + j];
      for (int p = 0; p < j; ++p) sdiag -= L[j * MAX_NCI + p] * L[j * MAX_NCI + p];
      if (!(sdiag > 0.0)) { bad = 1; sdiag = 1.0; }
      L[j * MAX_NCI + j] = sqrt(sdiag);
      for (int i = j + 1; i < nA; ++i) {
        double v = G[i * MAX_NCI + j];
        for (int p = 0; p < j; ++p) v -= L[i * MAX_NCI + p] * L[j * MAX_NCI + p];
        L[i * MAX_NCI + j] = v / L[j * MAX_NCI + j];
      }
    }
  }
  __syncthreads();
  // X = S_A^{-1} [I | E]: columns solved in parallel
  if (tid < nc && nA > 0) {
    const int c = tid;
    double y[MAX_NCI];
    for (int i = 0; i < nA; ++i) {
      double v = (c < nA) ? (i == c ? 1.0 : 0.0) : G[i * MAX_NCI + c];
      for (int p = 0; p < i; ++p) v -= L[i * MAX_NCI + p] * y[p];
      y[i] = v / L[i * MAX_NCI + i];
    }
    for (int i = nA - 1; i >= 0; --i) {
      double v = y[i];
      for (int p = i + 1; p < nA; ++p) v -= L[p * MAX_NCI + i] * y[p];
      y[i] = v / L[i * MAX_NCI + i];
    }
    for (int i = 0; i < nA; ++i) X[i * MAX_NCI + c] = y[i];
  }
  __syncthreads();
  double* so = sainv + int64_t(s) * MAX_NCI * MAX_NCI;
  double* se = sainve + int64_t(s) * MAX_NCI * MAX_NCI;
  double* ao = aci + int64_t(s) * MAX_NCI * MAX_NCI;
  const double* ap = app + int64_t(s) * MAX_NCI * MAX_NCI;
  double* co = cpp + int64_t(s) * MAX_NCI * MAX_NCI;
  for (int i = tid; i < MAX_NCI * MAX_NCI; i += 256) {
    int r = i / MAX_NCI, c = i % MAX_NCI;
    co[i] = (r < nP && c < nP) ? ap[i] - G[(nA + r) * MAX_NCI + nA + c] : 0.0;
    so[i] = (r < nA && c < nA) ? X[r * MAX_NCI + c] : 0.0;
    se[i] = (r < nA && c < nP) ? X[r * MAX_NCI + nA + c] : 0.0;
    double v = 0.0;
    if (r < nc && c < nc) {
      if (r < nA) {
        v = X[r * MAX_NCI + c];                       // S_A^{-1} [I | E]
      } else if (c < nA) {
        v = X[c * MAX_NCI + r];                       // (S_A^{-1} E)^T
      } else {
        const int p = r - nA, q = c - nA;
        v = ap[p * MAX_NCI + q] - G[r * MAX_NCI + c];
        for (int t = 0; t < nA; ++t) v += G[t * MAX_NCI + r] * X[t * MAX_NCI + c];
      }
    }
    ao[i] = v;
  }
  if (tid == 0 && bad) atomicOr(err, 8);
}

void launch_local_small(const MatDesc* mats, int nmats, const void* tiles, bool fp32, const double* app,
                        double* sainv, double* sainve, double* aci, double* cpp, int* err, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(local_small_kernel<float>, dim3(nmats), dim3(256), 0, st, mats, (const float*)tiles, app,
                       sainv, sainve, aci, cpp, err);
  else
    hipLaunchKernelGGL(local_small_kernel<double>, dim3(nmats), dim3(256), 0, st, mats, (const double*)tiles,
                       app, sainv, sainve, aci, cpp, err);
}

// ---------------------------------------------------------------------------
// Coarse matrix assembly (A_c = sum_i R_ci^T A_ci R_ci) into equilibrated tiles
// ---------------------------------------------------------------------------

__global__ void coarse_entries_kernel(const int32_t* src_ptr, const int32_t* src, const double* aci, double* val,
                                      int n) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double v = 0.0;
  for (int j = src_ptr[e]; j < src_ptr[e + 1]; ++j) v += aci[src[j]];
  val[e] = v;
}

__global__ void coarse_scale_kernel(const int32_t* diag, const double* val, double* dc, int nc, int* err) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nc) return;
  double d = val[diag[p]];
  if (!(d > 0.0)) { atomicOr(err, 16); d = 1.0; }
  dc[p] = 1.0 / sqrt(d);
}

__global__ void coarse_write_kernel(const int32_t* row, const int32_t* col, const double* val, const double* dc,
                                    double* tiles, int n) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  int p = row[e], q = col[e];
  tiles[tri_tile(p / NB, q / NB) * NB * NB + (p % NB) * NB + (q % NB)] = dc[p] * val[e] * dc[q];
}

void launch_coarse_assembly(const int32_t* src_ptr, const int32_t* src, const int32_t* row, const int32_t* col,
                            const int32_t* diag, int nentries, int nc, const double* aci, double* val, double* dc,
                            double* tiles, int* err, hipStream_t st) {
  if (nentries == 0) return;
  hipLaunchKernelGGL(coarse_entries_kernel, dim3((nentries + 255) / 256), dim3(256), 0, st, src_ptr, src, aci,
                     val, nentries);
  hipLaunchKernelGGL(coarse_scale_kernel, dim3((nc + 255) / 256), dim3(256), 0, st, diag, val, dc, nc, err);
  if (tiles)
    hipLaunchKernelGGL(coarse_write_kernel, dim3((nentries + 255) / 256), dim3(256), 0, st, row, col, val, dc,
                       tiles, nentries);
}

// ---------------------------------------------------------------------------
// Persistent sync-free blocked triangular solves
// ---------------------------------------------------------------------------
// Task (s, k): tile row k of matrix s.  Forward: y_k = Dinv_k (rhs_k - sum_{j<k}
// L_kj y_j); backward: x_k = Dinv_k^T (rhs_k - sum_{j>k} L_jk^T x_j).  Tiles are
// row-major; a wave owns 16 rows of a tile and every load instruction of a wave
// covers 1 KB of contiguous tile memory.

template <typename T, int MODE>
__global__ __launch_bounds__(256) void trsv_kernel(TrsvArgs A) {
  using V = typename Traits<T>::V;
  constexpr int VEC = Traits<T>::VEC;
  constexpr int LPR = NB / VEC;      // lanes per tile row
  constexpr int RPI = 64 / LPR;      // tile rows per wave instruction
  constexpr int NI = 16 / RPI;       // instructions per 16-row slab
  constexpr bool FWD = MODE == TRSV_FWD_RR;
  // FP32 forward passes take the backward layout (a wave owns 16 whole rows):
  // with a wave on 16 columns an FP32 tile row gives each wave 64 bytes of a
  // 128-byte line, and the streamed tiles are fetched about 1.4 times over
  constexpr bool ROWL = FWD && sizeof(T) == 4;
  static_assert(MODE != TRSV_FWD_II && MODE != TRSV_BWD_II, "interior passes: trsv2_kernel");

  __shared__ T s_rhs[NB];
  __shared__ T s_v[NB];
  __shared__ T s_out[NB];
  __shared__ T s_red[4][NB];
  __shared__ int s_task;

  if (A.done && *A.done) return;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int lr = lane / LPR, lc = lane % LPR;
  // Register layout of a tile.  Forward passes (row products) let wave w own
  // columns 16w..16w+15: lane = CPL * rg + cp holds rows rg + RG i, columns
  // 16w + VEC cp + e, so a row sum reduces over CPL lanes, then the four waves.
  // Backward passes (column products) let wave w own rows 16w..16w+15: lane =
  // LPR * lr + lc holds rows 16w + RPI i + lr, columns VEC lc + e, so a column sum
  // reduces over RPI lanes, then the four waves.  Both take NI loads per lane.
  // (ROWL: forward row sums in the backward layout reduce over LPR lanes and are
  // complete in the wave that owns the row.)
  constexpr int CPL = 16 / VEC, RG = 64 / CPL;
  static_assert(64 / RG == NI, "layouts differ in loads per lane");
  const int rg = lane / CPL, cp = lane % CPL;
  const int64_t lane_off =
      (FWD && !ROWL) ? (int64_t(rg) * NB + 16 * w + VEC * cp) : (int64_t(16 * w + lr) * NB + VEC * lc);
  constexpr int64_t STEP = (FWD && !ROWL) ? RG * NB : RPI * NB;   // between a lane's consecutive loads
  const int xcol = ROWL ? VEC * lc : 16 * w + VEC * cp;             // forward: first column of a lane's x values
  const T* tiles = reinterpret_cast<const T*>(A.tiles);
  const T* dinv = reinterpret_cast<const T*>(A.dinv);
  T* sol = reinterpret_cast<T*>(A.sol);
  const T* src = reinterpret_cast<const T*>(A.src);

  for (;;) {
    if (tid == 0) s_task = atomicAdd(A.ticket, 1u);
    __syncthreads();
    const int task = s_task;
    __syncthreads();
    if (task >= A.ntasks) return;
    const int s = A.tasks[2 * task], k = A.tasks[2 * task + 1];
    const MatDesc D = A.mats[s];
    const int T_rows = D.T;
    const int nlim = D.n_R;
    const int nlo = 0, j0 = 0;
    const int64_t tbase = D.tile_off;
    T* my_sol = sol + D.vec_off;

    // ---------------- prologue: right-hand side of tile row k ----------------
    if (tid < NB) {
      const int a = k * NB + tid;
      double rhs = 0.0;
      if (a >= nlo && a < nlim) {
        if (MODE == TRSV_FWD_RR) {
          const int64_t l = D.loc_off + a;
          rhs = A.wd[l] * A.rin[A.gmap[l]];
        } else {
          rhs = double(src[D.vec_off + a]);   // backward: the forward solution
        }
      }
      s_rhs[tid] = T(rhs);
    }
    if (MODE == TRSV_BWD_RR && D.n_ci > 0) {
      // rhs_k += W_k coef, W_k^T stored in the bordering tile row (rows = constraints)
      __syncthreads();
      const T* bt = tiles + env_tile(D, D.T, k) * int64_t(NB * NB);
      const double* cf = A.coef + int64_t(s) * MAX_NCI;
      if (tid < NB) {
        double v = 0.0;
        for (int c = 0; c < D.n_ci; ++c) v += double(bt[c * NB + tid]) * cf[c];
        if (k * NB + tid >= nlo && k * NB + tid < nlim) s_rhs[tid] += T(v);
      }
    }

    // the inverse diagonal tile does not depend on other tasks: load it before
    // waiting on any published value
    V dv[NI];
    {
      const T* dt = dinv + (D.dinv_off + k) * int64_t(NB * NB) + lane_off;
      for (int i = 0; i < NI; ++i) dv[i] = stream_load(reinterpret_cast<const V*>(dt + i * STEP));
    }

    // ---------------- main loop over off-diagonal tiles ----------------
    T acc[FWD ? NI : VEC];
    for (int i = 0; i < (FWD ? NI : VEC); ++i) acc[i] = T(0);
    // only the tiles inside the envelope: forward reads (k, jlo..k-1), backward
    // reads (jhi..k+1, k); the tiles outside are zero
    // (a column of the factor is not contiguous: below the band of the interior
    // rows, only the interface rows whose envelope reaches back to column k hold
    // nonzero tiles; the backward pass with a row list reads just those)
    const int jlo = (FWD && A.fcol) ? max(j0, int(A.fcol[D.vec_off / NB + k])) : j0;
    const int jhi = (!FWD && A.lrow) ? int(A.lrow[D.vec_off / NB + k]) : T_rows - 1;
    const bool list = !FWD && A.bptr != nullptr;
    const int b0 = list ? A.bptr[D.vec_off / NB + k] : 0;
    const int nt = FWD ? k - jlo : (list ? A.bptr[D.vec_off / NB + k + 1] - b0 : jhi - k);
    if (nt > 0) {
      // the backward row list is uniform per wave and read-only: scalar loads
      // (constant address space), which a wait for the polled values or the
      // tiles in flight does not include
      const cint32_t* lrow = (const cint32_t*)(A.brows) + b0;
      const cint32_t* ltil = (const cint32_t*)(A.btile) + b0;
      auto sol_row = [&](int jj) -> int { return FWD ? jlo + jj : (list ? int(lrow[jj]) : jhi - jj); };
      const int64_t ok = FWD ? row_origin(D, k) : 0;
      auto tile_ptr = [&](int jj) -> const T* {
        // forward: tile (k, jlo + jj), jj = 0..k-jlo-1, along the stored row; backward:
        // tile (j, k) of the listed rows j (its index is listed too), or j = jhi .. k+1
        const int64_t t =
            FWD ? ok + jlo + jj : (list ? D.tile_off + ltil[jj] : env_tile_s(D, jhi - jj, k));
        return tiles + t * int64_t(NB * NB) + lane_off;
      };
      V cur[NI], nxt[NI];
      {
        const T* p = tile_ptr(0);
        for (int i = 0; i < NI; ++i) cur[i] = stream_load(reinterpret_cast<const V*>(p + i * STEP));
      }
      for (int jj = 0; jj < nt; ++jj) {
        // the block's values are requested first, then the next tile; the wait
        // for the values leaves the next tile's loads in flight
        const T* ys = my_sol + sol_row(jj) * NB;
        const T* xs = FWD ? ys + xcol : ys + 16 * w + lr;
        constexpr int NX = FWD ? VEC : NI, XS = FWD ? 1 : RPI;
        T xv[NX];
        issue_published(xv, xs, XS);
        {
          // past the last tile the loads go to one shared address (a single
          // line), so that every step has the same loads in flight and the
          // wait for the values below never includes the next tile
          const bool more = jj + 1 < nt;
          const T* p = tile_ptr(more ? jj + 1 : jj);
          for (int i = 0; i < NI; ++i) nxt[i] = stream_load(reinterpret_cast<const V*>(more ? p + i * STEP : tiles));
        }
        __builtin_amdgcn_sched_barrier(0);   // every load above issues before the first test
        resolve_published(xv, xs, XS, A.spin, A.werr);
        if (FWD) {
          for (int i = 0; i < NI; ++i)
            for (int e = 0; e < VEC; ++e) acc[i] += cur[i][e] * xv[e];
        } else {
          for (int i = 0; i < NI; ++i)
            for (int e = 0; e < VEC; ++e) acc[e] += cur[i][e] * xv[i];
        }
        for (int i = 0; i < NI; ++i) cur[i] = nxt[i];
      }
    }
    // reduce partial sums into s_red
    if (ROWL) {
      for (int i = 0; i < NI; ++i) {
        T v = acc[i];
        for (int off = 1; off < LPR; off <<= 1) v += __shfl_xor(v, off, LPR);
        if (lc == 0) s_red[w][16 * w + RPI * i + lr] = v;
      }
    } else if (FWD) {
      for (int i = 0; i < NI; ++i) {
        T v = acc[i];
        for (int off = 1; off < CPL; off <<= 1) v += __shfl_xor(v, off, CPL);
        if (cp == 0) s_red[w][rg + RG * i] = v;
      }
    } else {
      for (int e = 0; e < VEC; ++e) {
        T v = acc[e];
        for (int off = LPR; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
        if (lr == 0) s_red[w][VEC * lc + e] = v;
      }
    }
    __syncthreads();
    if (tid < NB) {
      T red = ROWL ? s_red[tid >> 4][tid] : s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
      s_v[tid] = (k * NB + tid >= nlo && k * NB + tid < nlim) ? (s_rhs[tid] - red) : T(0);
    }
    __syncthreads();

    // ---------------- diagonal block: multiply by the inverse tile ----------------
    {
      if (ROWL) {
        for (int i = 0; i < NI; ++i) {
          T v = T(0);
          for (int e = 0; e < VEC; ++e) v += dv[i][e] * s_v[VEC * lc + e];
          for (int off = 1; off < LPR; off <<= 1) v += __shfl_xor(v, off, LPR);
          if (lc == 0) s_red[w][16 * w + RPI * i + lr] = v;
        }
      } else if (FWD) {
        for (int i = 0; i < NI; ++i) {
          T v = T(0);
          for (int e = 0; e < VEC; ++e) v += dv[i][e] * s_v[16 * w + VEC * cp + e];
          for (int off = 1; off < CPL; off <<= 1) v += __shfl_xor(v, off, CPL);
          if (cp == 0) s_red[w][rg + RG * i] = v;
        }
      } else {
        T a2[VEC];
        for (int e = 0; e < VEC; ++e) a2[e] = T(0);
        for (int i = 0; i < NI; ++i)
          for (int e = 0; e < VEC; ++e) a2[e] += dv[i][e] * s_v[16 * w + RPI * i + lr];
        for (int e = 0; e < VEC; ++e) {
          T v = a2[e];
          for (int off = LPR; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
          if (lr == 0) s_red[w][VEC * lc + e] = v;
        }
      }
      __syncthreads();
      if (tid < NB) {
        T o = ROWL ? s_red[tid >> 4][tid] : s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
        if (k * NB + tid >= nlim || k * NB + tid < nlo) o = T(0);
        s_out[tid] = o;
        store_published(my_sol + k * NB + tid, o);
      }
    }
    __syncthreads();

    // ---------------- epilogue ----------------
    if (MODE == TRSV_FWD_RR && D.n_ci > 0) {
      // partial border products h_c = sum_r W^T[c][r] y_k[r] for this tile row
      const T* bt = tiles + env_tile(D, D.T, k) * int64_t(NB * NB);
      for (int c = w; c < D.n_ci; c += 4) {   // one wave per constraint row, coalesced
        double v = double(bt[c * NB + lane]) * double(s_out[lane]);
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) A.part[(D.vec_off / NB + k) * MAX_NCI + c] = v;
      }
    } else if (MODE == TRSV_BWD_RR) {
      if (tid < NB) {
        const int a = k * NB + tid;
        if (a >= nlo && a < D.n_R) {
          const int64_t l = D.loc_off + a;
          A.ww[l] = A.wd[l] * double(s_out[tid]);
        }
      }
    }
    __syncthreads();
  }
}

// A launch whose dispatch records t0 / t1 (when given) at kernel start / end.
template <typename K, typename... Args>
static void launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t st, hipEvent_t t0, hipEvent_t t1,
                         Args... args) {
  if (t0)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, t0, t1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

// Interior passes with two tile rows per task (the task list holds every second
// row: forward k = 0, 2, 4, ... for rows k and k+1; backward k = T-1, T-3, ...
// for rows k and k-1).  A pass is a chain of tasks per subdomain, each link a
// publish to device memory and a poll by another workgroup (about 3 us); with
// two rows per task the second row takes the first row's block from LDS, so
// the chain has half as many links.  Everything a task multiplies before its
// last wait is in registers when that wait ends: both rows' inverse diagonal
// tiles, the tile coupling the two rows, and both rows' tiles of the next
// published block (double-buffered).  The register layouts, the envelope, the
// published values and the right-hand sides are those of trsv_kernel.  The
// inverse diagonal tiles are parked in LDS as soon as they arrive (each thread
// reads back only the entries it wrote, so no barrier guards them), which keeps
// the kernel within 256 registers per lane: two workgroups per CU, twice the
// tile loads in flight of a one-workgroup-per-CU kernel.
template <typename T, int MODE>
__global__ __launch_bounds__(256, 2) void trsv2_kernel(TrsvArgs A) {
  using V = typename Traits<T>::V;
  constexpr int VEC = Traits<T>::VEC;
  constexpr int LPR = NB / VEC;
  constexpr int RPI = 64 / LPR;
  constexpr int NI = 16 / RPI;
  constexpr bool FWD = MODE == TRSV_FWD_II;
  constexpr bool ROWL = FWD && sizeof(T) == 4;   // FP32 forward: a wave owns 16 whole rows, as in trsv_kernel
  static_assert(MODE == TRSV_FWD_II || MODE == TRSV_BWD_II, "interior passes only");
  constexpr int CPL = 16 / VEC, RG = 64 / CPL;
  constexpr int NACC = FWD ? NI : VEC;

  __shared__ T s_rhs[2][NB];
  __shared__ T s_v[NB];
  __shared__ T s_out[NB];
  __shared__ T s_red[4][NB];
  __shared__ V s_dv[2][NI][256];   // inverse diagonal tiles: entry [q][i][tid] is thread tid's own
  __shared__ int s_task;

  if (A.done && *A.done) return;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int lr = lane / LPR, lc = lane % LPR;
  const int rg = lane / CPL, cp = lane % CPL;
  const int64_t lane_off =
      (FWD && !ROWL) ? (int64_t(rg) * NB + 16 * w + VEC * cp) : (int64_t(16 * w + lr) * NB + VEC * lc);
  constexpr int64_t STEP = (FWD && !ROWL) ? RG * NB : RPI * NB;
  const int xcol = ROWL ? VEC * lc : 16 * w + VEC * cp;   // forward: first column of a lane's x values
  const T* tiles = reinterpret_cast<const T*>(A.tiles);
  const T* dinv = reinterpret_cast<const T*>(A.dinv);
  T* sol = reinterpret_cast<T*>(A.sol);
  const T* src = reinterpret_cast<const T*>(A.src);

  for (;;) {
    if (tid == 0) s_task = atomicAdd(A.ticket, 1u);
    __syncthreads();
    const int task = s_task;
    __syncthreads();
    if (task >= A.ntasks) return;
    const int s = A.tasks[2 * task], k0 = A.tasks[2 * task + 1];
    const MatDesc D = A.mats[s];
    const int TI = D.TI, nlim = D.n_I;
    const int64_t tbase = D.tile_off;
    T* my_sol = sol + D.vec_off;
    const int nr = FWD ? (k0 + 1 < TI ? 2 : 1) : (k0 >= 1 ? 2 : 1);
    const int kr0 = k0, kr1 = FWD ? k0 + 1 : k0 - 1;
    // forward: the task's two rows are read along their stored rows (one origin
    // each); backward: tile (j, k) of the rows j = k+1 .. lrow_ii[k], some of
    // which lie left of row j's envelope (the interior numbering starts a new
    // layer of rows that reach back to the first columns): those read the shared
    // zero tile
    const int64_t o0 = FWD ? row_origin(D, kr0) : 0;
    const int64_t o1 = (FWD && nr == 2) ? row_origin(D, kr1) : 0;
    auto tptr = [&](int k, int j) -> const T* {
      // forward: tile (k, j), j < k; backward: tile (j, k), j > k
      const int64_t t = FWD ? (k == kr0 ? o0 : o1) + j : env_tile_s(D, j, k);
      return tiles + t * int64_t(NB * NB) + lane_off;
    };
    auto load = [&](const T* p, V (&t)[NI]) {
      for (int i = 0; i < NI; ++i) t[i] = stream_load(reinterpret_cast<const V*>(p + i * STEP));
    };

    // blocks published by other tasks: forward row k reads tiles (k, lo..k-1),
    // backward row k reads tiles (k+1..hi, k); the external blocks of the task
    // are the union of both rows' ranges without the first row's own block
    int lo[2], hi[2];
    for (int q = 0; q < 2; ++q) {
      const int k = q == 0 ? kr0 : kr1;
      if (q < nr) {
        if (FWD) {
          lo[q] = A.fcol ? int(A.fcol[D.vec_off / NB + k]) : 0;
          hi[q] = k - 1;
        } else {
          lo[q] = k + 1;
          hi[q] = A.lrow ? int(A.lrow[D.vec_off / NB + k]) : TI - 1;
        }
      } else {
        lo[q] = 1;
        hi[q] = 0;
      }
    }
    const bool inner = nr > 1 && kr0 >= lo[1] && kr0 <= hi[1];
    const int ext_lo = FWD ? min(lo[0], nr > 1 ? lo[1] : lo[0]) : kr0 + 1;
    const int ext_hi = FWD ? kr0 - 1 : max(hi[0], nr > 1 ? hi[1] : hi[0]);
    // backward with a row list: the rows j > kr0 inside column kr0's envelope
    // (a superset of column kr1's rows beyond kr0), each with the tiles (j, kr0)
    // and (j, kr1) (-1: zero); no zero tile is read and no row is looked up
    const bool ilist = !FWD && A.iptr != nullptr;
    const int il0 = ilist ? A.iptr[D.vec_off / NB + kr0] : 0;
    const int nt = ilist ? A.iptr[D.vec_off / NB + kr0 + 1] - il0 : ext_hi - ext_lo + 1;
    // the list (up to 4 x 64 entries) is read once into registers, lane l of
    // register q holding entry 64 q + l, and each step takes its entry with a
    // lane read: no memory access between the steps of the chain
    constexpr int LREG = 4;
    const bool lreg = ilist && nt <= 64 * LREG;
    int erow[LREG], et0[LREG], et1[LREG];
    for (int q = 0; q < LREG; ++q) {
      const int e = 64 * q + lane;
      const bool ok = lreg && e < nt;
      erow[q] = ok ? A.irows[il0 + e] : 0;
      et0[q] = ok ? A.itile0[il0 + e] : 0;
      et1[q] = ok ? A.itile1[il0 + e] : -1;
    }
    auto ent = [&](const int (&a)[LREG], const int32_t* g, int jj) -> int {
      if (!lreg) return int(((const cint32_t*)g)[il0 + jj]);   // scalar load
      const int q = jj >> 6;
      const int v = q == 0 ? a[0] : q == 1 ? a[1] : q == 2 ? a[2] : a[3];
      return __builtin_amdgcn_readlane(v, jj & 63);
    };
    auto blk = [&](int jj) -> int { return ilist ? ent(erow, A.irows, jj) : (FWD ? ext_lo + jj : ext_hi - jj); };
    auto in0 = [&](int jj, int j) -> bool { return ilist ? true : (j >= lo[0] && j <= hi[0]); };
    auto in1 = [&](int jj, int j) -> bool {
      return ilist ? (nr > 1 && ent(et1, A.itile1, jj) >= 0) : (j >= lo[1] && j <= hi[1]);
    };
    auto tile0 = [&](int jj, int j) -> const T* {
      return ilist ? tiles + (D.tile_off + ent(et0, A.itile0, jj)) * int64_t(NB * NB) + lane_off : tptr(kr0, j);
    };
    auto tile1 = [&](int jj, int j) -> const T* {
      return ilist ? tiles + (D.tile_off + ent(et1, A.itile1, jj)) * int64_t(NB * NB) + lane_off : tptr(kr1, j);
    };

    // everything independent of other tasks first: both inverse diagonal tiles
    // (through the prefetch registers into LDS), the coupling tile, the first
    // external block's tiles
    V ti[NI], c0[NI], c1[NI], n0[NI], n1[NI];
    load(dinv + (D.dinv_off + kr0) * int64_t(NB * NB) + lane_off, n0);
    if (nr > 1) load(dinv + (D.dinv_off + kr1) * int64_t(NB * NB) + lane_off, n1);
    if (inner) load(tptr(kr1, kr0), ti);
    if (nt > 0) {
      const int j = blk(0);
      if (in0(0, j)) load(tile0(0, j), c0);
      if (in1(0, j)) load(tile1(0, j), c1);
    }
    for (int i = 0; i < NI; ++i) {
      s_dv[0][i][tid] = n0[i];
      if (nr > 1) s_dv[1][i][tid] = n1[i];
    }

    // right-hand sides of the task's rows
    for (int q = 0; q < nr; ++q) {
      const int k = q == 0 ? kr0 : kr1;
      if (FWD && A.v12) {
        // interior rows of r - A v12: four lanes per CSR row
        const int row = tid >> 2, sl = tid & 3;
        const int a = k * NB + row;
        double v = 0.0;
        int64_t l = 0;
        int g = 0;
        if (a < nlim) {
          l = D.loc_off + a;
          g = A.gmap[l];
          for (int j = A.rowptr[g] + sl; j < A.rowptr[g + 1]; j += 4) v += A.vals[j] * A.v12[A.colind[j]];
        }
        v += __shfl_xor(v, 1, 4);
        v += __shfl_xor(v, 2, 4);
        if (sl == 0) s_rhs[q][row] = a < nlim ? T(A.dsc[l] * (A.rin[g] - v)) : T(0);
      } else if (tid < NB) {
        const int a = k * NB + tid;
        double rhs = 0.0;
        if (a < nlim) {
          if (FWD) {
            const int64_t l = D.loc_off + a;
            rhs = A.dsc[l] * A.rin[A.gmap[l]];
          } else {
            rhs = double(src[D.vec_off + a]);   // the forward solution
          }
        }
        s_rhs[q][tid] = T(rhs);
      }
    }

    T acc0[NACC], acc1[NACC];
    for (int i = 0; i < NACC; ++i) {
      acc0[i] = T(0);
      acc1[i] = T(0);
    }
    auto mac = [&](T (&acc)[NACC], const V (&t)[NI], const T* xv) {
      if (FWD) {
        for (int i = 0; i < NI; ++i)
          for (int e = 0; e < VEC; ++e) acc[i] += t[i][e] * xv[e];
      } else {
        for (int i = 0; i < NI; ++i)
          for (int e = 0; e < VEC; ++e) acc[e] += t[i][e] * xv[i];
      }
    };
    for (int jj = 0; jj < nt; ++jj) {
      const int j = blk(jj);
      // the block's values are requested before the next tiles, so that the
      // wait for them leaves those loads in flight
      const T* ys = my_sol + j * NB;
      const T* xs = FWD ? ys + xcol : ys + 16 * w + lr;
      constexpr int NX = FWD ? VEC : NI, XS = FWD ? 1 : RPI;
      T xv[NX];
      issue_published(xv, xs, XS);
      {
        // a tile that is not needed (past the last block, or outside a row's
        // range) is replaced by loads of one shared address (a single line),
        // so that every step has the same loads in flight and the wait for the
        // values below never includes the next tiles
        const bool more = jj + 1 < nt;
        const int jm = more ? jj + 1 : jj;
        const int jn = blk(jm);
        const bool m0 = more && in0(jm, jn), m1 = more && in1(jm, jn);
        const T* p0 = m0 ? tile0(jm, jn) : tiles;
        const T* p1 = m1 ? tile1(jm, jn) : tiles;
        for (int i = 0; i < NI; ++i) n0[i] = stream_load(reinterpret_cast<const V*>(m0 ? p0 + i * STEP : tiles));
        for (int i = 0; i < NI; ++i) n1[i] = stream_load(reinterpret_cast<const V*>(m1 ? p1 + i * STEP : tiles));
      }
      __builtin_amdgcn_sched_barrier(0);   // every load above issues before the first test
      resolve_published(xv, xs, XS, A.spin, A.werr);
      if (in0(jj, j)) mac(acc0, c0, xv);
      if (in1(jj, j)) mac(acc1, c1, xv);
      for (int i = 0; i < NI; ++i) {
        c0[i] = n0[i];
        c1[i] = n1[i];
      }
    }

    // finish one row: reduce the partial sums, subtract from the right-hand
    // side, multiply by the inverse diagonal tile, publish, write the output
    auto finish = [&](int q, int k, const T (&acc)[NACC]) {
      const V (&dvq)[NI][256] = s_dv[q];
      if (ROWL) {
        for (int i = 0; i < NI; ++i) {
          T v = acc[i];
          for (int off = 1; off < LPR; off <<= 1) v += __shfl_xor(v, off, LPR);
          if (lc == 0) s_red[w][16 * w + RPI * i + lr] = v;
        }
      } else if (FWD) {
        for (int i = 0; i < NI; ++i) {
          T v = acc[i];
          for (int off = 1; off < CPL; off <<= 1) v += __shfl_xor(v, off, CPL);
          if (cp == 0) s_red[w][rg + RG * i] = v;
        }
      } else {
        for (int e = 0; e < VEC; ++e) {
          T v = acc[e];
          for (int off = LPR; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
          if (lr == 0) s_red[w][VEC * lc + e] = v;
        }
      }
      __syncthreads();
      if (tid < NB) {
        const T red = ROWL ? s_red[tid >> 4][tid] : s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
        s_v[tid] = k * NB + tid < nlim ? (s_rhs[q][tid] - red) : T(0);
      }
      __syncthreads();
      if (ROWL) {
        for (int i = 0; i < NI; ++i) {
          const V d = dvq[i][tid];
          T v = T(0);
          for (int e = 0; e < VEC; ++e) v += d[e] * s_v[VEC * lc + e];
          for (int off = 1; off < LPR; off <<= 1) v += __shfl_xor(v, off, LPR);
          if (lc == 0) s_red[w][16 * w + RPI * i + lr] = v;
        }
      } else if (FWD) {
        for (int i = 0; i < NI; ++i) {
          T v = T(0);
          const V d = dvq[i][tid];
          for (int e = 0; e < VEC; ++e) v += d[e] * s_v[16 * w + VEC * cp + e];
          for (int off = 1; off < CPL; off <<= 1) v += __shfl_xor(v, off, CPL);
          if (cp == 0) s_red[w][rg + RG * i] = v;
        }
      } else {
        T a2[VEC];
        for (int e = 0; e < VEC; ++e) a2[e] = T(0);
        for (int i = 0; i < NI; ++i) {
          const V d = dvq[i][tid];
          for (int e = 0; e < VEC; ++e) a2[e] += d[e] * s_v[16 * w + RPI * i + lr];
        }
        for (int e = 0; e < VEC; ++e) {
          T v = a2[e];
          for (int off = LPR; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
          if (lr == 0) s_red[w][VEC * lc + e] = v;
        }
      }
      __syncthreads();
      if (tid < NB) {
        T o = ROWL ? s_red[tid >> 4][tid] : s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
        if (k * NB + tid >= nlim) o = T(0);
        s_out[tid] = o;
        store_published(my_sol + k * NB + tid, o);
        if (!FWD) {
          const int a = k * NB + tid;
          if (a < nlim) {
            const int64_t l = D.loc_off + a;
            const int g = A.gmap[l];
            A.zout[g] = (A.base ? A.base[g] : 0.0) + A.dsc[l] * double(o);
          }
        }
      }
      __syncthreads();
    };

    finish(0, kr0, acc0);
    if (nr > 1) {
      if (inner) {
        // the first row's block, from LDS
        T xv[FWD ? VEC : NI];
        if (FWD) {
          for (int e = 0; e < VEC; ++e) xv[e] = s_out[xcol + e];
        } else {
          for (int i = 0; i < NI; ++i) xv[i] = s_out[16 * w + RPI * i + lr];
        }
        mac(acc1, ti, xv);
      }
      __syncthreads();   // s_out is overwritten by the second row
      finish(1, kr1, acc1);
    }
  }
}

template <typename T>
static void launch_trsv2_t(int mode, const TrsvArgs& a, int grid, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  const dim3 g(grid), b(256);
  if (mode == TRSV_FWD_II) launch_timed(trsv2_kernel<T, TRSV_FWD_II>, g, b, st, t0, t1, a);
  else launch_timed(trsv2_kernel<T, TRSV_BWD_II>, g, b, st, t0, t1, a);
}

void launch_trsv2(int mode, bool fp32, const TrsvArgs& a, int grid, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (a.ntasks <= 0) return;
  if (fp32) launch_trsv2_t<float>(mode, a, grid, st, t0, t1);
  else launch_trsv2_t<double>(mode, a, grid, st, t0, t1);
}

template <typename T>
static void launch_trsv_t(int mode, const TrsvArgs& a, int grid, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  const dim3 g(grid), b(256);
  switch (mode) {
    case TRSV_FWD_RR: launch_timed(trsv_kernel<T, TRSV_FWD_RR>, g, b, st, t0, t1, a); break;
    case TRSV_BWD_RR: launch_timed(trsv_kernel<T, TRSV_BWD_RR>, g, b, st, t0, t1, a); break;
  }
}

void launch_trsv(int mode, bool fp32, const TrsvArgs& a, int grid, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (a.ntasks <= 0) return;
  if (mode == TRSV_FWD_II || mode == TRSV_BWD_II) {
    launch_trsv2(mode, fp32, a, grid, st, t0, t1);
    return;
  }
  if (fp32)
    launch_trsv_t<float>(mode, a, grid, st, t0, t1);
  else
    launch_trsv_t<double>(mode, a, grid, st, t0, t1);
}

// The symmetric interface matrices of all subdomains form one stream of ntiles
// tiles; workgroup g of a mat-vec launch with nwg workgroups takes the tiles
// [g ntiles / nwg, (g+1) ntiles / nwg).  It stores the row product of every row
// piece it covers (a piece starts at a row's first tile or at a range start) in
// rowp[start tile * 64 + row].  This sums the pieces of the row whose len tiles
// start at tr0, in a fixed order.
// floor(a / b) for integers 0 <= a, 0 < b with a + b < 2^53, by one FP64
// division (a 64-bit integer division is a long instruction sequence here):
// a and b are exact doubles, and a quotient k + f that is not an integer lies
// at least 1/b below k + 1, while rounding moves it by less than (k + 1) 2^-53
// <= (a + b) / b 2^-53 < 1/b.
__device__ __forceinline__ int64_t small_div(int64_t a, int64_t b) { return int64_t(double(a) / double(b)); }
// Workgroup of a mat-vec launch whose range holds tile p: the g with
// g ntiles / nwg <= p < (g+1) ntiles / nwg (integer division).
__device__ __forceinline__ int64_t sym_wg(int64_t p, int64_t ntiles, int64_t nwg) {
  return small_div((p + 1) * nwg - 1, ntiles);
}
// Whether the slot of tile (i2, jj) holds a column product: for jj < lds_cols
// only the column's first tile in each workgroup range does (it holds the sum
// over the range's rows), for the other columns every tile.
__device__ __forceinline__ bool sym_col_first(const MatDesc& D, int i2, int jj, int64_t ntiles, int64_t nwg,
                                              int lds_cols) {
  if (jj >= lds_cols || i2 == jj) return true;
  return sym_wg(D.sg_off + tri_tile(i2, jj), ntiles, nwg) != sym_wg(D.sg_off + tri_tile(i2 - 1, jj), ntiles, nwg);
}

__device__ double sym_row_product(const double* rowp, int64_t tr0, int len, int64_t ntiles, int64_t nwg, int lane) {
  double v = 0.0;
  v += rowp[tr0 * NB + lane];
  for (int64_t g = small_div(tr0 * nwg, ntiles); g < nwg; ++g) {
    const int64_t b = small_div(g * ntiles, nwg);
    if (b <= tr0) continue;
    if (b >= tr0 + len) break;
    v += rowp[b * NB + lane];
  }
  return v;
}

// ---------------------------------------------------------------------------
// Coarse-level glue of the apply
// ---------------------------------------------------------------------------
// h = sum_k part[s][k] = W^T t (W = L^{-1} D B, t = L^{-1} D W_i f_R), then
//   g[A]  = S_A^{-1} h_A                        (also mu, the average multipliers)
//   g[Pi] = -h_Pi + (S_A^{-1} E)^T h_A + W_Pi r_Pi
// g = Phi_i^T W_i R_i r, the subdomain's share of the coarse residual r_c.
__global__ __launch_bounds__(256) void coarse_prep_kernel(const MatDesc* mats, const double* part,
                                                         const double* sainv, const double* sainve,
                                                         const int32_t* gmap, const double* wgt, const double* r,
                                                         double* gbuf, double* mu, const int* done,
                                                         const double* rowp, int64_t ntiles, int nwg) {
  const int dn = done ? *done : 0;   // tested once the loads are in flight
  const int s = blockIdx.x;
  const MatDesc D = mats[s];
  const int tid = threadIdx.x;
  __shared__ double h[MAX_NCI];
  __shared__ double hq[4][MAX_NCI];
  if (D.n_ci == 0) return;
  // constraint c = tid % 64; the whole-space partial products of the T tile
  // rows are split over the four waves (rows k = q, q + 4, ..., four loads in
  // flight each) and added in wave order
  const int c = tid & 63, q = tid >> 6;
  if (c < D.n_ci) {
    double v = 0.0;
    if (rowp) {
      // interface form: W^T t is the row product of constraint row n_G + c,
      // (W_G^T X) f
      if (q == 0) {
        const int R = D.n_R - D.n_I + c;
        v = sym_row_product(rowp, D.sg_off + tri_tile(R / NB, 0), R / NB + 1, ntiles, nwg, R % NB);
      }
    } else {
      const double* pp = part + (D.vec_off / NB) * MAX_NCI + c;
      int k = q;
      for (; k + 12 < D.T; k += 16) {
        const double a0 = pp[int64_t(k) * MAX_NCI], a1 = pp[int64_t(k + 4) * MAX_NCI],
                     a2 = pp[int64_t(k + 8) * MAX_NCI], a3 = pp[int64_t(k + 12) * MAX_NCI];
        v += a0;
        v += a1;
        v += a2;
        v += a3;
      }
      for (; k < D.T; k += 4) v += pp[int64_t(k) * MAX_NCI];
    }
    hq[q][c] = v;
  }
  if (dn) return;
  __syncthreads();
  if (tid < D.n_ci) h[tid] = hq[0][tid] + hq[1][tid] + hq[2][tid] + hq[3][tid];
  __syncthreads();
  const double* so = sainv + int64_t(s) * MAX_NCI * MAX_NCI;
  const double* se = sainve + int64_t(s) * MAX_NCI * MAX_NCI;
  const int nA = D.n_A;
  if (tid < D.n_ci) {
    double v;
    if (tid < nA) {
      v = 0.0;
      for (int t = 0; t < nA; ++t) v += so[tid * MAX_NCI + t] * h[t];
      mu[int64_t(s) * MAX_NCI + tid] = v;
    } else {
      const int p = tid - nA;
      v = -h[tid];
      for (int t = 0; t < nA; ++t) v += se[t * MAX_NCI + p] * h[t];
      const int64_t l = D.loc_off + D.n_R + p;
      v += wgt[l] * r[gmap[l]];
    }
    gbuf[D.coarse_off + tid] = v;
  }
}

// per subdomain: u = R_ci u_c; coef_A = -mu + S_A^{-1} u_A + S_A^{-1} E u_Pi;
// coef_Pi = -u_Pi; corner outputs w_Pi = u_Pi (weighted).  u_c is given as
// nsplit partial vectors of nc values (their sum, in order).
__global__ __launch_bounds__(64) void coarse_coef_kernel(const MatDesc* mats, const int32_t* rc, const double* uc,
                                                         int nc, int nsplit, const double* mu, const double* sainv,
                                                         const double* sainve, const double* wgt, double* coef,
                                                         double* ww, const int* done) {
  if (done && *done) return;
  const int s = blockIdx.x;
  const MatDesc D = mats[s];
  const int tid = threadIdx.x;
  __shared__ double u[MAX_NCI];
  if (D.n_ci == 0) return;
  if (tid < D.n_ci) {
    const int pc = rc[D.coarse_off + tid];
    double v = 0.0;
    for (int q = 0; q < nsplit; ++q) v += uc[int64_t(q) * nc + pc];
    u[tid] = v;
  }
  __syncthreads();
  const double* so = sainv + int64_t(s) * MAX_NCI * MAX_NCI;
  const double* se = sainve + int64_t(s) * MAX_NCI * MAX_NCI;
  const int nA = D.n_A, nP = D.n_P;
  if (tid < D.n_ci) {
    double v;
    if (tid < nA) {
      v = -mu[int64_t(s) * MAX_NCI + tid];
      for (int t = 0; t < nA; ++t) v += so[tid * MAX_NCI + t] * u[t];
      for (int p = 0; p < nP; ++p) v += se[tid * MAX_NCI + p] * u[nA + p];
    } else {
      v = -u[tid];
      const int64_t l = D.loc_off + D.n_R + (tid - nA);
      ww[l] = wgt[l] * u[tid];
    }
    coef[int64_t(s) * MAX_NCI + tid] = v;
  }
}

void launch_coarse_prep(const MatDesc* mats, int nmats, const double* part, const double* sainv,
                        const double* sainve, const int32_t* gmap, const double* wgt, const double* r,
                        double* gbuf, double* mu, const int* done, const double* rowp, int64_t ntiles, int nwg,
                        hipStream_t st) {
  hipLaunchKernelGGL(coarse_prep_kernel, dim3(nmats), dim3(256), 0, st, mats, part, sainv, sainve, gmap, wgt, r,
                     gbuf, mu, done, rowp, ntiles, nwg);
}

void launch_coarse_coef(const MatDesc* mats, int nmats, const int32_t* rc, const double* uc, int nc, int nsplit,
                        const double* mu, const double* sainv, const double* sainve, const double* wgt,
                        double* coef, double* ww, const int* done, hipStream_t st) {
  hipLaunchKernelGGL(coarse_coef_kernel, dim3(nmats), dim3(64), 0, st, mats, rc, uc, nc, nsplit, mu, sainv, sainve,
                     wgt, coef, ww, done);
}

// v12[g] = sum over the subdomains holding g of W_i w_i (gather through the inverse
// map, fixed order); interface entries of z get v12 directly (their v3 is 0).
__global__ void gather_v12_kernel(const int32_t* inv_ptr, const int32_t* inv, const double* ww,
                                  const uint8_t* kappa, double* v12, double* z, int64_t n, const int* done) {
  if (done && *done) return;
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < n; g += int64_t(gridDim.x) * blockDim.x) {
    double v = 0.0;
    for (int j = inv_ptr[g]; j < inv_ptr[g + 1]; ++j) v += ww[inv[j]];
    v12[g] = v;
    if (kappa[g] > 1) z[g] = v;
  }
}

void launch_gather_v12(const int32_t* inv_ptr, const int32_t* inv, const double* ww, const uint8_t* kappa,
                       double* v12, double* z, int64_t n, const int* done, hipStream_t st) {
  hipLaunchKernelGGL(gather_v12_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, inv_ptr, inv, ww, kappa,
                     v12, z, n, done);
}

// zero the interface entries (the static-condensation guess is zero there)
__global__ void zero_interface_kernel(const uint8_t* kappa, double* x, int64_t n) {
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < n; g += int64_t(gridDim.x) * blockDim.x)
    if (kappa[g] > 1) x[g] = 0.0;
}

__global__ void zero_interior_kernel(const uint8_t* kappa, double* x, int64_t n) {
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < n; g += int64_t(gridDim.x) * blockDim.x)
    if (kappa[g] < 2) x[g] = 0.0;
}

void launch_zero_interior(const uint8_t* kappa, double* x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_interior_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, kappa, x, n);
}

void launch_zero_interface(const uint8_t* kappa, double* x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_interface_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, kappa, x, n);
}

// ---------------------------------------------------------------------------
// CSR SpMV and the PCG vector kernels (FP64, deterministic reductions)
// ---------------------------------------------------------------------------
// A half-wave (32 lanes) per row: a 27-point row fits one pass.

constexpr int VBLK = 256;
constexpr int VGRID = 1024;   // fixed grid for the vector kernels: <= 1024 partial sums

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < VBLK / 64; ++i) t += sh[i];
  return t;
}

// every block re-reduces the partials of the previous kernel in the same order, so
// all blocks obtain the same bits
__device__ __forceinline__ double reduce_partials(const double* part, int np, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += VBLK) v += part[i];
  return block_sum(v, sh);
}

// CSR rows times x, each row by a group of ROW_LANES consecutive lanes.  A Q1
// row has at most 27 entries (3D), so every lane takes ROW_STEPS entries of each
// of its U rows with unconditional loads (addresses clamped into the row, the
// surplus terms dropped by a select): the loads of all U rows are in flight at
// once, where a loop over the entries waits for every trip's loads.  Longer rows
// (not produced by Q1 assembly) finish in a loop.  Rows >= n give 0.  Every row
// of the matrix is non-empty (it holds its diagonal), so clamped addresses stay
// inside the arrays.
constexpr int ROW_LANES = 4;
constexpr int ROW_STEPS = 7;
template <int U>
__device__ __forceinline__ void rows_dot(const int32_t* rowptr, const int32_t* col, const double* val,
                                         const double* x, const int64_t (&row)[U], int64_t n, int sl,
                                         double (&v)[U]) {
  int b[U], e[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t rw = row[u] < n ? row[u] : n - 1;
    b[u] = rowptr[rw];
    e[u] = row[u] < n ? rowptr[rw + 1] : b[u];
  }
  int cc[U][ROW_STEPS];
  double cv[U][ROW_STEPS];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int k = 0; k < ROW_STEPS; ++k) {
      const int j = min(b[u] + sl + ROW_LANES * k, max(e[u] - 1, b[u]));
      cc[u][k] = col[j];
      cv[u][k] = val[j];
    }
  double xv[U][ROW_STEPS];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int k = 0; k < ROW_STEPS; ++k) xv[u][k] = x[cc[u][k]];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < ROW_STEPS; ++k) {
      const double t = cv[u][k] * xv[u][k];
      s += b[u] + sl + ROW_LANES * k < e[u] ? t : 0.0;
    }
    for (int j = b[u] + sl + ROW_LANES * ROW_STEPS; j < e[u]; j += ROW_LANES) s += val[j] * x[col[j]];
    for (int off = ROW_LANES / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, ROW_LANES);
    v[u] = s;
  }
}
constexpr int ROW_U = 2;   // rows per lane group and step of the SpMV loops

__global__ __launch_bounds__(VBLK) void spmv_kernel(const int32_t* rowptr, const int32_t* col, const double* val,
                                                    const double* x, double* y, int64_t n) {
  const int sl = threadIdx.x % ROW_LANES;
  const int64_t hw = (blockIdx.x * int64_t(VBLK) + threadIdx.x) / ROW_LANES;
  const int64_t nhw = (int64_t(gridDim.x) * VBLK) / ROW_LANES;
  for (int64_t row0 = hw; row0 < n; row0 += ROW_U * nhw) {
    int64_t rows[ROW_U];
    double v[ROW_U];
    for (int u = 0; u < ROW_U; ++u) rows[u] = row0 + u * nhw;
    rows_dot<ROW_U>(rowptr, col, val, x, rows, n, sl, v);
    if (sl == 0)
      for (int u = 0; u < ROW_U; ++u)
        if (rows[u] < n) y[rows[u]] = v[u];
  }
}

void launch_spmv(const int32_t* rowptr, const int32_t* col, const double* val, const double* x, double* y, int64_t n,
                 hipStream_t st) {
  int64_t g = (n * 32 + VBLK - 1) / VBLK;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(spmv_kernel, dim3(g), dim3(VBLK), 0, st, rowptr, col, val, x, y, n);
}

// r = b - A x, partial sums of r.r and b.b
__global__ __launch_bounds__(VBLK) void residual_kernel(const int32_t* rowptr, const int32_t* col,
                                                        const double* val, const double* x, const double* b,
                                                        double* r, double* part_rr, double* part_bb, int64_t n,
                                                        const uint8_t* iface_only) {
  __shared__ double sh[VBLK / 64];
  const int sl = threadIdx.x % ROW_LANES;
  const int64_t hw = (blockIdx.x * int64_t(VBLK) + threadIdx.x) / ROW_LANES;
  const int64_t nhw = (int64_t(gridDim.x) * VBLK) / ROW_LANES;
  double rr = 0.0, bb = 0.0;
  for (int64_t row0 = hw; row0 < n; row0 += ROW_U * nhw) {
    int64_t rows[ROW_U];
    double v[ROW_U];
    for (int u = 0; u < ROW_U; ++u) rows[u] = row0 + u * nhw;
    rows_dot<ROW_U>(rowptr, col, val, x, rows, n, sl, v);
    if (sl == 0)
      for (int u = 0; u < ROW_U; ++u) {
        const int64_t row = rows[u];
        if (row >= n) break;
        double rv = (iface_only && iface_only[row] < 2) ? 0.0 : b[row] - v[u];
        r[row] = rv;
        rr += rv * rv;
        bb += b[row] * b[row];
      }
  }
  double t = block_sum(rr, sh);
  double u = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part_rr[blockIdx.x] = t;
    part_bb[blockIdx.x] = u;
  }
}

void launch_residual(const int32_t* rowptr, const int32_t* col, const double* val, const double* x, const double* b,
                     double* r, double* part_rr, double* part_bb, int64_t n, hipStream_t st,
                     const uint8_t* iface_only) {
  hipLaunchKernelGGL(residual_kernel, dim3(VGRID), dim3(VBLK), 0, st, rowptr, col, val, x, b, r, part_rr, part_bb,
                     n, iface_only);
}

// scalars: per-iteration slots (rz[it], pq[it], rr[it], alpha[it], beta[it])
// p = z + beta p, q = A z + beta q (beta = rz[it]/rz[it-1]; it == 0: p = z, q = A z),
// partial sums of p.q
__global__ __launch_bounds__(VBLK) void pcg_dir_kernel(const int32_t* rowptr, const int32_t* col, const double* val,
                                                       const double* z, double* p, double* q, const double* part_rz,
                                                       double* part_pq, PcgScalars* sc, int it, int fresh,
                                                       int64_t n) {
  __shared__ double sh[VBLK / 64];
  if (sc->done) return;
  const double rz = reduce_partials(part_rz, VGRID, sh);
  double beta = 0.0;
  if (!fresh) beta = rz / sc->rz[it - 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rz[it] = rz;
    if (!fresh) sc->beta[it - 1] = beta;
  }
  const int sl = threadIdx.x % ROW_LANES;
  const int64_t hw = (blockIdx.x * int64_t(VBLK) + threadIdx.x) / ROW_LANES;
  const int64_t nhw = (int64_t(gridDim.x) * VBLK) / ROW_LANES;
  double pq = 0.0;
  for (int64_t row0 = hw; row0 < n; row0 += ROW_U * nhw) {
    int64_t rows[ROW_U];
    double az[ROW_U];
    for (int u = 0; u < ROW_U; ++u) rows[u] = row0 + u * nhw;
    rows_dot<ROW_U>(rowptr, col, val, z, rows, n, sl, az);
    if (sl == 0)
      for (int u = 0; u < ROW_U; ++u) {
        const int64_t row = rows[u];
        if (row >= n) break;
        double pv = z[row] + (fresh ? 0.0 : beta * p[row]);
        double qv = az[u] + (fresh ? 0.0 : beta * q[row]);
        p[row] = pv;
        q[row] = qv;
        pq += pv * qv;
      }
  }
  double t = block_sum(pq, sh);
  if (threadIdx.x == 0) part_pq[blockIdx.x] = t;
}

// alpha = rz/pq; x += alpha p; r -= alpha q; partial sums of r.r
__global__ __launch_bounds__(VBLK) void pcg_update_kernel(double* x, double* r, const double* p, const double* q,
                                                          const double* part_pq, double* part_rr, PcgScalars* sc,
                                                          int it, int64_t n) {
  __shared__ double sh[VBLK / 64];
  if (sc->done) return;
  const double pq = reduce_partials(part_pq, VGRID, sh);
  const double rz = sc->rz[it];
  const double alpha = rz / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->pq[it] = pq;
    sc->alpha[it] = alpha;
  }
  double rr = 0.0;
  if (pq > 0.0 && rz > 0.0) {
    for (int64_t i = blockIdx.x * int64_t(VBLK) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VBLK) {
      x[i] += alpha * p[i];
      double rv = r[i] - alpha * q[i];
      r[i] = rv;
      rr += rv * rv;
    }
  }
  double t = block_sum(rr, sh);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = t;
}

// finalise rr (convergence / breakdown decision) in a single block; later kernels
// of the iteration see sc->done
// Tells the host that the solve has ended (a word of mapped pinned host memory;
// a system-scope store, visible to the host once the kernel has completed).
__device__ __forceinline__ void signal_host(int* hdone) {
  if (hdone) __hip_atomic_store(hdone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(VBLK) void pcg_check_kernel(const double* part_rr, PcgScalars* sc, int it,
                                                         int* hdone) {
  __shared__ double sh[VBLK / 64];
  if (sc->done) return;
  const double rr = reduce_partials(part_rr, VGRID, sh);
  if (threadIdx.x == 0) {
    sc->rr[it] = rr;
    const double pq = sc->pq[it], rz = sc->rz[it];
    sc->iters = it + 1;
    if (!(pq > 0.0) || !(rz > 0.0) || !(rr == rr)) {
      sc->done = 2;
      sc->iters = it;     // the update of this iteration was not applied
      signal_host(hdone);
    } else if (rr <= sc->tol2) {
      sc->done = 1;
      signal_host(hdone);
    }
  }
}

// partial sums of r.z (it == 0: also stores rz[0])
__global__ __launch_bounds__(VBLK) void dot_kernel(const double* a, const double* b, double* part, int64_t n,
                                                   const int* done) {
  __shared__ double sh[VBLK / 64];
  if (done && *done) return;
  double v = 0.0;
  for (int64_t i = blockIdx.x * int64_t(VBLK) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VBLK) v += a[i] * b[i];
  double t = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(VBLK) void finish_dot_kernel(const double* part, double* out) {
  __shared__ double sh[VBLK / 64];
  const double v = reduce_partials(part, VGRID, sh);
  if (threadIdx.x == 0) *out = v;
}

void launch_pcg_dir(const int32_t* rowptr, const int32_t* col, const double* val, const double* z, double* p,
                    double* q, const double* part_rz, double* part_pq, PcgScalars* sc, int it, int fresh, int64_t n,
                    hipStream_t st) {
  hipLaunchKernelGGL(pcg_dir_kernel, dim3(VGRID), dim3(VBLK), 0, st, rowptr, col, val, z, p, q, part_rz, part_pq,
                     sc, it, fresh, n);
}

// tolerance from ||b||^2, initial residual check
__global__ __launch_bounds__(VBLK) void pcg_init_kernel(const double* part_rr, const double* part_bb, PcgScalars* sc,
                                                        double rtol2) {
  __shared__ double sh[VBLK / 64];
  const double rr = reduce_partials(part_rr, VGRID, sh);
  const double bb = reduce_partials(part_bb, VGRID, sh);
  if (threadIdx.x == 0) {
    sc->bb = bb;
    sc->rr0 = rr;
    sc->tol2 = rtol2 * bb;
    sc->iters = 0;
    sc->done = (rr <= rtol2 * bb) ? 1 : 0;
  }
}

void launch_pcg_init(const double* part_rr, const double* part_bb, PcgScalars* sc, double rtol2, hipStream_t st) {
  hipLaunchKernelGGL(pcg_init_kernel, dim3(1), dim3(VBLK), 0, st, part_rr, part_bb, sc, rtol2);
}
void launch_pcg_update(double* x, double* r, const double* p, const double* q, const double* part_pq,
                       double* part_rr, PcgScalars* sc, int it, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(pcg_update_kernel, dim3(VGRID), dim3(VBLK), 0, st, x, r, p, q, part_pq, part_rr, sc, it, n);
}
// End of a CG segment: the scalars the host reads, written straight into mapped
// pinned host memory (one launch instead of several copies): out[0..3] = tol2,
// bb, rr0, (done, iters) as two ints; out[4] = the true r.r; out[5] = the device
// status word (as an int); then alpha, beta and rr of iterations seg .. seg+n-1.
__global__ void pack_readback_kernel(const PcgScalars* sc, const double* rr_true, const int* werr, int seg, int n,
                                     double* out) {
  const int t = threadIdx.x;
  if (t == 0) {
    out[0] = sc->tol2;
    out[1] = sc->bb;
    out[2] = sc->rr0;
    int* w = reinterpret_cast<int*>(out + 3);
    w[0] = sc->done;
    w[1] = sc->iters;
    out[4] = *rr_true;
    int* e = reinterpret_cast<int*>(out + 5);
    e[0] = *werr;
    e[1] = 0;
  }
  for (int i = t; i < n; i += blockDim.x) {
    out[6 + i] = sc->alpha[seg + i];
    out[6 + n + i] = sc->beta[seg + i];
    out[6 + 2 * n + i] = sc->rr[seg + i];
  }
}

void launch_pack_readback(const PcgScalars* sc, const double* rr_true, const int* werr, int seg, int n,
                          double* out, hipStream_t st) {
  hipLaunchKernelGGL(pack_readback_kernel, dim3(1), dim3(256), 0, st, sc, rr_true, werr, seg, n, out);
}

void launch_pcg_check(const double* part_rr, PcgScalars* sc, int it, int* hdone, hipStream_t st) {
  hipLaunchKernelGGL(pcg_check_kernel, dim3(1), dim3(VBLK), 0, st, part_rr, sc, it, hdone);
}
void launch_dot(const double* a, const double* b, double* part, int64_t n, const int* done, hipStream_t st) {
  hipLaunchKernelGGL(dot_kernel, dim3(VGRID), dim3(VBLK), 0, st, a, b, part, n, done);
}
void launch_finish_dot(const double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(finish_dot_kernel, dim3(1), dim3(VBLK), 0, st, part, out);
}

// ---------------------------------------------------------------------------
// Interface (Schur-complement) form, FP64 local factors
// ---------------------------------------------------------------------------
// With B = interface (G = non-corner, Pi = corners) and the bordered factor of
// the equilibrated A_RR (interior first), the trailing block L_GG is
// chol(D_G S_GG D_G) and the border rows give W = L^{-1} D [C_AR^T | A_RPi], so
//   (S p)_G  = D^{-1} L_GG q,  q = L_GG^T D^{-1} p_G + W_Pi,G p_Pi
//   (S p)_Pi = W_Pi,G^T q + (A_PiPi - W_Pi^T W_Pi) p_Pi
// and the preconditioner needs L_GG^{-T} (L_GG^{-1} D f_G + W_G coef).  Setup forms
// X = inverse of the tile-aligned trailing block of L, then both operators as
// explicit symmetric matrices (the Schur complement itself and X^T X with the
// border row W_G^T X), so each application streams one triangle of tiles.

// X(ii, jj) = -Dinv_i sum_{kk=jj}^{ii-1} L(i, k) X(kk, jj), X(ii, ii) = Dinv_i
// (i = j0 + ii, k = j0 + kk); one launch per block row ii, one task per (matrix, jj)
__global__ __launch_bounds__(256) void trailing_inverse_kernel(const MatDesc* mats, const double* tiles,
                                                               const double* dinv, double* xg, int ii) {
  const MatDesc D = mats[blockIdx.y];
  const int j0 = D.n_I / NB;
  const int TG = D.T - j0;
  const int jj = blockIdx.x;
  if (ii >= TG || jj > ii) return;
  double* out = xg + (D.xg_off + tri_tile(ii, jj)) * int64_t(NB * NB);
  const double* di = dinv + (D.dinv_off + j0 + ii) * int64_t(NB * NB);
  if (jj == ii) {
    for (int e = threadIdx.x; e < NB * NB; e += 256) out[e] = di[e];
    return;
  }
  __shared__ double sa[NB * LDT];
  __shared__ double sb[NB * LDT];
  d4v acc[2][2];
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q) acc[p][q] = d4v(0);
  for (int kk = jj; kk < ii; ++kk) {
    __syncthreads();
    const double* a = tiles + env_tile(D, j0 + ii, j0 + kk) * int64_t(NB * NB);
    const double* b = xg + (D.xg_off + tri_tile(kk, jj)) * int64_t(NB * NB);
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
      sa[(e / NB) * LDT + (e % NB)] = a[e];
      sb[(e % NB) * LDT + (e / NB)] = b[e];      // transposed: gemm_nt then gives A B
    }
    __syncthreads();
    gemm_nt_tile<double>(sa, sb, acc);
  }
  __syncthreads();
  // C (in acc) -> transposed into sb; Dinv_i into sa; out = -Dinv_i C
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q)
      for (int it = 0; it < 4; ++it) {
        const int r = r0 + 16 * p + Acc4<double>::row(lane, it), c = c0 + 16 * q + (lane & 15);
        sb[c * LDT + r] = acc[p][q][it];
      }
  for (int e = threadIdx.x; e < NB * NB; e += 256) sa[(e / NB) * LDT + (e % NB)] = di[e];
  __syncthreads();
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q) acc[p][q] = d4v(0);
  gemm_nt_tile<double>(sa, sb, acc);
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q)
      for (int it = 0; it < 4; ++it) {
        const int r = r0 + 16 * p + Acc4<double>::row(lane, it), c = c0 + 16 * q + (lane & 15);
        out[r * NB + c] = -acc[p][q][it];
      }
}

void launch_trailing_inverse(const MatDesc* mats, int nmats, int maxTG, const double* tiles, const double* dinv,
                             double* xg, hipStream_t st) {
  for (int ii = 0; ii < maxTG; ++ii)
    hipLaunchKernelGGL(trailing_inverse_kernel, dim3(ii + 1, nmats), dim3(256), 0, st, mats, tiles, dinv, xg, ii);
}

// Explicit coarse inverse: A_c^{-1} = D X^T X D with X = L_c^{-1} (L_c the
// Cholesky factor of the equilibrated D A_c D, X lower triangular in tiles, the
// diagonal tiles with zeros above the diagonal), row-major dense.  One workgroup
// per output tile (I, J): the sum over K >= max(I, J) of X(K, I)^T X(K, J) on
// MFMA, both tiles transposed into LDS.
__global__ __launch_bounds__(256) void coarse_inverse_kernel(const double* xg, const double* dc, int nc,
                                                             double* ainv) {
  const int I = blockIdx.y, J = blockIdx.x;
  const int Tc = (nc + NB - 1) / NB;
  __shared__ double sa[NB * LDT];
  __shared__ double sb[NB * LDT];
  d4v acc[2][2];
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q) acc[p][q] = d4v(0);
  for (int K = max(I, J); K < Tc; ++K) {
    __syncthreads();
    const double* a = xg + tri_tile(K, I) * int64_t(NB * NB);
    const double* b = xg + tri_tile(K, J) * int64_t(NB * NB);
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
      sa[(e % NB) * LDT + (e / NB)] = a[e];   // X(K, I)^T
      sb[(e % NB) * LDT + (e / NB)] = b[e];   // X(K, J)^T: gemm_nt gives X(K, I)^T X(K, J)
    }
    __syncthreads();
    gemm_nt_tile<double>(sa, sb, acc);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q)
      for (int it = 0; it < 4; ++it) {
        const int i = I * NB + r0 + 16 * p + Acc4<double>::row(lane, it), j = J * NB + c0 + 16 * q + (lane & 15);
        if (i < nc && j < nc) ainv[int64_t(i) * nc + j] = dc[i] * acc[p][q][it] * dc[j];
      }
}

void launch_coarse_inverse(const double* xg, const double* dc, int nc, double* ainv, hipStream_t st) {
  if (nc <= 0) return;
  const int Tc = (nc + NB - 1) / NB;
  hipLaunchKernelGGL(coarse_inverse_kernel, dim3(Tc, Tc), dim3(256), 0, st, xg, dc, nc, ainv);
}

constexpr int CG_RW = 8;   // rows of A_c^{-1} per wave of the coarse GEMV
// u_c = A_c^{-1} r_c with r_c = sum_i R_ci^T g_i gathered per column block; block
// (4 CG_RW rows, column split s) writes its partial u into upart[s*nc + i]
__global__ __launch_bounds__(256) void coarse_gemv_kernel(const double* ainv, int nc, int cs,
                                                          const int32_t* cinv_ptr, const int32_t* cinv,
                                                          const double* gbuf, double* upart, const int* done) {
  __shared__ double rcs[COARSE_SPLIT_COLS];
  const int dn = done ? *done : 0;   // tested once the loads are in flight
  const int s = blockIdx.y;
  const int j0 = s * cs, j1 = min(nc, j0 + cs);
  // CG_RW rows per wave, loaded while the coarse residual is assembled (the
  // assembly of a column slice is repeated by every block of the slice, so a
  // block takes many rows)
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = (blockIdx.x * 4 + w) * CG_RW;
  constexpr int PER_LANE = COARSE_SPLIT_COLS / 64;
  double rv[CG_RW][PER_LANE];
  for (int k = 0; k < CG_RW; ++k) {
    const double* row = ainv + int64_t(min(i0 + k, nc - 1)) * nc;
    for (int q = 0; q < PER_LANE; ++q) {
      const int j = j0 + lane + 64 * q;
      rv[k][q] = j < j1 ? row[j] : 0.0;
    }
  }
  for (int j = j0 + threadIdx.x; j < j1; j += 256) {
    double v = 0.0;
    for (int q = cinv_ptr[j]; q < cinv_ptr[j + 1]; ++q) v += gbuf[cinv[q]];
    rcs[j - j0] = v;
  }
  if (dn) return;
  __syncthreads();
  for (int k = 0; k < CG_RW; ++k) {
    const int i = i0 + k;
    if (i >= nc) break;
    double v = 0.0;
    for (int q = 0; q < PER_LANE; ++q)
      if (j0 + lane + 64 * q < j1) v += rv[k][q] * rcs[lane + 64 * q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) upart[int64_t(s) * nc + i] = v;
  }
}

void launch_coarse_gemv(const double* ainv, int nc, int nsplit, const int32_t* cinv_ptr, const int32_t* cinv,
                        const double* gbuf, double* upart, const int* done, hipStream_t st) {
  if (nc <= 0) return;
  const int cs = (nc + nsplit - 1) / nsplit;
  hipLaunchKernelGGL(coarse_gemv_kernel, dim3((nc + 4 * CG_RW - 1) / (4 * CG_RW), nsplit), dim3(256), 0, st, ainv,
                     nc, cs, cinv_ptr,
                     cinv, gbuf, upart, done);
}

// The coarse problem by CG (the paper's choice; an option beside the explicit
// inverse): A_c u_c = r_c with r_c = sum of the subdomain shares gbuf over the
// coarse inverse map, CG preconditioned by diag(A_c)^{-1} = dc^2 from u_c = 0
// until ||r|| <= tol ||r_c|| or maxit mat-vecs, in one workgroup.  The iteration
// is the single-reduction form of Chronopoulos and Gear (same iterates as CG in
// exact arithmetic): with u = M r and w = A u, gamma = (r, u), delta = (w, u),
// beta = gamma / gamma_old, alpha = gamma / (delta - beta gamma / alpha_old),
// p = u + beta p, s = w + beta s (= A p), x += alpha p, r -= alpha s, so that one
// block reduction (gamma, delta and ||r||^2 together) serves an iteration.  fval
// is the full symmetric A_c in CSR (rowptr, col), gathered once at setup from the
// stored lower triangle.  A group of CCG_G lanes forms each row's product and the
// group's first lane owns that row in every vector operation, so u is the only
// vector that threads share.  When the seven vectors (r, u, p, s, w, dc^2, x) and
// the CSR fit in CCG_LDS_DBL doubles of LDS they are all kept there (the CSR is
// copied in once per launch, so an iteration touches no global memory); else the
// vectors live in work (7 nc doubles) and the CSR is read through L2.
constexpr int CCG_BLK = 1024;
constexpr int CCG_G = 2;
constexpr int CCG_NG = CCG_BLK / CCG_G;
constexpr int CCG_LDS_DBL = 19200;   // 150 KB of the 160 KB of LDS of a CDNA4 compute unit

__device__ __forceinline__ void ccg_sum3(double& a, double& b, double& c, double* sh) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
    c += __shfl_xor(c, off, 64);
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    sh[3 * w] = a;
    sh[3 * w + 1] = b;
    sh[3 * w + 2] = c;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  c = 0.0;
  for (int i = 0; i < CCG_BLK / 64; ++i) {
    a += sh[3 * i];
    b += sh[3 * i + 1];
    c += sh[3 * i + 2];
  }
}

template <bool SH>
__global__ __launch_bounds__(CCG_BLK) void coarse_cg_kernel(const int32_t* rowptr_g, const int32_t* col_g,
                                                           const double* fval_g, int nnz, const double* dc, int nc,
                                                           const int32_t* cinv_ptr, const int32_t* cinv,
                                                           const double* gbuf, double* uc, double* work, double tol2,
                                                           int maxit, const int* done, int* werr) {
  __shared__ double sh[3 * (CCG_BLK / 64)];
  __shared__ double sv[SH ? CCG_LDS_DBL : 1];
  if (done && *done) return;
  const int ld = nc;
  double* r = SH ? sv : work;
  const double* fval = fval_g;
  const int32_t* col = col_g;
  const int32_t* rowptr = rowptr_g;
  if (SH) {
    double* fs = sv + 7 * int64_t(nc);
    int32_t* cs = reinterpret_cast<int32_t*>(fs + nnz);
    int32_t* rs = cs + nnz;
    for (int k = threadIdx.x; k < nnz; k += CCG_BLK) {
      fs[k] = fval_g[k];
      cs[k] = col_g[k];
    }
    for (int k = threadIdx.x; k <= nc; k += CCG_BLK) rs[k] = rowptr_g[k];
    fval = fs;
    col = cs;
    rowptr = rs;
  }
  double* u = r + ld;
  double* p = r + 2 * ld;
  double* s = r + 3 * ld;
  double* w = r + 4 * ld;
  double* dd = r + 5 * ld;
  double* x = r + 6 * ld;
  const int t = threadIdx.x, g = t / CCG_G, l = t % CCG_G;
  const bool own = (l == 0);
  if (own)
    for (int i = g; i < nc; i += CCG_NG) {
      double v = 0.0;
      for (int k = cinv_ptr[i]; k < cinv_ptr[i + 1]; ++k) v += gbuf[cinv[k]];
      const double d2 = dc[i] * dc[i];
      r[i] = v;
      dd[i] = d2;
      u[i] = d2 * v;
      x[i] = 0.0;
    }
  double bb = 0.0, gam_old = 1.0, alpha = 1.0;
  for (int it = 0; it <= maxit; ++it) {
    __syncthreads();   // u complete
    double gam = 0.0, del = 0.0, rr = 0.0;
    for (int i = g; i < nc; i += CCG_NG) {
      double v = 0.0;
#pragma unroll 4
      for (int k = rowptr[i] + l; k < rowptr[i + 1]; k += CCG_G) v += fval[k] * u[col[k]];
      for (int o = CCG_G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, CCG_G);
      if (own) {
        w[i] = v;
        const double ui = u[i], ri = r[i];
        gam += ri * ui;
        del += v * ui;
        rr += ri * ri;
      }
    }
    ccg_sum3(gam, del, rr, sh);
    if (it == 0) bb = rr;
    if (!(bb > 0.0) || rr <= tol2 * bb) break;
    const double beta = it == 0 ? 0.0 : gam / gam_old;
    const double den = del - beta * gam / alpha;
    if (it == maxit || !(gam > 0.0) || !(den > 0.0)) {
      // not converged: iteration limit or breakdown (A_c not positive definite)
      if (threadIdx.x == 0) atomicOr(werr, DEV_COARSE_NOCONV);
      break;
    }
    alpha = gam / den;
    gam_old = gam;
    if (own)
      for (int i = g; i < nc; i += CCG_NG) {
        const double pi = it == 0 ? u[i] : u[i] + beta * p[i];
        const double si = it == 0 ? w[i] : w[i] + beta * s[i];
        p[i] = pi;
        s[i] = si;
        x[i] += alpha * pi;
        const double ri = r[i] - alpha * si;
        r[i] = ri;
        u[i] = dd[i] * ri;
      }
  }
  if (own)
    for (int i = g; i < nc; i += CCG_NG) uc[i] = x[i];
}

// The same CG spread over CCG_GRID workgroups when A_c does not fit one
// workgroup's LDS: workgroup g owns a contiguous block of rows, keeps that
// block's CSR and its rows of r, p, s, w, dc^2 and x in LDS, and copies the
// shared vector u into LDS for each mat-vec.  An iteration meets twice at a
// grid-wide barrier: after the partial sums of (gamma, delta, ||r||^2) are
// written (every workgroup then adds all partials in the same order, so all
// take the same decisions), and after every workgroup has written its rows of
// the new u.  u and the partial sums are written and read with device-scope
// atomic accesses.  A barrier wait gives up after `spin` polls, marks the
// status word and ends the workgroup's iteration, so that the kernel finishes
// instead of hanging; the 64 workgroups, one per compute unit by their LDS
// size, are normally co-resident, and otherwise the late ones start as the
// earlier kernels on the device drain.
constexpr int CCG_GRID = 64;          // workgroups
constexpr int CCG_GBLK = 256;         // threads per workgroup
constexpr int CCG_GG = 4;             // lanes per row of the mat-vec
constexpr int CCG_GROWS = 256;        // rows per workgroup held in LDS
constexpr int CCG_GLDS_DBL = 12000;   // LDS doubles for u, the block's CSR values and columns
static_assert(CCG_GRID <= 64, "one lane per workgroup in the reduction of the partial sums");

__device__ __forceinline__ bool ccg_grid_barrier(unsigned* bar, unsigned& gen, int spin, int* werr) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  __shared__ int s_ok;
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned g = gen;
    const unsigned n = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
    if (n == gridDim.x) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&bar[1], g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      int n = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (n++ >= spin) {
          atomicOr(werr, DEV_WAIT_GAVE_UP);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    gen = g + 1;
    s_ok = ok;
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(s_ok) != 0;
}

__global__ __launch_bounds__(CCG_GBLK) void coarse_cg_grid_kernel(const int32_t* rowptr, const int32_t* col,
                                                                 const double* fval, const double* dc, int nc,
                                                                 const int32_t* cinv_ptr, const int32_t* cinv,
                                                                 const double* gbuf, double* uc, double* work,
                                                                 unsigned* bar, double tol2, int maxit,
                                                                 int spin, const int* done, int* werr) {
  __shared__ double sh[3 * (CCG_GBLK / 64)];
  __shared__ double sv[CCG_GLDS_DBL];
  __shared__ double rv[6 * CCG_GROWS];
  if (done && *done) return;
  const int G = gridDim.x, b = blockIdx.x, t = threadIdx.x;
  const int r0 = int(int64_t(nc) * b / G), r1 = int(int64_t(nc) * (b + 1) / G);
  const int nr = r1 - r0;
  const int k0 = rowptr[r0], nk = rowptr[r1] - k0;
  // LDS: u (nc), then the block's CSR values and columns when they fit
  const bool csr_lds = nc + nk + (nk + 1) / 2 <= CCG_GLDS_DBL;
  double* us = sv;
  double* fs = sv + nc;
  int32_t* cs = reinterpret_cast<int32_t*>(sv + nc + nk);
  if (csr_lds)
    for (int k = t; k < nk; k += CCG_GBLK) {
      fs[k] = fval[k0 + k];
      cs[k] = col[k0 + k];
    }
  double* r = rv;
  double* p = rv + CCG_GROWS;
  double* s = rv + 2 * CCG_GROWS;
  double* w = rv + 3 * CCG_GROWS;
  double* dd = rv + 4 * CCG_GROWS;
  double* x = rv + 5 * CCG_GROWS;
  double* ug = work;                 // shared u (nc)
  double* part = work + nc;          // 3 partial sums per workgroup
  for (int i = t; i < nr; i += CCG_GBLK) {
    double v = 0.0;
    for (int k = cinv_ptr[r0 + i]; k < cinv_ptr[r0 + i + 1]; ++k) v += gbuf[cinv[k]];
    const double d2 = dc[r0 + i] * dc[r0 + i];
    r[i] = v;
    dd[i] = d2;
    x[i] = 0.0;
    store_agent(ug + r0 + i, d2 * v);
  }
  unsigned gen = 0;
  bool ok = ccg_grid_barrier(bar, gen, spin, werr);
  const int g = t / CCG_GG, l = t % CCG_GG;
  constexpr int NG = CCG_GBLK / CCG_GG;
  double bb = 0.0, gam_old = 1.0, alpha = 1.0;
  for (int it = 0; ok && it <= maxit; ++it) {
    // u into LDS, eight loads in flight per thread
    constexpr int UB = 8;
    for (int i0 = t; i0 < nc; i0 += UB * CCG_GBLK) {
      double v[UB];
#pragma unroll
      for (int q = 0; q < UB; ++q) {
        v[q] = load_agent(ug + min(i0 + q * CCG_GBLK, nc - 1));   // unconditional: no branch between the loads
      }
#pragma unroll
      for (int q = 0; q < UB; ++q) {
        const int i = i0 + q * CCG_GBLK;
        if (i < nc) us[i] = v[q];
      }
    }
    __syncthreads();
    double gam = 0.0, del = 0.0, rr = 0.0;
    for (int i = g; i < nr; i += NG) {
      double v = 0.0;
      const int a = rowptr[r0 + i] - k0, e = rowptr[r0 + i + 1] - k0;
      if (csr_lds)
        for (int k = a + l; k < e; k += CCG_GG) v += fs[k] * us[cs[k]];
      else
        for (int k = a + l; k < e; k += CCG_GG) v += fval[k0 + k] * us[col[k0 + k]];
      for (int o = CCG_GG / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, CCG_GG);
      if (l == 0) {
        w[i] = v;
        const double ui = us[r0 + i], ri = r[i];
        gam += ri * ui;
        del += v * ui;
        rr += ri * ri;
      }
    }
    // block partial sums, in a fixed order
    for (int off = 32; off > 0; off >>= 1) {
      gam += __shfl_xor(gam, off, 64);
      del += __shfl_xor(del, off, 64);
      rr += __shfl_xor(rr, off, 64);
    }
    if ((t & 63) == 0) {
      sh[3 * (t >> 6)] = gam;
      sh[3 * (t >> 6) + 1] = del;
      sh[3 * (t >> 6) + 2] = rr;
    }
    __syncthreads();
    if (t < 3) {
      double v = 0.0;
      for (int q = 0; q < CCG_GBLK / 64; ++q) v += sh[3 * q + t];
      store_agent(part + 3 * b + t, v);
    }
    if (!ccg_grid_barrier(bar, gen, spin, werr)) break;
    // every wave reads the G partial sums (lane q those of workgroup q) and adds
    // them by a butterfly: IEEE addition is commutative, so every lane of every
    // wave of every workgroup ends with the same bits
    {
      const int q = t & 63, qc = min(q, G - 1);
      const double g0 = load_agent(part + 3 * qc), d0 = load_agent(part + 3 * qc + 1),
                   r0v = load_agent(part + 3 * qc + 2);
      gam = q < G ? g0 : 0.0;
      del = q < G ? d0 : 0.0;
      rr = q < G ? r0v : 0.0;
      for (int off = 32; off > 0; off >>= 1) {
        gam += __shfl_xor(gam, off, 64);
        del += __shfl_xor(del, off, 64);
        rr += __shfl_xor(rr, off, 64);
      }
    }
    if (it == 0) bb = rr;
    // every lane holds the same sums; the decisions are read as scalars so that
    // the compiler keeps the loop and its barriers uniform
    if (__builtin_amdgcn_readfirstlane(int(!(bb > 0.0) || rr <= tol2 * bb))) break;
    const double beta = it == 0 ? 0.0 : gam / gam_old;
    const double den = del - beta * gam / alpha;
    if (__builtin_amdgcn_readfirstlane(int(it == maxit || !(gam > 0.0) || !(den > 0.0)))) {
      if (b == 0 && t == 0) atomicOr(werr, DEV_COARSE_NOCONV);
      break;
    }
    alpha = gam / den;
    gam_old = gam;
    for (int i = t; i < nr; i += CCG_GBLK) {
      const double ui = us[r0 + i];
      const double pi = it == 0 ? ui : ui + beta * p[i];
      const double si = it == 0 ? w[i] : w[i] + beta * s[i];
      p[i] = pi;
      s[i] = si;
      x[i] += alpha * pi;
      const double ri = r[i] - alpha * si;
      r[i] = ri;
      store_agent(ug + r0 + i, dd[i] * ri);
    }
    ok = ccg_grid_barrier(bar, gen, spin, werr);
  }
  for (int i = t; i < nr; i += CCG_GBLK) uc[r0 + i] = x[i];
}

__global__ void coarse_cg_matrix_kernel(const int32_t* fsrc, const double* val, double* fval, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) fval[k] = val[fsrc[k]];
}

void launch_coarse_cg_matrix(const int32_t* fsrc, const double* val, double* fval, int nnz, hipStream_t st) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(coarse_cg_matrix_kernel, dim3((nnz + 255) / 256), dim3(256), 0, st, fsrc, val, fval, nnz);
}

void launch_coarse_cg(const int32_t* rowptr, const int32_t* col, const double* fval, int nnz, const double* dc,
                      int nc, const int32_t* cinv_ptr, const int32_t* cinv, const double* gbuf, double* u,
                      double* work, double tol, int maxit, int spin, const int* done, int* werr,
                      hipStream_t st) {
  if (nc <= 0) return;
  // LDS bytes of the resident variant: 7 nc + nnz doubles, nnz + nc + 1 ints
  const int64_t need = 8 * (7 * int64_t(nc) + nnz) + 4 * (int64_t(nnz) + nc + 1);
  if (need <= 8 * int64_t(CCG_LDS_DBL)) {
    hipLaunchKernelGGL(coarse_cg_kernel<true>, dim3(1), dim3(CCG_BLK), 0, st, rowptr, col, fval, nnz, dc, nc,
                       cinv_ptr, cinv, gbuf, u, work, tol * tol, maxit, done, werr);
  } else if (coarse_cg_grid_fits(nc)) {
    // the grid variant's barrier words sit after its shared vectors
    unsigned* bar = reinterpret_cast<unsigned*>(work + nc + 3 * CCG_GRID);
    launch_fill<unsigned>(bar, 0u, 2, st);
    hipLaunchKernelGGL(coarse_cg_grid_kernel, dim3(CCG_GRID), dim3(CCG_GBLK), 0, st, rowptr, col, fval, dc, nc,
                       cinv_ptr, cinv, gbuf, u, work, bar, tol * tol, maxit, spin, done, werr);
  } else {
    hipLaunchKernelGGL(coarse_cg_kernel<false>, dim3(1), dim3(CCG_BLK), 0, st, rowptr, col, fval, nnz, dc, nc,
                       cinv_ptr, cinv, gbuf, u, work, tol * tol, maxit, done, werr);
  }
}

bool coarse_cg_grid_fits(int nc) {
  // every workgroup holds u and at most CCG_GROWS rows of the six row vectors
  return nc < CCG_GLDS_DBL && (nc + CCG_GRID - 1) / CCG_GRID <= CCG_GROWS;
}

// Symmetric interface matrices of a subdomain, lower tile triangle over
// sym_tile_rows tile rows.  Rows (and columns) 0..n_G-1 are the interface rows
// (local dofs n_I + r), rows n_G + c the constraints c < n_ci.  M = K K^T with
// K of n_G columns (the interface rows again):
//   SYM_OP: K(r, k) = L(n_I+r, n_I+k) (k <= r), K(n_G+c, k) = W^T(c, n_I+k) for the
//           corners c >= n_A (zero for the averages); A_PiPi - W_Pi^T W_Pi is added
//           to the corner block.  M is the equilibrated local Schur complement on
//           [G | Pi]: L_GG L_GG^T, W_Pi,G^T L_GG^T, cpp + W_Pi,G^T W_Pi,G.
//   SYM_PC: K(r, k) = X(n_I+k, n_I+r) (k >= r), K(n_G+c, k) = W^T(c, n_I+k) for all
//           constraints, so M_GG = X_GG^T X_GG = (L_GG L_GG^T)^{-1} and the
//           constraint rows hold W_G^T X_GG = (L_GG^{-T} W_G)^T.
// (X, the inverse of the tile-aligned trailing block of L, acts on the interface
// rows through its block X_GG = L_GG^{-1}.)  One workgroup per output tile, MFMA.
template <int MODE>
__device__ void load_k_tile(double* dst, const MatDesc& D, const double* tiles, const double* xg, int ii, int kk) {
  const int nG = D.n_R - D.n_I, j0 = D.n_I / NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int rl = e / NB, cl = e % NB;
    const int r = ii * NB + rl, k = kk * NB + cl;
    double v = 0.0;
    if (k < nG) {
      const int b = D.n_I + k;
      if (r < nG) {
        const int a = D.n_I + r;
        if (MODE == SYM_OP) {
          if (k <= r) v = tiles[env_tile(D, a / NB, b / NB) * (NB * NB) + (a % NB) * NB + b % NB];
        } else {
          if (k >= r) v = xg[(D.xg_off + tri_tile(b / NB - j0, a / NB - j0)) * (NB * NB) + (b % NB) * NB + a % NB];
        }
      } else {
        const int c = r - nG;
        if (c < D.n_ci && (MODE == SYM_PC || c >= D.n_A))
          v = tiles[env_tile(D, D.T, b / NB) * (NB * NB) + c * NB + b % NB];
      }
    }
    dst[rl * LDT + cl] = v;
  }
}

template <int MODE, typename TO>
__global__ __launch_bounds__(256) void sym_build_kernel(const MatDesc* mats, const double* tiles, const double* xg,
                                                         const double* cpp, TO* out) {
  const int s = blockIdx.y;
  const MatDesc D = mats[s];
  const int TS = sym_tile_rows(D), nG = D.n_R - D.n_I;
  const int KG = (nG + NB - 1) / NB;
  const int64_t pidx = blockIdx.x;
  if (pidx >= tri_tile(TS, 0)) return;
  int ii = int((sqrt(8.0 * double(pidx) + 1.0) - 1.0) * 0.5);
  while (tri_tile(ii, 0) > pidx) --ii;
  while (tri_tile(ii + 1, 0) <= pidx) ++ii;
  const int jj = int(pidx - tri_tile(ii, 0));
  // K(ii, kk) and K(jj, kk) (jj <= ii) are both nonzero only for kk in [k0, k1);
  // a tile row without constraint rows is triangular in K
  const bool pure_i = (ii + 1) * NB <= nG, pure_j = (jj + 1) * NB <= nG;
  int k0 = 0, k1 = KG;
  if (MODE == SYM_OP) {
    if (pure_j) k1 = min(jj + 1, KG);
  } else {
    k0 = max(pure_i ? ii : 0, pure_j ? jj : 0);
  }
  __shared__ double sa[NB * LDT];
  __shared__ double sb[NB * LDT];
  d4v acc[2][2];
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q) acc[p][q] = d4v(0);
  for (int kk = k0; kk < k1; ++kk) {
    __syncthreads();
    load_k_tile<MODE>(sa, D, tiles, xg, ii, kk);
    if (jj != ii) load_k_tile<MODE>(sb, D, tiles, xg, jj, kk);
    __syncthreads();
    gemm_nt_tile<double>(sa, jj != ii ? sb : sa, acc);
  }
  TO* o = out + (D.sg_off + pidx) * int64_t(NB * NB);
  const double* m = cpp + int64_t(s) * MAX_NCI * MAX_NCI;
  const int p0 = nG + D.n_A, p1 = nG + D.n_ci;   // corner rows
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q)
      for (int it = 0; it < 4; ++it) {
        const int r = r0 + 16 * p + Acc4<double>::row(lane, it), c = c0 + 16 * q + (lane & 15);
        double v = acc[p][q][it];
        const int R = ii * NB + r, C = jj * NB + c;
        if (MODE == SYM_OP && R >= p0 && R < p1 && C >= p0 && C < p1) v += m[(R - p0) * MAX_NCI + (C - p0)];
        o[sizeof(TO) == 4 ? sym_f32_off(r, c) : r * NB + c] = TO(v);
      }
}

void launch_sym_build(int mode, const MatDesc* mats, int nmats, int maxTS, const double* tiles, const double* xg,
                      const double* cpp, void* out, bool out32, hipStream_t st) {
  if (maxTS <= 0 || nmats <= 0) return;   // no interface (a single subdomain)
  const dim3 grid(unsigned(tri_tile(maxTS, 0)), nmats);
  if (mode == SYM_OP)
    hipLaunchKernelGGL((sym_build_kernel<SYM_OP, double>), grid, dim3(256), 0, st, mats, tiles, xg, cpp,
                       static_cast<double*>(out));
  else if (out32)
    hipLaunchKernelGGL((sym_build_kernel<SYM_PC, float>), grid, dim3(256), 0, st, mats, tiles, xg, cpp,
                       static_cast<float*>(out));
  else
    hipLaunchKernelGGL((sym_build_kernel<SYM_PC, double>), grid, dim3(256), 0, st, mats, tiles, xg, cpp,
                       static_cast<double*>(out));
}

// Lane reductions of the interface mat-vec (no LDS crossbar).  A double moves
// as two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
// the sum over lane bits 4 and 5 by the row and half-wave swaps (each swap
// returns both halves, whose sum is the same in every lane)
__device__ __forceinline__ double sum_hi_bits(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  v = __hiloint2double(ph[0], pl[0]) + __hiloint2double(ph[1], pl[1]);
  lo = __double2loint(v);
  hi = __double2hiint(v);
  pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(ph[0], pl[0]) + __hiloint2double(ph[1], pl[1]);
}
__device__ __forceinline__ float sum_hi_bits(float v) {
  auto p = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
  v = __int_as_float(p[0]) + __int_as_float(p[1]);
  p = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
  return __int_as_float(p[0]) + __int_as_float(p[1]);
}
// FP64 layout: the sum over lane bits 0..2 (two quad permutations, then the
// mirror inside each half-row of eight lanes: after the first two steps every
// lane of a quad holds the quad's sum) and over lane bits 3..5 (a rotation by
// 8 inside each row of 16 lanes, then the swaps).
__device__ __forceinline__ double sum_cp(double v) {
  v += dpp_f64<0xB1>(v);    // quad permutation [1,0,3,2]
  v += dpp_f64<0x4E>(v);    // quad permutation [2,3,0,1]
  v += dpp_f64<0x141>(v);   // mirror inside each half-row
  return v;
}
__device__ __forceinline__ double sum_rg(double v) {
  v += dpp_f64<0x128>(v);   // row rotation by 8
  return sum_hi_bits(v);
}
// FP32 layout: the sum over lane bits 0..1 (the quad permutations) and over
// lane bits 2..5 (rotations by 4 and 8 inside each row, then the swaps).
__device__ __forceinline__ float sum_cp(float v) {
  v += dpp_f32<0xB1>(v);
  v += dpp_f32<0x4E>(v);
  return v;
}
__device__ __forceinline__ float sum_rg(float v) {
  v += dpp_f32<0x124>(v);   // row rotation by 4
  v += dpp_f32<0x128>(v);   // row rotation by 8
  return sum_hi_bits(v);
}

// Lane layout of the interface mat-vec for matrix elements of type T: a lane
// loads VEC consecutive columns (16 bytes), CPL lanes cover the 16 columns of
// a wave, and lane = CPL * rg + cp holds rows rg + RG t (t < KR).  Products
// accumulate in T (an FP32 matrix is applied with FP32 accumulation); the
// partial results are stored in FP64.
template <typename T> struct SymLayout;
template <> struct SymLayout<double> {
  using V = d2v;
  static constexpr int VEC = 2, CPL = 8, RG = 8, KR = 8;
};
template <> struct SymLayout<float> {
  using V = f4v;
  static constexpr int VEC = 4, CPL = 4, RG = 16, KR = 4;
};

// y = M v for the symmetric interface matrices, all subdomains at once.  The
// launch splits the tile stream into equal contiguous ranges (no tickets):
// every tile (ii, jj) is read once and used twice, for the row product
// sum_jj M(ii, jj) v_jj (kept in registers along a row piece, see
// sym_row_product) and the column product M(ii, jj)^T v_ii.  A diagonal tile
// counts its lower triangle in the row product and its strict lower triangle in
// the column product.  Output row k of a subdomain is then its row product plus
// the column products of the tiles (i, k), i >= k.  Inputs come from padded
// per-row vectors (zero where a row has no interface dof).
// Wave w owns columns 16w..16w+15 of every tile (lane layout: SymLayout), so a
// column product reduces over the RG row-group lanes of one wave and a row
// product over the CPL column lanes.  The partial products are a write stream
// beside the tile reads, and on MI355X such writes cost the reads far more than
// their share of the bytes, so they are staged in LDS:
//  - the column products of a column jj < A.lds_cols (at most SYM_LDS_COLS) are
//    summed over the rows of the range and stored once, at the column's first
//    tile in the range (sym_col_first tells those slots apart); the other
//    columns store one product per tile;
//  - a row piece's sums are added over the four waves (one barrier per piece)
//    and the range's first pieces are stored as whole lines when it is done.
// Rows that hold nothing are not read: past the matrix's last row, in a zero
// row range (the average-constraint rows of the operator), and in a diagonal
// tile the row blocks above wave w's columns.
// Tile descriptors are uniform per wave and read-only: scalar loads (constant
// address space), which complete independently of the vector memory counter.
template <typename T>
__global__ __launch_bounds__(256) void sym_mv_kernel(IfaceArgs A) {
  using L = SymLayout<T>;
  using V = typename L::V;
  constexpr int VEC = L::VEC, CPL = L::CPL, RG = L::RG, KR = L::KR;
  if (A.sc->done) return;
  if (A.check_it >= 0) {
    // the convergence decision of CG iteration check_it, taken by every
    // workgroup from the same partial sums of r.r (workgroup 0 records it)
    __shared__ double sh[VBLK / 64];
    const int it = A.check_it;
    PcgScalars* sc = const_cast<PcgScalars*>(A.sc);
    const double pq = sc->pq[it], rz = sc->rz[it];
    const double rr = reduce_partials(A.part_rr, A.nparts_rr, sh);
    const bool bad = !(pq > 0.0) || !(rz > 0.0) || !(rr == rr);
    const bool conv = rr <= sc->tol2;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->rr[it] = rr;
      sc->iters = bad ? it : it + 1;   // a breakdown leaves this iteration's update unapplied
      if (bad) sc->done = 2;
      else if (conv) sc->done = 1;
      if (bad || conv) signal_host(A.hdone);
    }
    if (bad || conv) return;
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rg = lane / CPL, cp = lane % CPL;
  const int col = 16 * w + VEC * cp;
  // column sums of this range (wave w keeps its own 16 columns, so the waves
  // share nothing), the first tile of each column in the range (per wave), and
  // the columns touched since the range or the subdomain started
  __shared__ double s_col[SYM_LDS_COLS][NB];
  __shared__ int32_t s_first[4][SYM_LDS_COLS];
  uint64_t touched = 0;
  static_assert(SYM_LDS_COLS <= 64, "one bit per column");
  // a row piece's sums: the four waves' partial sums (double-buffered) are added
  // in a fixed order after a barrier; the range's first A.row_pieces pieces
  // (at most SYM_ROW_PIECES) are stored as whole lines when the range is done,
  // later ones at once
  __shared__ double s_rpart[2][4][NB];
  __shared__ double s_row[SYM_ROW_PIECES][NB];
  __shared__ int32_t s_pstart[SYM_ROW_PIECES];
  int npieces = 0;
  const int64_t N = A.ntiles, G = gridDim.x;
  const int64_t t0 = blockIdx.x * N / G, t1 = (blockIdx.x + 1) * N / G;
  if (t0 >= t1) return;
  const T* mat = static_cast<const T*>(A.m);
  const double* xv = A.xpad;
  const cint32_t* tinfo = (const cint32_t*)(A.tinfo);
  const cint32_t* trows = (const cint32_t*)(A.trows);
  int cur_row = tinfo[t0] >> 8;
  int64_t pstart = t0;
  T xi[KR], racc[KR];
  for (int t = 0; t < KR; ++t) {
    xi[t] = T(xv[int64_t(cur_row) * NB + rg + RG * t]);
    racc[t] = T(0);
  }
  // (every wave of the workgroup meets the same row changes: the barrier is
  // uniform.  A buffer of s_rpart is written again two pieces later, after the
  // next barrier, which wave 0 reaches only once it has read the buffer.)
  auto flush = [&]() {
    const int b = npieces & 1;
    for (int t = 0; t < KR; ++t) {
      const T v = sum_cp(racc[t]);
      if (cp == 0) s_rpart[b][w][rg + RG * t] = double(v);
      racc[t] = T(0);
    }
    __syncthreads();
    if (w == 0) {
      const double y = ((s_rpart[b][0][lane] + s_rpart[b][1][lane]) + s_rpart[b][2][lane]) + s_rpart[b][3][lane];
      if (npieces < A.row_pieces) {
        s_row[npieces][lane] = y;
        if (lane == 0) s_pstart[npieces] = int32_t(pstart);
      } else {
        A.rowp[pstart * NB + lane] = y;
      }
    }
    ++npieces;
  };
  auto flush_cols = [&]() {
    for (uint64_t m = touched; m != 0; m &= m - 1) {
      const int jj = __builtin_ctzll(m);
      const int64_t slot = s_first[w][jj];
      if (rg == 0)
        for (int j = 0; j < VEC; j += 2) {
          d2v o2;
          o2[0] = s_col[jj][col + j];
          o2[1] = s_col[jj][col + j + 1];
          *reinterpret_cast<d2v*>(A.part + slot * NB + col + j) = o2;
        }
    }
    touched = 0;
  };
  // the tile descriptors run one tile ahead, so that every load of a tile (its
  // elements, its inputs, the inputs of a row that starts at it) issues at once
  int inf_next = tinfo[t0], rws_next = trows[t0];
  for (int64_t t = t0; t < t1; ++t) {
    const int inf = inf_next, rws = rws_next;
    const int row = inf >> 8, d = inf & 255;
    const int jt = int(unsigned(rws) >> 24);   // the tile's column in its subdomain
    if (jt == 0 && d == 0) flush_cols();        // tile (0, 0): a new subdomain
    V b[KR];
    {
      // FP64 tiles are row-major (a wave's 16 columns of a row: one 128-byte
      // line); FP32 tiles are stored by 16-column blocks (sym_f32_off), so that a
      // wave reads whole lines of its own block
      constexpr int RS = sizeof(T) == 4 ? 16 : NB;   // row stride
      const T* p = mat + t * (NB * NB) + (sizeof(T) == 4 ? sym_f32_off(0, 16 * w) + VEC * cp : col) + rg * RS;
      // rows kept: r < h, outside [z0, z1), and (diagonal tile) r >= 16 w
      const int h = rws & 255, z0 = (rws >> 8) & 255, z1 = (rws >> 16) & 255;
      const int rmin = d == 0 ? 16 * w : 0;
      for (int k = 0; k < KR; ++k) {
        const int r = rg + RG * k;
        V v = V(T(0));
        if (r < h && r >= rmin && (r < z0 || r >= z1)) v = stream_load(reinterpret_cast<const V*>(p + k * RG * RS));
        b[k] = v;
      }
    }
    T xx[VEC];
    for (int j = 0; j < VEC; j += 2) {
      const d2v x2 = *reinterpret_cast<const d2v*>(xv + int64_t(row - d) * NB + col + j);
      xx[j] = T(x2[0]);
      xx[j + 1] = T(x2[1]);
    }
    // a new row's inputs (the old ones are dead once the row changes: the
    // flush reads only the row sums); FP32 takes them through FP64 registers
    constexpr bool XD = sizeof(T) == sizeof(double);
    double xn[XD ? 1 : KR];
    if (row != cur_row)
      for (int k = 0; k < KR; ++k) {
        const double v = xv[int64_t(row) * NB + rg + RG * k];
        if constexpr (XD) xi[k] = v;
        else xn[k] = v;
      }
    {
      const int64_t tn = min(t + 1, t1 - 1);
      inf_next = tinfo[tn];
      rws_next = trows[tn];
    }
    if (row != cur_row) {
      flush();
      pstart = t;
      cur_row = row;
      if constexpr (!XD)
        for (int k = 0; k < KR; ++k) xi[k] = T(xn[k]);
    }
    T c[VEC];
    for (int j = 0; j < VEC; ++j) c[j] = T(0);
    if (d > 0) {
      for (int k = 0; k < KR; ++k) {
        T s = b[k][0] * xx[0];
        for (int j = 1; j < VEC; ++j) s += b[k][j] * xx[j];
        racc[k] += s;
        for (int j = 0; j < VEC; ++j) c[j] += b[k][j] * xi[k];
      }
    } else {
      // diagonal tile: lower triangle (c <= r) in the row product, strict lower
      // triangle (c < r) in the column product
      for (int k = 0; k < KR; ++k) {
        const int r = rg + RG * k;
        T m[VEC];
        for (int j = 0; j < VEC; ++j) m[j] = col + j <= r ? b[k][j] : T(0);
        T s = m[0] * xx[0];
        for (int j = 1; j < VEC; ++j) s += m[j] * xx[j];
        racc[k] += s;
        for (int j = 0; j < VEC; ++j) c[j] += (col + j < r ? m[j] : T(0)) * xi[k];
      }
    }
    double o[VEC];
    for (int j = 0; j < VEC; ++j) o[j] = double(sum_rg(c[j]));
    if (jt < A.lds_cols) {
      const bool first = !((touched >> jt) & 1);
      touched |= uint64_t(1) << jt;
      if (rg == 0)
        for (int j = 0; j < VEC; ++j) s_col[jt][col + j] = first ? o[j] : s_col[jt][col + j] + o[j];
      if (first && lane == 0) s_first[w][jt] = int32_t(t);
    } else if (rg == 0) {
      for (int j = 0; j < VEC; j += 2) {
        d2v o2;
        o2[0] = o[j];
        o2[1] = o[j + 1];
        *reinterpret_cast<d2v*>(A.part + t * NB + col + j) = o2;
      }
    }
  }
  flush();
  flush_cols();
  if (w == 0)
    for (int q = 0; q < min(npieces, A.row_pieces); ++q) A.rowp[int64_t(s_pstart[q]) * NB + lane] = s_row[q][lane];
}

// Output row ii of a subdomain's symmetric matrix: the row product (over its
// pieces) plus the column products of tiles (i2, ii), i2 = ii .. TS-1; the
// four waves take every fourth term, the result is in s_red[0..3] (summed by
// the caller in that fixed order).
__device__ __forceinline__ void sum_row(const IfaceArgs& A, const MatDesc& D, int ii, int TS, double (*s_red)[NB]) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double y = 0.0;
  if (w == 0) y = sym_row_product(A.rowp, D.sg_off + tri_tile(ii, 0), ii + 1, A.ntiles, A.nwg, lane);
  const double* pp = A.part + D.sg_off * NB + lane;
  for (int i2 = ii + w; i2 < TS; i2 += 4)
    if (sym_col_first(D, i2, ii, A.ntiles, A.nwg, A.lds_cols)) y += pp[tri_tile(i2, ii) * NB];
  s_red[w][lane] = y;
}

// (S z) per local dof: sploc = D^{-1} y on the interface rows, y itself on the
// corners.
__global__ __launch_bounds__(256) void op_finish_kernel(IfaceArgs A) {
  __shared__ double s_red[4][NB];
  const int dn = A.sc->done;   // tested once the loads are in flight
  const int s = A.tasks[2 * blockIdx.x], ii = A.tasks[2 * blockIdx.x + 1];
  const MatDesc D = A.mats[s];
  const int TS = sym_tile_rows(D), nG = D.n_R - D.n_I, tid = threadIdx.x;
  const int r = ii * NB + tid;
  const double ds = tid < NB && r < nG ? A.dsc[D.loc_off + D.n_I + r] : 1.0;
  sum_row(A, D, ii, TS, s_red);
  if (dn) return;
  __syncthreads();
  if (tid >= NB) return;
  const double y = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
  if (r < nG) {
    A.sploc[D.loc_off + D.n_I + r] = y / ds;
  } else if (r - nG >= D.n_A && r - nG < D.n_ci) {
    A.sploc[D.loc_off + D.n_R + (r - nG - D.n_A)] = y;
  }
}

// Preconditioner output on the interface rows of tile row ii:
//   x = (X^T X f)_r + sum_c (W^T X)(c, r) coef_c,  ww = W D x,
// with the coefficients of the coarse correction from coarse_coef_kernel
// (which also writes the corner outputs).  (Products with the constraint rows
// vanish: their input is zero.)
__global__ __launch_bounds__(256) void pc_finish_kernel(IfaceArgs A) {
  __shared__ double cf[MAX_NCI];
  __shared__ double s_red[4][NB];
  const int dn = A.sc->done;   // tested once the loads are in flight
  const int s = A.tasks[2 * blockIdx.x], ii = A.tasks[2 * blockIdx.x + 1];
  const MatDesc D = A.mats[s];
  const int TS = sym_tile_rows(D), nG = D.n_R - D.n_I, tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  if (ii * NB >= nG) return;   // a tile row of constraint rows only: no output
  const int nci = D.n_ci;
  // the partial sums of the output row, the constraint rows M(n_G + c, r) for
  // c = w, w + 4, ... (M(n_G + c, r) lies in tile ((n_G + c) / 64, ii)), the
  // output weight and the coefficients, all loaded before the first barrier
  constexpr int CPW = MAX_NCI / 4;
  double mc[CPW];
  double wdr = 0.0;
  const int r_out = ii * NB + lane;
  sum_row(A, D, ii, TS, s_red);
  for (int q = 0; q < CPW; ++q) {
    const int c = w + 4 * q;
    double m = 0.0;
    if (c < nci) {
      const int R = nG + c;
      const int64_t t = (D.sg_off + tri_tile(R / NB, ii)) * int64_t(NB * NB);
      m = A.m32 ? double(static_cast<const float*>(A.m)[t + sym_f32_off(R % NB, lane)])
                : static_cast<const double*>(A.m)[t + (R % NB) * NB + lane];
    }
    mc[q] = m;
  }
  if (w == 0 && r_out < nG) wdr = A.wd[D.loc_off + D.n_I + r_out];
  if (tid < nci) cf[tid] = A.coef[int64_t(s) * MAX_NCI + tid];
  if (dn) return;
  __syncthreads();
  // constraint rows: wave w takes c = w, w+4, ...
  {
    double v = 0.0;
    for (int q = 0; q < CPW; ++q)
      if (w + 4 * q < nci) v += mc[q] * cf[w + 4 * q];
    s_red[w][lane] += v;
  }
  __syncthreads();
  if (tid >= NB) return;
  if (r_out < nG) {
    const double x = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
    A.ww[D.loc_off + D.n_I + r_out] = wdr * x;
  }
}

void launch_sym_mv(const IfaceArgs& a, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (a.ntiles <= 0 || a.nwg <= 0) return;
  if (a.m32) launch_timed(sym_mv_kernel<float>, dim3(a.nwg), dim3(256), st, t0, t1, a);
  else launch_timed(sym_mv_kernel<double>, dim3(a.nwg), dim3(256), st, t0, t1, a);
}

void launch_op_finish(const IfaceArgs& a, hipStream_t st) {
  if (a.ntasks <= 0) return;
  hipLaunchKernelGGL(op_finish_kernel, dim3(a.ntasks), dim3(256), 0, st, a);
}

void launch_pc_finish(const IfaceArgs& a, hipStream_t st) {
  if (a.ntasks <= 0) return;
  hipLaunchKernelGGL(pc_finish_kernel, dim3(a.ntasks), dim3(256), 0, st, a);
}
// ---------------------------------------------------------------------------
// Interface-form vector kernels over the interface dofs only: the interface
// iterate, residual and directions vanish on subdomain interiors.  Interface dof
// k has global index ifc_g[k] and IFC_MAXC copy slots (-1 past its last copy):
// local dof, slot in the operator's padded input, slot in the preconditioner's.
// ---------------------------------------------------------------------------
struct IfcCopies {
  int32_t l[IFC_MAXC];
};
__device__ __forceinline__ IfcCopies load_copies(const int32_t* a, int64_t k) {
  IfcCopies c;
  const int4* p = reinterpret_cast<const int4*>(a + k * IFC_MAXC);
  const int4 u = p[0], v = p[1];
  c.l[0] = u.x; c.l[1] = u.y; c.l[2] = u.z; c.l[3] = u.w;
  c.l[4] = v.x; c.l[5] = v.y; c.l[6] = v.z; c.l[7] = v.w;
  return c;
}

// per copy slot: equilibration and weighted equilibration of its local dof
__global__ void ifc_setup_kernel(const int32_t* ifc_l, const double* dsc, const double* wd, double* ifc_dsc,
                                 double* ifc_wd, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t l = ifc_l[i];
    ifc_dsc[i] = l >= 0 ? dsc[l] : 1.0;
    ifc_wd[i] = l >= 0 ? wd[l] : 0.0;
  }
}

// z = sum_i R_i^T W_i w_i on interface dofs, D^{-1} z into the operator's padded
// input, partial sums of r.z
__global__ __launch_bounds__(VBLK) void gather_z_ifc_kernel(IfcArgs A) {
  __shared__ double sh[VBLK / 64];
  // the end-of-solve word is tested once the thread's first loads are in flight
  const int dn = A.sc->done;
  const int64_t k0 = blockIdx.x * int64_t(VBLK) + threadIdx.x, ks = int64_t(gridDim.x) * VBLK;
  int g = 0;
  IfcCopies sz;
  double v = 0.0, rv = 0.0;
  auto load = [&](int64_t k) {
    g = A.g[k];
    const IfcCopies l = load_copies(A.l, k);
    sz = load_copies(A.slotz, k);
    v = 0.0;
    for (int c = 0; c < IFC_MAXC; ++c)
      if (l.l[c] >= 0) v += A.ww[l.l[c]];
    rv = A.r[g];
  };
  if (k0 < A.n) load(k0);
  if (dn) return;
  double rz = 0.0;
  for (int64_t k = k0; k < A.n; k += ks) {
    if (k != k0) load(k);
    A.z[g] = v;
    rz += rv * v;
    for (int c = 0; c < IFC_MAXC; ++c)
      if (sz.l[c] >= 0) A.zpad[sz.l[c]] = v / A.dsc[k * IFC_MAXC + c];
  }
  const double t = block_sum(rz, sh);
  if (threadIdx.x == 0) A.part_out[blockIdx.x] = t;
}

// q = S p = sum_i R_i^T (S_i z)_i + beta q, p = z + beta p on interface dofs (beta
// from the partial sums of r.z), partial sums of p.q
__global__ __launch_bounds__(VBLK) void gather_sp_ifc_kernel(IfcArgs A) {
  __shared__ double sh[VBLK / 64];
  PcgScalars* sc = A.sc;
  const int dn = sc->done;   // tested once the first loads are in flight
  // the data of an interface dof does not depend on beta: the loads of the
  // thread's first dof are issued before the reduction of the r.z partial sums
  const int64_t k0 = blockIdx.x * int64_t(VBLK) + threadIdx.x, ks = int64_t(gridDim.x) * VBLK;
  int g = 0;
  double v = 0.0, zv = 0.0, pv0 = 0.0, qv0 = 0.0;
  auto load = [&](int64_t k) {
    g = A.g[k];
    const IfcCopies l = load_copies(A.l, k);
    v = 0.0;
    for (int c = 0; c < IFC_MAXC; ++c)
      if (l.l[c] >= 0) v += A.sploc[l.l[c]];
    zv = A.z[g];
    if (!A.fresh) {
      pv0 = A.p[g];
      qv0 = A.q[g];
    }
  };
  if (k0 < A.n) load(k0);
  if (dn) return;
  const double rz = reduce_partials(A.part_in, gridDim.x, sh);
  const double beta = A.fresh ? 0.0 : rz / sc->rz[A.it - 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rz[A.it] = rz;
    if (!A.fresh) sc->beta[A.it - 1] = beta;
  }
  double pq = 0.0;
  for (int64_t k = k0; k < A.n; k += ks) {
    if (k != k0) load(k);
    const double pv = A.fresh ? zv : zv + beta * pv0;
    const double qv = A.fresh ? v : v + beta * qv0;
    A.p[g] = pv;
    A.q[g] = qv;
    pq += pv * qv;
  }
  const double t = block_sum(pq, sh);
  if (threadIdx.x == 0) A.part_out[blockIdx.x] = t;
}

// alpha = rz/pq; x += alpha p; r -= alpha q on interface dofs; W D r into the
// preconditioner's padded input; partial sums of r.r
__global__ __launch_bounds__(VBLK) void pcg_update_ifc_kernel(IfcArgs A) {
  __shared__ double sh[VBLK / 64];
  PcgScalars* sc = A.sc;
  const int dn = sc->done;   // tested once the first loads are in flight
  // the thread's first interface dof is loaded before the reduction of the p.q
  // partial sums (its data does not depend on alpha)
  const int64_t k0 = blockIdx.x * int64_t(VBLK) + threadIdx.x, ks = int64_t(gridDim.x) * VBLK;
  int g = 0;
  IfcCopies sf;
  double xv = 0.0, pv = 0.0, rv0 = 0.0, qv = 0.0, wd[IFC_MAXC];
  auto load = [&](int64_t k) {
    g = A.g[k];
    sf = load_copies(A.slotf, k);
    xv = A.x[g];
    pv = A.p[g];
    rv0 = A.r[g];
    qv = A.q[g];
    const d2v* wp = reinterpret_cast<const d2v*>(A.wd + k * IFC_MAXC);
    for (int c = 0; c < IFC_MAXC; c += 2) {
      const d2v w2 = wp[c / 2];
      wd[c] = w2[0];
      wd[c + 1] = w2[1];
    }
  };
  const double rz = sc->rz[A.it];
  if (k0 < A.n) load(k0);
  if (dn) return;
  const double pq = reduce_partials(A.part_in, gridDim.x, sh);
  const double alpha = rz / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->pq[A.it] = pq;
    sc->alpha[A.it] = alpha;
  }
  double rr = 0.0;
  if (pq > 0.0 && rz > 0.0) {
    for (int64_t k = k0; k < A.n; k += ks) {
      if (k != k0) load(k);
      A.x[g] = xv + alpha * pv;
      const double rv = rv0 - alpha * qv;
      A.r[g] = rv;
      rr += rv * rv;
      for (int c = 0; c < IFC_MAXC; ++c)
        if (sf.l[c] >= 0) A.fpad[sf.l[c]] = wd[c] * rv;
    }
  }
  const double t = block_sum(rr, sh);
  if (threadIdx.x == 0) A.part_out[blockIdx.x] = t;
}

// W D r into the preconditioner's padded input (start of a CG segment)
__global__ void scatter_f_ifc_kernel(IfcArgs A) {
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < A.n; k += int64_t(gridDim.x) * blockDim.x) {
    const double rv = A.r[A.g[k]];
    const IfcCopies sf = load_copies(A.slotf, k);
    for (int c = 0; c < IFC_MAXC; ++c)
      if (sf.l[c] >= 0) A.fpad[sf.l[c]] = A.wd[k * IFC_MAXC + c] * rv;
  }
}

void launch_ifc_setup(const int32_t* ifc_l, const double* dsc, const double* wd, double* ifc_dsc, double* ifc_wd,
                      int64_t n_ifc, hipStream_t st) {
  const int64_t n = n_ifc * IFC_MAXC;
  if (n <= 0) return;
  hipLaunchKernelGGL(ifc_setup_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, ifc_l, dsc, wd, ifc_dsc,
                     ifc_wd, n);
}
// The three kernels use the same grid, ifc_blocks(n): each reduces the partial
// sums of the previous one, one per block.
int ifc_blocks(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>(VGRID, (n + VBLK - 1) / VBLK))); }
void launch_gather_z_ifc(const IfcArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(gather_z_ifc_kernel, dim3(ifc_blocks(a.n)), dim3(VBLK), 0, st, a);
}
void launch_gather_sp_ifc(const IfcArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(gather_sp_ifc_kernel, dim3(ifc_blocks(a.n)), dim3(VBLK), 0, st, a);
}
void launch_pcg_update_ifc(const IfcArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(pcg_update_ifc_kernel, dim3(ifc_blocks(a.n)), dim3(VBLK), 0, st, a);
}
void launch_scatter_f_ifc(const IfcArgs& a, hipStream_t st) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(scatter_f_ifc_kernel, dim3(grid_for(a.n, 256, 4096)), dim3(256), 0, st, a);
}

// sentinel fill of the published buffers and zero tickets, one launch
template <typename T>
__global__ void reset_kernel(T* pub, int64_t n_pub, double* pubc, int64_t n_pubc, unsigned* tickets,
                             const int* done, const uint8_t* kappa, double* zero_iface, double* zero_all,
                             int64_t n) {
  if (done && *done) return;
  using U = typename Traits<T>::U;
  U* q = reinterpret_cast<U*>(pub);
  unsigned long long* qc = reinterpret_cast<unsigned long long*>(pubc);
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t i0 = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  for (int64_t i = i0; i < n_pub; i += stride) q[i] = Traits<T>::SENT;
  for (int64_t i = i0; i < n_pubc; i += stride) qc[i] = Traits<double>::SENT;
  if (i0 < 8) tickets[i0] = 0u;
  for (int64_t i = i0; i < n; i += stride) {
    if (zero_all) zero_all[i] = 0.0;
    if (zero_iface && kappa[i] > 1) zero_iface[i] = 0.0;
  }
}

void launch_reset(bool fp32, void* pub, int64_t n_pub, double* pubc, int64_t n_pubc, unsigned* tickets,
                  const int* done, hipStream_t st, const uint8_t* kappa, double* zero_iface, double* zero_all,
                  int64_t n) {
  int64_t m = n_pub > n_pubc ? n_pub : n_pubc;
  if (n > m) m = n;
  const int g = grid_for(m, 256, 2048);
  if (fp32)
    hipLaunchKernelGGL(reset_kernel<float>, dim3(g), dim3(256), 0, st, (float*)pub, n_pub, pubc, n_pubc, tickets,
                       done, kappa, zero_iface, zero_all, n);
  else
    hipLaunchKernelGGL(reset_kernel<double>, dim3(g), dim3(256), 0, st, (double*)pub, n_pub, pubc, n_pubc, tickets,
                       done, kappa, zero_iface, zero_all, n);
}






// ---------------------------------------------------------------------------
// Per-element gradient g_e = -lam_e^T K_ref u_e
// ---------------------------------------------------------------------------
__global__ void elem_grad_kernel(MeshDev M, const double* lam, const double* u, double* g, int64_t nel) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < nel; e += int64_t(gridDim.x) * blockDim.x) {
    int ec[3];
    int64_t r = e;
    ec[0] = int(r % M.nel[0]);
    r /= M.nel[0];
    if (M.dim == 3) {
      ec[1] = int(r % M.nel[1]);
      ec[2] = int(r / M.nel[1]);
    } else {
      ec[1] = int(r);
      ec[2] = 0;
    }
    const int nn = 1 << M.dim;
    double lv[8], uv[8];
    for (int a = 0; a < nn; ++a) {
      int c[3] = {ec[0] + (a & 1), ec[1] + ((a >> 1) & 1), M.dim == 3 ? ec[2] + ((a >> 2) & 1) : 0};
      int64_t q = free_of(M, c);
      lv[a] = q >= 0 ? lam[q] : 0.0;
      uv[a] = q >= 0 ? u[q] : 0.0;
    }
    double s = 0.0;
    for (int a = 0; a < nn; ++a) {
      double t = 0.0;
      for (int b = 0; b < nn; ++b) t += kref(M, a, b) * uv[b];
      s += lv[a] * t;
    }
    g[e] = -s;
  }
}

void launch_elem_grad(const MeshDevHost& mh, const double* lam, const double* u, double* g, int64_t nel,
                      hipStream_t st) {
  MeshDev M{mh.dim, {mh.nel[0], mh.nel[1], mh.nel[2]}, {mh.h[0], mh.h[1], mh.h[2]}};
  hipLaunchKernelGGL(elem_grad_kernel, dim3(grid_for(nel)), dim3(256), 0, st, M, lam, u, g, nel);
}

// Fixed device workspace of the allocation-free apply (bddc_apply_noalloc):
// the published-solution buffers, coarse solution buffers and ticket counters
// of one preconditioner application.  Every GPU the library runs on holds its
// own copy for the life of the process.  In host code `scratch` names a
// host-side stand-in, never the device memory: kernels get the per-device
// address that static_scratch_address obtains from the runtime.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

int static_scratch_address(void** ptr) {
  static std::mutex mtx;
  static std::map<int, void*> by_device;
  *ptr = nullptr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  std::lock_guard<std::mutex> lock(mtx);
  auto it = by_device.find(dev);
  if (it != by_device.end()) {
    *ptr = it->second;
    return 0;
  }
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
  by_device[dev] = p;
  *ptr = p;
  return 0;
}

}  // namespace bddc
