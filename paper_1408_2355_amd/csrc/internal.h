// Internal types of libsegpart (not part of the C ABI).
#pragma once

#include <array>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "segpart.h"

namespace sp {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SP_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::sp::Error(SP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define SP_REQUIRE(cond, code, msg) \
  do {                              \
    if (!(cond)) throw ::sp::Error((code), (msg)); \
  } while (0)

// Device allocation: owned (alloc, freed on release) or a view of memory
// someone else owns (adopt, never freed here).
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  bool owned = true;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), owned(o.owned) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; owned = o.owned; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    owned = true;
    if (count == 0) return;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error(SP_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    n = count;
  }
  void adopt(T* ptr, size_t count) {
    release();
    p = count ? ptr : nullptr;
    n = count;
    owned = false;
  }
  void release() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// Device memory handed out in order from one region owned elsewhere (no
// allocation): pieces 256-byte aligned; take() throws SP_ENOMEM once the
// region is exhausted.
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
  const char* what = "arena";
  template <class T>
  T* take(size_t count) {
    const size_t at = (used + 255) & ~size_t(255);
    const size_t bytes = count * sizeof(T);
    if (at > size || bytes > size - at)
      throw Error(SP_ENOMEM, std::string(what) + ": the batch needs more than its " +
                                 std::to_string(size >> 20) + " MiB (" +
                                 std::to_string((at + bytes) >> 20) + " MiB so far)");
    used = at + bytes;
    return reinterpret_cast<T*>(base + at);
  }
};

// The allocation-free entry point's work area on the current device: a
// file-scope device array of kScratchBytes (noalloc.hip), located once per
// device with hipGetSymbolAddress.  Calls on one device share it.
constexpr size_t kScratchBytes = size_t(128) << 20;
Arena noalloc_scratch();

// Row x column tiling of an [n][rp] column-interleaved array for the
// row-parallel kernels.  A thread owns 4 consecutive columns of one row; a
// 256-thread workgroup covers tr rows x tg column groups per pass.  The rows
// are split into 8 contiguous ranges (one per XCD) of xrows rows; within a
// range, chunks of ch rows go to the range's nper workgroups cyclically.
// Every workgroup walks all nct column tiles and writes one partial sum per
// column, so partial arrays have nchunk = nblk rows.
struct Tile {
  int n = 0;       // rows
  int rp = 0;      // padded columns (multiple of 4)
  int G = 0;       // column groups (rp / 4)
  int tg = 1;      // column groups per tile (power of two, <= 64)
  int tr = 256;    // rows per pass (256 / tg)
  int nct = 1;     // column tiles
  int xrows = 0;   // rows per XCD range (ceil(n / 8))
  int ch = 256;    // rows per chunk (multiple of tr)
  int nchx = 1;    // chunks per XCD range
  int nper = 1;    // workgroups per XCD range
  int nblk = 8;    // workgroups (8 * nper)
  int nchunk = 8;  // rows of the partial-sum arrays (= nblk)
};
constexpr int kMaxPer = 256;  // workgroups per XCD range at most (partials sized for 8 x this)
// tg_cap: lanes-per-row cap (1..64, rounded to a power of two); passes: row
// passes per chunk; nper_cap: workgroups per XCD range.
Tile make_tile(int n, int rp, int tg_cap = 64, int passes = 1, int nper_cap = kMaxPer);

// Per-time-step matrices for one tau: K = M + tau A in float64 and float32,
// the inverse diagonals used by the Jacobi preconditioner and, once a solver
// asks for it, the polynomial preconditioner P = D^-1 (c0 I + c1 K D^-1) on
// K's pattern (precond.cpp).
struct TauMats {
  double tau = 0;
  DevBuf<double> K64, dinv64;
  DevBuf<float> K32, dinv32;
  double pc0 = 0, pc1 = 0;
  DevBuf<double> P64;
  DevBuf<float> P32;
};

struct Mesh {
  int64_t n = 0, nt = 0, nnz = 0;
  int W = 0;           // ELL width (max row length); slot 0 holds the diagonal
  double area = 0;
  std::vector<int32_t> perm;   // perm[new] = caller index
  std::vector<int32_t> iperm;  // iperm[caller] = new
  std::vector<int32_t> h_cols; // [W][n] host copy of the pattern (new numbering)
  DevBuf<int32_t> cols;        // [W][n]; padding slots repeat the row index, value 0
  DevBuf<double> M64, A64;     // [W][n]
  DevBuf<int32_t> tri;         // [nt][3] (new numbering, sorted for locality)
  DevBuf<double> tarea;        // [nt]
  DevBuf<int32_t> perm_d, iperm_d;
  std::vector<double> h_xyz;   // [n][3] caller numbering (refinement)
  std::vector<int32_t> h_tri;  // [nt][3] caller numbering
  // made by refinement: new vertex n_coarse + j is the midpoint of edge
  // (parents[2j], parents[2j+1]) of the coarse mesh (caller numbering)
  int64_t n_coarse = 0;
  std::vector<int32_t> parents;
  DevBuf<int32_t> parents_d;
  int device = 0;
  std::mutex mu;
  std::vector<std::unique_ptr<TauMats>> kcache;
  // with_precond: P64/P32 built too (once per tau)
  TauMats* tau_mats(double tau, bool with_precond = false);
  // coefficients of the CG's degree-1 Chebyshev preconditioner for
  // K = M + tau A (precond.cpp); host work, cached per tau
  void cheb_coefs(double tau, double* c0, double* c1);
  std::mutex pmu;
  std::vector<std::array<double, 3>> pcache;  // (tau, c0, c1)
};

Mesh* mesh_create(int64_t n, const double* xyz, int64_t nt, const int32_t* tri);
// 4-fold midpoint refinement (continuation.cpp); project (nullable) moves the
// new vertices onto the surface.
typedef void (*ProjectFn)(double* xyz, int64_t n, void* ctx);
Mesh* mesh_refine(const Mesh& coarse, ProjectFn project, void* ctx);

// Kernel launchers (kernels.hip).
struct ColTables;  // forward
namespace k {
void assemble(const Mesh& m, const double* xyz_new, const int32_t* inc_ptr, const int32_t* inc,
              hipStream_t s);
void tau_mats(const Mesh& m, TauMats& t, hipStream_t s);
// t.P64 / t.P32 from t.K64, t.dinv64 and t.pc0 / t.pc1
void precond_mats(const Mesh& m, TauMats& t, hipStream_t s);
void fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s);
void fill_f64(double* p, double v, size_t n, hipStream_t s);
void fill_f32(float* p, float v, size_t n, hipStream_t s);
// u_fine [cols][fine.n] from u_coarse [cols][fine.n_coarse] (prolong.hip)
void prolong(const Mesh& fine, int cols, const double* u_coarse, double* u_fine, hipStream_t s);
}  // namespace k

}  // namespace sp
