// HIP kernels of the segregation time step for CDNA4 (gfx950).
//
// Vector layout: [n][rp], the rp column values of one vertex contiguous, so a
// 64-lane wavefront reading one row reads one long contiguous run.  Matrices
// are ELL, slot-major ([W][n]), slot 0 = diagonal.  The work is bound by HBM
// bandwidth: no MFMA (there is no dense contraction on this path).
//
// Row-parallel kernels use the Tile mapping of internal.h: each thread owns 4
// consecutive columns of a row; per-column dot products are reduced inside
// the workgroup (fixed tree order) and written as one partial per row chunk;
// small column-parallel kernels add the chunk partials in chunk order.  All
// reductions are float64 and deterministic for a fixed tiling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "kernels.h"

namespace sp {

namespace {

constexpr int kBlock = 256;

template <typename T>
struct V4 {
  T v[4];
};

__device__ __forceinline__ V4<double> ld4(const double* p) {
  const double2* q = reinterpret_cast<const double2*>(p);
  double2 a = q[0], b = q[1];
  return {{a.x, a.y, b.x, b.y}};
}
__device__ __forceinline__ V4<float> ld4(const float* p) {
  float4 a = *reinterpret_cast<const float4*>(p);
  return {{a.x, a.y, a.z, a.w}};
}
__device__ __forceinline__ void st4(double* p, const V4<double>& x) {
  double2* q = reinterpret_cast<double2*>(p);
  q[0] = make_double2(x.v[0], x.v[1]);
  q[1] = make_double2(x.v[2], x.v[3]);
}
__device__ __forceinline__ void st4(float* p, const V4<float>& x) {
  *reinterpret_cast<float4*>(p) = make_float4(x.v[0], x.v[1], x.v[2], x.v[3]);
}
// Nontemporal (nt) forms, for data touched once per launch: every operand
// of the streaming kernels, the output of the gathering kernels and their
// row's own operands.  They do not displace the gathered operand's rows
// from L2, where the reuse between neighbouring rows happens (the matrix
// product runs about 15% faster with them, the time step about 8%).
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st4_nt(float* p, const V4<float>& x) {
  f4v v = {x.v[0], x.v[1], x.v[2], x.v[3]};
  __builtin_nontemporal_store(v, reinterpret_cast<f4v*>(p));
}
__device__ __forceinline__ void st4_nt(double* p, const V4<double>& x) {
  d2v a = {x.v[0], x.v[1]}, b = {x.v[2], x.v[3]};
  __builtin_nontemporal_store(a, reinterpret_cast<d2v*>(p));
  __builtin_nontemporal_store(b, reinterpret_cast<d2v*>(p) + 1);
}
__device__ __forceinline__ V4<float> ld4_nt(const float* p) {
  f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
  return {{v.x, v.y, v.z, v.w}};
}
__device__ __forceinline__ V4<double> ld4_nt(const double* p) {
  d2v a = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
  d2v b = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p) + 1);
  return {{a.x, a.y, b.x, b.y}};
}
// bfloat16 storage (the inner float32 CG's directions and preconditioner
// output): the upper 16 bits of the float32, rounded to nearest even; 4
// values in 8 bytes, widened to float32 on load.
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;  // NaN stays a NaN
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ V4<float> bf16_unpack(uint32_t lo, uint32_t hi) {
  return {{__uint_as_float(lo << 16), __uint_as_float(lo & 0xffff0000u),
           __uint_as_float(hi << 16), __uint_as_float(hi & 0xffff0000u)}};
}
typedef uint32_t u2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ V4<float> ld4(const bf16_t* p) {
  const u2v w = *reinterpret_cast<const u2v*>(p);
  return bf16_unpack(w.x, w.y);
}
__device__ __forceinline__ V4<float> ld4_nt(const bf16_t* p) {
  const u2v w = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(p));
  return bf16_unpack(w.x, w.y);
}
__device__ __forceinline__ void st4_nt(bf16_t* p, const V4<float>& x) {
  u2v w = {bf16_bits(x.v[0]) | (bf16_bits(x.v[1]) << 16),
           bf16_bits(x.v[2]) | (bf16_bits(x.v[3]) << 16)};
  __builtin_nontemporal_store(w, reinterpret_cast<u2v*>(p));
}
// Split float32 storage (the inner float32 CG's residual r under the
// polynomial preconditioner), in the bytes of an n x rp float32 array: plane 0
// (its first n*rp 16-bit words, laid out [n][rp]) holds each value rounded to
// bfloat16 (nearest, ties away from zero: bits + 0x8000, upper half), plane 1
// (the next n*rp words) the difference of the bit patterns, which lies in
// [-0x8000, 0x7fff] and is kept as a signed 16-bit word, so
// bits = (plane 0 << 16) + plane 1 restores the float32 exactly.  The
// residual recursion reads and writes both planes (the bytes of float32); the
// preconditioner pass gathers the neighbours' values from plane 0 alone, a
// bf16 array half the size of the float32 one, and takes the row's own value
// exactly.  (Measured in the time step: the gather from the separate plane is
// about 10% faster; interleaving the two halves inside a row, in blocks of
// 64 to 256 columns or as half rows, left it as slow as the float32 gather.)
__device__ __forceinline__ uint32_t split_join(uint32_t hi, uint32_t lo) {
  return (hi << 16) + uint32_t(int32_t(int16_t(uint16_t(lo & 0xffffu))));
}
__device__ __forceinline__ V4<float> split_join4(const V4<float>& hi, u2v lo) {
  return {{__uint_as_float(split_join(__float_as_uint(hi.v[0]) >> 16, lo.x)),
           __uint_as_float(split_join(__float_as_uint(hi.v[1]) >> 16, lo.x >> 16)),
           __uint_as_float(split_join(__float_as_uint(hi.v[2]) >> 16, lo.y)),
           __uint_as_float(split_join(__float_as_uint(hi.v[3]) >> 16, lo.y >> 16))}};
}
// plane 1 words at element offset o (plane = n*rp)
__device__ __forceinline__ u2v ld_plane1(const float* r, size_t plane, size_t o) {
  const uint16_t* b = reinterpret_cast<const uint16_t*>(r) + plane + o;
  return __builtin_nontemporal_load(reinterpret_cast<const u2v*>(b));
}
__device__ __forceinline__ V4<float> ld4_split(const float* r, size_t plane, size_t o) {
  return split_join4(ld4_nt(reinterpret_cast<const bf16_t*>(r) + o), ld_plane1(r, plane, o));
}
__device__ __forceinline__ void st4_split(float* r, size_t plane, size_t o, const V4<float>& x) {
  uint32_t h[4], l[4];
  for (int j = 0; j < 4; ++j) {
    const uint32_t u = __float_as_uint(x.v[j]);
    h[j] = (u + 0x8000u) >> 16;
    l[j] = (u - (h[j] << 16)) & 0xffffu;
  }
  uint16_t* b = reinterpret_cast<uint16_t*>(r);
  const u2v wh = {h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
  const u2v wl = {l[0] | (l[1] << 16), l[2] | (l[3] << 16)};
  __builtin_nontemporal_store(wh, reinterpret_cast<u2v*>(b + o));
  __builtin_nontemporal_store(wl, reinterpret_cast<u2v*>(b + plane + o));
}
// Values as they come back from storage type S (bf16: float32).
template <typename S>
using V4of = decltype(ld4(static_cast<const S*>(nullptr)));

template <typename S>
__device__ __forceinline__ V4of<S> ld4g(const S* p) { return ld4_nt(p); }  // own row, gathering kernel
template <typename S, typename V>
__device__ __forceinline__ void st4g(S* p, const V& x) { st4_nt(p, x); }  // gathering kernel
template <typename S>
__device__ __forceinline__ V4of<S> ld4s(const S* p) { return ld4_nt(p); }  // streaming kernel
template <typename S, typename V>
__device__ __forceinline__ void st4s(S* p, const V& x) { st4_nt(p, x); }  // streaming kernel

// Row traversal of the row-parallel kernels.  Workgroups are handed to the
// 8 XCDs round-robin by id, so workgroup b runs on XCD b % 8.  The rows are
// split into 8 contiguous ranges, one per XCD; inside its range an XCD's
// workgroups take chunks of ch rows cyclically (chunk j -> workgroup j mod
// nper), so at any moment they work on one compact window of rows and the
// neighbour rows they gather stay in that XCD's L2.  Each workgroup walks
// every column tile in turn (the caller's loop over ct).
template <typename F>
__device__ __forceinline__ void for_rows(const Tile& t, F&& f) {
  const int xcd = blockIdx.x & 7, kb = blockIdx.x >> 3;
  const int rbeg = xcd * t.xrows, rend = min(rbeg + t.xrows, t.n);
  if (t.tg == 64) {
    // one row per wavefront: the row index is wave-uniform, so the row's
    // matrix indices and values come through scalar loads and the vector
    // memory pipe carries only the 16-byte column gathers
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int j = kb; j < t.nchx; j += t.nper) {
      const int r1 = min(rbeg + (j + 1) * t.ch, rend);
      for (int row = rbeg + j * t.ch + wv; row < r1; row += kBlock / 64) f(row);
    }
    return;
  }
  const int rl = threadIdx.x / t.tg;
  for (int j = kb; j < t.nchx; j += t.nper) {
    const int r1 = min(rbeg + (j + 1) * t.ch, rend);
    for (int row = rbeg + j * t.ch + rl; row < r1; row += t.tr) f(row);
  }
}

__device__ __forceinline__ size_t part_off(const Tile& t, int d) {
  return size_t(d) * size_t(t.nchunk) * size_t(t.rp);
}

// Reduce ND x 4 per-thread sums over the tr rows of the workgroup (tree,
// fixed order) and store them as the chunk's partials.
template <int ND>
__device__ void block_store(const Tile& t, double (&s)[ND][4], double* part, int chunk, int ct) {
  __shared__ double red[kBlock * 4];
  const int tid = threadIdx.x, rl = tid / t.tg, gl = tid % t.tg;
  const int g = ct * t.tg + gl;
  for (int d = 0; d < ND; ++d) {
    for (int j = 0; j < 4; ++j) red[tid * 4 + j] = s[d][j];
    for (int st = t.tr >> 1; st >= 1; st >>= 1) {
      __syncthreads();
      if (rl < st)
        for (int j = 0; j < 4; ++j) red[tid * 4 + j] += red[(tid + st * t.tg) * 4 + j];
    }
    __syncthreads();
    if (rl == 0 && g < t.G)
      for (int j = 0; j < 4; ++j)
        part[part_off(t, d) + size_t(chunk) * t.rp + 4 * g + j] = red[tid * 4 + j];
    __syncthreads();
  }
}

// Column reductions over the chunk partials: a workgroup serves kRC columns
// with kRL lanes each; lane l adds chunks l, l + kRL, ... and lane 0 adds
// the lane sums in order (fixed order, so results are reproducible).  Every
// thread of the block must call red_sum; the total is valid in lane 0.
// (32 lanes: the streaming kernels write up to 2048 partial rows, and each
// lane's chain of dependent loads sets the reduction's latency)
constexpr int kRL = 32;
constexpr int kRC = kBlock / kRL;

__device__ __forceinline__ int red_col() { return blockIdx.x * kRC + threadIdx.x % kRC; }
__device__ __forceinline__ bool red_lead() { return threadIdx.x < kRC; }

__device__ __forceinline__ double red_sum(const double* p, int nchunk, int rp, int c) {
  __shared__ double sh[kBlock];
  const int lane = threadIdx.x / kRC, cl = threadIdx.x % kRC;
  // 8 independent accumulators (chunk lane + 8 kRL j + i kRL goes to s[i]),
  // combined in fixed order: the loads of 8 chunks are in flight together
  double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (c < rp) {
    int ch = lane;
    for (; ch + 7 * kRL < nchunk; ch += 8 * kRL) {
#pragma unroll
      for (int i = 0; i < 8; ++i) s8[i] += p[size_t(ch + i * kRL) * rp + c];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (ch + i * kRL < nchunk) s8[i] += p[size_t(ch + i * kRL) * rp + c];
  }
  const double s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
  sh[threadIdx.x] = s;
  __syncthreads();
  double tot = 0.0;
  if (lane == 0)
    for (int l = 0; l < kRL; ++l) tot += sh[l * kRC + cl];
  __syncthreads();
  return tot;
}

// x * s rounded on its own, never fused with a following add: a column factor
// applied as a value is read (deferred normalisation) then gives bit for bit
// the value a scaled copy of the state holds (k_scale), whichever route a step
// takes.
__device__ __forceinline__ double mul_alone(double x, double s) {
#pragma clang fp contract(off)
  return x * s;
}

// Count the columns for which flag is set, into *counter (one atomic per wave).
__device__ __forceinline__ void count_active(int flag, int* counter) {
  unsigned long long bal = __ballot(flag);
  if ((threadIdx.x & 63) == 0 && bal) atomicAdd(counter, __popcll(bal));
}

// ELL row product helper.  The ELL width W is a multiple of kSlots (the mesh
// pads it; padding slots point at the row itself with value 0), so slots are
// walked in groups of kSlots with straight-line code: all indices of a group
// are loaded, then all neighbour vectors are requested, then used, so a
// thread keeps kSlots gathers in flight.  The last slot of a group, when it
// is padding (index = row), requests nothing and hands f zeros: on a
// triangle mesh of valence 6 every row has 7 entries, so one gather in 8 is
// saved, and the gathers are what bounds the product.  (Only the last slot
// is tested, after all indices of the group are loaded, so the other loads
// of the group stay in flight together.)  f(k, x_k, o) gets the slot, the
// neighbour's 4 column values and the matrix offset o = k*n + row.
constexpr int kSlots = 8;

// Load of matrix data (pattern and values), which no kernel of the time step
// writes: read through the constant address space, so a wave-uniform address
// becomes a scalar load.
template <typename T>
__device__ __forceinline__ T ldm(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}

template <typename S, typename F>
__device__ __forceinline__ void for_neighbors(const StepArgs& a, int row, int c0,
                                              const S* __restrict__ x, F&& f) {
  const int n = a.t.n, rp = a.t.rp;
  for (int kb = 0; kb < a.W; kb += kSlots) {
    int idx[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) idx[k] = ldm(a.cols + size_t(kb + k) * n + row);
    V4of<S> xv[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots - 1; ++k) xv[k] = ld4(x + size_t(idx[k]) * rp + c0);
    constexpr int kl = kSlots - 1;
    xv[kl] = idx[kl] != row ? ld4(x + size_t(idx[kl]) * rp + c0) : V4of<S>{};
#pragma unroll
    for (int k = 0; k < kSlots; ++k) f(kb + k, xv[k], size_t(kb + k) * n + row);
  }
}

// --------------------------------------------------------------- assembly --
// One thread per row.  P1 element matrices on a flat triangle with corners
// x0, x1, x2 and edges e_a opposite corner a (e0 = x2 - x1, e1 = x0 - x2,
// e2 = x1 - x0):
//   mass       |T|/12 (1 + delta_ab)
//   stiffness  (e_a . e_b) / (4 |T|)     (the gradient of corner a's hat
//              function is the in-plane rotation of e_a over 2|T|)
// Contributions are added in the fixed incident-triangle order of the row.
__global__ __launch_bounds__(kBlock) void k_assemble(int n, int W, const int* __restrict__ cols,
                                                     const double* __restrict__ xyz,
                                                     const int* __restrict__ tri,
                                                     const int* __restrict__ inc_ptr,
                                                     const int* __restrict__ inc,
                                                     double* __restrict__ M, double* __restrict__ A,
                                                     double* __restrict__ tarea) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < W; ++k) {
    M[size_t(k) * n + i] = 0.0;
    A[size_t(k) * n + i] = 0.0;
  }
  for (int e = inc_ptr[i]; e < inc_ptr[i + 1]; ++e) {
    const int code = inc[e], t = code / 3, a = code % 3;
    int v[3];
    double x[3][3];
    for (int c = 0; c < 3; ++c) {
      v[c] = tri[3 * t + c];
      for (int d = 0; d < 3; ++d) x[c][d] = xyz[3 * size_t(v[c]) + d];
    }
    double ed[3][3];
    for (int d = 0; d < 3; ++d) {
      ed[0][d] = x[2][d] - x[1][d];
      ed[1][d] = x[0][d] - x[2][d];
      ed[2][d] = x[1][d] - x[0][d];
    }
    // (x1 - x0) x (x2 - x0) = e2 x (-e1)
    double cx = -(ed[2][1] * ed[1][2] - ed[2][2] * ed[1][1]);
    double cy = -(ed[2][2] * ed[1][0] - ed[2][0] * ed[1][2]);
    double cz = -(ed[2][0] * ed[1][1] - ed[2][1] * ed[1][0]);
    double area = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    if (a == 0) tarea[t] = area;
    for (int b = 0; b < 3; ++b) {
      int slot = 0;
      for (int k = 0; k < W; ++k)
        if (cols[size_t(k) * n + i] == v[b]) { slot = k; break; }
      double dot = ed[a][0] * ed[b][0] + ed[a][1] * ed[b][1] + ed[a][2] * ed[b][2];
      M[size_t(slot) * n + i] += area * (a == b ? 2.0 : 1.0) / 12.0;
      A[size_t(slot) * n + i] += dot / (4.0 * area);
    }
  }
}

__global__ void k_tau_mats(size_t total, int n, double tau, const double* __restrict__ M,
                           const double* __restrict__ A, double* __restrict__ K64,
                           float* __restrict__ K32, double* __restrict__ dinv64,
                           float* __restrict__ dinv32) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  double k = M[i] + tau * A[i];
  K64[i] = k;
  K32[i] = float(k);
  if (i < size_t(n)) {
    double d = 1.0 / k;
    dinv64[i] = d;
    dinv32[i] = float(d);
  }
}

// P = D^-1 (c0 I + c1 K D^-1) on K's pattern: slot 0 (the diagonal)
// d_i (c0 + c1 K_ii d_i), off-diagonal slots c1 d_i K_ij d_j (padding: 0).
__global__ void k_precond_mats(size_t total, int n, double c0, double c1,
                               const int* __restrict__ cols, const double* __restrict__ K,
                               const double* __restrict__ dinv, double* __restrict__ P64,
                               float* __restrict__ P32) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int row = int(i % size_t(n));
  const double di = dinv[row], dj = dinv[cols[i]];
  const double v = i < size_t(n) ? di * (c0 + c1 * K[i] * dj) : c1 * di * K[i] * dj;
  P64[i] = v;
  P32[i] = float(v);
}

// Marks a solve that ended with columns still active (iteration cap hit).
__global__ void k_flag_nonconv(const int* counter, long long* stat) {
  if (threadIdx.x == 0 && *counter != 0) stat[2] = 1;
}

template <typename T>
__global__ void k_fill(T* p, T v, size_t n) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------- float64 CG --
// r0 = b - K u = M u - (M + tau A) u = -tau A u (no cancellation), z0 = D r0,
// p0 = z0; partials ||M u||^2, r.z, r.r.
__global__ __launch_bounds__(kBlock) void k_init_fp64(StepArgs a, const double* __restrict__ u,
                                                      double* __restrict__ r,
                                                      double* __restrict__ p) {
  const Tile& t = a.t64;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  double s[3][4] = {};
  if (g < t.G) {
    const int c0 = 4 * g;
    double lv0[4];
    for (int j = 0; j < 4; ++j) lv0[j] = a.ct.live[c0 + j] ? 1.0 : 0.0;
    for_rows(t, [&](int row) {
      double au[4] = {}, mu[4] = {};
      for_neighbors(a, row, c0, u, [&](int, const V4<double>& x, size_t o) {
        const double va = ldm(a.A64 + o), vm = ldm(a.M64 + o);
        for (int j = 0; j < 4; ++j) {
          au[j] = fma(va, x.v[j], au[j]);
          mu[j] = fma(vm, x.v[j], mu[j]);
        }
      });
      const double di = a.dinv64[row];
      double lv[4] = {lv0[0], lv0[1], lv0[2], lv0[3]};
      if (a.mask)  // restricted solve: b and r0 live on the column's region
        for (int j = 0; j < 4; ++j) lv[j] *= double(a.mask[size_t(row) * t.rp + c0 + j]);
      V4<double> rv, pv;
      for (int j = 0; j < 4; ++j) {
        rv.v[j] = -a.tau * au[j] * lv[j];
        pv.v[j] = di * rv.v[j];
        s[0][j] += mu[j] * mu[j] * lv[j];
        s[1][j] += rv.v[j] * pv.v[j];
        s[2][j] += rv.v[j] * rv.v[j];
      }
      st4g(r + size_t(row) * t.rp + c0, rv);
      if (p) st4g(p + size_t(row) * t.rp + c0, pv);
    });
  }
  block_store<3>(t, s, a.part, blockIdx.x, ct);
  }
}

__global__ void k_red_init_fp64(StepArgs a) {
  const int c = red_col();
  const Tile& t = a.t64;
  const double bb = red_sum(a.part + part_off(t, 0), t.nchunk, t.rp, c);
  const double rz = red_sum(a.part + part_off(t, 1), t.nchunk, t.rp, c);
  const double rr = red_sum(a.part + part_off(t, 2), t.nchunk, t.rp, c);
  int act = 0;
  if (red_lead() && c < a.t64.rp) {
    a.cg.bb[c] = bb;
    a.cg.rz[c] = rz;
    a.cg.tol2[c] = a.rtol2 * bb;
    act = (a.ct.live[c] && rr > a.rtol2 * bb) ? 1 : 0;
    a.cg.act[c] = act;
    a.cg.alpha[c] = 0.0;
    a.cg.beta[c] = 0.0;
  }
  count_active(act, a.ring + 0);
}

// q = K p, partial p.q (per column).  p stored as S (float32 CG: bf16).
template <typename T, typename S = T>
__global__ __launch_bounds__(kBlock) void k_cg_spmm(StepArgs a, int slot, const T* __restrict__ K,
                                                    const S* __restrict__ p, T* __restrict__ q) {
  if (a.ring[slot] == 0) return;
  const Tile& t = a.tm;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  double s[1][4] = {};
  if (g < t.G) {
    const int c0 = 4 * g;
    const int any = a.cg.act[c0] | a.cg.act[c0 + 1] | a.cg.act[c0 + 2] | a.cg.act[c0 + 3];
    if (any) {
      for_rows(t, [&](int row) {
        V4<T> acc = {}, pd = {};
        for_neighbors(a, row, c0, p, [&](int k, const V4<T>& x, size_t o) {
          const T v = ldm(K + o);
          if (k == 0) pd = x;
          for (int j = 0; j < 4; ++j) acc.v[j] = fma(v, x.v[j], acc.v[j]);
        });
        if constexpr (sizeof(T) == 8) {
          if (a.mask)  // restricted solve: the product keeps the region's rows
            for (int j = 0; j < 4; ++j)
              if (!a.mask[size_t(row) * t.rp + c0 + j]) acc.v[j] = 0.0;
        }
        st4g(q + size_t(row) * t.rp + c0, acc);
        for (int j = 0; j < 4; ++j) s[0][j] += double(pd.v[j]) * double(acc.v[j]);
      });
    }
  }
  block_store<1>(t, s, a.part, blockIdx.x, ct);
  }
}

// alpha = r.z / p.q per active column; ah (nullable) also receives it (the
// direction ring's coefficient row of this iteration, zero when the
// iteration does no work).
__global__ void k_red_alpha(StepArgs a, int slot, int next, double* __restrict__ ah) {
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ring[next] = 0;
  if (a.ring[slot] == 0) {
    const int c = red_col();
    if (ah && red_lead() && c < a.tm.rp) ah[c] = 0.0;
    return;
  }
  // columns this iteration works on, summed over iterations (traffic model)
  if (blockIdx.x == 0 && threadIdx.x == 0) a.stat[3] += a.ring[slot];
  const int c = red_col();
  const bool act = c < a.tm.rp && a.cg.act[c];
  const double pq = red_sum(a.part, act ? a.tm.nchunk : 0, a.tm.rp, c);
  if (!red_lead() || c >= a.tm.rp) return;
  double al = 0.0;
  if (act && pq > 0.0) al = a.cg.rz[c] / pq;
  a.cg.alpha[c] = al;
  if (ah) ah[c] = al;
}

// x += alpha p, r -= alpha q, z = D r; partials r.z and r.r (Poly: r.r only,
// the preconditioner's pass forms z and r.z).
template <typename T, bool Poly>
__global__ __launch_bounds__(kBlock) void k_cg_update(StepArgs a, int slot, T* __restrict__ x,
                                                      T* __restrict__ r, const T* __restrict__ p,
                                                      const T* __restrict__ q,
                                                      const T* __restrict__ dinv) {
  if (a.ring[slot] == 0) return;
  const Tile& t = a.t;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  double s[Poly ? 1 : 2][4] = {};
  if (g < t.G) {
    const int c0 = 4 * g;
    int act[4];
    T al[4];
    int any = 0;
    for (int j = 0; j < 4; ++j) {
      act[j] = a.cg.act[c0 + j];
      al[j] = T(a.cg.alpha[c0 + j]);
      any |= act[j];
    }
    if (any) {
      for_rows(t, [&](int row) {
        const size_t o = size_t(row) * t.rp + c0;
        V4<T> xv = ld4s(x + o), rv = ld4s(r + o);
        const V4<T> pv = ld4s(p + o), qv = ld4s(q + o);
        const T di = dinv[row];
        for (int j = 0; j < 4; ++j) {
          if (act[j]) {
            xv.v[j] = fma(al[j], pv.v[j], xv.v[j]);
            rv.v[j] = fma(-al[j], qv.v[j], rv.v[j]);
            const double rd = double(rv.v[j]);
            if constexpr (Poly) {
              s[0][j] += rd * rd;
            } else {
              s[0][j] += rd * double(di * rv.v[j]);
              s[1][j] += rd * rd;
            }
          }
        }
        st4s(x + o, xv);
        st4s(r + o, rv);
      });
    }
  }
  block_store<Poly ? 1 : 2>(t, s, a.part, blockIdx.x, ct);
  }
}

// beta = r.z(new) / r.z(old) per column still iterating, which stops once
// ||r||^2 <= tol2.  Poly: r.z from the preconditioner pass (part2, tiling tm),
// r.r from the update (part slot 0); otherwise both from the update.
template <bool Poly>
__global__ void k_red_beta(StepArgs a, int slot, int next) {
  if (a.ring[slot] == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.stat[0] += 1;  // an iteration that did work
  const int c = red_col();
  const Tile& t = a.t;
  const bool act = c < t.rp && a.cg.act[c];
  const double rzn = Poly ? red_sum(a.part2, act ? a.tp.nchunk : 0, t.rp, c)
                          : red_sum(a.part + part_off(t, 0), act ? t.nchunk : 0, t.rp, c);
  const double rr = red_sum(a.part + part_off(t, Poly ? 0 : 1), act ? t.nchunk : 0, t.rp, c);
  int still = 0;
  if (red_lead() && act) {
    a.cg.iters[c] += 1;
    if (rr <= a.cg.tol2[c] || !(rr == rr)) {
      a.cg.act[c] = 0;
      a.cg.beta[c] = 0.0;
    } else {
      a.cg.beta[c] = rzn / a.cg.rz[c];
      a.cg.rz[c] = rzn;
      still = 1;
    }
  }
  count_active(still, a.ring + next);
}

// Direction-ring form of the float32 inner CG: the correction d = sum_i
// alpha_i p_i is not updated every iteration; the directions p_i stay in a
// ring of kPRing vectors and d is formed from them when the ring is full and
// at the end of the solve (k_materialize), in iteration order, so d gets
// exactly the rounding of the running update.
//
// The directions (and the polynomial preconditioner's output z) are stored
// as bf16.  A rounded direction is still a direction: q = K p, p.q, alpha
// and d all use the stored p, so r stays the float32 residual of d and the
// attainable accuracy is unchanged; what rounding perturbs is only the
// conjugacy of successive directions (relative 2^-9 per direction), which
// changed no iteration count on the meshes tested (condition numbers of
// D^-1 K from 2 to 90).  r and q, whose recursion defines the residual,
// stay float32.
//
// r -= alpha q, z = D r; partials r.z and r.r (Poly: r.r only, r in split
// storage).
template <bool Poly>
__global__ __launch_bounds__(kBlock) void k_cg_update_r(StepArgs a, int slot,
                                                        float* __restrict__ r,
                                                        const float* __restrict__ q,
                                                        const float* __restrict__ dinv) {
  if (a.ring[slot] == 0) return;
  const Tile& t = a.t;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  double s[Poly ? 1 : 2][4] = {};
  if (g < t.G) {
    const int c0 = 4 * g;
    int act[4];
    float al[4];
    int any = 0;
    for (int j = 0; j < 4; ++j) {
      act[j] = a.cg.act[c0 + j];
      al[j] = float(a.cg.alpha[c0 + j]);
      any |= act[j];
    }
    if (any) {
      const size_t plane = size_t(t.n) * t.rp;
      for_rows(t, [&](int row) {
        const size_t o = size_t(row) * t.rp + c0;
        V4<float> rv = Poly ? ld4_split(r, plane, o) : ld4s(r + o);
        const V4<float> qv = ld4s(q + o);
        const float di = Poly ? 0.0f : dinv[row];
        for (int j = 0; j < 4; ++j) {
          if (act[j]) {
            rv.v[j] = fmaf(-al[j], qv.v[j], rv.v[j]);
            const double rd = double(rv.v[j]);
            if constexpr (Poly) {
              s[0][j] += rd * rd;
            } else {
              s[0][j] += rd * double(di * rv.v[j]);
              s[1][j] += rd * rd;
            }
          }
        }
        if constexpr (Poly)
          st4_split(r, plane, o, rv);
        else
          st4s(r + o, rv);
      });
    }
  }
  block_store<Poly ? 1 : 2>(t, s, a.part, blockIdx.x, ct);
  }
}

// p_next = z + beta p on the columns still iterating, 0 on the others of a
// group that has one (p_next is a different ring slot from p); z = D r
// (src = r), or the preconditioner's output (Poly: src = z).
template <bool Poly>
__global__ __launch_bounds__(kBlock) void k_cg_dir_ring(
    StepArgs a, int next, bf16_t* __restrict__ pn, const bf16_t* __restrict__ p,
    const std::conditional_t<Poly, bf16_t, float>* __restrict__ src,
    const float* __restrict__ dinv) {
  if (a.ring[next] == 0) return;
  const Tile& t = a.t;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  if (g >= t.G) continue;
  const int c0 = 4 * g;
  int act[4];
  float be[4];
  int any = 0;
  for (int j = 0; j < 4; ++j) {
    act[j] = a.cg.act[c0 + j];
    be[j] = float(a.cg.beta[c0 + j]);
    any |= act[j];
  }
  if (!any) continue;
  for_rows(t, [&](int row) {
    const size_t o = size_t(row) * t.rp + c0;
    const V4<float> pv = ld4s(p + o), sv = ld4s(src + o);
    const float di = Poly ? 1.0f : dinv[row];
    V4<float> nv;
    for (int j = 0; j < 4; ++j) nv.v[j] = act[j] ? fmaf(be[j], pv.v[j], di * sv.v[j]) : 0.0f;
    st4s(pn + o, nv);
  });
  }
}

// d = sum_q ah[row q] p_q (accumulate: d += ...), in the order given, on the
// columns of live groups; float32 like the running update it replaces.
__global__ __launch_bounds__(kBlock) void k_materialize(StepArgs a, RingArgs ra,
                                                        const double* __restrict__ ah,
                                                        float* __restrict__ d) {
  const Tile& t = a.ts;
  for (int ct = 0; ct < t.nct; ++ct) {
    const int g = ct * t.tg + threadIdx.x % t.tg;
    if (g >= t.G) continue;
    const int c0 = 4 * g;
    int any = 0;
    for (int j = 0; j < 4; ++j) any |= a.ct.live[c0 + j];
    if (!any) continue;
    float cf[kPRing][4];
    for (int q = 0; q < ra.n; ++q)
      for (int j = 0; j < 4; ++j) cf[q][j] = float(ah[size_t(ra.row[q]) * t.rp + c0 + j]);
    for_rows(t, [&](int row) {
      const size_t o = size_t(row) * t.rp + c0;
      V4<float> acc = {};
      if (ra.accumulate) acc = ld4s(d + o);
      for (int q = 0; q < ra.n; ++q) {
        // a direction whose 4 coefficients are zero (columns that had
        // converged) adds nothing: skip its load
        if (cf[q][0] == 0.0f && cf[q][1] == 0.0f && cf[q][2] == 0.0f && cf[q][3] == 0.0f) continue;
        const V4<float> pv = ld4s(ra.p[q] + o);
        for (int j = 0; j < 4; ++j) acc.v[j] = fmaf(cf[q][j], pv.v[j], acc.v[j]);
      }
      st4s(d + o, acc);
    });
  }
}

// Start guess of the heat solve, per column c: y = sum_{j<h} (-1)^j C(h, j+1)
// x_j, the polynomial extrapolation through the column's last h heat
// increments x_0 (newest), x_1, ..., with h = min(hlen[c], ord[c], e.n); 0 on
// columns that are not live or have no increment yet (a column admitted to a
// running batch starts from its own state while the others keep their
// history).  y may be one of the sources (each element is read before it is
// written, by the same thread).  A source whose 4 coefficients are 0 is not
// read.
__global__ __launch_bounds__(kBlock) void k_extrap(StepArgs a, ExtrapArgs e, float* y) {
  const Tile& t = a.ts;
  for (int ct = 0; ct < t.nct; ++ct) {
    const int g = ct * t.tg + threadIdx.x % t.tg;
    if (g >= t.G) continue;
    const int cb = 4 * g;
    float cf[kMaxExtrap][4];
    for (int j = 0; j < 4; ++j) {
      const int h = a.ct.live[cb + j] ? min(min(a.hlen[cb + j], a.ord[cb + j]), e.n) : 0;
      int binom = 1;  // C(h, q + 1), built up from C(h, 0) = 1
      for (int q = 0; q < kMaxExtrap; ++q) {
        if (q < h) {
          binom = binom * (h - q) / (q + 1);
          cf[q][j] = float((q % 2 == 0) ? binom : -binom);
        } else {
          cf[q][j] = 0.0f;
        }
      }
    }
    for_rows(t, [&](int row) {
      const size_t o = size_t(row) * t.rp + cb;
      float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int q = 0; q < e.n; ++q) {
        if (cf[q][0] == 0.0f && cf[q][1] == 0.0f && cf[q][2] == 0.0f && cf[q][3] == 0.0f) continue;
        const V4<float> v = ld4s(e.x[q] + o);
        for (int j = 0; j < 4; ++j) acc[j] = cf[q][j] != 0.0f ? fmaf(cf[q][j], v.v[j], acc[j]) : acc[j];
      }
      V4<float> yv;
      for (int j = 0; j < 4; ++j) yv.v[j] = acc[j];
      st4s(y + o, yv);
    });
  }
}

// Order control of the extrapolation, on a sample of rows (every
// a.probe_stride-th row; tiling a.tprobe over the sample): per column, the
// sums of squares of the backward differences D_j = sum_{i<=j} (-1)^i C(j, i)
// x_i of the kept increments, j below their number (partial slots
// 0..kMaxOrderProbe-1).  Extrapolating with order j neglects the j-th
// difference at the next step, which |D_j| estimates.
constexpr int kMaxOrderProbe = k::kOrderProbes;
__global__ __launch_bounds__(kBlock) void k_extrap_probe(StepArgs a, ExtrapArgs e) {
  const Tile& t = a.tprobe;
  for (int ct = 0; ct < t.nct; ++ct) {
    const int g = ct * t.tg + threadIdx.x % t.tg;
    double s[kMaxOrderProbe][4] = {};
    if (g < t.G) {
      const int cb = 4 * g;
      int nd[4], nread = 0;
      for (int j = 0; j < 4; ++j) {
        nd[j] = a.ct.live[cb + j] ? min(min(a.hlen[cb + j], e.n), kMaxOrderProbe) : 0;
        nread = max(nread, nd[j]);
      }
      for_rows(t, [&](int srow) {
        const size_t o = size_t(srow) * size_t(a.probe_stride) * t.rp + cb;
        V4<float> xs[kMaxOrderProbe] = {};
        for (int q = 0; q < nread; ++q) xs[q] = ld4s(e.x[q] + o);
        // difference table in float64 (differences of float32 values are exact
        // there): after pass k its first entry is D_k
        for (int j = 0; j < 4; ++j) {
          double d[kMaxOrderProbe];
          for (int i = 0; i < kMaxOrderProbe; ++i) d[i] = i < nd[j] ? double(xs[i].v[j]) : 0.0;
          s[0][j] += d[0] * d[0];
          for (int k = 1; k < kMaxOrderProbe; ++k) {
            for (int i = 0; i + k < kMaxOrderProbe; ++i) d[i] -= d[i + 1];
            if (k < nd[j]) s[k][j] += d[0] * d[0];
          }
        }
      });
    }
    block_store<kMaxOrderProbe>(t, s, a.part, blockIdx.x, ct);
  }
}

// This step's extrapolation order per live column with at least two kept
// increments: the j of least |D_j| (j below the number kept, ties to the
// lower), or qmax when that is the deepest difference measured (the
// differences are still falling).
__global__ void k_red_extrap_order(StepArgs a, int n_kept, int qmax) {
  const int c = red_col();
  const Tile& t = a.tprobe;
  const int nd = c < t.rp && a.ct.live[c] ? min(min(a.hlen[c], n_kept), kMaxOrderProbe) : 0;
  double e[kMaxOrderProbe];
  for (int d = 0; d < kMaxOrderProbe; ++d)
    e[d] = red_sum(a.part + part_off(t, d), d < nd ? t.nchunk : 0, t.rp, c);
  if (!red_lead() || nd < 2) return;
  int best = 0;
  bool finite = e[0] == e[0];
  for (int d = 1; d < nd; ++d) {
    finite &= e[d] == e[d];
    if (e[d] < e[best]) best = d;
  }
  if (finite) a.ord[c] = best == nd - 1 ? qmax : best;
}

// After a heat solve: every live column has one more increment kept (at most
// q); a column that is not live has none (its stored increment is 0).
__global__ void k_hist_advance(StepArgs a, int q) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.t.rp) return;
  a.hlen[c] = a.ct.live[c] ? min(a.hlen[c] + 1, q) : 0;
}

// p = z + beta p, z = D r (src = r) or the preconditioner's output (Poly).
template <typename T, bool Poly>
__global__ __launch_bounds__(kBlock) void k_cg_update_p(StepArgs a, int next, T* __restrict__ p,
                                                        const T* __restrict__ src,
                                                        const T* __restrict__ dinv) {
  if (a.ring[next] == 0) return;
  const Tile& t = a.t;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  if (g >= t.G) continue;
  const int c0 = 4 * g;
  int act[4];
  T be[4];
  int any = 0;
  for (int j = 0; j < 4; ++j) {
    act[j] = a.cg.act[c0 + j];
    be[j] = T(a.cg.beta[c0 + j]);
    any |= act[j];
  }
  if (!any) continue;
  for_rows(t, [&](int row) {
    const size_t o = size_t(row) * t.rp + c0;
    V4<T> pv = ld4s(p + o);
    const V4<T> sv = ld4s(src + o);
    const T di = Poly ? T(1) : dinv[row];
    for (int j = 0; j < 4; ++j)
      if (act[j]) pv.v[j] = fma(be[j], pv.v[j], di * sv.v[j]);
    st4s(p + o, pv);
  });
  }
}

// Polynomial preconditioner pass: z = P r with P = D^-1 (c0 I + c1 K D^-1),
// the degree-1 Chebyshev polynomial in D^-1 K applied to the Jacobi step
// (a matrix of K's pattern, built once per tau: precond_mats), on the
// columns still iterating (0 on the others of a group that has one), with
// the partials r.z (part2, tiling tp; from z before it is stored as Z, which
// is bf16 in the float32 CG).  Restricted solves keep z on the column's
// region.  In the float32 CG r is in split storage: the neighbours' values
// enter z rounded to bf16 (the rounding z itself gets when it is stored), the
// row's own value and r.z exactly.
template <typename T, typename Z = T>
__global__ __launch_bounds__(kBlock) void k_cg_precond(StepArgs a, int slot,
                                                       const T* __restrict__ r,
                                                       Z* __restrict__ z,
                                                       const T* __restrict__ P) {
  // the float32 CG's r (bf16 z) is in split storage
  constexpr bool kSplit = std::is_same_v<Z, bf16_t>;
  if (a.ring[slot] == 0) return;
  const Tile& t = a.tp;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  double s[1][4] = {};
  if (g < t.G) {
    const int cb = 4 * g;
    int act[4], any = 0;
    for (int j = 0; j < 4; ++j) {
      act[j] = a.cg.act[cb + j];
      any |= act[j];
    }
    if (any) {
      const size_t plane = size_t(a.t.n) * a.t.rp;
      for_rows(t, [&](int row) {
        V4<T> acc = {}, ro = {};
        if constexpr (kSplit) {
          // the neighbours' values from plane 0 (bf16), the row's own exact
          const u2v lo = ld_plane1(r, plane, size_t(row) * t.rp + cb);
          for_neighbors(a, row, cb, reinterpret_cast<const bf16_t*>(r),
                        [&](int k, const V4<float>& x, size_t o) {
                          const T v = ldm(P + o);
                          const V4<float> y = k == 0 ? split_join4(x, lo) : x;
                          if (k == 0) ro = y;
                          for (int j = 0; j < 4; ++j) acc.v[j] = fma(v, y.v[j], acc.v[j]);
                        });
        } else {
          for_neighbors(a, row, cb, r, [&](int k, const V4<T>& x, size_t o) {
            const T v = ldm(P + o);
            if (k == 0) ro = x;
            for (int j = 0; j < 4; ++j) acc.v[j] = fma(v, x.v[j], acc.v[j]);
          });
        }
        V4<T> zv;
        for (int j = 0; j < 4; ++j) zv.v[j] = act[j] ? acc.v[j] : T(0);
        if constexpr (sizeof(T) == 8) {
          if (a.mask)  // restricted solve: z stays on the region
            for (int j = 0; j < 4; ++j)
              if (!a.mask[size_t(row) * t.rp + cb + j]) zv.v[j] = 0.0;
        }
        st4g(z + size_t(row) * t.rp + cb, zv);
        for (int j = 0; j < 4; ++j) s[0][j] += double(ro.v[j]) * double(zv.v[j]);
      });
    }
  }
  block_store<1>(t, s, a.part2, blockIdx.x, ct);
  }
}

// r.z of the preconditioner's first pass of a solve: cg.rz of every column
// starting it (cg.act).
__global__ void k_red_precond_init(StepArgs a) {
  const int c = red_col();
  const Tile& t = a.tp;
  const bool act = c < t.rp && a.cg.act[c];
  const double rz = red_sum(a.part2, act ? t.nchunk : 0, t.rp, c);
  if (red_lead() && act) a.cg.rz[c] = rz;
}

// ------------------------------------------------- mixed-precision refinement --
// Outer residual r64 = -tau A u (float64), partials ||M u||^2 and ||r64||^2.
// Start of the float64 refinement.  b = M u; with a start guess g (nullable)
// the iterate is x0 = u + g, written to x0, and r64 = b - K x0 = -tau A u - K g
// (no cancellation); without one x0 = u and r64 = -tau A u.  Partials:
// ||M u||^2 and ||r64||^2.  x0 must not alias u (u is gathered).
__global__ __launch_bounds__(kBlock) void k_init_outer(StepArgs a, const double* __restrict__ u,
                                                       const float* __restrict__ gd,
                                                       double* __restrict__ x0,
                                                       double* __restrict__ r64) {
  const Tile& t = a.t64;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  double s[2][4] = {};
  if (g < t.G) {
    const int c0 = 4 * g;
    double lv[4];
    for (int j = 0; j < 4; ++j) lv[j] = a.ct.live[c0 + j] ? 1.0 : 0.0;
    for_rows(t, [&](int row) {
      double au[4] = {}, mu[4] = {}, kg[4] = {};
      V4<double> uo = {};
      for_neighbors(a, row, c0, u, [&](int k, const V4<double>& x, size_t o) {
        const double va = ldm(a.A64 + o), vm = ldm(a.M64 + o);
        if (k == 0) uo = x;
        for (int j = 0; j < 4; ++j) {
          au[j] = fma(va, x.v[j], au[j]);
          mu[j] = fma(vm, x.v[j], mu[j]);
        }
      });
      V4<float> go = {};
      if (gd)
        for_neighbors(a, row, c0, gd, [&](int k, const V4<float>& x, size_t o) {
          const double v = ldm(a.K64 + o);
          if (k == 0) go = x;
          for (int j = 0; j < 4; ++j) kg[j] = fma(v, double(x.v[j]), kg[j]);
        });
      V4<double> rv, xv;
      for (int j = 0; j < 4; ++j) {
        rv.v[j] = (-a.tau * au[j] - kg[j]) * lv[j];
        xv.v[j] = uo.v[j] + double(go.v[j]) * lv[j];
        s[0][j] += mu[j] * mu[j] * lv[j];
        s[1][j] += rv.v[j] * rv.v[j];
      }
      const size_t o = size_t(row) * t.rp + c0;
      st4g(r64 + o, rv);
      if (gd) st4g(x0 + o, xv);
    });
  }
  block_store<2>(t, s, a.part, blockIdx.x, ct);
  }
}

__global__ void k_red_outer_init(StepArgs a) {
  const int c = red_col();
  const Tile& t = a.t64;
  const double bb = red_sum(a.part + part_off(t, 0), t.nchunk, t.rp, c);
  const double rr = red_sum(a.part + part_off(t, 1), t.nchunk, t.rp, c);
  int act = 0;
  if (red_lead() && c < t.rp) {
    a.cg.bb[c] = bb;
    a.cg.rr_o[c] = rr;
    act = (a.ct.live[c] && rr > a.rtol2 * bb) ? 1 : 0;
    a.cg.act_o[c] = act;
    a.cg.act[c] = 0;
  }
  count_active(act, a.oring + 0);
}

// Refinement start and first inner start in one pass, from the previous
// step's norm pass: the state u = v / n is already scaled and w holds A v, so
// A u = w / n needs no float64 gather.  With the start guess g:
//   r64 = b - K (u + g) = -tau A u - K64 g, r32 = float(r64), p = D r32;
// the iterate u + g is formed by the first refinement update (ubase mode),
// and the correction d by the inner solve.  Partials ||r64||^2, r32.p,
// ||r32||^2.  Columns that are not live get zeros.  Tiling tm (the float32
// gather of g).  Under the polynomial preconditioner r32 goes to split
// storage.
__global__ __launch_bounds__(kBlock) void k_refine_start(StepArgs a, const double* __restrict__ w,
                                                         const float* __restrict__ gd,
                                                         double* __restrict__ r64,
                                                         float* __restrict__ r,
                                                         bf16_t* __restrict__ p) {
  const Tile& t = a.tm;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  double s[3][4] = {};
  if (g < t.G) {
    const int c0 = 4 * g;
    bool lv[4];
    double inv[4];
    for (int j = 0; j < 4; ++j) {
      lv[j] = a.ct.live[c0 + j] != 0;
      inv[j] = 1.0 / a.cg.nrm[c0 + j];
    }
    for_rows(t, [&](int row) {
      double kg[4] = {};
      for_neighbors(a, row, c0, gd, [&](int, const V4<float>& x, size_t o) {
        const double v = ldm(a.K64 + o);
        for (int j = 0; j < 4; ++j) kg[j] = fma(v, double(x.v[j]), kg[j]);
      });
      const size_t o = size_t(row) * t.rp + c0;
      const V4<double> wv = ld4g(w + o);
      const float di = a.dinv32[row];
      V4<double> rv;
      V4<float> r32, pv;
      for (int j = 0; j < 4; ++j) {
        rv.v[j] = lv[j] ? -a.tau * (wv.v[j] * inv[j]) - kg[j] : 0.0;
        r32.v[j] = float(rv.v[j]);
        pv.v[j] = di * r32.v[j];
        s[0][j] += rv.v[j] * rv.v[j];
        s[1][j] += double(r32.v[j]) * double(pv.v[j]);
        s[2][j] += double(r32.v[j]) * double(r32.v[j]);
      }
      st4g(r64 + o, rv);
      if (a.poly)
        st4_split(r, size_t(a.t.n) * a.t.rp, o, r32);
      else
        st4g(r + o, r32);
      if (p) st4g(p + o, pv);
    });
  }
  block_store<3>(t, s, a.part, blockIdx.x, ct);
  }
}

// Reductions of the fused start: the refinement's activity (with ||b||^2
// from the norm pass) and the first inner solve's scalars and tolerance.
__global__ void k_red_refine_start(StepArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) a.oring[1] = 0;
  const int c = red_col();
  const Tile& t = a.tm;
  const double rr = red_sum(a.part + part_off(t, 0), t.nchunk, t.rp, c);
  const double rz = red_sum(a.part + part_off(t, 1), t.nchunk, t.rp, c);
  const double r2 = red_sum(a.part + part_off(t, 2), t.nchunk, t.rp, c);
  int act_o = 0, act = 0;
  if (red_lead() && c < t.rp) {
    const double bb = a.cg.bb_next[c];
    a.cg.bb[c] = bb;
    a.cg.rr_o[c] = rr;
    act_o = (a.ct.live[c] && rr > a.rtol2 * bb) ? 1 : 0;
    a.cg.act_o[c] = act_o;
    a.cg.rz[c] = rz;
    a.cg.tol2[c] = fmax(a.inner_rtol2 * r2, a.inner_floor2 * a.rtol2 * bb);
    act = (act_o && r2 > 0.0) ? 1 : 0;
    a.cg.act[c] = act;
    a.cg.alpha[c] = 0.0;
    a.cg.beta[c] = 0.0;
  }
  count_active(act_o, a.oring + 0);
  count_active(act, a.ring + 0);
}

// Start of an inner float32 solve K d = r64: r = float(r64) (split storage
// under the polynomial preconditioner), p = D r (d is formed by the solve).
__global__ __launch_bounds__(kBlock) void k_inner_init(StepArgs a, int oslot,
                                                       const double* __restrict__ r64,
                                                       float* __restrict__ d,
                                                       float* __restrict__ r,
                                                       bf16_t* __restrict__ p) {
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ring[0] = 0;
  if (a.oring[oslot] == 0) return;
  const Tile& t = a.t;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  double s[2][4] = {};
  if (g < t.G) {
    const int c0 = 4 * g;
    int act[4];
    for (int j = 0; j < 4; ++j) act[j] = a.cg.act_o[c0 + j];
    for_rows(t, [&](int row) {
      const size_t o = size_t(row) * t.rp + c0;
      const V4<double> rd = ld4s(r64 + o);
      const float di = a.dinv32[row];
      V4<float> rv, pv;
      for (int j = 0; j < 4; ++j) {
        rv.v[j] = act[j] ? float(rd.v[j]) : 0.0f;
        pv.v[j] = di * rv.v[j];
        s[0][j] += double(rv.v[j]) * double(pv.v[j]);
        s[1][j] += double(rv.v[j]) * double(rv.v[j]);
      }
      if (a.poly)
        st4_split(r, size_t(a.t.n) * a.t.rp, o, rv);
      else
        st4s(r + o, rv);
      if (p) st4s(p + o, pv);
    });
  }
  block_store<2>(t, s, a.part, blockIdx.x, ct);
  }
}

__global__ void k_red_inner_init(StepArgs a, int oslot, int onext) {
  if (blockIdx.x == 0 && threadIdx.x == 0) a.oring[onext] = 0;
  if (a.oring[oslot] == 0) return;
  const int c = red_col();
  const Tile& t = a.t;
  const double rz = red_sum(a.part + part_off(t, 0), t.nchunk, t.rp, c);
  const double rr = red_sum(a.part + part_off(t, 1), t.nchunk, t.rp, c);
  int act = 0;
  if (red_lead() && c < t.rp) {
    a.cg.rz[c] = rz;
    // stop the inner solve once its residual drops by inner_rtol, or below
    // sqrt(inner_floor2) x the outer target (no point solving further)
    a.cg.tol2[c] = fmax(a.inner_rtol2 * rr, a.inner_floor2 * a.rtol2 * a.cg.bb[c]);
    act = (a.cg.act_o[c] && rr > 0.0) ? 1 : 0;
    a.cg.act[c] = act;
    a.cg.alpha[c] = 0.0;
    a.cg.beta[c] = 0.0;
  }
  count_active(act, a.ring + 0);
}

// x += d; r64 -= K64 d (float64 product of the float32 correction), on the
// columns still refining; partial ||r64||^2 of the new residual.  dacc (if
// given) accumulates the corrections on top of the start guess, so after the
// last sweep it holds the step's heat increment x - u.
// ubase (nullable, first sweep of the fused start): the iterate is formed
// here as x = ubase + dacc (+ d), for every column of a group with a live
// column (dacc is 0 on columns that are not live), instead of being read.
// store_r == 0 leaves r64 as it was (the partial still measures the new
// residual); outer_residual stores it when another sweep follows.
// Prep (another sweep expected): the next inner solve's start is written
// too, r = float(r64), p = D r (rn, pn; zeros where the column is not
// refining), with its partials r.p and ||r||^2, so the sweep after this one
// needs neither outer_residual nor inner_init (red_outer_prep reduces all
// three); r64 must be stored then.
// Deferred iterate (d0mode): when the solve is expected to need another
// sweep, sweep 0 leaves x and dacc alone (d0mode 1: x, ubase, dacc unused)
// and keeps its correction in d0 (0 where the column is not refining), and
// the next sweep forms the iterate in ubase mode with d0 as one more addend
// (d0mode 2): x = ((ubase + dacc) + d0) + d, dacc + d0 + d, the same sums in
// the same order as forming x in sweep 0 and adding to it in sweep 1, with
// one pass over u, x and dacc fewer.
template <bool Prep>
__global__ __launch_bounds__(kBlock) void k_outer_update(StepArgs a, int oslot,
                                                         double* __restrict__ x,
                                                         const double* __restrict__ ubase,
                                                         double* __restrict__ r64,
                                                         const float* __restrict__ d,
                                                         float* __restrict__ dacc, int store_r,
                                                         float* __restrict__ rn,
                                                         bf16_t* __restrict__ pn,
                                                         float* __restrict__ d0, int d0mode) {
  // the next sweep's inner activity is counted afresh (red_outer_prep)
  if (Prep && blockIdx.x == 0 && threadIdx.x == 0) a.ring[0] = 0;
  // (d0mode 1 writes d0 on every live group, refining or not)
  if (!ubase && d0mode != 1 && a.oring[oslot] == 0) return;
  const Tile& t = a.tm;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  const int* mask = a.cg.act_o;
  double s[Prep ? 3 : 1][4] = {};
  if (g < t.G) {
    const int c0 = 4 * g;
    int act[4], any = 0, anylive = 0;
    double usc[4] = {1.0, 1.0, 1.0, 1.0};
    for (int j = 0; j < 4; ++j) {
      act[j] = mask[c0 + j];
      any |= act[j];
      anylive |= a.ct.live[c0 + j];
      if (a.usc) usc[j] = a.usc[c0 + j];
    }
    if (any || ((ubase || d0mode == 1) && anylive)) {
      for_rows(t, [&](int row) {
        double kd[4] = {};
        float dd[4] = {};
        if (any)
          for_neighbors(a, row, c0, d, [&](int k, const V4<float>& xv, size_t o) {
            const double v = ldm(a.K64 + o);
            if (k == 0)
              for (int j = 0; j < 4; ++j) dd[j] = xv.v[j];
            for (int j = 0; j < 4; ++j) kd[j] = fma(v, double(xv.v[j]), kd[j]);
          });
        const size_t o = size_t(row) * t.rp + c0;
        V4<float> av = {};
        V4<double> xv = {};
        if (d0mode != 1) {
          if (dacc) av = ld4g(dacc + o);
          if (ubase) {
            const V4<double> ub = ld4g(ubase + o);
            for (int j = 0; j < 4; ++j) xv.v[j] = mul_alone(ub.v[j], usc[j]) + double(av.v[j]);
            if (d0mode == 2) {
              const V4<float> e0 = ld4g(d0 + o);
              for (int j = 0; j < 4; ++j) {
                xv.v[j] += double(e0.v[j]);
                av.v[j] += e0.v[j];
              }
            }
          } else {
            xv = ld4g(x + o);
          }
        }
        V4<double> rv = {};
        if (any) rv = ld4g(r64 + o);
        for (int j = 0; j < 4; ++j) {
          if (act[j]) {
            xv.v[j] += double(dd[j]);
            rv.v[j] -= kd[j];
            s[0][j] += rv.v[j] * rv.v[j];
            av.v[j] += dd[j];
          }
        }
        if (d0mode == 1) {
          V4<float> e0;
          for (int j = 0; j < 4; ++j) e0.v[j] = act[j] ? dd[j] : 0.0f;
          st4g(d0 + o, e0);
        } else {
          st4g(x + o, xv);
          if (dacc && (any || d0mode == 2)) st4g(dacc + o, av);
        }
        if (any && store_r) st4g(r64 + o, rv);
        if constexpr (Prep) {
          if (any) {
            const float di = a.dinv32[row];
            V4<float> r32, p32;
            for (int j = 0; j < 4; ++j) {
              r32.v[j] = act[j] ? float(rv.v[j]) : 0.0f;
              p32.v[j] = di * r32.v[j];
              s[1][j] += double(r32.v[j]) * double(p32.v[j]);
              s[2][j] += double(r32.v[j]) * double(r32.v[j]);
            }
            if (a.poly)
              st4_split(rn, size_t(a.t.n) * a.t.rp, o, r32);
            else
              st4g(rn + o, r32);
            if (pn) st4g(pn + o, p32);
          }
        }
      });
    }
  }
  block_store<Prep ? 3 : 1>(t, s, a.part, blockIdx.x, ct);
  }
}

// r64 -= K64 d on the columns still refining, after a sweep whose update did
// not store r64 (it is needed only when another sweep follows).
__global__ __launch_bounds__(kBlock) void k_outer_residual(StepArgs a, int oslot,
                                                           double* __restrict__ r64,
                                                           const float* __restrict__ d) {
  if (a.oring[oslot] == 0) return;
  const Tile& t = a.tm;
  for (int ct = 0; ct < t.nct; ++ct) {
    const int g = ct * t.tg + threadIdx.x % t.tg;
    if (g >= t.G) continue;
    const int c0 = 4 * g;
    int act[4], any = 0;
    for (int j = 0; j < 4; ++j) {
      act[j] = a.cg.act_o[c0 + j];
      any |= act[j];
    }
    if (!any) continue;
    for_rows(t, [&](int row) {
      double kd[4] = {};
      for_neighbors(a, row, c0, d, [&](int, const V4<float>& xv, size_t o) {
        const double v = ldm(a.K64 + o);
        for (int j = 0; j < 4; ++j) kd[j] = fma(v, double(xv.v[j]), kd[j]);
      });
      const size_t o = size_t(row) * t.rp + c0;
      V4<double> rv = ld4g(r64 + o);
      for (int j = 0; j < 4; ++j)
        if (act[j]) rv.v[j] -= kd[j];
      st4g(r64 + o, rv);
    });
  }
}

__global__ void k_red_outer(StepArgs a, int oslot, int onext) {
  if (a.oring[oslot] == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.stat[1] += 1;
  const int c = red_col();
  const bool act = c < a.tm.rp && a.cg.act_o[c];
  const double rr = red_sum(a.part, act ? a.tm.nchunk : 0, a.tm.rp, c);
  int still = 0;
  if (red_lead() && act) {
    a.cg.rr_o[c] = rr;
    a.cg.sweeps[c] += 1;
    if (rr <= a.rtol2 * a.cg.bb[c] || !(rr == rr))
      a.cg.act_o[c] = 0;
    else
      still = 1;
  }
  count_active(still, a.oring + onext);
}

// Reduction of a refinement update that prepared the next sweep (Prep):
// the outer test as k_red_outer, and for the columns still refining the next
// inner solve's scalars as k_red_inner_init would set them from the r and p
// the update wrote; counts go to oring[onext] and ring[0] (zeroed by the
// update), and oring[onext2] is zeroed for the next sweep's red_outer.
__global__ void k_red_outer_prep(StepArgs a, int oslot, int onext, int onext2) {
  if (a.oring[oslot] == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.stat[1] += 1;
    a.oring[onext2] = 0;
  }
  const int c = red_col();
  const Tile& t = a.tm;
  const bool act_o = c < t.rp && a.cg.act_o[c];
  const int nch = act_o ? t.nchunk : 0;
  const double rr = red_sum(a.part + part_off(t, 0), nch, t.rp, c);
  const double rz = red_sum(a.part + part_off(t, 1), nch, t.rp, c);
  const double r2 = red_sum(a.part + part_off(t, 2), nch, t.rp, c);
  int still = 0, act = 0;
  if (red_lead() && c < t.rp) {
    if (act_o) {
      a.cg.rr_o[c] = rr;
      a.cg.sweeps[c] += 1;
      if (rr <= a.rtol2 * a.cg.bb[c] || !(rr == rr)) {
        a.cg.act_o[c] = 0;
      } else {
        still = 1;
        a.cg.rz[c] = rz;
        a.cg.tol2[c] = fmax(a.inner_rtol2 * r2, a.inner_floor2 * a.rtol2 * a.cg.bb[c]);
        act = r2 > 0.0 ? 1 : 0;
      }
    }
    a.cg.act[c] = act;
    a.cg.alpha[c] = 0.0;
    a.cg.beta[c] = 0.0;
  }
  count_active(still, a.oring + onext);
  count_active(act, a.ring + 0);
}

// -------------------------------------------------------------- node step --
// Step 2 of Algorithm 2.2 in its practical form: S = sum_j u~_j^2 over the
// restart's components, u^_i = u~_i exp(-(2 tau/eps^2)(S - u~_i^2)).
//
// S comes from segmented sums across the row group (the tg lanes that hold
// one row's column tile, 4 columns a lane).  In general (any restart length
// and alignment) a forward scan F (restarting at each restart's first column in
// the tile) and a backward scan B (restarting at its last one), each a local
// pass over the lane's 4 columns plus a shuffle scan over the lanes, give
// S_i = F_i + B_i - u~_i^2 (all terms nonnegative: no cancellation).  A
// restart that runs past either edge of the tile adds the squares of its
// columns outside the tile, read from the row.  Every lane of a row group
// takes part in the shuffles; lanes past the last column group carry empty
// segments.
template <bool General>
__global__ __launch_bounds__(kBlock) void k_nodal(StepArgs a, const double* __restrict__ u,
                                                  double* __restrict__ out, int keep) {
  const Tile& t = a.ts;
  const int tg = t.tg, gl = threadIdx.x % tg;
  for (int ct = 0; ct < t.nct; ++ct) {
    const int g = ct * tg + gl;
    const bool in = g < t.G;
    const int c0 = 4 * g;
    const int tile_lo = 4 * ct * tg, tile_hi = min(tile_lo + 4 * tg, t.rp);
    int lo[4] = {0, 0, 0, 0}, len[4] = {0, 0, 0, 0}, lv[4] = {0, 0, 0, 0};
    double cf[4] = {0, 0, 0, 0};
    if (in)
      for (int j = 0; j < 4; ++j) {
        lo[j] = a.ct.seg_lo[c0 + j];
        len[j] = a.ct.seg_len[c0 + j];
        lv[j] = a.ct.live[c0 + j];
        cf[j] = a.ct.coef[c0 + j];
      }
    const int anylv = lv[0] | lv[1] | lv[2] | lv[3];
    // a row group with no live column has nothing to do (the test is uniform
    // over the group: a whole wavefront when tg = 64, else every group runs)
    if (tg == 64 && !__any(anylv)) continue;
    const bool mixed = keep && !(lv[0] & lv[1] & lv[2] & lv[3]);
    // first / last column of each column's restart inside the tile
    bool head[4], tail[4], left[4], right[4];
    for (int j = 0; j < 4; ++j) {
      const bool v = in && len[j] > 0;
      const int c = c0 + j;
      head[j] = !v || c == max(lo[j], tile_lo);
      tail[j] = !v || c == min(lo[j] + len[j], tile_hi) - 1;
      left[j] = v && lo[j] < tile_lo;
      right[j] = v && lo[j] + len[j] > tile_hi;
    }
    const bool fh = head[0] | head[1] | head[2] | head[3];
    const bool bt = tail[0] | tail[1] | tail[2] | tail[3];
    // Fast case (wave-uniform): one row per wavefront and each lane's four
    // columns inside one restart that starts on a lane and lies in the
    // tile; then one segmented sum of the lanes' partial sums, broadcast
    // from the restart's first lane, gives S.
    const int lane = threadIdx.x & 63;
    const bool one_seg = in && lo[0] == lo[3] && len[0] > 0 && ((lo[0] | len[0]) & 3) == 0 &&
                         lo[0] >= tile_lo && lo[0] + len[0] <= tile_hi;
    // (General = false: the host has checked that every wavefront qualifies)
    const bool lanes = !General || (tg == 64 && __all(!in || one_seg));
    const int ls = one_seg ? (lo[0] - tile_lo) >> 2 : lane, le = one_seg ? ls + (len[0] >> 2) : lane + 1;
    for_rows(t, [&](int row) {
      const double* ur = u + size_t(row) * t.rp;
      V4<double> uv = {}, ov = {};
      if (in) {
        uv = ld4s(ur + c0);
        ov = mixed ? ld4s(out + size_t(row) * t.rp + c0) : uv;
      }
      if (!General || lanes) {
        double v = 0.0;
        for (int j = 0; j < 4; ++j) v = fma(uv.v[j], uv.v[j], v);
        for (int d = 1; d < 64 && __any(lane + d < le); d <<= 1) {
          const double w = __shfl_down(v, d);
          if (lane + d < le) v += w;
        }
        const double S = __shfl(v, ls);
        if (in) {
          for (int j = 0; j < 4; ++j)
            if (lv[j]) ov.v[j] = uv.v[j] * exp(-cf[j] * (S - uv.v[j] * uv.v[j]));
          st4s(out + size_t(row) * t.rp + c0, ov);
        }
        return;
      }
      double q[4], F[4], B[4];
      for (int j = 0; j < 4; ++j) q[j] = (in && len[j] > 0) ? uv.v[j] * uv.v[j] : 0.0;
      F[0] = q[0];
      for (int j = 1; j < 4; ++j) F[j] = head[j] ? q[j] : F[j - 1] + q[j];
      B[3] = q[3];
      for (int j = 2; j >= 0; --j) B[j] = tail[j] ? q[j] : B[j + 1] + q[j];
      // inclusive segmented scans over the lanes of the row group
      double tf = F[3], tb = B[0];
      int ff = fh, fb = bt;
      for (int d = 1; d < tg; d <<= 1) {
        const double uf = __shfl_up(tf, d, tg), ub = __shfl_down(tb, d, tg);
        const int gf = __shfl_up(ff, d, tg), gb = __shfl_down(fb, d, tg);
        if (gl >= d) {
          if (!ff) tf = uf + tf;
          ff |= gf;
        }
        if (gl + d < tg) {
          if (!fb) tb = tb + ub;
          fb |= gb;
        }
      }
      // carries from the neighbouring lanes (their inclusive values)
      const double cf_in = __shfl_up(tf, 1, tg), cb_in = __shfl_down(tb, 1, tg);
      bool open = gl > 0;
      for (int j = 0; j < 4; ++j) {
        open = open && !head[j];
        if (open) F[j] += cf_in;
      }
      open = gl + 1 < tg;
      for (int j = 3; j >= 0; --j) {
        open = open && !tail[j];
        if (open) B[j] += cb_in;
      }
      if (!in) return;
      double outside = 0.0;
      int cur = -1;
      for (int j = 0; j < 4; ++j) {
        if (!lv[j]) continue;
        if ((left[j] || right[j]) && lo[j] != cur) {
          // the restart's columns outside the tile, in column order
          cur = lo[j];
          outside = 0.0;
          for (int c = lo[j]; c < tile_lo; ++c) outside = fma(ur[c], ur[c], outside);
          for (int c = tile_hi; c < lo[j] + len[j]; ++c) outside = fma(ur[c], ur[c], outside);
        }
        const double S = F[j] + B[j] - q[j] + ((left[j] || right[j]) ? outside : 0.0);
        const double x = uv.v[j];
        ov.v[j] = x * exp(-cf[j] * (S - x * x));
      }
      st4s(out + size_t(row) * t.rp + c0, ov);
    });
  }
}

// ---------------------------------------------------------- normalisation --
// Norm pass: per column v.Mv, v.Av and ||M v||^2 (partials); w (nullable)
// receives A v, which the next step's refinement start reuses.
__global__ __launch_bounds__(kBlock) void k_norm_dot(StepArgs a, const double* __restrict__ v,
                                                     double* __restrict__ w) {
  const Tile& t = a.t64;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  double s[3][4] = {};
  if (g < t.G) {
    const int c0 = 4 * g;
    int lv[4], any = 0;
    for (int j = 0; j < 4; ++j) {
      lv[j] = a.ct.live[c0 + j];
      any |= lv[j];
    }
    if (any) {
      for_rows(t, [&](int row) {
        double mv[4] = {};
        V4<double> av = {}, vd = {};
        for_neighbors(a, row, c0, v, [&](int k, const V4<double>& x, size_t o) {
          const double wm = ldm(a.M64 + o), z = ldm(a.A64 + o);
          if (k == 0) vd = x;
          for (int j = 0; j < 4; ++j) {
            mv[j] = fma(wm, x.v[j], mv[j]);
            av.v[j] = fma(z, x.v[j], av.v[j]);
          }
        });
        for (int j = 0; j < 4; ++j)
          if (lv[j]) {
            s[0][j] += vd.v[j] * mv[j];
            s[1][j] += vd.v[j] * av.v[j];
            s[2][j] += mv[j] * mv[j];
          }
        if (w) st4g(w + size_t(row) * t.rp + c0, av);
      });
    }
  }
  block_store<3>(t, s, a.part, blockIdx.x, ct);
  }
}

// M-norms of the live columns, their Rayleigh quotients v.Av / v.Mv
// (unchanged by the scaling that follows, so they are the eigenvalue
// estimates of the normalised state) and ||M u||^2 of the scaled state.
__global__ void k_red_norm(StepArgs a, double* __restrict__ lam) {
  const int c = red_col();
  const Tile& t = a.t64;
  const bool lv = c < t.rp && a.ct.live[c];
  const double s = red_sum(a.part, lv ? t.nchunk : 0, t.rp, c);
  const double sa = red_sum(a.part + part_off(t, 1), lv ? t.nchunk : 0, t.rp, c);
  const double sm = red_sum(a.part + part_off(t, 2), lv ? t.nchunk : 0, t.rp, c);
  if (!red_lead() || c >= t.rp) return;
  a.cg.nrm[c] = lv ? sqrt(s) : 1.0;
  a.cg.isc[c] = lv ? 1.0 / sqrt(s) : 1.0;
  if (lv && lam) lam[c] = sa / s;
  // ||M u||^2 of the scaled state u = v / ||v||_M (the next solve's ||b||^2)
  if (lv) a.cg.bb_next[c] = sm / s;
}

// u *= mask, every column (region restriction of a state).
__global__ __launch_bounds__(kBlock) void k_apply_mask(StepArgs a, double* __restrict__ u) {
  const size_t total = size_t(a.t.n) * a.t.rp;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < total;
       i += size_t(gridDim.x) * kBlock)
    if (!a.mask[i]) u[i] = 0.0;
}

// Region adjacency: one thread per (row, restart); every neighbour of the row
// with another valid label marks the pair (all writers store 1).
__global__ __launch_bounds__(kBlock) void k_region_graph(StepArgs a, const int32_t* __restrict__ lab,
                                                         const int* __restrict__ off,
                                                         const int* __restrict__ mres, int nres,
                                                         uint8_t* __restrict__ adj) {
  const int n = a.t.n;
  const size_t total = size_t(n) * nres;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < total;
       i += size_t(gridDim.x) * kBlock) {
    const int r = int(i / n), row = int(i - size_t(r) * n);
    const int m = mres[r];
    const int32_t* lr = lab + size_t(r) * n;
    const int li = lr[row];
    if (li < 0 || li >= m) continue;
    for (int k = 1; k < a.W; ++k) {
      const int w = a.cols[size_t(k) * n + row];
      const int lw = lr[w];
      if (lw >= 0 && lw < m && lw != li) adj[off[r] + li * m + lw] = 1;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_scale(StepArgs a, const double* v, double* u) {
  const Tile& t = a.ts;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  if (g >= t.G) continue;
  const int c0 = 4 * g;
  int lv[4], any = 0;
  double inv[4];
  for (int j = 0; j < 4; ++j) {
    lv[j] = a.ct.live[c0 + j];
    any |= lv[j];
    inv[j] = 1.0 / a.cg.nrm[c0 + j];
  }
  if (!any) continue;
  const bool all = lv[0] && lv[1] && lv[2] && lv[3];
  for_rows(t, [&](int row) {
    const size_t o = size_t(row) * t.rp + c0;
    const V4<double> vv = ld4s(v + o);
    // columns that are not live keep their value (read only where needed)
    V4<double> uv = all ? vv : ld4s(u + o);
    for (int j = 0; j < 4; ++j)
      if (lv[j]) uv.v[j] = vv.v[j] * inv[j];
    st4s(u + o, uv);
  });
  }
}

// ---------------------------------------------------------------- energies --
// Rayleigh quotient parts u.Au and u.Mu per column.
__global__ __launch_bounds__(kBlock) void k_energy_rq(StepArgs a, const double* __restrict__ u) {
  const Tile& t = a.t64;
  for (int ct = 0; ct < t.nct; ++ct) {
  const int g = ct * t.tg + threadIdx.x % t.tg;
  double s[2][4] = {};
  if (g < t.G) {
    const int c0 = 4 * g;
    int lv[4], any = 0;
    for (int j = 0; j < 4; ++j) {
      lv[j] = a.ct.seg_len[c0 + j] > 0;
      any |= lv[j];
    }
    if (any) {
      for_rows(t, [&](int row) {
        double au[4] = {}, mu[4] = {};
        V4<double> ud = {};
        for_neighbors(a, row, c0, u, [&](int k, const V4<double>& x, size_t o) {
          const double va = ldm(a.A64 + o), vm = ldm(a.M64 + o);
          if (k == 0) ud = x;
          for (int j = 0; j < 4; ++j) {
            au[j] = fma(va, x.v[j], au[j]);
            mu[j] = fma(vm, x.v[j], mu[j]);
          }
        });
        for (int j = 0; j < 4; ++j)
          if (lv[j]) {
            s[0][j] += ud.v[j] * au[j];
            s[1][j] += ud.v[j] * mu[j];
          }
      });
    }
  }
  block_store<2>(t, s, a.part, blockIdx.x, ct);
  }
}

// Triangle traversal of the S_eps kernels.  Triangles are cut into chunks
// of sp.tchunk (they are sorted by their lowest vertex, so a chunk touches a
// compact set of rows); the chunks are split into 8 contiguous ranges, one
// per XCD (workgroup b runs on XCD b % 8), and an XCD's sp.nper workgroups
// take the chunks of its range cyclically, restart tile by restart tile, so
// at any moment an XCD works on one window of rows, which stays in its L2.
// f(tile, first chunk, end chunk, stride) runs once per tile; each
// workgroup writes one partial row (its index) per tile.
template <typename F>
__device__ __forceinline__ void for_seps_chunks(const SepsPlan& sp, F&& f) {
  const int xcd = blockIdx.x & 7, kb = blockIdx.x >> 3;
  const int cpx = (sp.nchunk + 7) / 8;
  const int cbeg = xcd * cpx, cend = min(cbeg + cpx, sp.nchunk);
  for (int tile = 0; tile < sp.ntile; ++tile) f(tile, cbeg + kb, cend, sp.nper);
}

// S_eps element kernel.  On a triangle T the P1 functions are u_i = sum_p
// a_ip b_p in the barycentric coordinates b_p, and
//   int_T b^alpha = 2|T| alpha! / (|alpha| + 2)!.
// For symmetric 3x3 G, H the quartic moment
//   B(G, H) = (360/|T|) sum_{pqrs} G_pq H_rs int_T b_p b_q b_r b_s
// equals, summing over the 24 permutations of the four slots,
//   S_G S_H + tr_G S_H + S_G tr_H + tr_G tr_H + 2 <G,H> + 4 g.h
//     + 4 dG.h + 4 g.dH + 6 dG.dH
// with S = 1^T X 1, tr = trace, g = G 1, h = H 1, dX = diag X.  Then
//   int_T sum_{i != j} u_i^2 u_j^2 = (2|T|/360) sum_i B(G_{<i}, a_i a_i^T),
//   G_{<i} = sum_{j<i} a_j a_j^T,
// a sum of nonnegative terms for nonnegative u (no cancellation).
// QuarticPairs accumulates sum_i B(G_{<i}, a_i a_i^T) over the components of
// one restart, fed in component order with their three corner values.
struct QuarticPairs {
  double g00 = 0, g11 = 0, g22 = 0, g01 = 0, g02 = 0, g12 = 0, acc = 0;
  __device__ __forceinline__ void add(double x0, double x1, double x2) {
    const double s1 = x0 + x1 + x2;
    const double q0 = x0 * x0, q1 = x1 * x1, q2 = x2 * x2;
    const double s2 = q0 + q1 + q2;
    const double trG = g00 + g11 + g22;
    const double SG = trG + 2.0 * (g01 + g02 + g12);
    const double gv0 = g00 + g01 + g02, gv1 = g01 + g11 + g12, gv2 = g02 + g12 + g22;
    const double ga = gv0 * x0 + gv1 * x1 + gv2 * x2;
    const double da = g00 * x0 + g11 * x1 + g22 * x2;
    const double gq = gv0 * q0 + gv1 * q1 + gv2 * q2;
    const double dq = g00 * q0 + g11 * q1 + g22 * q2;
    const double aGa = dq + 2.0 * (x0 * x1 * g01 + x0 * x2 * g02 + x1 * x2 * g12);
    acc += (SG + trG) * s1 * s1 + (SG + trG) * s2 + 2.0 * aGa + 4.0 * s1 * (ga + da) +
           4.0 * gq + 6.0 * dq;
    g00 += q0;
    g11 += q1;
    g22 += q2;
    g01 += x0 * x1;
    g02 += x0 * x2;
    g12 += x1 * x2;
  }
};

// The sum for one restart of m components whose corner values start at u0,
// u1, u2 (rows of global memory).  With 16-byte aligned starts the values
// are read two at a time (half the load instructions; each lane's loads walk
// one cache line).
// Sum over the triangle's component pairs for one restart of m components
// (corner rows u0, u1, u2); w (Scaled) holds per-component factors the
// values are multiplied by as they are read (deferred normalisation).
template <bool Scaled, typename WP = const double*>
__device__ __forceinline__ double quartic_pairs(const double* u0, const double* u1,
                                                const double* u2, WP w, int m) {
  QuarticPairs qp;
  int i = 0;
  if (((reinterpret_cast<size_t>(u0) | reinterpret_cast<size_t>(u1) |
        reinterpret_cast<size_t>(u2)) & 15) == 0) {
    // 8 components at a time: all 12 loads are issued before the recursion
    // uses them
    for (; i + 7 < m; i += 8) {
      double2 a0[4], a1[4], a2[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        a0[h] = *reinterpret_cast<const double2*>(u0 + i + 2 * h);
        a1[h] = *reinterpret_cast<const double2*>(u1 + i + 2 * h);
        a2[h] = *reinterpret_cast<const double2*>(u2 + i + 2 * h);
      }
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        if constexpr (Scaled) {
          const double wx = w[i + 2 * h], wy = w[i + 2 * h + 1];
          qp.add(a0[h].x * wx, a1[h].x * wx, a2[h].x * wx);
          qp.add(a0[h].y * wy, a1[h].y * wy, a2[h].y * wy);
        } else {
          qp.add(a0[h].x, a1[h].x, a2[h].x);
          qp.add(a0[h].y, a1[h].y, a2[h].y);
        }
      }
    }
    for (; i + 1 < m; i += 2) {
      const double2 a0 = *reinterpret_cast<const double2*>(u0 + i);
      const double2 a1 = *reinterpret_cast<const double2*>(u1 + i);
      const double2 a2 = *reinterpret_cast<const double2*>(u2 + i);
      if constexpr (Scaled) {
        const double wx = w[i], wy = w[i + 1];
        qp.add(a0.x * wx, a1.x * wx, a2.x * wx);
        qp.add(a0.y * wy, a1.y * wy, a2.y * wy);
      } else {
        qp.add(a0.x, a1.x, a2.x);
        qp.add(a0.y, a1.y, a2.y);
      }
    }
  }
  for (; i < m; ++i) {
    if constexpr (Scaled)
      qp.add(u0[i] * w[i], u1[i] * w[i], u2[i] * w[i]);
    else
      qp.add(u0[i], u1[i], u2[i]);
  }
  return qp.acc;
}

// Element kernel with LDS staging.  Thread (tb, rr) of a workgroup runs the
// quartic of restart rr of the tile on triangle tb of the current pass (TB =
// 256 / nr triangles per pass, so every thread works).  The components are
// taken kSepsPiece at a time: the workgroup first copies, for every
// (triangle, corner, restart), the restart's next kSepsPiece values of that
// corner row (contiguous in memory, 16-byte loads) into LDS rows padded to an
// odd length, so the threads of a wave read different banks; the quartic
// state stays in registers between pieces.
constexpr int kSepsPiece = 8;
constexpr int kSepsPad = kSepsPiece + 1;
constexpr int kSepsCols = 256;  // column budget of a restart tile

__global__ __launch_bounds__(kBlock) void k_energy_seps(StepArgs a, SepsPlan sp,
                                                        const int* __restrict__ tri,
                                                        const double* __restrict__ tarea,
                                                        const double* __restrict__ u,
                                                        double* __restrict__ part_s) {
  constexpr int kHalves = kSepsPiece / 2;        // 16-byte items per staged row
  __shared__ double sh[kBlock * 3 * kSepsPad];   // staged rows (triangle, corner, restart)
  __shared__ long long s_off[kBlock * 3];        // their source offsets (-1: no triangle)
  __shared__ int s_len[kBlock * 3];              // and their restart's m
  __shared__ int s_lo[64], s_m[64];              // the tile's restarts
  __shared__ double red[kBlock];
  const int rp = a.t.rp;
  const int tid = threadIdx.x;
  for_seps_chunks(sp, [&](int tile, int cb, int ce, int stride) {
    const int4 tl = sp.tiles[tile];
    const int r0 = tl.x, nr = max(tl.y - tl.x, 1);
    const int TB = kBlock / nr;
    const int tb = tid / nr, rr = tid % nr;
    const bool worker = tb < TB;
    const int nrow = TB * 3 * nr;
    if (tid < nr) {
      s_lo[tid] = a.ct.res_lo[r0 + tid];
      s_m[tid] = a.ct.res_len[r0 + tid];
    }
    __syncthreads();
    int mmax = 0;
    for (int q = 0; q < nr; ++q) mmax = max(mmax, s_m[q]);
    const int lo = worker ? s_lo[rr] : 0, m = worker ? s_m[rr] : 0;
    double acc = 0.0;
    for (int chunk = cb; chunk < ce; chunk += stride) {
      const int t_beg = chunk * sp.tchunk, t_end = min(t_beg + sp.tchunk, sp.nt);
      for (int t0 = t_beg; t0 < t_end; t0 += TB) {
        // row (bq * 3 + k) * nr + q: corner k of triangle t0 + bq, restart q
        for (int row3 = tid; row3 < nrow; row3 += kBlock) {
          const int q = row3 % nr, bk = row3 / nr;
          const int bq = bk / 3, k = bk - 3 * bq;
          const int tt = t0 + bq;
          s_off[row3] = tt < t_end ? (long long)tri[3 * tt + k] * rp + s_lo[q] : -1;
          s_len[row3] = s_m[q];
        }
        const int t = t0 + tb;
        QuarticPairs qp;
        for (int i0 = 0; i0 < mmax; i0 += kSepsPiece) {
          __syncthreads();
          for (int it = tid; it < nrow * kHalves; it += kBlock) {
            const int row3 = it / kHalves, h = it % kHalves;
            const long long off = s_off[row3];
            const int i = i0 + 2 * h, len = s_len[row3];
            double vx = 0.0, vy = 0.0;
            if (off >= 0) {
              const int cl = s_lo[row3 % nr] + i;
              if (i < len) vx = u[off + i] * (a.usc ? a.usc[cl] : 1.0);
              if (i + 1 < len) vy = u[off + i + 1] * (a.usc ? a.usc[cl + 1] : 1.0);
            }
            double* dst = sh + row3 * kSepsPad + 2 * h;
            dst[0] = vx;
            dst[1] = vy;
          }
          __syncthreads();
          if (worker && t < t_end) {
            const double* b0 = sh + ((tb * 3 + 0) * nr + rr) * kSepsPad;
            const double* b1 = sh + ((tb * 3 + 1) * nr + rr) * kSepsPad;
            const double* b2 = sh + ((tb * 3 + 2) * nr + rr) * kSepsPad;
            const int n = min(kSepsPiece, m - i0);
            for (int i = 0; i < n; ++i) qp.add(b0[i], b1[i], b2[i]);
          }
        }
        if (worker && t < t_end && m > 0) acc += qp.acc * tarea[t] * (1.0 / 180.0);
        __syncthreads();
      }
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < nr) {
      double sum = 0.0;
      for (int bq = 0; bq < TB; ++bq) sum += red[bq * nr + tid];
      part_s[size_t(blockIdx.x) * sp.nres_p + r0 + tid] = sum;
    }
    __syncthreads();
  });
}

// Direct variant: no staging.  A workgroup holds 256/nrp triangles x nrp
// restart lanes (nrp = restarts of the tile rounded up to a power of two);
// each lane reads its restart's m corner values straight from global memory
// (lanes of one triangle read adjacent segments of the same rows).
template <bool Scaled>
__global__ __launch_bounds__(kBlock) void k_energy_seps_direct(StepArgs a, SepsPlan sp,
                                                               const int* __restrict__ tri,
                                                               const double* __restrict__ tarea,
                                                               const double* __restrict__ u,
                                                               double* __restrict__ part_s) {
  __shared__ double red[kBlock];
  __shared__ double s_w[kSepsCols];  // the tile's column factors (Scaled)
  const int rp = a.t.rp;
  const int tid = threadIdx.x;
  for_seps_chunks(sp, [&](int tile, int cb, int ce, int stride) {
    const int4 tl = sp.tiles[tile];
    if (Scaled) {
      // the host flushes the factors instead when a tile is wider
      for (int c = tid; c < tl.w - tl.z; c += kBlock) s_w[c] = a.usc[tl.z + c];
      __syncthreads();
    }
    const int r0 = tl.x, nr = tl.y - tl.x;
    int nrp = 1;
    while (nrp < nr) nrp <<= 1;
    const int TB = kBlock / nrp;
    const int tb = tid / nrp, rr = tid % nrp;
    int lo = 0, m = 0;
    if (rr < nr) {
      lo = a.ct.res_lo[r0 + rr];
      m = a.ct.res_len[r0 + rr];
    }
    double acc = 0.0;
    if (m > 0) {
      typedef const __attribute__((address_space(3))) double* LdsPtr;
      const LdsPtr w = (LdsPtr)(s_w + (Scaled ? lo - tl.z : 0));
      for (int chunk = cb; chunk < ce; chunk += stride) {
        const int t_beg = chunk * sp.tchunk, t_end = min(t_beg + sp.tchunk, sp.nt);
        for (int t = t_beg + tb; t < t_end; t += TB)
          acc += quartic_pairs<Scaled>(u + size_t(tri[3 * t + 0]) * rp + lo,
                                       u + size_t(tri[3 * t + 1]) * rp + lo,
                                       u + size_t(tri[3 * t + 2]) * rp + lo, w, m) *
                 tarea[t] * (1.0 / 180.0);
      }
    }
    red[tid] = acc;
    for (int st = TB >> 1; st >= 1; st >>= 1) {
      __syncthreads();
      if (tb < st) red[tid] += red[tid + st * nrp];
    }
    __syncthreads();
    if (tb == 0 && rr < nr) part_s[size_t(blockIdx.x) * sp.nres_p + r0 + rr] = red[tid];
    __syncthreads();
  });
}

// Lane-split variant for tiles whose restarts start and end on 4-column
// boundaries.  One wavefront takes one triangle and one restart tile (at most
// 256 columns = 64 lanes x 4): lane l owns columns c0 + 4l .. +3, so the
// wavefront reads each corner row of the tile as one contiguous run.  A lane
// runs the prefix recursion over its 4 components from zero (local sum and
// H_l = sum a a^T), the lanes of each restart take an exclusive prefix of H
// (shuffles), and since B is bilinear the lane's share is
//   local + B(G_before, H_l),  G_before = sum of H over the restart's lower lanes.
// Scaled: the lane's four column factors (deferred normalisation) are read
// once per tile.  The kernel is bound by load latency, so its registers are
// capped for 7 waves per SIMD; the triangle index is wave-uniform, so the
// corner indices and areas come through scalar loads.
__device__ __forceinline__ double quartic_b(const double (&G)[6], const double (&H)[6]) {
  // symmetric 3x3 as (00, 11, 22, 01, 02, 12)
  const double trG = G[0] + G[1] + G[2], trH = H[0] + H[1] + H[2];
  const double SG = trG + 2.0 * (G[3] + G[4] + G[5]), SH = trH + 2.0 * (H[3] + H[4] + H[5]);
  const double gi[3] = {G[0] + G[3] + G[4], G[3] + G[1] + G[5], G[4] + G[5] + G[2]};
  const double hi[3] = {H[0] + H[3] + H[4], H[3] + H[1] + H[5], H[4] + H[5] + H[2]};
  const double GH = G[0] * H[0] + G[1] * H[1] + G[2] * H[2] +
                    2.0 * (G[3] * H[3] + G[4] * H[4] + G[5] * H[5]);
  double gh = 0, dgh = 0, gdh = 0, dgdh = 0;
  for (int q = 0; q < 3; ++q) {
    gh += gi[q] * hi[q];
    dgh += G[q] * hi[q];
    gdh += gi[q] * H[q];
    dgdh += G[q] * H[q];
  }
  return (SG + trG) * (SH + trH) + 2.0 * GH + 4.0 * (gh + dgh + gdh) + 6.0 * dgdh;
}

template <bool Scaled>
__global__ __launch_bounds__(kBlock, 7) void k_energy_seps_lanes(StepArgs a, SepsPlan sp,
                                                              const int* __restrict__ tri,
                                                              const double* __restrict__ tarea,
                                                              const double* __restrict__ u,
                                                              double* __restrict__ part_s) {
  __shared__ double red[kBlock];
  const int rp = a.t.rp;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int kW = kBlock / 64;
  for_seps_chunks(sp, [&](int tile, int cb, int ce, int stride) {
    const int4 tl = sp.tiles[tile];
    const int r0 = tl.x, c0 = tl.z, ncol = tl.w - tl.z;
    const int c = c0 + 4 * lane;
    const bool on = 4 * lane < ncol;
    // the lane's restart and its position among the restart's lanes; lanes
    // per restart at most kmax (the prefix needs log2(kmax) shuffle steps)
    int k = 0;
    if (on) k = (c - a.ct.seg_lo[c]) >> 2;
    int kmax = 1;
    for (int q = tl.x; q < tl.y; ++q) kmax = max(kmax, a.ct.res_len[q] >> 2);
    double acc = 0.0;
    V4<double> w = {};  // the lane's column factors (Scaled), loaded once per tile
    if (Scaled && on) w = ld4(a.usc + c);
    for (int chunk = cb; chunk < ce; chunk += stride) {
      const int t_beg = chunk * sp.tchunk, t_end = min(t_beg + sp.tchunk, sp.nt);
      for (int t = t_beg + wave; t < t_end; t += kW) {
        double H[6] = {0, 0, 0, 0, 0, 0}, loc = 0.0;
        if (on) {
          const double* p0 = u + size_t(tri[3 * t + 0]) * rp + c;
          const double* p1 = u + size_t(tri[3 * t + 1]) * rp + c;
          const double* p2 = u + size_t(tri[3 * t + 2]) * rp + c;
          V4<double> x0 = ld4(p0), x1 = ld4(p1), x2 = ld4(p2);
          if constexpr (Scaled) {
            for (int j = 0; j < 4; ++j) {
              x0.v[j] *= w.v[j];
              x1.v[j] *= w.v[j];
              x2.v[j] *= w.v[j];
            }
          }
          QuarticPairs qp;
          for (int j = 0; j < 4; ++j) qp.add(x0.v[j], x1.v[j], x2.v[j]);
          loc = qp.acc;
          H[0] = qp.g00;
          H[1] = qp.g11;
          H[2] = qp.g22;
          H[3] = qp.g01;
          H[4] = qp.g02;
          H[5] = qp.g12;
        }
        // inclusive prefix of H over the restart's lanes (k = position)
        double P[6];
        for (int q = 0; q < 6; ++q) P[q] = H[q];
        for (int d = 1; d < kmax; d <<= 1) {
          double up[6];
          for (int q = 0; q < 6; ++q) up[q] = __shfl_up(P[q], d);
          if (k >= d)
            for (int q = 0; q < 6; ++q) P[q] += up[q];
        }
        double G[6];
        for (int q = 0; q < 6; ++q) G[q] = P[q] - H[q];  // exclusive
        if (on && k > 0) loc += quartic_b(G, H);
        if (on) acc += loc * tarea[t] * (1.0 / 180.0);
      }
    }
    // per restart: its lanes, then the workgroup's wavefronts, in order
    red[tid] = acc;
    __syncthreads();
    const int nr = tl.y - tl.x;
    if (tid < nr) {
      const int lo = a.ct.res_lo[r0 + tid], m = a.ct.res_len[r0 + tid];
      double sum = 0.0;
      if (m > 0) {
        const int l0 = (lo - c0) >> 2, l1 = (lo - c0 + m) >> 2;
        for (int w = 0; w < kW; ++w)
          for (int l = l0; l < l1; ++l) sum += red[w * 64 + l];
      }
      part_s[size_t(blockIdx.x) * sp.nres_p + r0 + tid] = sum;
    }
    __syncthreads();
  });
}

// Coupling term of the Lagrange multipliers: P_i = int u_i^2 sum_{j != i}
// u_j^2 per column, = (|T|/360) B(G - a_i a_i^T, a_i a_i^T) per triangle with
// G = sum_j a_j a_j^T over the restart's components (B as above).  Layout of
// the direct S_eps kernel (one lane per restart and triangle); components in
// blocks of 8 accumulated in registers, G recomputed per block; the block
// loop runs to the tile's largest m so every thread reaches the barriers.
// part [8 nper][rp]: one partial per workgroup and column (lane order fixed).
__global__ __launch_bounds__(kBlock) void k_multipliers(StepArgs a, SepsPlan sp,
                                                        const int* __restrict__ tri,
                                                        const double* __restrict__ tarea,
                                                        const double* __restrict__ u,
                                                        double* __restrict__ part) {
  __shared__ double red[kBlock];
  const int rp = a.t.rp;
  const int tid = threadIdx.x;
  for_seps_chunks(sp, [&](int tile, int cb, int ce, int stride) {
    const int4 tl = sp.tiles[tile];
    const int r0 = tl.x, nr = tl.y - tl.x;
    int nrp = 1;
    while (nrp < nr) nrp <<= 1;
    const int TB = kBlock / nrp;
    const int tb = tid / nrp, rr = tid % nrp;
    int lo = 0, m = 0, mmax = 0;
    for (int q = 0; q < nr; ++q) mmax = max(mmax, a.ct.res_len[r0 + q]);
    if (rr < nr) {
      lo = a.ct.res_lo[r0 + rr];
      m = a.ct.res_len[r0 + rr];
    }
    for (int kb = 0; kb < mmax; kb += 8) {
      double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (kb < m)
        for (int chunk = cb; chunk < ce; chunk += stride) {
          const int t_beg = chunk * sp.tchunk, t_end = min(t_beg + sp.tchunk, sp.nt);
          for (int t = t_beg + tb; t < t_end; t += TB) {
            const double* c0 = u + size_t(tri[3 * t + 0]) * rp + lo;
            const double* c1 = u + size_t(tri[3 * t + 1]) * rp + lo;
            const double* c2 = u + size_t(tri[3 * t + 2]) * rp + lo;
            double G[6] = {0, 0, 0, 0, 0, 0};
            for (int i = 0; i < m; ++i) {
              const double x0 = c0[i], x1 = c1[i], x2 = c2[i];
              G[0] = fma(x0, x0, G[0]);
              G[1] = fma(x1, x1, G[1]);
              G[2] = fma(x2, x2, G[2]);
              G[3] = fma(x0, x1, G[3]);
              G[4] = fma(x0, x2, G[4]);
              G[5] = fma(x1, x2, G[5]);
            }
            const double w = tarea[t] * (1.0 / 360.0);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              if (kb + j >= m) break;
              const double x0 = c0[kb + j], x1 = c1[kb + j], x2 = c2[kb + j];
              const double H[6] = {x0 * x0, x1 * x1, x2 * x2, x0 * x1, x0 * x2, x1 * x2};
              double R[6];
              for (int q = 0; q < 6; ++q) R[q] = G[q] - H[q];
              acc[j] = fma(quartic_b(R, H), w, acc[j]);
            }
          }
        }
      for (int j = 0; j < 8; ++j) {
        red[tid] = acc[j];
        for (int st = TB >> 1; st >= 1; st >>= 1) {
          __syncthreads();
          if (tb < st) red[tid] += red[tid + st * nrp];
        }
        __syncthreads();
        if (tb == 0 && rr < nr && kb + j < m) part[size_t(blockIdx.x) * rp + lo + kb + j] = red[tid];
        __syncthreads();
      }
    }
  });
}

// lambda^eps_c = lambda_c + (2 / eps^2) sum over workgroups of the partials
// (fixed order); 2 / eps^2 = coef / tau.
__global__ void k_red_multipliers(StepArgs a, SepsPlan sp, const double* __restrict__ part,
                                  const double* __restrict__ lam, double* __restrict__ out) {
  const int c = red_col();
  const bool real = c < a.t.rp && a.ct.seg_len[c] > 0;
  const double p = red_sum(part, real ? 8 * sp.nper : 0, a.t.rp, c);
  if (!red_lead() || c >= a.t.rp) return;
  out[c] = real ? lam[c] + (a.ct.coef[c] / a.tau) * p : 0.0;
}

__global__ void k_red_lambda(StepArgs a, double* __restrict__ lam) {
  const int c = red_col();
  const Tile& t = a.t64;
  const bool real = c < t.rp && a.ct.seg_len[c] > 0;
  const double num = red_sum(a.part + part_off(t, 0), real ? t.nchunk : 0, t.rp, c);
  const double den = red_sum(a.part + part_off(t, 1), real ? t.nchunk : 0, t.rp, c);
  if (!red_lead() || c >= t.rp) return;
  lam[c] = real ? num / den : 0.0;
}

__global__ void k_red_seps(StepArgs a, SepsPlan sp, const double* __restrict__ part_s,
                           const double* __restrict__ lam, double* __restrict__ seps,
                           double* __restrict__ energy) {
  // one partial per element-kernel workgroup and restart, summed by
  // kRL lanes per restart in a fixed order
  const int r = red_col();
  const double ps = red_sum(part_s, r < a.ct.nres ? 8 * sp.nper : 0, sp.nres_p, r);
  if (!red_lead() || r >= a.ct.nres) return;
  const double s = ps * a.ct.res_ieps2[r];
  double e = s;
  const int lo = a.ct.res_lo[r], m = a.ct.res_len[r];
  for (int i = 0; i < m; ++i) e += lam[lo + i];
  seps[r] = s;
  energy[r] = e;
}

// ------------------------------------------------ small batches, one launch --
// Whole time steps of a small batch (n * rp <= kSmallMaxValues) in one
// workgroup that stays resident for all the steps of the launch: the float64
// CG from x0 = u (as the plain float64 form), the node step, the norm pass,
// the scaling and, at the energy cadence, Rayleigh quotients (from the norm
// pass), S_eps and E.  Phases are separated by workgroup barriers instead of
// kernel launches, and there is no host round trip per CG iteration.
//
// Thread mapping: column group g = tid % gp (gp = G rounded up to a power of
// two; lanes with g >= G idle) and row lane tid / gp, rows row-lane, + RL, ...
// Per-column sums in a fixed order (small_sum), so results do not depend on
// timing.
constexpr int kSmallBlock = 512;

struct SmallScal {
  double rz[kSmallMaxCols], tol2[kSmallMaxCols], alpha[kSmallMaxCols], beta[kSmallMaxCols];
  double nrm[kSmallMaxCols];
  int act[kSmallMaxCols];
  int nact;
};

// Sum v (4 columns per thread) over the threads of each column group: a
// butterfly inside each wavefront (lanes l and l ^ off, off a multiple of gp,
// share the group), the sums of lane l < gp of every wavefront into LDS, then
// one thread per column adds the wavefronts in order.  The total of column c
// is left in tot[c].  Every thread must call it.
constexpr int kSmallWaves = kSmallBlock / 64;

__device__ __forceinline__ void small_sum(double* red, double* tot, double v0, double v1,
                                          double v2, double v3, int gp) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double v[4] = {v0, v1, v2, v3};
  for (int off = 32; off >= gp; off >>= 1)
    for (int j = 0; j < 4; ++j) v[j] += __shfl_xor(v[j], off);
  if (lane < gp)
    for (int j = 0; j < 4; ++j) red[(wave * gp + lane) * 4 + j] = v[j];
  __syncthreads();
  if (tid < 4 * gp) {
    const int gq = tid >> 2, j = tid & 3;
    double sum = 0.0;
    for (int w = 0; w < kSmallWaves; ++w) sum += red[(w * gp + gq) * 4 + j];
    tot[tid] = sum;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kSmallBlock) void k_small_steps(StepArgs a, SmallArgs sa) {
  __shared__ double red[kSmallWaves * 64 * 4];
  __shared__ double tot[4 * 64];
  __shared__ SmallScal cs;
  const int tid = threadIdx.x;
  const int n = a.t.n, rp = a.t.rp, G = rp / 4, W = a.W;
  int gp = 1;
  while (gp < G) gp <<= 1;
  const int g = tid % gp, RL = kSmallBlock / gp, rl = tid / gp;
  const bool valid = g < G;
  const int c0 = 4 * g;
  double* u = sa.u;
  double* r = sa.r;
  double* p = sa.p;
  double* q = sa.q;
  int lv[4] = {0, 0, 0, 0}, seg_lo[4] = {0, 0, 0, 0}, seg_len[4] = {0, 0, 0, 0};
  double coef[4] = {0, 0, 0, 0};
  int any_live = 0;
  if (valid)
    for (int j = 0; j < 4; ++j) {
      lv[j] = a.ct.live[c0 + j];
      seg_lo[j] = a.ct.seg_lo[c0 + j];
      seg_len[j] = a.ct.seg_len[c0 + j];
      coef[j] = a.ct.coef[c0 + j];
      any_live |= lv[j];
    }
  // gather helper: acc_k += sum over the row's slots of mat[slot] * x[col]
  auto gather = [&](int row, const double* x, auto&& f) {
    for (int k = 0; k < W; ++k) {
      const size_t o = size_t(k) * n + row;
      const int cidx = ldm(a.cols + o);
      f(k, o, ld4(x + size_t(cidx) * rp + c0));
    }
  };

  for (int step = 0; step < sa.nsteps; ++step) {
    // ---- heat: CG on (M + tau A) x = M u from x = u, r = -tau A u
    {
      double sb[4] = {}, sz[4] = {}, sr[4] = {};
      if (valid && any_live)
        for (int row = rl; row < n; row += RL) {
          double au[4] = {}, mu[4] = {};
          gather(row, u, [&](int, size_t o, const V4<double>& x) {
            const double va = ldm(a.A64 + o), vm = ldm(a.M64 + o);
            for (int j = 0; j < 4; ++j) {
              au[j] = fma(va, x.v[j], au[j]);
              mu[j] = fma(vm, x.v[j], mu[j]);
            }
          });
          const double di = a.dinv64[row];
          V4<double> rv, pv;
          for (int j = 0; j < 4; ++j) {
            rv.v[j] = lv[j] ? -a.tau * au[j] : 0.0;
            pv.v[j] = di * rv.v[j];
            if (lv[j]) sb[j] += mu[j] * mu[j];
            sz[j] += rv.v[j] * pv.v[j];
            sr[j] += rv.v[j] * rv.v[j];
          }
          st4(r + size_t(row) * rp + c0, rv);
          st4(p + size_t(row) * rp + c0, pv);
        }
      double bb = 0, rz = 0, rr = 0;
      small_sum(red, tot, sb[0], sb[1], sb[2], sb[3], gp);
      if (tid < rp) bb = tot[tid];
      __syncthreads();
      small_sum(red, tot, sz[0], sz[1], sz[2], sz[3], gp);
      if (tid < rp) rz = tot[tid];
      __syncthreads();
      small_sum(red, tot, sr[0], sr[1], sr[2], sr[3], gp);
      if (tid < rp) rr = tot[tid];
      if (tid == 0) cs.nact = 0;
      __syncthreads();
      if (tid < rp) {
        const int act = (a.ct.live[tid] && rr > a.rtol2 * bb) ? 1 : 0;
        a.cg.bb[tid] = bb;
        cs.rz[tid] = rz;
        cs.tol2[tid] = a.rtol2 * bb;
        cs.act[tid] = act;
        cs.alpha[tid] = 0.0;
        cs.beta[tid] = 0.0;
        if (act) atomicAdd(&cs.nact, 1);
      }
      __syncthreads();
    }
    for (int it = 0; it < sa.max_iter && cs.nact > 0; ++it) {
      if (tid == 0) {
        a.stat[0] += 1;
        a.stat[3] += cs.nact;
      }
      int act[4] = {0, 0, 0, 0}, any = 0;
      if (valid)
        for (int j = 0; j < 4; ++j) {
          act[j] = cs.act[c0 + j];
          any |= act[j];
        }
      // q = K p, p.q
      double spq[4] = {};
      if (any)
        for (int row = rl; row < n; row += RL) {
          V4<double> acc = {}, pd = {};
          gather(row, p, [&](int k, size_t o, const V4<double>& x) {
            const double v = ldm(a.K64 + o);
            if (k == 0) pd = x;
            for (int j = 0; j < 4; ++j) acc.v[j] = fma(v, x.v[j], acc.v[j]);
          });
          st4(q + size_t(row) * rp + c0, acc);
          for (int j = 0; j < 4; ++j)
            if (act[j]) spq[j] += pd.v[j] * acc.v[j];
        }
      small_sum(red, tot, spq[0], spq[1], spq[2], spq[3], gp);
      if (tid < rp) cs.alpha[tid] = (cs.act[tid] && tot[tid] > 0.0) ? cs.rz[tid] / tot[tid] : 0.0;
      __syncthreads();
      // x += alpha p, r -= alpha q, z = D r; r.z and r.r
      double al[4] = {0, 0, 0, 0};
      for (int j = 0; j < 4; ++j) al[j] = valid ? cs.alpha[c0 + j] : 0.0;
      double szn[4] = {}, srn[4] = {};
      if (any)
        for (int row = rl; row < n; row += RL) {
          const size_t o = size_t(row) * rp + c0;
          V4<double> xv = ld4(u + o), rv = ld4(r + o);
          const V4<double> pv = ld4(p + o), qv = ld4(q + o);
          const double di = a.dinv64[row];
          for (int j = 0; j < 4; ++j)
            if (act[j]) {
              xv.v[j] = fma(al[j], pv.v[j], xv.v[j]);
              rv.v[j] = fma(-al[j], qv.v[j], rv.v[j]);
              szn[j] += rv.v[j] * (di * rv.v[j]);
              srn[j] += rv.v[j] * rv.v[j];
            }
          st4(u + o, xv);
          st4(r + o, rv);
        }
      double rzn = 0, rrn = 0;
      small_sum(red, tot, szn[0], szn[1], szn[2], szn[3], gp);
      if (tid < rp) rzn = tot[tid];
      __syncthreads();
      small_sum(red, tot, srn[0], srn[1], srn[2], srn[3], gp);
      if (tid < rp) rrn = tot[tid];
      if (tid == 0) cs.nact = 0;
      __syncthreads();
      if (tid < rp && cs.act[tid]) {
        a.cg.iters[tid] += 1;
        if (rrn <= cs.tol2[tid] || !(rrn == rrn)) {
          cs.act[tid] = 0;
          cs.beta[tid] = 0.0;
        } else {
          cs.beta[tid] = rzn / cs.rz[tid];
          cs.rz[tid] = rzn;
          atomicAdd(&cs.nact, 1);
        }
      }
      __syncthreads();
      // p = D r + beta p on the columns still iterating
      int still[4] = {0, 0, 0, 0}, anys = 0;
      double be[4] = {0, 0, 0, 0};
      if (valid)
        for (int j = 0; j < 4; ++j) {
          still[j] = cs.act[c0 + j];
          be[j] = cs.beta[c0 + j];
          anys |= still[j];
        }
      if (anys)
        for (int row = rl; row < n; row += RL) {
          const size_t o = size_t(row) * rp + c0;
          V4<double> pv = ld4(p + o);
          const V4<double> rv = ld4(r + o);
          const double di = a.dinv64[row];
          for (int j = 0; j < 4; ++j)
            if (still[j]) pv.v[j] = fma(be[j], pv.v[j], di * rv.v[j]);
          st4(p + o, pv);
        }
      __syncthreads();
    }
    if (tid == 0 && cs.nact > 0) a.stat[2] = 1;  // iteration cap hit
    __syncthreads();
    // ---- node step (into r): u^_i = u~_i exp(-coef (S - u~_i^2))
    if (valid && any_live)
      for (int row = rl; row < n; row += RL) {
        const double* ur = u + size_t(row) * rp;
        V4<double> uv = ld4(ur + c0), ov = uv;
        double S = 0.0;
        int cur = -1;
        for (int j = 0; j < 4; ++j) {
          if (!lv[j]) continue;
          if (seg_lo[j] != cur) {
            cur = seg_lo[j];
            S = 0.0;
            for (int i = 0; i < seg_len[j]; ++i) {
              const double w = ur[seg_lo[j] + i];
              S = fma(w, w, S);
            }
          }
          const double x = uv.v[j];
          ov.v[j] = x * exp(-coef[j] * (S - x * x));
        }
        st4(r + size_t(row) * rp + c0, ov);
      }
    __syncthreads();
    // ---- norm pass: v.Mv, v.Av of v = u^ (gathered from r)
    {
      double sm[4] = {}, sa2[4] = {};
      if (valid && any_live)
        for (int row = rl; row < n; row += RL) {
          double mv[4] = {}, av[4] = {};
          V4<double> vd = {};
          gather(row, r, [&](int k, size_t o, const V4<double>& x) {
            const double wm = ldm(a.M64 + o), z = ldm(a.A64 + o);
            if (k == 0) vd = x;
            for (int j = 0; j < 4; ++j) {
              mv[j] = fma(wm, x.v[j], mv[j]);
              av[j] = fma(z, x.v[j], av[j]);
            }
          });
          for (int j = 0; j < 4; ++j)
            if (lv[j]) {
              sm[j] += vd.v[j] * mv[j];
              sa2[j] += vd.v[j] * av[j];
            }
        }
      double vm = 0, va = 0;
      small_sum(red, tot, sm[0], sm[1], sm[2], sm[3], gp);
      if (tid < rp) vm = tot[tid];
      __syncthreads();
      small_sum(red, tot, sa2[0], sa2[1], sa2[2], sa2[3], gp);
      if (tid < rp) va = tot[tid];
      if (tid < rp) {
        const bool l = a.ct.live[tid] != 0;
        cs.nrm[tid] = l ? sqrt(vm) : 1.0;
        a.cg.nrm[tid] = cs.nrm[tid];
        if (l) sa.lam[tid] = va / vm;
      }
      __syncthreads();
    }
    // ---- scale: u = u^ / ||u^||_M on the live columns
    if (valid && any_live) {
      double inv[4];
      for (int j = 0; j < 4; ++j) inv[j] = 1.0 / cs.nrm[c0 + j];
      for (int row = rl; row < n; row += RL) {
        const size_t o = size_t(row) * rp + c0;
        const V4<double> vv = ld4(r + o);
        V4<double> uv = ld4(u + o);
        for (int j = 0; j < 4; ++j)
          if (lv[j]) uv.v[j] = vv.v[j] * inv[j];
        st4(u + o, uv);
      }
    }
    __syncthreads();
    // ---- energy at the cadence: S_eps per restart, E = sum lambda + S_eps
    if (sa.every > 0 && (sa.step0 + step + 1) % sa.every == 0) {
      const int nres = a.ct.nres;
      int np2 = 1;
      while (np2 < nres) np2 <<= 1;
      const int rr = tid % np2, tl = tid / np2, TL = kSmallBlock / np2;
      double acc[4] = {0, 0, 0, 0};
      if (rr < nres) {
        const int lo = a.ct.res_lo[rr], m = a.ct.res_len[rr];
        if (m > 0)
          for (int t = tl; t < sa.nt; t += TL)
            acc[0] += quartic_pairs<false>(u + size_t(sa.tri[3 * t + 0]) * rp + lo,
                                           u + size_t(sa.tri[3 * t + 1]) * rp + lo,
                                           u + size_t(sa.tri[3 * t + 2]) * rp + lo, nullptr, m) *
                      sa.tarea[t] * (1.0 / 180.0);
      }
      // per-restart sums: small_sum with np2 as the group width (slot 0)
      small_sum(red, tot, acc[0], 0.0, 0.0, 0.0, np2);
      if (tid < nres) {
        const double se = tot[tid * 4] * a.ct.res_ieps2[tid];
        const int lo = a.ct.res_lo[tid], m = a.ct.res_len[tid];
        double e = se;
        for (int i = 0; i < m; ++i) e += sa.lam[lo + i];
        sa.seps[tid] = se;
        sa.energy[tid] = e;
        if (sa.hist) sa.hist[size_t(step) * a.ct.nres_p + tid] = e;
      }
      __syncthreads();
    }
  }
}

// ----------------------------------------------------------------- labels --
// Equation (vi): v_i = u_i - sum_{j != i} u_j = 2 u_i - sum_j u_j; label =
// argmax_i v_i if positive else -1; second labelling = argmax_i u_i (lowest
// index wins ties in both).
__global__ void k_labels(StepArgs a, const double* __restrict__ u, const int* __restrict__ perm,
                         int* __restrict__ lab, int* __restrict__ lab_am) {
  const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t nres = size_t(a.ct.nres);
  if (idx >= size_t(a.t.n) * nres) return;
  const int row = int(idx / nres), r = int(idx % nres);
  const int lo = a.ct.res_lo[r], m = a.ct.res_len[r];
  const double* ur = u + size_t(row) * a.t.rp + lo;
  double tot = 0.0;
  for (int i = 0; i < m; ++i) tot += ur[i];
  int best = 0, am = 0;
  double vb = 2.0 * ur[0] - tot, ub = ur[0];
  for (int i = 1; i < m; ++i) {
    const double v = 2.0 * ur[i] - tot;
    if (v > vb) { vb = v; best = i; }
    if (ur[i] > ub) { ub = ur[i]; am = i; }
  }
  const size_t o = size_t(r) * a.t.n + perm[row];
  if (lab) lab[o] = vb > 0.0 ? best : -1;
  if (lab_am) lab_am[o] = am;
}

// ---------------------------------------------------------- layout changes --
// Caller layout [Rq][n] (component-major, caller vertex numbering) <->
// columns [c_lo, c_lo + Rq) of the [n][rp] state (renumbered rows).
__global__ void k_pack(size_t total, int rp, int n, int c_lo, int Rq, const double* __restrict__ u0,
                       const int* __restrict__ perm, double* __restrict__ u) {
  const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int row = int(idx / Rq), c = int(idx % Rq);
  u[size_t(row) * rp + c_lo + c] = u0[size_t(c) * n + perm[row]];
}

__global__ void k_unpack(size_t total, int rp, int n, int c_lo, int Rq, const double* __restrict__ u,
                         const int* __restrict__ perm, double* __restrict__ out) {
  const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int row = int(idx / Rq), c = int(idx % Rq);
  out[size_t(c) * n + perm[row]] = u[size_t(row) * rp + c_lo + c];
}

inline unsigned nblocks(size_t work, int bs = kBlock) { return unsigned((work + bs - 1) / bs); }
// blocks of the column reductions (kRC columns per block)
inline unsigned colblocks(const Tile& t) { return nblocks(size_t(t.rp), kRC); }

#define SP_LAUNCH_CHECK() SP_HIP(hipGetLastError())

}  // namespace

Tile make_tile(int n, int rp, int tg_cap, int passes, int nper_cap) {
  Tile t;
  t.n = n;
  t.rp = rp;
  t.G = rp / 4;
  tg_cap = std::max(1, std::min(tg_cap, 64));
  int tg = 1;
  while (tg < t.G && tg < tg_cap) tg <<= 1;
  t.tg = tg;
  t.tr = kBlock / tg;
  t.nct = (t.G + tg - 1) / tg;
  t.xrows = (n + 7) / 8;
  passes = std::max(1, passes);
  t.ch = t.tr * passes;
  t.nchx = std::max(1, (t.xrows + t.ch - 1) / t.ch);
  t.nper = std::max(1, std::min(t.nchx, std::min(nper_cap, kMaxPer)));
  t.nblk = 8 * t.nper;
  t.nchunk = t.nblk;
  return t;
}

namespace k {

void assemble(const Mesh& m, const double* xyz_new, const int32_t* inc_ptr, const int32_t* inc,
              hipStream_t s) {
  hipLaunchKernelGGL(k_assemble, dim3(nblocks(m.n)), dim3(kBlock), 0, s, int(m.n), m.W, m.cols.p,
                     xyz_new, m.tri.p, inc_ptr, inc, m.M64.p, m.A64.p, m.tarea.p);
  SP_LAUNCH_CHECK();
}

void tau_mats(const Mesh& m, TauMats& t, hipStream_t s) {
  size_t total = size_t(m.W) * m.n;
  hipLaunchKernelGGL(k_tau_mats, dim3(nblocks(total)), dim3(kBlock), 0, s, total, int(m.n), t.tau,
                     m.M64.p, m.A64.p, t.K64.p, t.K32.p, t.dinv64.p, t.dinv32.p);
  SP_LAUNCH_CHECK();
}

void precond_mats(const Mesh& m, TauMats& t, hipStream_t s) {
  const size_t total = size_t(m.W) * size_t(m.n);
  hipLaunchKernelGGL(k_precond_mats, dim3(nblocks(total)), dim3(kBlock), 0, s, total, int(m.n),
                     t.pc0, t.pc1, m.cols.p, t.K64.p, t.dinv64.p, t.P64.p, t.P32.p);
  SP_LAUNCH_CHECK();
}

void fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(nblocks(n)), dim3(kBlock), 0, s, p, v, n);
  SP_LAUNCH_CHECK();
}

void fill_f64(double* p, double v, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill<double>, dim3(nblocks(n)), dim3(kBlock), 0, s, p, v, n);
  SP_LAUNCH_CHECK();
}

void fill_f32(float* p, float v, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill<float>, dim3(nblocks(n)), dim3(kBlock), 0, s, p, v, n);
  SP_LAUNCH_CHECK();
}

void flag_nonconv(const StepArgs& a, const int* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_flag_nonconv, dim3(1), dim3(64), 0, s, counter, a.stat);
  SP_LAUNCH_CHECK();
}

void init_fp64(const StepArgs& a, const double* u, double* r, double* p, hipStream_t s) {
  hipLaunchKernelGGL(k_init_fp64, dim3(a.t64.nblk), dim3(kBlock), 0, s, a, u, r, p);
  SP_LAUNCH_CHECK();
}

void red_init_fp64(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_red_init_fp64, dim3(colblocks(a.t)), dim3(kBlock), 0, s, a);
  SP_LAUNCH_CHECK();
}

template <typename T, typename Z>
void precond_init(const StepArgs& a, const T* r, Z* p, const T* P, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_precond<T, Z>), dim3(a.tp.nblk), dim3(kBlock), 0, s, a, 0, r, p, P);
  hipLaunchKernelGGL(k_red_precond_init, dim3(colblocks(a.tp)), dim3(kBlock), 0, s, a);
  SP_LAUNCH_CHECK();
}
template void precond_init<double, double>(const StepArgs&, const double*, double*, const double*,
                                           hipStream_t);
template void precond_init<float, bf16_t>(const StepArgs&, const float*, bf16_t*, const float*,
                                          hipStream_t);

template <typename T>
void cg_iter(const StepArgs& a, int it, T* x, T* r, T* p, T* q, T* z, const T* K, const T* dinv,
             const T* P, hipStream_t s, const hipEvent_t* ev) {
  const int slot = it % kRing, next = (it + 1) % kRing;
  const dim3 nb(a.t.nblk), rb(colblocks(a.t)), bl(kBlock);
  if (ev) SP_HIP(hipEventRecord(ev[0], s));
  hipLaunchKernelGGL(k_cg_spmm<T>, dim3(a.tm.nblk), bl, 0, s, a, slot, K, (const T*)p, q);
  if (ev) SP_HIP(hipEventRecord(ev[1], s));
  hipLaunchKernelGGL(k_red_alpha, rb, bl, 0, s, a, slot, next, (double*)nullptr);
  if (ev) SP_HIP(hipEventRecord(ev[2], s));
  if (a.poly) {
    hipLaunchKernelGGL((k_cg_update<T, true>), nb, bl, 0, s, a, slot, x, r, (const T*)p,
                       (const T*)q, dinv);
    if (ev) SP_HIP(hipEventRecord(ev[3], s));
    if (ev) SP_HIP(hipEventRecord(ev[6], s));
    hipLaunchKernelGGL(k_cg_precond<T>, dim3(a.tp.nblk), bl, 0, s, a, slot, (const T*)r, z, P);
    if (ev) SP_HIP(hipEventRecord(ev[7], s));
  } else {
    hipLaunchKernelGGL((k_cg_update<T, false>), nb, bl, 0, s, a, slot, x, r, (const T*)p,
                       (const T*)q, dinv);
    if (ev) SP_HIP(hipEventRecord(ev[3], s));
  }
  if (a.poly)
    hipLaunchKernelGGL(k_red_beta<true>, rb, bl, 0, s, a, slot, next);
  else
    hipLaunchKernelGGL(k_red_beta<false>, rb, bl, 0, s, a, slot, next);
  if (ev) SP_HIP(hipEventRecord(ev[4], s));
  if (a.poly)
    hipLaunchKernelGGL((k_cg_update_p<T, true>), nb, bl, 0, s, a, next, p, (const T*)z, dinv);
  else
    hipLaunchKernelGGL((k_cg_update_p<T, false>), nb, bl, 0, s, a, next, p, (const T*)r, dinv);
  if (ev) SP_HIP(hipEventRecord(ev[5], s));
  SP_LAUNCH_CHECK();
}

template <typename T, typename S>
void matvec(const StepArgs& a, const T* K, const S* p, T* q, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_spmm<T, S>), dim3(a.tm.nblk), dim3(kBlock), 0, s, a, 0, K, p, q);
  SP_LAUNCH_CHECK();
}
template void matvec<double, double>(const StepArgs&, const double*, const double*, double*,
                                     hipStream_t);
template void matvec<float, bf16_t>(const StepArgs&, const float*, const bf16_t*, float*,
                                    hipStream_t);

void cg_iter_ring(const StepArgs& a, int it, float* r, bf16_t* const* pring, float* q, bf16_t* z,
                  double* ah, float* d, int* flushed, hipStream_t s, const hipEvent_t* ev) {
  const int slot = it % kRing, next = (it + 1) % kRing;
  const int ps = it % kPRing, pn = (it + 1) % kPRing;
  const dim3 nb(a.t.nblk), rb(colblocks(a.t)), bl(kBlock);
  if (ev) SP_HIP(hipEventRecord(ev[0], s));
  hipLaunchKernelGGL((k_cg_spmm<float, bf16_t>), dim3(a.tm.nblk), bl, 0, s, a, slot, a.K32,
                     (const bf16_t*)pring[ps], q);
  if (ev) SP_HIP(hipEventRecord(ev[1], s));
  hipLaunchKernelGGL(k_red_alpha, rb, bl, 0, s, a, slot, next, ah + size_t(ps) * a.t.rp);
  if (ev) SP_HIP(hipEventRecord(ev[2], s));
  if (a.poly) {
    hipLaunchKernelGGL(k_cg_update_r<true>, nb, bl, 0, s, a, slot, r, (const float*)q, a.dinv32);
    if (ev) SP_HIP(hipEventRecord(ev[3], s));
    if (ev) SP_HIP(hipEventRecord(ev[6], s));
    hipLaunchKernelGGL((k_cg_precond<float, bf16_t>), dim3(a.tp.nblk), bl, 0, s, a, slot,
                       (const float*)r, z, a.P32);
    if (ev) SP_HIP(hipEventRecord(ev[7], s));
  } else {
    hipLaunchKernelGGL(k_cg_update_r<false>, nb, bl, 0, s, a, slot, r, (const float*)q, a.dinv32);
    if (ev) SP_HIP(hipEventRecord(ev[3], s));
  }
  if (a.poly)
    hipLaunchKernelGGL(k_red_beta<true>, rb, bl, 0, s, a, slot, next);
  else
    hipLaunchKernelGGL(k_red_beta<false>, rb, bl, 0, s, a, slot, next);
  if (pn == 0) {
    // the ring is full: fold its directions into d before slot 0 is reused
    materialize(a, pring, ah, 0, kPRing, *flushed, d, s);
    *flushed = 1;
  }
  if (ev) SP_HIP(hipEventRecord(ev[4], s));
  if (a.poly)
    hipLaunchKernelGGL(k_cg_dir_ring<true>, nb, bl, 0, s, a, next, pring[pn],
                       (const bf16_t*)pring[ps], (const bf16_t*)z, a.dinv32);
  else
    hipLaunchKernelGGL(k_cg_dir_ring<false>, nb, bl, 0, s, a, next, pring[pn],
                       (const bf16_t*)pring[ps], (const float*)r, a.dinv32);
  if (ev) SP_HIP(hipEventRecord(ev[5], s));
  SP_LAUNCH_CHECK();
}

void materialize(const StepArgs& a, bf16_t* const* pring, const double* ah, int first, int count,
                 int accumulate, float* d, hipStream_t s) {
  RingArgs ra;
  ra.n = count;
  ra.accumulate = accumulate;
  for (int q = 0; q < count; ++q) {
    const int sl = (first + q) % kPRing;
    ra.p[q] = pring[sl];
    ra.row[q] = sl;
  }
  hipLaunchKernelGGL(k_materialize, dim3(a.ts.nblk), dim3(kBlock), 0, s, a, ra, ah, d);
  SP_LAUNCH_CHECK();
}

template void cg_iter<double>(const StepArgs&, int, double*, double*, double*, double*, double*,
                              const double*, const double*, const double*, hipStream_t,
                              const hipEvent_t*);

void init_outer(const StepArgs& a, const double* u, const float* g, double* x0, double* r64,
                hipStream_t s) {
  hipLaunchKernelGGL(k_init_outer, dim3(a.t64.nblk), dim3(kBlock), 0, s, a, u, g, x0, r64);
  SP_LAUNCH_CHECK();
}

void red_outer_init(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_red_outer_init, dim3(colblocks(a.t)), dim3(kBlock), 0, s, a);
  SP_LAUNCH_CHECK();
}

void refine_start(const StepArgs& a, const double* w, const float* g, double* r64, float* r,
                  bf16_t* p, hipStream_t s) {
  hipLaunchKernelGGL(k_refine_start, dim3(a.tm.nblk), dim3(kBlock), 0, s, a, w, g, r64, r, p);
  hipLaunchKernelGGL(k_red_refine_start, dim3(colblocks(a.t)), dim3(kBlock), 0, s, a);
  SP_LAUNCH_CHECK();
}

void inner_init(const StepArgs& a, int o, const double* r64, float* d, float* r, bf16_t* p,
                hipStream_t s) {
  hipLaunchKernelGGL(k_inner_init, dim3(a.t.nblk), dim3(kBlock), 0, s, a, o % kRing, r64, d, r, p);
  SP_LAUNCH_CHECK();
}

void red_inner_init(const StepArgs& a, int o, hipStream_t s) {
  hipLaunchKernelGGL(k_red_inner_init, dim3(colblocks(a.t)), dim3(kBlock), 0, s, a, o % kRing,
                     (o + 1) % kRing);
  SP_LAUNCH_CHECK();
}

void outer_update(const StepArgs& a, int o, double* x, const double* ubase, double* r64,
                  const float* d, float* dacc, bool store_r, float* rn, bf16_t* pn, float* d0,
                  int d0mode, hipStream_t s) {
  if (rn)
    hipLaunchKernelGGL(k_outer_update<true>, dim3(a.tm.nblk), dim3(kBlock), 0, s, a, o % kRing, x,
                       ubase, r64, d, dacc, 1, rn, pn, d0, d0mode);
  else
    hipLaunchKernelGGL(k_outer_update<false>, dim3(a.tm.nblk), dim3(kBlock), 0, s, a, o % kRing,
                       x, ubase, r64, d, dacc, int(store_r), nullptr, nullptr, d0, d0mode);
  SP_LAUNCH_CHECK();
}

void red_outer_prep(const StepArgs& a, int o, hipStream_t s) {
  hipLaunchKernelGGL(k_red_outer_prep, dim3(colblocks(a.tm)), dim3(kBlock), 0, s, a, o % kRing,
                     (o + 1) % kRing, (o + 2) % kRing);
  SP_LAUNCH_CHECK();
}

void outer_residual(const StepArgs& a, int o, double* r64, const float* d, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_residual, dim3(a.tm.nblk), dim3(kBlock), 0, s, a, o % kRing, r64, d);
  SP_LAUNCH_CHECK();
}

void extrap(const StepArgs& a, const ExtrapArgs& e, float* y, int qmax, hipStream_t s) {
  if (qmax >= 2) {
    hipLaunchKernelGGL(k_extrap_probe, dim3(a.tprobe.nblk), dim3(kBlock), 0, s, a, e);
    hipLaunchKernelGGL(k_red_extrap_order, dim3(colblocks(a.tprobe)), dim3(kBlock), 0, s, a, e.n,
                       qmax);
  }
  hipLaunchKernelGGL(k_extrap, dim3(a.ts.nblk), dim3(kBlock), 0, s, a, e, y);
  SP_LAUNCH_CHECK();
}

void hist_advance(const StepArgs& a, int q, hipStream_t s) {
  hipLaunchKernelGGL(k_hist_advance, dim3((a.t.rp + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a, q);
  SP_LAUNCH_CHECK();
}

void red_outer(const StepArgs& a, int o, hipStream_t s) {
  hipLaunchKernelGGL(k_red_outer, dim3(colblocks(a.t)), dim3(kBlock), 0, s, a, o % kRing,
                     (o + 1) % kRing);
  SP_LAUNCH_CHECK();
}

void nodal(const StepArgs& a, const double* u, double* out, bool keep, hipStream_t s) {
  if (a.nodal_fast && a.ts.tg == 64)
    hipLaunchKernelGGL(k_nodal<false>, dim3(a.ts.nblk), dim3(kBlock), 0, s, a, u, out, int(keep));
  else
    hipLaunchKernelGGL(k_nodal<true>, dim3(a.ts.nblk), dim3(kBlock), 0, s, a, u, out, int(keep));
  SP_LAUNCH_CHECK();
}

void norm_dot(const StepArgs& a, const double* v, double* w, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_dot, dim3(a.t64.nblk), dim3(kBlock), 0, s, a, v, w);
  SP_LAUNCH_CHECK();
}

void red_norm(const StepArgs& a, double* lam, hipStream_t s) {
  hipLaunchKernelGGL(k_red_norm, dim3(colblocks(a.t)), dim3(kBlock), 0, s, a, lam);
  SP_LAUNCH_CHECK();
}

void apply_mask(const StepArgs& a, double* u, hipStream_t s) {
  const size_t total = size_t(a.t.n) * a.t.rp;
  hipLaunchKernelGGL(k_apply_mask, dim3(std::min<size_t>(nblocks(total), 65536)), dim3(kBlock), 0,
                     s, a, u);
  SP_LAUNCH_CHECK();
}

void region_graph(const StepArgs& a, const int32_t* labels, const int* off, const int* mres,
                  int nres, uint8_t* adj, hipStream_t s) {
  const size_t total = size_t(a.t.n) * nres;
  hipLaunchKernelGGL(k_region_graph, dim3(std::min<size_t>(nblocks(total), 65536)), dim3(kBlock), 0,
                     s, a, labels, off, mres, nres, adj);
  SP_LAUNCH_CHECK();
}

void multipliers(const StepArgs& a, const SepsPlan& sp, const int32_t* tri, const double* tarea,
                 const double* u, double* part, const double* lam, double* out, hipStream_t s) {
  if (sp.ntile > 0)
    hipLaunchKernelGGL(k_multipliers, dim3(8 * sp.nper), dim3(kBlock), 0, s, a, sp, tri, tarea, u,
                       part);
  hipLaunchKernelGGL(k_red_multipliers, dim3(colblocks(a.t)), dim3(kBlock), 0, s, a, sp,
                     part, lam, out);
  SP_LAUNCH_CHECK();
}

void scale(const StepArgs& a, const double* v, double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(a.ts.nblk), dim3(kBlock), 0, s, a, v, u);
  SP_LAUNCH_CHECK();
}

void energy_rq(const StepArgs& a, const double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_rq, dim3(a.t64.nblk), dim3(kBlock), 0, s, a, u);
  SP_LAUNCH_CHECK();
}

void energy_seps(const StepArgs& a, const SepsPlan& sp, const int32_t* tri, const double* tarea,
                 const double* u, double* part_s, hipStream_t s) {
  if (sp.ntile == 0) return;
  if (sp.direct == 2 && sp.lanes_ok) {
    if (a.usc)
      hipLaunchKernelGGL(k_energy_seps_lanes<true>, dim3(8 * sp.nper), dim3(kBlock), 0, s, a, sp,
                         tri, tarea, u, part_s);
    else
      hipLaunchKernelGGL(k_energy_seps_lanes<false>, dim3(8 * sp.nper), dim3(kBlock), 0, s, a, sp,
                         tri, tarea, u, part_s);
  } else if (sp.direct && a.usc)
    hipLaunchKernelGGL(k_energy_seps_direct<true>, dim3(8 * sp.nper), dim3(kBlock), 0, s, a, sp,
                       tri, tarea, u, part_s);
  else if (sp.direct)
    hipLaunchKernelGGL(k_energy_seps_direct<false>, dim3(8 * sp.nper), dim3(kBlock), 0, s, a, sp,
                       tri, tarea, u, part_s);
  else
    hipLaunchKernelGGL(k_energy_seps, dim3(8 * sp.nper), dim3(kBlock), 0, s, a, sp, tri, tarea, u,
                       part_s);
  SP_LAUNCH_CHECK();
}

int seps_resident_groups() {
  // workgroups of the lane-split element kernel that fit on one XCD at once
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  SP_HIP(hipGetDevice(&dev));
  SP_HIP(hipGetDeviceProperties(&prop, dev));
  SP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_energy_seps_lanes<true>, kBlock, 0));
  return std::max(1, per_cu * prop.multiProcessorCount / 8);
}

void red_energy(const StepArgs& a, const SepsPlan& sp, const double* part_s, bool with_lambda,
                double* lam, double* seps, double* energy, hipStream_t s) {
  if (with_lambda)
    hipLaunchKernelGGL(k_red_lambda, dim3(colblocks(a.t)), dim3(kBlock), 0, s, a, lam);
  hipLaunchKernelGGL(k_red_seps, dim3(nblocks(size_t(a.ct.nres), kRC)), dim3(kBlock), 0, s, a, sp,
                     part_s, (const double*)lam, seps, energy);
  SP_LAUNCH_CHECK();
}

std::vector<int4> seps_tiles(const std::vector<int>& res_lo, const std::vector<int>& res_len,
                             int nres) {
  // contiguous runs of restarts whose columns fit in kSepsCols (at most 64
  // restarts, so every restart of a run gets a worker thread per triangle)
  std::vector<int4> tiles;
  int r = 0;
  while (r < nres) {
    int r1 = r, c0 = 0, c1 = 0;
    bool any = false;
    while (r1 < nres && r1 - r < 64) {
      const int lo = res_lo[r1], len = res_len[r1];
      if (len > 0) {
        const int n0 = any ? std::min(c0, lo) : lo, n1 = any ? std::max(c1, lo + len) : lo + len;
        if (any && n1 - n0 > kSepsCols) break;
        c0 = n0;
        c1 = n1;
        any = true;
      }
      ++r1;
    }
    if (r1 == r) r1 = r + 1;  // a single restart wider than the stage
    tiles.push_back(make_int4(r, r1, c0, c1));
    r = r1;
  }
  return tiles;
}

void small_steps(const StepArgs& a, const SmallArgs& sa, hipStream_t s) {
  hipLaunchKernelGGL(k_small_steps, dim3(1), dim3(kSmallBlock), 0, s, a, sa);
  SP_LAUNCH_CHECK();
}

void labels(const StepArgs& a, const double* u, const int32_t* perm, int32_t* lab, int32_t* lab_am,
            hipStream_t s) {
  size_t total = size_t(a.t.n) * size_t(a.ct.nres);
  hipLaunchKernelGGL(k_labels, dim3(nblocks(total)), dim3(kBlock), 0, s, a, u, perm, lab, lab_am);
  SP_LAUNCH_CHECK();
}

void pack(const Tile& t, int c_lo, int Rq, const double* u0, const int32_t* perm, double* u,
          hipStream_t s) {
  size_t total = size_t(t.n) * Rq;
  if (!total) return;
  hipLaunchKernelGGL(k_pack, dim3(nblocks(total)), dim3(kBlock), 0, s, total, t.rp, t.n, c_lo, Rq,
                     u0, perm, u);
  SP_LAUNCH_CHECK();
}

void unpack(const Tile& t, int c_lo, int Rq, const double* u, const int32_t* perm, double* out,
            hipStream_t s) {
  size_t total = size_t(t.n) * Rq;
  if (!total) return;
  hipLaunchKernelGGL(k_unpack, dim3(nblocks(total)), dim3(kBlock), 0, s, total, t.rp, t.n, c_lo, Rq,
                     u, perm, out);
  SP_LAUNCH_CHECK();
}

}  // namespace k
}  // namespace sp
