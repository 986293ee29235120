// Connected components of the threshold graph on D (Sec. 7, Conclusions and
// perspectives: the reads are the vertices, (i, j) is an edge iff
// d(i, j) <= theta, and the components are candidate clusters; linear in the
// number of entries of D).  A second HBM-bound pass over the same resident D.
//
// Union-find with union by index: a root is only ever hooked under a root of
// smaller index, and path halving only moves a pointer to an ancestor, so
// every parent pointer is at most its vertex, the forest stays a forest
// under concurrent updates, and the root of a component is its smallest
// vertex.  The labels are therefore canonical (label = smallest index in
// the component) whatever order the edges are processed in.
//
//   k_cc_tiles: one workgroup per 128 x 128 tile of D on and above the
//     diagonal (the whole matrix with the full-matrix flag).  The tile's edges
//     are first joined in a union-find over its 256 (diagonal tile: 128)
//     vertices in LDS; then each vertex whose local root differs from it is
//     joined with that root in the global forest (at most 255 global unions
//     per tile, however dense the tile).  The global forest is the labels
//     array itself; its reads are atomic (they bypass the non-coherent L1) and
//     a hook is a compare-and-swap on a root.
//   k_cc_finalize: labels[i] = root of i; counts the roots.
// D is read once (half of it by default) in whole 512-byte row segments.
#include "mds_internal.h"

namespace mds {
namespace {

constexpr int kCT = 128;       // tile edge
constexpr int kCThreads = 256;

// ---- global forest (labels) --------------------------------------------------
__device__ __forceinline__ int32_t gload(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t gfind(int32_t* L, int32_t v) {
  int32_t p = gload(&L[v]);
  while (p != v) {
    const int32_t gp = gload(&L[p]);
    if (gp != p) __hip_atomic_store(&L[v], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // halving
    v = gp;
    p = gload(&L[v]);
  }
  return v;
}
__device__ void gunion(int32_t* L, int32_t a, int32_t b) {
  while (true) {
    a = gfind(L, a);
    b = gfind(L, b);
    if (a == b) return;
    if (a > b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    // hook root b under a (a < b); fails if b stopped being a root meanwhile
    int32_t expected = b;
    if (__hip_atomic_compare_exchange_strong(&L[b], &expected, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
}

// ---- local forest (LDS) ------------------------------------------------------
__device__ __forceinline__ int lfind(volatile int* lp, int v) {
  int p = lp[v];
  while (p != v) {
    const int gp = lp[p];
    if (gp != p) lp[v] = gp;
    v = gp;
    p = lp[v];
  }
  return v;
}
__device__ void lunion(int* lp, int a, int b) {
  volatile int* vl = lp;
  while (true) {
    a = lfind(vl, a);
    b = lfind(vl, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    if (atomicCAS(&lp[b], b, a) == b) return;
  }
}

// four entries of a row (cnt of them inside D; the others read as NaN: no edge)
template <typename DT>
__device__ __forceinline__ void load4(const DT* p, bool vec, DT (&v)[4], int cnt) {
  if (vec && cnt == 4) {
    if constexpr (sizeof(DT) == 4) {
      const float4 x = *reinterpret_cast<const float4*>(p);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else {
      const double2 x = reinterpret_cast<const double2*>(p)[0], y = reinterpret_cast<const double2*>(p)[1];
      v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = e < cnt ? p[e] : (DT)__builtin_nan("");
  }
}

// full: every tile (I, J); else the tiles with I <= J (upper triangle, strict
// above the diagonal inside diagonal tiles)
template <typename DT>
__global__ __launch_bounds__(kCThreads) void k_cc_tiles(const DT* __restrict__ D, int64_t n, double theta,
                                                        int full, int vec, int32_t* __restrict__ labels) {
  __shared__ int lp[2 * kCT];
  const int64_t nt = (n + kCT - 1) / kCT;
  int64_t I, J;
  if (full) {
    I = (int64_t)blockIdx.x / nt;
    J = (int64_t)blockIdx.x % nt;
  } else {
    upper_tile((int64_t)blockIdx.x, nt, I, J);
  }
  const bool diag = I == J;
  const int nloc = diag ? kCT : 2 * kCT;
  const int tid = threadIdx.x;
  for (int v = tid; v < nloc; v += kCThreads) lp[v] = v;
  __syncthreads();
  const int64_t r0 = I * kCT, c0 = J * kCT;
  // rows of 128 entries as 32 pieces of 4: thread (rr, pc) reads piece pc of
  // rows rr, rr + 8, ..; the 8 loads of a batch are issued before any of
  // their entries is examined
  constexpr int kRowStep = kCThreads / 32, kBatch = 8;
  const int pc = tid & 31, rr = tid >> 5;
  const int64_t j = c0 + 4 * pc;
  const int cnt = j >= n ? 0 : (j + 4 <= n ? 4 : (int)(n - j));
  for (int b0 = 0; b0 < kCT / kRowStep; b0 += kBatch) {
    DT v[kBatch][4];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int64_t i = r0 + rr + (b0 + b) * kRowStep;
      const int c = i < n ? cnt : 0;
      load4<DT>(D + (c ? i * n + j : 0), vec != 0, v[b], c);
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int r = rr + (b0 + b) * kRowStep;  // local row
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int cl = 4 * pc + e;  // local column
        if (!((double)v[b][e] <= theta)) continue;  // no edge (NaN included)
        if (diag) {
          if (cl == r) continue;
          if (!full && cl < r) continue;
          lunion(lp, r, cl);
        } else {
          lunion(lp, r, kCT + cl);
        }
      }
    }
  }
  __syncthreads();
  for (int v = tid; v < nloc; v += kCThreads) {
    const int root = lfind(lp, v);
    if (root == v) continue;
    const int64_t gv = v < kCT ? r0 + v : c0 + (v - kCT);
    const int64_t gr = root < kCT ? r0 + root : c0 + (root - kCT);
    gunion(labels, (int32_t)gv, (int32_t)gr);
  }
}

__global__ __launch_bounds__(256) void k_cc_init(int32_t* __restrict__ labels, int64_t n,
                                                 unsigned long long* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) labels[i] = (int32_t)i;
  if (i == 0 && count) *count = 0;
}

__global__ __launch_bounds__(256) void k_cc_finalize(int32_t* __restrict__ labels, int64_t n,
                                                     unsigned long long* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int32_t r = gfind(labels, (int32_t)i);
  __hip_atomic_store(&labels[i], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (count && r == (int32_t)i) atomicAdd(count, 1ull);
}

}  // namespace

hipError_t launch_components(const void* D, bool f64, int64_t n, double theta, bool full, int32_t* labels,
                             int64_t* n_components, hipStream_t s) {
  const unsigned eb = (unsigned)((n + 255) / 256);
  auto* cnt = reinterpret_cast<unsigned long long*>(n_components);
  hipLaunchKernelGGL(k_cc_init, dim3(eb), dim3(256), 0, s, labels, n, cnt);
  const int64_t nt = (n + kCT - 1) / kCT;
  const int64_t tiles = full ? nt * nt : nt * (nt + 1) / 2;
  const int vec = (n % 4 == 0 && ((uintptr_t)D % (f64 ? 32 : 16)) == 0) ? 1 : 0;
  if (f64)
    hipLaunchKernelGGL(k_cc_tiles<double>, dim3((unsigned)tiles), dim3(kCThreads), 0, s, (const double*)D, n, theta,
                       full ? 1 : 0, vec, labels);
  else
    hipLaunchKernelGGL(k_cc_tiles<float>, dim3((unsigned)tiles), dim3(kCThreads), 0, s, (const float*)D, n, theta,
                       full ? 1 : 0, vec, labels);
  hipLaunchKernelGGL(k_cc_finalize, dim3(eb), dim3(256), 0, s, labels, n, cnt);
  return hipGetLastError();
}

}  // namespace mds
