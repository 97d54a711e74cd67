// Constant-weight greedy codes over words of up to 64 coordinates (MI355X,
// gfx950).
//
// Section "Brief overview of the Greedy Algorithm and Codes": a
// constant-weight code takes only the vectors of weight w as candidates; the
// rule is the greedy one of section "Greedy Algorithms and Different
// Orderings" (a candidate joins the code when its Hamming distance, section
// "Hamming Distance", to every word already in the code is at least d).
// Section "Some Examples" reports such codes up to length 35, past 32-bit
// words.  Candidates are the weight-w vectors in increasing value.
//
// One cooperative launch walks the candidates in blocks of kCands positions:
//   1. every workgroup unranks the block's candidates (combinatorial number
//      system) and screens them against its own slice of the committed code;
//      a clash sets the candidate's bit in a dead mask (device atomics);
//   2. grid barrier;
//   3. workgroup 0 takes the block's live candidates in order, accepts each
//      one that no word accepted earlier in the block is closer than d to
//      (the sequential rule inside the block), and appends them to the code;
//   4. grid barrier.
// The code is the sequential greedy one: a candidate is accepted exactly when
// no earlier accepted word (of an earlier block: step 1; of its own block:
// step 3) is closer than d.  This path favours simplicity over speed; the
// 32-bit windowed screen is the fast path.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gc_internal.h"
#include "greedy_code.h"

namespace gcimpl {

int acquire_workspace(size_t bytes, char **ptr, int *slot);
void release_workspace(int slot);

namespace {

constexpr int kCwBlock = 256;                     // threads per workgroup
constexpr int kCands = 1024;                      // candidate positions per block
constexpr int kPerThread = kCands / kCwBlock;     // candidates a thread screens
constexpr unsigned long long kMaxPositions = 1ull << 32;

struct CwState {                 // device workspace (zeroed before the launch)
  unsigned long long m;          // committed words
  int status;                    // GC_OK or GC_ECAPACITY
  int pad;
  uint32_t dead[kCands / 32];    // the block's dead mask
};

struct CwParams {
  int n, w, d;
  unsigned long long total;      // C(n, w) candidate positions
  uint64_t *words;
  unsigned long long capacity;
  uint64_t *count;               // may be null
  CwState *st;
};

__device__ __forceinline__ unsigned long long ld_dev(unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The r-th weight-w vector of length n in increasing value: r is written as
// C(c_w, w) + ... + C(c_1, 1) with c_w > ... > c_1 >= 0 (combinatorial
// number system), and the vector has ones at c_1 .. c_w.
__device__ __forceinline__ uint64_t unrank(const unsigned long long (*C)[65], int n, int w, unsigned long long r) {
  uint64_t x = 0;
  int c = n;
  for (int i = w; i >= 1; --i) {
    int cc = c - 1;
    while (C[cc][i] > r) --cc;  // C(i - 1, i) = 0 <= r ends the search
    x |= 1ull << cc;
    r -= C[cc][i];
    c = cc;
  }
  return x;
}

__global__ void __launch_bounds__(kCwBlock) cw64_kernel(CwParams P) {
  __shared__ unsigned long long C[65][65];  // binomials C(a, b), a, b <= 64 (Pascal's rule)
  __shared__ uint64_t cand[kCands];         // workgroup 0: the block's candidates
  __shared__ uint64_t acc[kCands];          // workgroup 0: words accepted in this block
  __shared__ uint32_t deadw[kCands / 32];
  __shared__ unsigned long long m_s;
  __shared__ int stop_s;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int tid = threadIdx.x;
  if (tid == 0) {
    for (int a = 0; a <= 64; ++a) {
      C[a][0] = 1;
      for (int b = 1; b <= 64; ++b) C[a][b] = a == 0 ? 0ull : C[a - 1][b - 1] + C[a - 1][b];
    }
  }
  __syncthreads();
  const unsigned int d = (unsigned int)P.d;
  for (unsigned long long p0 = 0; p0 < P.total; p0 += kCands) {
    const unsigned int nb = (unsigned int)(P.total - p0 < (unsigned long long)kCands ? P.total - p0 : kCands);
    if (tid == 0) {
      m_s = ld_dev(&P.st->m);
      stop_s = __hip_atomic_load(&P.st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (stop_s != 0) break;  // every workgroup reads the same state after the barrier
    const unsigned long long m = m_s;

    // 1. Screen against this workgroup's slice of code[0, m).
    uint64_t x[kPerThread];
    bool live[kPerThread];
    int nlive = 0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const unsigned int idx = (unsigned int)(k * kCwBlock + tid);
      live[k] = idx < nb;
      x[k] = live[k] ? unrank(C, P.n, P.w, p0 + idx) : 0ull;
      nlive += live[k];
    }
    const unsigned long long lo = m * blockIdx.x / gridDim.x, hi = m * (blockIdx.x + 1) / gridDim.x;
    for (unsigned long long j = lo; j < hi && nlive > 0; ++j) {
      const uint64_t c = P.words[j];
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        if (live[k] && (unsigned int)__builtin_popcountll(x[k] ^ c) < d) {
          live[k] = false;
          --nlive;
          const unsigned int idx = (unsigned int)(k * kCwBlock + tid);
          __hip_atomic_fetch_or(&P.st->dead[idx >> 5], 1u << (idx & 31), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    grid.sync();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

    // 3. Workgroup 0: the block in order.
    if (blockIdx.x == 0) {
      for (unsigned int i = tid; i < nb; i += kCwBlock) cand[i] = unrank(C, P.n, P.w, p0 + i);
      for (int i = tid; i < kCands / 32; i += kCwBlock)
        deadw[i] = __hip_atomic_load(&P.st->dead[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      unsigned int na = 0;  // the same in every thread
      for (unsigned int i = 0; i < nb; ++i) {
        if ((deadw[i >> 5] >> (i & 31)) & 1u) continue;
        const uint64_t y = cand[i];
        bool clash = false;
        for (unsigned int a = tid; a < na; a += kCwBlock)
          clash |= (unsigned int)__builtin_popcountll(y ^ acc[a]) < d;
        if (!__syncthreads_or(clash)) {
          if (tid == 0) acc[na] = y;
          ++na;
          __syncthreads();
        }
      }
      const unsigned long long room = P.capacity > m ? P.capacity - m : 0;
      const unsigned int nput = (unsigned long long)na < room ? na : (unsigned int)room;
      for (unsigned int a = tid; a < nput; a += kCwBlock) P.words[m + a] = acc[a];
      for (int i = tid; i < kCands / 32; i += kCwBlock) P.st->dead[i] = 0;
      if (tid == 0) {
        P.st->m = m + nput;
        if (nput < na) P.st->status = GC_ECAPACITY;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    grid.sync();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  if (blockIdx.x == 0 && tid == 0 && P.count) *P.count = ld_dev(&P.st->m);
}

// C(a, b), or kMaxPositions + 1 once it exceeds kMaxPositions.  After step i
// the product is C(a - b + i, i), exact, increasing with i and at most
// 2^32 before the multiplication (so the product stays below 2^39).
unsigned long long positions(int a, int b) {
  if (b < 0 || b > a) return 0;
  if (b > a - b) b = a - b;
  unsigned long long r = 1;
  for (int i = 1; i <= b; ++i) {
    r = r * (unsigned long long)(a - b + i) / (unsigned long long)i;
    if (r > kMaxPositions) return kMaxPositions + 1;
  }
  return r;
}

}  // namespace
}  // namespace gcimpl

using namespace gcimpl;

extern "C" int greedy_code_cw64(int n, int w, int d, uint64_t *d_words, uint64_t capacity, uint64_t *d_count,
                                void *hip_stream) {
  if (n < 1 || n > 64) return fail(GC_EINVAL, "n = %d is outside 1..64", n);
  if (w < 0 || w > n) return fail(GC_EINVAL, "weight %d is outside 0..%d", w, n);
  if (d < 1) return fail(GC_EINVAL, "d = %d is below 1", d);
  if (!d_words && capacity) return fail(GC_EINVAL, "d_words is NULL with capacity %llu",
                                        (unsigned long long)capacity);
  if (reinterpret_cast<uintptr_t>(d_words) % 8) return fail(GC_EINVAL, "d_words is not 8-byte aligned");
  // The walk's length: at most 2^32 positions, as for the 32-bit walks.
  const unsigned long long total = positions(n, w);
  if (total > kMaxPositions) return fail(GC_EINVAL, "C(%d, %d) positions exceed 2^32", n, w);
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  int dev = 0, cus = 0, coop = 0, bpc = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(GC_EDEVICE, "hipGetDevice failed");
  if (int rc = device_info(dev, &cus, &coop, &bpc)) return rc;
  if (!coop) return fail(GC_EDEVICE, "device %d has no cooperative launch", dev);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, cw64_kernel, kCwBlock, 0) != hipSuccess || per_cu < 1)
    return fail(GC_EDEVICE, "the constant-weight kernel does not fit a compute unit");
  const unsigned int grid = (unsigned int)cus;  // one workgroup per CU: co-resident by the check above
  char *ws = nullptr;
  int slot = -1;
  if (int rc = acquire_workspace(sizeof(CwState), &ws, &slot)) return rc;
  CwState *st = reinterpret_cast<CwState *>(ws);
  CwParams P{n, w, d, total, d_words, capacity, d_count, st};
  void *args[] = {&P};
  hipError_t e = hipMemsetAsync(st, 0, sizeof(CwState), stream);
  if (e == hipSuccess)
    e = hipLaunchCooperativeKernel((const void *)cw64_kernel, dim3(grid), dim3(kCwBlock), args, 0, stream);
  int status = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&status, &st->status, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  release_workspace(slot);
  if (e != hipSuccess) return fail(GC_EDEVICE, "constant-weight launch failed: %s", hipGetErrorString(e));
  if (status == GC_ECAPACITY) return fail(GC_ECAPACITY, "the code exceeds capacity %llu",
                                          (unsigned long long)capacity);
  return GC_OK;
}
