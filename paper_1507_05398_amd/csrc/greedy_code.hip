// greedy_code.hip -- MI355X (gfx950) greedy binary code construction.
//
// Operation (Paliwal et al., arXiv:1507.05398, section "Greedy Algorithms and
// Different Orderings"): walk the 2^n vectors of F_2^n in a fixed ordering and
// append a vector to the code C when popcount(x XOR c) >= d for every word c
// already in C (section "Hamming Distance").  The result is one ordered list.
//
// Device design (one cooperative persistent launch per code):
//
//   The ordering is cut into windows of consecutive positions.  For a window
//   starting with m0 committed words:
//
//   A  near screen   every window candidate is compared with the newest
//                    `near_depth` committed words (2-D work items: 256
//                    candidates x a code chunk, newest chunk first); a conflict
//                    sets the candidate's bit in a window "dead" mask.
//   C  survivors     every workgroup rebuilds the ordered survivor list in LDS
//                    (capped at kSMax, the window is cut at the cap) and the
//                    grid computes the in-window conflict graph among survivors
//                    as 64x64-bit tiles (earlier-neighbour masks).
//   D  resolve       one wave computes the lexicographically first maximal
//                    independent set of the survivor graph in position order,
//                    which is exactly sequential greedy restricted to the
//                    window, treating survivors whose deep status is unknown as
//                    passing.
//   E  deep scan     tentatively accepted survivors whose status is unknown
//                    are compared with the older code words [0, m0-near_depth)
//                    (2-D items again); D then runs again with the new facts.
//                    When every tentatively accepted survivor is known to pass,
//                    the set is the greedy result for the window: it is
//                    appended to the code and the next window starts.
//
//   Between phases the grid synchronises with a bounded-wait barrier.  The
//   paper launched two kernels per candidate and copied |C| to the host each
//   time (sections "Parallel Implementation", "Removing Wasted Threads",
//   "Dynamic Parallelism"); here |C| stays on the device and one launch covers
//   all 2^n positions.  Its "selective kernel launch" (check part of the code
//   first, the rest only if that passes) becomes the near screen / deep scan
//   split, reordered newest-first.
//
// Distance checks run on the vector ALUs: v_xor_b32, v_bcnt_u32_b32 and
// v_min3_u32 (2.5 instructions per check).  No matrix cores: this is bit-packed
// popcount work, not a dense contraction.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>

#include "greedy_code.h"

#define GC_VERSION_STRING "greedy_code 0.1.0 (gfx950)"

namespace gcimpl {

constexpr int kBlock = 1024;                          // threads per workgroup
constexpr int kWaves = kBlock / 64;                   // waves per workgroup
constexpr int kTile = 256;                            // candidates per screen tile (4 rows of 64)
constexpr int kRows = kTile / 64;
constexpr int kSeg = 64 * kWaves;                     // code words per screen segment (64 per wave)
constexpr int kMaxXcd = 16;
constexpr int kSMax = 1024;                           // survivors per window (resolve capacity)
constexpr int kNb = kSMax / 64;                       // survivor blocks of 64
constexpr int kAdjWords = 64 * kNb * (kNb + 1) / 2;   // lower-triangular block adjacency
constexpr unsigned long long kWMin = 256;
constexpr unsigned long long kWMax = 1ull << 18;
constexpr unsigned int kDefaultTarget = 768;
constexpr unsigned long long kDefaultNear = 16384;
constexpr unsigned int kDefaultSpin = 1u << 25;

enum : int { ST_UNKNOWN = 0, ST_PASS = 1, ST_FAIL = 2 };
enum : int { ACT_NEXT = 0, ACT_DEEP = 1, ACT_STOP = 2 };
enum : int { MODE_TENTATIVE = 1, MODE_DEEP_ALL = 2 };

// Grid barrier state: one counter/generation pair per XCD (each on its own
// 256-byte line) and one pair across XCD leaders.
struct Bar {
  unsigned int join_count;   // one-time membership count
  unsigned int top_count;
  unsigned int top_gen;
  unsigned int pad0[61];
  unsigned int xcd[kMaxXcd][64];   // [x][0] count, [x][1] generation, [x][2] members
};

struct Ctl {
  unsigned long long m;   // committed words
  unsigned long long p;   // start of the next window
  unsigned long long w;   // length of the next window
  unsigned int pad_bar[2];
  int status;
  int action;
  unsigned int ndeep;
  unsigned int pad;
  unsigned long long stat_windows, stat_rounds, stat_surv, stat_near, stat_deep, stat_pairs;
};

struct Params {
  int n, d, ord, mode;
  unsigned long long total;   // 2^n
  uint32_t *code;
  unsigned long long capacity;
  Ctl *ctl;
  Bar *bar;
  unsigned long long *count_out;
  uint32_t *win_dead;             // kWMax / 32 words
  unsigned long long *adj;        // kAdjWords
  uint32_t *deep_word;            // kSMax
  uint32_t *deep_idx;             // kSMax
  uint32_t *deep_fail;            // kSMax / 32
  unsigned long long near_depth;
  unsigned int target;
  unsigned int spin_limit;
};

struct Tables {
  uint32_t binom[33][33];              // C(a, b)
  unsigned long long off[34];          // off[w] = number of words of weight < w
};

// Screen tile: candidate words and ids (double-buffered for compaction), code
// segment (double-buffered), per-wave conflict masks.
struct TileLds {
  alignas(16) uint32_t seg[2][kSeg];
  uint32_t cw[2][kTile];
  uint32_t ci[2][kTile];
  unsigned long long killw[kWaves][kRows];
  unsigned int wcnt[kWaves];
};

// In-window resolve (workgroup 0 only).
struct ResolveLds {
  unsigned long long adj[kAdjWords];   // survivor adjacency (earlier-neighbour masks)
  unsigned long long accm[kNb];        // accepted mask per block
  uint32_t tlist[kSMax];               // tentatively accepted words
};

struct Lds {
  uint32_t s1w[kSMax];                 // window survivors, in position order
  uint8_t st[kSMax];                   // deep status of each survivor (resolve only)
  Tables tab;
  unsigned long long p0, m0, w, pe, lo;
  unsigned int s, s_tot, ndeep, round, tcount, truncated;
  int status, action;
  unsigned int xcd, xcd_members, nxcd;
  unsigned int wsum[kWaves];
  union alignas(16) {
    TileLds t;
    ResolveLds r;
  } u;
};

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }
// min(min(a, b), c) lowers to one v_min3_u32.
__device__ __forceinline__ uint32_t umin3(uint32_t a, uint32_t b, uint32_t c) {
  return umin(umin(a, b), c);
}
__device__ __forceinline__ uint32_t dist(uint32_t a, uint32_t b) { return __builtin_popcount(a ^ b); }

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ unsigned int lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long lanemask_lt() {
  unsigned int l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

template <typename T>
__device__ __forceinline__ T ld_acquire(T *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_relaxed(T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_status(Ctl *ctl, int code) {
  int expected = 0;
  __hip_atomic_compare_exchange_strong(&ctl->status, &expected, code, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned int xcc_id() {
  unsigned int v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(v));
  return v & (kMaxXcd - 1);
}

// Bounded spin until *p != old; records GC_ETIMEOUT and gives up after
// spin_limit polls so that no wait can hang the device.
__device__ __forceinline__ void wait_change(unsigned int *p, unsigned int old, Ctl *ctl,
                                            unsigned int spin_limit) {
  unsigned int spins = 0;
  while (ld_relaxed(p) == old) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > spin_limit) {
      set_status(ctl, GC_ETIMEOUT);
      break;
    }
  }
}

// One-time registration: every workgroup counts itself on its XCD, then all
// wait until the whole grid has registered, so that each XCD leader knows how
// many workgroups to expect (no assumption about the block -> XCD mapping).
__device__ void barrier_join(Lds &L, Bar *B, Ctl *ctl, unsigned int spin_limit) {
  if (threadIdx.x == 0) {
    const unsigned int x = xcc_id();
    __hip_atomic_fetch_add(&B->xcd[x][2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&B->join_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned int spins = 0;
    while (ld_relaxed(&B->join_count) < gridDim.x) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > spin_limit) {
        set_status(ctl, GC_ETIMEOUT);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    unsigned int nx = 0;
    for (int i = 0; i < kMaxXcd; ++i) nx += ld_relaxed(&B->xcd[i][2]) > 0;
    L.xcd = x;
    L.xcd_members = ld_relaxed(&B->xcd[x][2]);
    L.nxcd = nx;
  }
  __syncthreads();
}

// Grid-wide barrier for a cooperative launch, two levels.  Workgroups of one
// XCD meet on that XCD's counter; the last to arrive (the XCD leader) makes
// the XCD's writes visible device-wide (release), meets the other leaders,
// acquires, and releases its XCD.  Every workgroup then acquires at agent
// scope before reading data written elsewhere.  All waits are bounded.
__device__ void grid_barrier(Lds &L, Bar *B, Ctl *ctl, unsigned int spin_limit) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int *xc = &B->xcd[L.xcd][0];
    unsigned int *xg = &B->xcd[L.xcd][1];
    const unsigned int g = ld_relaxed(xg);
    const unsigned int a = __hip_atomic_fetch_add(xc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a + 1 == L.xcd_members) {
      __hip_atomic_store(xc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned int tg = ld_relaxed(&B->top_gen);
      const unsigned int b =
          __hip_atomic_fetch_add(&B->top_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (b + 1 == L.nxcd) {
        __hip_atomic_store(&B->top_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&B->top_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        wait_change(&B->top_gen, tg, ctl, spin_limit);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __builtin_amdgcn_s_waitcnt(0);
      __hip_atomic_fetch_add(xg, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      wait_change(xg, g, ctl, spin_limit);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Orderings: position -> word
// ---------------------------------------------------------------------------

// The r-th (from 0) n-bit integer of weight k in increasing order
// (combinatorial number system: the top bit is the largest b with
// C(b, k) <= r).
__device__ __forceinline__ uint32_t unrank_weight(const Tables &L, unsigned long long r, int k, int n) {
  uint32_t x = 0;
  for (int b = n - 1; b >= 0 && k > 0; --b) {
    unsigned long long c = L.binom[b][k];
    if (r >= c) {
      x |= 1u << b;
      r -= c;
      --k;
    }
  }
  return x;
}

__device__ __forceinline__ uint32_t position_word(const Tables &L, int n, int ord, unsigned long long p) {
  if (ord == GC_LEX) return (uint32_t)p;
  if (ord == GC_GRAY) return (uint32_t)(p ^ (p >> 1));
  int w = 0;
  while (w < n && L.off[w + 1] <= p) ++w;
  unsigned long long r = p - L.off[w];
  if (ord == GC_GRLEX) return unrank_weight(L, r, w, n);
  // GREVLEX: inside weight w, the r-th word is the bit-reversed complement of
  // the r-th weight-(n-w) integer (complement reverses the increasing order,
  // bit reversal turns "differs first at the top" into "at the bottom").
  uint32_t y = unrank_weight(L, r, n - w, n);
  uint32_t mask = n == 32 ? 0xffffffffu : ((1u << n) - 1u);
  return __builtin_bitreverse32(~y & mask) >> (32 - n);
}

// Fill the binomial and weight-offset tables (whole workgroup).
__device__ void init_tables(Tables &T, int n) {
  for (int i = threadIdx.x; i < 33 * 33; i += blockDim.x) {
    const int a = i / 33, b = i % 33;
    // C(a, b) by the multiplicative formula, exact in 64 bits for a <= 32.
    unsigned long long c = 0;
    if (b <= a) {
      c = 1;
      for (int t = 1; t <= b; ++t) c = c * (unsigned long long)(a - b + t) / (unsigned long long)t;
    }
    T.binom[a][b] = (uint32_t)c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long acc = 0;
    for (int w = 0; w < 34; ++w) {
      T.off[w] = acc;
      if (w <= n) acc += T.binom[n][w];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// The screen: a tile of candidates against code[a, b), whole workgroup
// ---------------------------------------------------------------------------

// Candidates of a screen: window positions (id = offset from the window
// start) or the deep list (id = index into deep_word).  `dead` holds one bit
// per id; a set bit means "closer than d to a committed word".
struct Source {
  const Tables *tab;
  int n, ord;
  unsigned long long p0;
  const uint32_t *words;  // deep list, or null for window positions
  uint32_t *dead;
  __device__ uint32_t word(uint32_t id) const {
    return words ? words[id] : position_word(*tab, n, ord, p0 + id);
  }
  __device__ bool is_dead(uint32_t id) const { return (ld_relaxed(&dead[id >> 5]) >> (id & 31)) & 1; }
  __device__ void kill(uint32_t id) const {
    __hip_atomic_fetch_or(&dead[id >> 5], 1u << (id & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

// Workgroup compaction: threads of the first kRows waves offer (keep, word,
// id); kept entries go densely and in order to buffer dst.  Returns the count.
__device__ unsigned int tile_compact(TileLds &T, int dst, bool keep, uint32_t word, uint32_t id) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const unsigned long long m = ballot(keep);
  if (lane == 0 && wave < kRows) T.wcnt[wave] = (unsigned int)__builtin_popcountll(m);
  __syncthreads();
  unsigned int base = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kRows; ++w) {
    if (w < wave) base += T.wcnt[w];
    total += T.wcnt[w];
  }
  if (keep) {
    const unsigned int pos = base + (unsigned int)__builtin_popcountll(m & lanemask_lt());
    T.cw[dst][pos] = word;
    T.ci[dst][pos] = id;
  }
  __syncthreads();
  return total;
}

// One wave against its 64 words of the staged segment, ROWS rows of 64 live
// candidates; m[r] gets the lanes of row r closer than d to one of the words.
template <int ROWS>
__device__ __forceinline__ void segment_rows(const TileLds &T, int cur, int buf, unsigned int live,
                                             uint32_t d, unsigned long long (&m)[kRows]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x[ROWS], acc[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    const unsigned int idx = 64u * r + lane;
    x[r] = idx < live ? T.cw[cur][idx] : 0u;
    acc[r] = 0xffffffffu;
  }
  const uint4 *sp = reinterpret_cast<const uint4 *>(&T.seg[buf][64 * wave]);
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    const uint4 c = sp[i];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      acc[r] = umin3(acc[r], dist(x[r], c.x), dist(x[r], c.y));
      acc[r] = umin3(acc[r], dist(x[r], c.z), dist(x[r], c.w));
    }
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r) m[r] = 0;
#pragma unroll
  for (int r = 0; r < ROWS; ++r) m[r] = ballot(acc[r] < d && 64u * r + lane < live);
}

// Screen candidates id0 .. id0+nc-1 of `src` (nc <= kTile) against
// code[a, b), newest segment first, with the whole workgroup: each wave takes
// 64 words of a 1024-word segment staged in LDS (the next segment is
// prefetched into registers meanwhile).  After every segment the conflicts of
// all waves are merged, killed candidates are marked in `src`, candidates
// killed elsewhere are dropped, and the survivors are compacted, so the work
// per segment follows the live count and the loop stops when none is left.
// Returns the executed checks (candidate slots x words).
__device__ unsigned long long tile_screen(Lds &L, const Source &src, const uint32_t *code, uint32_t id0,
                                          uint32_t nc, unsigned long long a, unsigned long long b,
                                          uint32_t d) {
  TileLds &T = L.u.t;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  bool keep = false;
  uint32_t word = 0, id = 0;
  if (tid < (int)nc) {
    id = id0 + tid;
    keep = !src.is_dead(id);
    if (keep) word = src.word(id);
  }
  unsigned int live = tile_compact(T, 0, keep, word, id);
  int cur = 0, buf = 0;
  unsigned long long checks = 0;
  unsigned long long hi = b;
  uint32_t nxt = 0;
  if (live > 0 && hi > a) {
    const unsigned long long lo_s = hi > a + kSeg ? hi - kSeg : a;
    const unsigned long long idx = lo_s + tid;
    nxt = code[idx < hi ? idx : hi - 1];
  }
  while (live > 0 && hi > a) {
    const unsigned long long lo_s = hi > a + kSeg ? hi - kSeg : a;
    T.seg[buf][tid] = nxt;
    __syncthreads();
    if (lo_s > a) {  // prefetch the next (older) segment
      const unsigned long long lo2 = lo_s > a + kSeg ? lo_s - kSeg : a;
      const unsigned long long idx = lo2 + tid;
      nxt = code[idx < lo_s ? idx : lo_s - 1];
    }
    unsigned long long m[kRows];
    const unsigned int rows = (live + 63) / 64;
    if (rows == 1) segment_rows<1>(T, cur, buf, live, d, m);
    else if (rows == 2) segment_rows<2>(T, cur, buf, live, d, m);
    else if (rows == 3) segment_rows<3>(T, cur, buf, live, d, m);
    else segment_rows<4>(T, cur, buf, live, d, m);
    if (lane == 0) {
#pragma unroll
      for (int r = 0; r < kRows; ++r) T.killw[wave][r] = m[r];
    }
    checks += 64ull * rows * kSeg;
    __syncthreads();
    keep = false;
    if (tid < (int)live) {
      unsigned long long k = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) k |= T.killw[w][tid >> 6];
      const bool killed = (k >> (tid & 63)) & 1;
      word = T.cw[cur][tid];
      id = T.ci[cur][tid];
      if (killed) src.kill(id);
      keep = !killed && !src.is_dead(id);
    }
    live = tile_compact(T, cur ^ 1, keep, word, id);
    cur ^= 1;
    buf ^= 1;
    hi = lo_s;
  }
  return checks;
}

// Split of a 2-D screen (tiles x code range of `len` words) into items for
// the grid: enough range parts to give every workgroup an item, each part a
// whole number of segments.
struct Split {
  unsigned long long tiles, parts, plen;
};

__device__ __forceinline__ Split make_split(unsigned long long ncand, unsigned long long len) {
  Split sp;
  sp.tiles = (ncand + kTile - 1) / kTile;
  unsigned long long parts = (gridDim.x + sp.tiles - 1) / sp.tiles;
  const unsigned long long maxparts = (len + kSeg - 1) / kSeg;
  if (parts > maxparts) parts = maxparts;
  if (parts < 1) parts = 1;
  sp.plen = ((len + parts - 1) / parts + kSeg - 1) / kSeg * kSeg;
  sp.parts = (len + sp.plen - 1) / sp.plen;
  return sp;
}

// ---------------------------------------------------------------------------
// Phase D: in-window resolve on workgroup 0
// ---------------------------------------------------------------------------

__device__ void resolve_window(const Params &P, Lds &L) {
  const int tid = threadIdx.x;
  const unsigned int s = L.s;
  const int nb = (int)((s + 63) / 64);
  const int nadj = 64 * nb * (nb + 1) / 2;

  ResolveLds &R = L.u.r;
  if (L.round == 0) {
    for (unsigned int j = tid; j < s; j += kBlock) L.st[j] = L.lo == 0 ? ST_PASS : ST_UNKNOWN;
    if (P.mode == MODE_DEEP_ALL && L.lo > 0 && s > 0) {
      // Scan every survivor once; the resolve after that round has every fact.
      for (unsigned int k = tid; k < s; k += kBlock) {
        P.deep_word[k] = L.s1w[k];
        P.deep_idx[k] = k;
      }
      for (unsigned int k = tid; k < (s + 31) / 32; k += kBlock) P.deep_fail[k] = 0;
      if (tid == 0) {
        L.ndeep = s;
        P.ctl->ndeep = s;
        P.ctl->action = ACT_DEEP;
        P.ctl->stat_rounds += 1;
      }
      __syncthreads();
      return;
    }
  } else {
    for (unsigned int k = tid; k < L.ndeep; k += kBlock) {
      uint32_t word = ld_relaxed(&P.deep_fail[k >> 5]);
      L.st[P.deep_idx[k]] = (word >> (k & 31)) & 1 ? ST_FAIL : ST_PASS;
    }
  }
  for (int i = tid; i < nadj; i += kBlock) R.adj[i] = P.adj[i];
  __syncthreads();

  if (tid < 64) {
    const unsigned int lane = tid;
    unsigned int tcount = 0, ndeep = 0;
    for (int I = 0; I < nb; ++I) {
      const unsigned int j = 64u * I + lane;
      const int base = 64 * I * (I + 1) / 2;
      const bool valid = j < s;
      const int st = valid ? L.st[j] : ST_FAIL;
      bool killed = st == ST_FAIL;
      for (int J = 0; J < I; ++J) killed |= (R.adj[base + 64 * J + lane] & R.accm[J]) != 0;
      unsigned long long alive = ballot(!killed);
      const unsigned long long own = R.adj[base + 64 * I + lane];  // earlier neighbours in block
      unsigned long long acc = 0;
      while (alive) {
        const int i = __builtin_ctzll(alive);
        acc |= 1ull << i;
        alive &= ~(1ull << i);
        alive &= ~ballot((own >> i) & 1);
      }
      if (lane == 0) R.accm[I] = acc;
      const bool mine = (acc >> lane) & 1;
      const unsigned long long need = ballot(mine && st == ST_UNKNOWN);
      if (mine) R.tlist[tcount + __builtin_popcountll(acc & lanemask_lt())] = L.s1w[j];
      if (mine && st == ST_UNKNOWN) {
        const unsigned int k = ndeep + __builtin_popcountll(need & lanemask_lt());
        P.deep_word[k] = L.s1w[j];
        P.deep_idx[k] = j;
      }
      tcount += __builtin_popcountll(acc);
      ndeep += __builtin_popcountll(need);
    }
    if (lane == 0) {
      L.tcount = tcount;
      L.ndeep = ndeep;
    }
  }
  __syncthreads();

  const unsigned int tcount = L.tcount, ndeep = L.ndeep;
  if (ndeep > 0) {
    for (unsigned int k = tid; k < (ndeep + 31) / 32; k += kBlock) P.deep_fail[k] = 0;
    if (tid == 0) {
      P.ctl->ndeep = ndeep;
      P.ctl->action = ACT_DEEP;
      P.ctl->stat_rounds += 1;
    }
    __syncthreads();
    return;
  }

  // Commit: every tentatively accepted survivor is known to pass.
  const unsigned long long m0 = L.m0;
  unsigned long long room = P.capacity > m0 ? P.capacity - m0 : 0;
  const unsigned int nput = tcount < room ? tcount : (unsigned int)room;
  for (unsigned int k = tid; k < nput; k += kBlock) P.code[m0 + k] = R.tlist[k];

  // Next window length: aim for `target` survivors from this window's density.
  const unsigned long long nwin = L.pe - L.p0;
  unsigned long long next;
  if (L.truncated) {
    next = nwin * 3 / 4;
  } else if (L.s_tot == 0) {
    next = 2 * L.w;
  } else {
    next = L.w * P.target / L.s_tot;
    if (next > 2 * L.w) next = 2 * L.w;
  }
  if (next < kWMin) next = kWMin;
  if (next > kWMax) next = kWMax;
  next = (next + 63) & ~63ull;
  for (unsigned long long k = tid; k < (next + 31) / 32; k += kBlock) P.win_dead[k] = 0;

  if (tid == 0) {
    Ctl *ctl = P.ctl;
    ctl->stat_windows += 1;
    ctl->stat_surv += L.s;
    if (nput < tcount) {
      ctl->m = m0 + nput;
      set_status(ctl, GC_ECAPACITY);
      ctl->action = ACT_STOP;
    } else {
      ctl->m = m0 + tcount;
      ctl->p = L.pe;
      ctl->w = next;
      ctl->action = ACT_NEXT;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// The persistent kernel
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) greedy_kernel(Params P) {
  __shared__ Lds L;
  const int tid = threadIdx.x;
  const unsigned int lane = tid & 63;
  const unsigned long long gwave = (unsigned long long)blockIdx.x * kWaves + (tid >> 6);
  const unsigned long long nwaves = (unsigned long long)gridDim.x * kWaves;
  const uint32_t d = (uint32_t)P.d;
  unsigned long long my_near = 0, my_deep = 0, my_pairs = 0;

  init_tables(L.tab, P.n);
  barrier_join(L, P.bar, P.ctl, P.spin_limit);

  for (;;) {
    if (tid == 0) {
      L.p0 = ld_relaxed(&P.ctl->p);
      L.m0 = ld_relaxed(&P.ctl->m);
      L.w = ld_relaxed(&P.ctl->w);
      L.status = ld_relaxed(&P.ctl->status);
      L.round = 0;
    }
    __syncthreads();
    if (L.status != 0 || L.p0 >= P.total) break;
    const unsigned long long p0 = L.p0, m0 = L.m0;
    const unsigned long long pe0 = p0 + L.w < P.total ? p0 + L.w : P.total;
    const unsigned long long nwin = pe0 - p0;
    const unsigned long long lo = m0 > P.near_depth ? m0 - P.near_depth : 0;
    if (tid == 0) L.lo = lo;

    // ---- A: near screen of [p0, pe0) against code[lo, m0) -----------------
    if (m0 > lo) {
      const Split sp = make_split(nwin, m0 - lo);
      const Source src{&L.tab, P.n, P.ord, p0, nullptr, P.win_dead};
      for (unsigned long long it = blockIdx.x; it < sp.tiles * sp.parts; it += gridDim.x) {
        const unsigned long long part = it / sp.tiles, tile = it % sp.tiles;
        const unsigned long long b = m0 - part * sp.plen;
        const unsigned long long a = b > lo + sp.plen ? b - sp.plen : lo;
        const unsigned long long id0 = tile * kTile;
        const uint32_t nc = (uint32_t)(nwin - id0 < (unsigned long long)kTile ? nwin - id0 : kTile);
        my_near += tile_screen(L, src, P.code, (uint32_t)id0, nc, a, b, d);
      }
    }
    grid_barrier(L, P.bar, P.ctl, P.spin_limit);

    // ---- C: survivor list (every workgroup) and in-window pairs ------------
    {
      if (tid == 0) {
        L.s_tot = 0;
        L.truncated = 0;
        L.pe = pe0;
      }
      __syncthreads();
      const unsigned long long nwords = (nwin + 31) / 32;
      for (unsigned long long w0 = 0; w0 < nwords; w0 += kBlock) {
        const unsigned long long wi = w0 + tid;
        uint32_t liveb = 0;
        if (wi < nwords) {
          const uint32_t dead = ld_relaxed(&P.win_dead[wi]);
          const unsigned long long rem = nwin - wi * 32;
          const uint32_t valid = rem >= 32 ? 0xffffffffu : ((1u << rem) - 1u);
          liveb = ~dead & valid;
        }
        // workgroup exclusive scan of popcounts
        const unsigned int cnt = __builtin_popcount(liveb);
        unsigned int incl = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const unsigned int y = __shfl_up(incl, off);
          if ((int)lane >= off) incl += y;
        }
        if (lane == 63) L.wsum[tid >> 6] = incl;
        __syncthreads();
        unsigned int before = L.s_tot;
        for (int wv = 0; wv < (tid >> 6); ++wv) before += L.wsum[wv];
        unsigned int idx = before + incl - cnt;
        while (liveb) {
          const int bpos = __builtin_ctz(liveb);
          liveb &= liveb - 1;
          const unsigned long long off = wi * 32 + bpos;
          if (idx < (unsigned int)kSMax) {
            L.s1w[idx] = position_word(L.tab, P.n, P.ord, p0 + off);
          } else if (idx == (unsigned int)kSMax) {
            L.pe = p0 + off;  // the window ends before the first survivor that does not fit
            L.truncated = 1;
          }
          ++idx;
        }
        __syncthreads();
        if (tid == 0) {
          unsigned int tot = 0;
          for (int wv = 0; wv < kWaves; ++wv) tot += L.wsum[wv];
          L.s_tot += tot;
        }
        __syncthreads();
        if (L.truncated) break;
      }
      if (tid == 0) L.s = L.s_tot < (unsigned int)kSMax ? L.s_tot : (unsigned int)kSMax;
      __syncthreads();

      const unsigned int s = L.s;
      const unsigned int nb = (s + 63) / 64;
      const unsigned int ntiles = nb * (nb + 1) / 2;
      for (unsigned long long t = gwave; t < ntiles; t += nwaves) {
        unsigned int I = 0;
        while ((I + 1) * (I + 2) / 2 <= t) ++I;
        const unsigned int J = (unsigned int)t - I * (I + 1) / 2;
        const unsigned int j = 64 * I + lane;
        const uint32_t xj = j < s ? L.s1w[j] : 0u;
        const unsigned int cmax = J == I ? lane : (s - 64 * J < 64 ? s - 64 * J : 64);
        unsigned long long mask = 0;
        for (unsigned int c = 0; c < 64; ++c) {
          const uint32_t y = L.s1w[64 * J + c < s ? 64 * J + c : 0];
          if (c < cmax && dist(xj, y) < d) mask |= 1ull << c;
        }
        if (j >= s) mask = 0;
        P.adj[64 * (I * (I + 1) / 2) + 64 * J + lane] = mask;
        my_pairs += 64 * 64;
      }
    }
    grid_barrier(L, P.bar, P.ctl, P.spin_limit);

    // ---- D / E rounds ------------------------------------------------------
    for (;;) {
      if (blockIdx.x == 0) resolve_window(P, L);
      grid_barrier(L, P.bar, P.ctl, P.spin_limit);
      if (tid == 0) {
        L.action = ld_relaxed(&P.ctl->action);
        L.ndeep = ld_relaxed(&P.ctl->ndeep);
        L.status = ld_relaxed(&P.ctl->status);
      }
      __syncthreads();
      if (L.action != ACT_DEEP || L.status != 0) break;

      // ---- E: deep scan of the listed survivors against code[0, lo) ----------
      {
        const unsigned long long nd = L.ndeep;
        const Split sp = make_split(nd, lo);
        const Source src{&L.tab, P.n, P.ord, 0, P.deep_word, P.deep_fail};
        for (unsigned long long it = blockIdx.x; it < sp.tiles * sp.parts; it += gridDim.x) {
          const unsigned long long part = it / sp.tiles, tile = it % sp.tiles;
          const unsigned long long b = lo - part * sp.plen;
          const unsigned long long a = b > sp.plen ? b - sp.plen : 0;
          const unsigned long long id0 = tile * kTile;
          const uint32_t nc = (uint32_t)(nd - id0 < (unsigned long long)kTile ? nd - id0 : kTile);
          my_deep += tile_screen(L, src, P.code, (uint32_t)id0, nc, a, b, d);
        }
      }
      if (tid == 0) L.round += 1;
      grid_barrier(L, P.bar, P.ctl, P.spin_limit);
    }
    if (L.action == ACT_STOP || L.status != 0) break;
  }

  if (tid == 0) {
    __hip_atomic_fetch_add(&P.ctl->stat_near, my_near, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&P.ctl->stat_deep, my_deep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (lane == 0)
    __hip_atomic_fetch_add(&P.ctl->stat_pairs, my_pairs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (blockIdx.x == 0 && tid == 0 && P.count_out) *P.count_out = ld_relaxed(&P.ctl->m);
}

// Workspace initialisation (a kernel rather than memset, so that it can live
// in captured graphs).
__global__ void init_kernel(Ctl *ctl, Bar *bar, uint32_t *win_dead, unsigned long long w0) {
  const unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
  if (i == 0) {
    Ctl c;
    memset(&c, 0, sizeof(c));
    c.w = w0;
    *ctl = c;
  }
  for (unsigned long long k = i; k < sizeof(Bar) / sizeof(unsigned int);
       k += (unsigned long long)gridDim.x * blockDim.x)
    reinterpret_cast<unsigned int *>(bar)[k] = 0;
  for (unsigned long long k = i; k < kWMax / 32; k += (unsigned long long)gridDim.x * blockDim.x)
    win_dead[k] = 0;
}

// d = 1: every pair of distinct words is at distance >= 1, so the code is the
// whole ordering.
__global__ void emit_ordering_kernel(int n, int ord, uint32_t *code, unsigned long long count,
                                     unsigned long long *count_out) {
  __shared__ Tables T;
  init_tables(T, n);
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long p = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; p < count;
       p += stride)
    code[p] = position_word(T, n, ord, p);
  if (blockIdx.x == 0 && threadIdx.x == 0 && count_out) *count_out = count;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(GC_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                               \
  } while (0)

struct DeviceInfo {
  int cus = 0;
  int coop = 0;
  int max_blocks_per_cu = 0;
};

std::mutex g_info_mu;
DeviceInfo g_info[64];

int device_info(int dev, DeviceInfo *out) {
  std::lock_guard<std::mutex> lk(g_info_mu);
  if (dev < 0 || dev >= 64) return fail(GC_EDEVICE, "device ordinal %d out of range", dev);
  DeviceInfo &di = g_info[dev];
  if (di.cus == 0) {
    HIP_TRY(hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&di.coop, hipDeviceAttributeCooperativeLaunch, dev));
    int nb = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, greedy_kernel, kBlock, 0));
    di.max_blocks_per_cu = nb;
  }
  *out = di;
  return GC_OK;
}

unsigned long long binom_host(int a, int b) {
  if (b < 0 || b > a) return 0;
  unsigned long long c = 1;
  for (int t = 1; t <= b; ++t) c = c * (unsigned long long)(a - b + t) / (unsigned long long)t;
  return c;
}

}  // namespace gcimpl

using namespace gcimpl;

extern "C" {

const char *gc_last_error(void) { return g_error.c_str(); }

const char *gc_version(void) { return GC_VERSION_STRING; }

uint64_t greedy_code_capacity(int n, int d) {
  if (n < 1 || n > 32 || d < 1) return 0;
  if (d == 1) return 1ull << n;
  if (d > n) return 1;
  int nn = n, dd = d;
  if (dd % 2 == 0) {  // A(n, d) = A(n-1, d-1) for even d
    nn -= 1;
    dd -= 1;
  }
  const int t = (dd - 1) / 2;
  unsigned long long v = 0;
  for (int i = 0; i <= t; ++i) v += binom_host(nn, i);
  return (1ull << nn) / v;
}

int greedy_code_device_ex(int n, int d, int ordering, uint32_t *d_words, uint64_t capacity,
                          uint64_t *d_count, void *hip_stream, const gc_tuning *tuning,
                          gc_stats *stats) {
  g_error.clear();
  if (n < 1 || n > 32) return fail(GC_EINVAL, "n=%d outside [1, 32]", n);
  if (d < 1) return fail(GC_EINVAL, "d=%d must be >= 1", d);
  if (ordering < GC_LEX || ordering > GC_GREVLEX) return fail(GC_EINVAL, "unknown ordering %d", ordering);
  if (!d_count) return fail(GC_EINVAL, "d_count is NULL");
  if (!d_words && capacity > 0) return fail(GC_EINVAL, "d_words is NULL");
  if (((uintptr_t)d_words & 15u) != 0) return fail(GC_EINVAL, "d_words must be 16-byte aligned");
  if (capacity == 0) return fail(GC_ECAPACITY, "capacity 0 cannot hold the zero word");
  hipStream_t stream = (hipStream_t)hip_stream;
  if (stats) memset(stats, 0, sizeof(*stats));

  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DeviceInfo di;
  int rc = device_info(dev, &di);
  if (rc) return rc;

  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  HIP_TRY(hipEventCreate(&ev0));
  HIP_TRY(hipEventCreate(&ev1));
  const unsigned long long total = 1ull << n;

  if (d == 1) {
    const unsigned long long count = total < capacity ? total : capacity;
    HIP_TRY(hipEventRecord(ev0, stream));
    unsigned long long blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(emit_ordering_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, n,
                       ordering, d_words, count, (unsigned long long *)d_count);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(ev1, stream));
    HIP_TRY(hipEventSynchronize(ev1));
    if (stats) {
      stats->count = count;
      HIP_TRY(hipEventElapsedTime(&stats->kernel_ms, ev0, ev1));
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (count < total) return fail(GC_ECAPACITY, "code has %llu words, capacity %llu", total, capacity);
    return GC_OK;
  }

  if (!di.coop) return fail(GC_EDEVICE, "device %d does not support cooperative launch", dev);
  if (di.max_blocks_per_cu < 1) return fail(GC_EDEVICE, "kernel does not fit on a compute unit");
  unsigned int grid = (unsigned int)di.cus;
  if (tuning && tuning->grid_blocks) grid = tuning->grid_blocks;
  if (grid > (unsigned int)(di.cus * di.max_blocks_per_cu))
    return fail(GC_EINVAL, "grid_blocks %u exceeds co-resident limit %d", grid,
                di.cus * di.max_blocks_per_cu);

  // Workspace: control block, window dead mask, adjacency, deep lists.
  const size_t off_ctl = 0;
  const size_t off_bar = 512;
  const size_t off_dead = off_bar + ((sizeof(Bar) + 255) / 256) * 256;
  const size_t off_adj = off_dead + (kWMax / 32) * sizeof(uint32_t);
  const size_t off_dword = off_adj + kAdjWords * sizeof(unsigned long long);
  const size_t off_didx = off_dword + kSMax * sizeof(uint32_t);
  const size_t off_dfail = off_didx + kSMax * sizeof(uint32_t);
  const size_t ws_bytes = off_dfail + (kSMax / 32) * sizeof(uint32_t) + 256;
  char *ws = nullptr;
  HIP_TRY(hipMallocAsync((void **)&ws, ws_bytes, stream));

  Params P;
  memset(&P, 0, sizeof(P));
  P.n = n;
  P.d = d;
  P.ord = ordering;
  P.total = total;
  P.code = d_words;
  P.capacity = capacity;
  P.ctl = (Ctl *)(ws + off_ctl);
  P.bar = (Bar *)(ws + off_bar);
  P.count_out = (unsigned long long *)d_count;
  P.win_dead = (uint32_t *)(ws + off_dead);
  P.adj = (unsigned long long *)(ws + off_adj);
  P.deep_word = (uint32_t *)(ws + off_dword);
  P.deep_idx = (uint32_t *)(ws + off_didx);
  P.deep_fail = (uint32_t *)(ws + off_dfail);
  P.near_depth = (tuning && tuning->near_depth) ? tuning->near_depth : kDefaultNear;
  P.target = (tuning && tuning->target_survivors) ? tuning->target_survivors : kDefaultTarget;
  if (P.target > (unsigned int)kSMax) P.target = kSMax;
  if (P.target < 16) P.target = 16;
  P.spin_limit = kDefaultSpin;
  // Resolve mode: graded orders reject many survivors deep in the code, so
  // scanning every survivor once beats repeated tentative rounds there.
  P.mode = (ordering == GC_GRLEX || ordering == GC_GREVLEX) ? MODE_DEEP_ALL : MODE_TENTATIVE;
  if (tuning && tuning->resolve_mode) P.mode = tuning->resolve_mode == 2 ? MODE_DEEP_ALL : MODE_TENTATIVE;
  if (const char *env = getenv("GC_SPIN_LIMIT")) P.spin_limit = (unsigned int)strtoul(env, nullptr, 0);

  int status = GC_OK;
  hipLaunchKernelGGL(init_kernel, dim3(8), dim3(256), 0, stream, P.ctl, P.bar, P.win_dead,
                     (unsigned long long)kWMin);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(ev0, stream);
  if (e == hipSuccess) {
    void *args[] = {&P};
    e = hipLaunchCooperativeKernel((const void *)greedy_kernel, dim3(grid), dim3(kBlock), args, 0,
                                   stream);
  }
  if (e == hipSuccess) e = hipEventRecord(ev1, stream);
  Ctl host_ctl;
  memset(&host_ctl, 0, sizeof(host_ctl));
  if (e == hipSuccess) e = hipMemcpyAsync(&host_ctl, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  hipError_t ef = hipFreeAsync(ws, stream);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    return fail(GC_EDEVICE, "greedy kernel failed: %s", hipGetErrorString(e));
  }
  if (ef != hipSuccess) return fail(GC_EDEVICE, "hipFreeAsync failed: %s", hipGetErrorString(ef));
  if (stats) {
    stats->count = host_ctl.m;
    stats->windows = host_ctl.stat_windows;
    stats->resolve_rounds = host_ctl.stat_rounds;
    stats->survivors = host_ctl.stat_surv;
    stats->checks_near = host_ctl.stat_near;
    stats->checks_deep = host_ctl.stat_deep;
    stats->checks_pairs = host_ctl.stat_pairs;
    (void)hipEventElapsedTime(&stats->kernel_ms, ev0, ev1);
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  status = host_ctl.status;
  if (status == GC_ECAPACITY)
    return fail(GC_ECAPACITY, "code exceeds capacity %llu", (unsigned long long)capacity);
  if (status == GC_ETIMEOUT) return fail(GC_ETIMEOUT, "device barrier wait expired");
  if (status != 0) return fail(GC_EDEVICE, "device status %d", status);
  return GC_OK;
}

int greedy_code_device(int n, int d, int ordering, uint32_t *d_words, uint64_t capacity,
                       uint64_t *d_count, void *hip_stream) {
  return greedy_code_device_ex(n, d, ordering, d_words, capacity, d_count, hip_stream, nullptr,
                               nullptr);
}

int greedy_code(int n, int d, int ordering, uint32_t *out_words, uint64_t *out_count) {
  g_error.clear();
  if (!out_count) return fail(GC_EINVAL, "out_count is NULL");
  const uint64_t bound = greedy_code_capacity(n, d);
  if (bound == 0) return fail(GC_EINVAL, "invalid n=%d or d=%d", n, d);
  if (ordering < GC_LEX || ordering > GC_GREVLEX) return fail(GC_EINVAL, "unknown ordering %d", ordering);
  const uint64_t cap = *out_count;
  if (!out_words && cap > 0) return fail(GC_EINVAL, "out_words is NULL");
  const uint64_t dcap = cap < bound ? cap : bound;
  if (dcap == 0) {
    *out_count = bound;
    return fail(GC_ECAPACITY, "capacity 0 cannot hold the zero word");
  }
  uint32_t *dw = nullptr;
  uint64_t *dc = nullptr;
  HIP_TRY(hipMalloc((void **)&dw, dcap * sizeof(uint32_t)));
  hipError_t e = hipMalloc((void **)&dc, sizeof(uint64_t));
  if (e != hipSuccess) {
    (void)hipFree(dw);
    return fail(GC_ENOMEM, "hipMalloc failed: %s", hipGetErrorString(e));
  }
  int rc = greedy_code_device(n, d, ordering, dw, dcap, dc, nullptr);
  if (rc == GC_OK) {
    uint64_t count = 0;
    e = hipMemcpy(&count, dc, sizeof(count), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(out_words, dw, count * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = fail(GC_EDEVICE, "hipMemcpy failed: %s", hipGetErrorString(e));
    else *out_count = count;
  } else if (rc == GC_ECAPACITY) {
    *out_count = bound;
  }
  (void)hipFree(dw);
  (void)hipFree(dc);
  return rc;
}

}  // extern "C"
