// server.hip -- continuous-batching job server over the persistent kernel.
//
// Jobs (codes to build) are admitted when the device arena has room for their
// worst-case code (greedy_code_capacity words); admitted jobs are published
// into a ring of job descriptors in coherent pinned host memory, where the
// running persistent kernel's teams claim them.  A job that arrives while
// others are being built is picked up by the first team that frees up, so
// builds of different codes overlap on the device.  Finished codes stay in the
// arena until released.  The kernel exits after a bounded idle period and is
// relaunched when new work is published.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <stdlib.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <list>
#include <iterator>
#include <thread>
#include <map>
#include <mutex>
#include <set>
#include <vector>

#include "gc_internal.h"
#include "greedy_code.h"

namespace gcimpl {

constexpr unsigned int kServerSlots = 1u << 16;   // jobs over the life of one server
constexpr unsigned int kServerIdlePolls = 50000;  // about 0.1 s of empty queue before the kernel exits
// A job whose exhaustive work bound 2^n * capacity(n, d) reaches this is
// "wide": it goes to the wide ring, which the team spanning half of the XCDs
// serves first (on one XCD's team it would take up to eight times longer and
// stretch the makespan); the other jobs go to the narrow ring, served by the
// teams of the other half and, when no wide job waits, by the wide team too.
constexpr double kWideWork = 274877906944.0;  // 2^38
// Narrow jobs may be admitted past a wide job that waits for arena space,
// until that wide job has waited this long; then admission stops behind it
// until it fits.
constexpr double kWideAdmitWaitS = 1.0;

struct Ticket {
  int n, d, ord;
  std::chrono::steady_clock::time_point submitted;
  size_t bytes = 0, offset = 0;
  bool has_space = false;   // owns `bytes` of the arena at `offset`
  int state = GC_JOB_WAITING;
  int status = 0;           // GC_OK, or the failure code once FAILED
  int slot = -1;
};

}  // namespace gcimpl

struct gc_server {
  std::mutex mu;
  int teams = 8;            // as passed to gc_server_create
  int launch_teams = 1;     // teams of a launch: `teams`, or 1 wide + `teams` narrow (one XCD each)
  bool stopped = false;     // a bounded device-side wait expired: no further launches
  unsigned int grid = 0;
  hipStream_t stream = nullptr;
  hipEvent_t kernel_done = nullptr;
  bool launched = false;
  // device
  char *dev = nullptr;            // Bar | DevQueue | team workspaces
  gcimpl::Bar *bar = nullptr;
  gcimpl::DevQueue *dq = nullptr;
  char *team_ws = nullptr;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  // pinned host mirror of the arena: the kernel writes each finished code
  // there too, so fetching a result needs no device copy
  char *mirror = nullptr;
  char *mirror_dev = nullptr;
  // pinned host (device-visible)
  gcimpl::HostQueue *hq = nullptr;
  gcimpl::Job *jobs = nullptr;
  gcimpl::HostQueue *hq_dev = nullptr;
  gcimpl::Job *jobs_dev = nullptr;
  unsigned int *ring = nullptr, *ring_dev = nullptr;            // narrow ring (pinned, mapped)
  unsigned int *ring_wide = nullptr, *ring_wide_dev = nullptr;  // wide ring
  unsigned int published = 0, published_narrow = 0, published_wide = 0;
  // host bookkeeping
  std::map<size_t, size_t> free_ranges;   // offset -> length
  std::map<uint64_t, gcimpl::Ticket> tickets;
  std::list<uint64_t> waiting;
  std::set<uint64_t> inflight;            // admitted, not yet seen finished
  std::vector<uint64_t> slot_ticket;
  uint64_t next_ticket = 1;
};

namespace gcimpl {

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

bool arena_alloc(gc_server *s, size_t bytes, size_t *off) {
  for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      s->free_ranges.erase(it);
      if (rest) s->free_ranges[at] = rest;
      return true;
    }
  }
  return false;
}

void arena_free(gc_server *s, size_t off, size_t bytes) {
  auto it = s->free_ranges.emplace(off, bytes).first;
  auto next = std::next(it);
  if (next != s->free_ranges.end() && it->first + it->second == next->first) {
    it->second += next->second;
    s->free_ranges.erase(next);
  }
  if (it != s->free_ranges.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      s->free_ranges.erase(it);
    }
  }
}

bool kernel_running(gc_server *s) {
  if (!s->launched) return false;
  return hipEventQuery(s->kernel_done) == hipErrorNotReady;
}

// Wide XCDs of a server: teams 2 and 4 split the 8 XCDs into one wide team
// of 8 - teams XCDs and `teams` narrow teams of one XCD; teams 1 and 8 have
// equal teams (one team spanning the GPU, or one per XCD) and one queue.
int wide_xcds(int teams) { return teams == 2 || teams == 4 ? 8 - teams : 0; }

bool is_wide(const gc_server *s, int n, int d) {
  return wide_xcds(s->teams) > 0 && std::ldexp((double)greedy_code_capacity(n, d), n) >= kWideWork;
}

int launch_server_kernel(gc_server *s) {
  Params P;
  memset(&P, 0, sizeof(P));
  P.jobs = s->jobs_dev;
  P.hq = s->hq_dev;
  P.dq = s->dq;
  P.bar = s->bar;
  P.njobs_fixed = -1;
  P.nteams = s->launch_teams;
  P.split = wide_xcds(s->teams);
  P.ring = s->ring_dev;
  P.ring_wide = s->ring_wide_dev;
  P.spin_limit = 1u << 25;
  if (const char *env = getenv("GC_SPIN_LIMIT")) P.spin_limit = (unsigned int)strtoul(env, nullptr, 0);
  P.idle_limit = kServerIdlePolls;
  P.team_ws = s->team_ws;
  P.team_ws_stride = team_workspace_bytes();
  hipError_t e = launch_init(s->bar, s->dq, 0, s->stream);
  if (e == hipSuccess) e = launch_persistent(P, s->grid, s->stream, LaunchKind::kServer);
  if (e == hipSuccess) e = hipEventRecord(s->kernel_done, s->stream);
  if (e != hipSuccess) return fail(GC_EDEVICE, "server launch failed: %s", hipGetErrorString(e));
  s->launched = true;
  return GC_OK;
}

// Every job not yet finished fails with `code` (waiting ones included), and
// the server launches nothing more.  Jobs the device did finish keep their
// results.
void fail_unfinished(gc_server *s, int code) {
  s->stopped = true;
  for (uint64_t id : s->inflight) {
    Ticket &t = s->tickets[id];
    const Job &J = s->jobs[t.slot];
    if (__atomic_load_n(&J.done, __ATOMIC_ACQUIRE)) {
      t.status = J.status;
      t.state = t.status == 0 ? GC_JOB_DONE : GC_JOB_FAILED;
    } else {
      t.state = GC_JOB_FAILED;
      t.status = code;
    }
  }
  s->inflight.clear();
  for (uint64_t id : s->waiting) {
    Ticket &t = s->tickets[id];
    t.state = GC_JOB_FAILED;
    t.status = code;
  }
  s->waiting.clear();
}

// Admit waiting jobs in arrival order while the arena has room, publish them,
// and make sure a kernel is running while published work is unfinished.
int pump(gc_server *s) {
  if (s->stopped) return GC_OK;
  bool published_any = false;
  // Arrival order, except that a narrow job may pass a wide job that waits
  // for arena space (for at most kWideAdmitWaitS, so wide jobs do not
  // starve).
  const auto now = std::chrono::steady_clock::now();
  bool blocked_wide = false;
  for (auto it = s->waiting.begin(); it != s->waiting.end();) {
    const uint64_t id = *it;
    Ticket &t = s->tickets[id];
    const bool wide = is_wide(s, t.n, t.d);
    if (!wide && blocked_wide) break;
    size_t off = 0;
    if (!arena_alloc(s, t.bytes, &off)) {
      if (!wide) break;  // narrow jobs are admitted in order
      const double waited = std::chrono::duration<double>(now - t.submitted).count();
      if (waited > kWideAdmitWaitS) blocked_wide = true;
      ++it;
      continue;
    }
    if (s->published >= kServerSlots) {
      arena_free(s, off, t.bytes);
      return fail(GC_ENOMEM, "server job slots exhausted (%u)", kServerSlots);
    }
    it = s->waiting.erase(it);
    t.offset = off;
    t.has_space = true;
    t.slot = (int)s->published;
    t.state = GC_JOB_ADMITTED;
    Job *J = &s->jobs[t.slot];
    memset(J, 0, sizeof(*J));
    J->n = t.n;
    J->d = t.d;
    J->ord = t.ord;
    J->code = reinterpret_cast<uint32_t *>(s->arena + off);
    J->capacity = greedy_code_capacity(t.n, t.d);
    J->count = nullptr;
    J->host_copy = reinterpret_cast<uint32_t *>(s->mirror_dev + off);
    J->wide = wide ? 1 : 0;
    if (J->wide) s->ring_wide[s->published_wide++] = (unsigned int)t.slot;
    else s->ring[s->published_narrow++] = (unsigned int)t.slot;
    gc_tuning tu;
    if (tuned_for(t.n, t.d, t.ord, &tu)) {
      J->near_depth = tu.near_depth;
      J->target = tu.target_survivors;
      J->mode = (int)tu.resolve_mode;
      J->deep_tile = tu.deep_tile;
      J->valu_screen = tu.valu_screen;
    }
    s->slot_ticket[t.slot] = id;
    s->inflight.insert(id);
    ++s->published;
    published_any = true;
  }
  if (published_any) {
    std::atomic_thread_fence(std::memory_order_seq_cst);
    __atomic_store_n(&s->hq->submitted_wide, s->published_wide, __ATOMIC_RELEASE);
    __atomic_store_n(&s->hq->submitted, s->published_narrow, __ATOMIC_RELEASE);
  }
  // Relaunch if published jobs are unfinished and no kernel is running (the
  // previous one may have gone idle just before the publication, stopped at
  // a job of the other kind, or given up on a bounded wait).
  if (!kernel_running(s)) {
    bool unfinished = false;
    for (uint64_t id : s->inflight)
      if (!__atomic_load_n(&s->jobs[s->tickets[id].slot].done, __ATOMIC_ACQUIRE)) {
        unfinished = true;
        break;
      }
    if (!unfinished) return GC_OK;
    // The last launch has finished: its queue state tells where to resume.
    DevQueue dq;
    memset(&dq, 0, sizeof(dq));
    hipError_t e = hipSuccess;
    if (s->launched) {
      e = hipMemcpyAsync(&dq, s->dq, sizeof(dq), hipMemcpyDeviceToHost, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return fail(GC_EDEVICE, "server queue read failed: %s", hipGetErrorString(e));
    }
    if (dq.abort) {
      // A device-side wait expired: the jobs that launch claimed are lost,
      // and the device made no guaranteed progress; stop here rather than
      // relaunch.
      fail_unfinished(s, GC_ETIMEOUT);
      return GC_OK;
    }
    return launch_server_kernel(s);
  }
  return GC_OK;
}

void refresh(gc_server *s, uint64_t id, Ticket &t) {
  if (t.state == GC_JOB_ADMITTED && __atomic_load_n(&s->jobs[t.slot].done, __ATOMIC_ACQUIRE)) {
    t.status = s->jobs[t.slot].status;
    t.state = t.status == 0 ? GC_JOB_DONE : GC_JOB_FAILED;
    s->inflight.erase(id);
  }
}

}  // namespace gcimpl

using namespace gcimpl;

extern "C" {

int gc_server_create(size_t arena_bytes, int teams, gc_server **out) {
  g_error.clear();
  if (!out) return fail(GC_EINVAL, "out is NULL");
  *out = nullptr;
  if (teams != 1 && teams != 2 && teams != 4 && teams != 8)
    return fail(GC_EINVAL, "teams must be 1, 2, 4 or 8 (got %d)", teams);
  if (arena_bytes < 256) return fail(GC_EINVAL, "arena of %zu bytes is too small", arena_bytes);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(GC_EDEVICE, "no HIP device");
  int cus = 0, coop = 0, bpc = 0;
  int rc = device_info(dev, &cus, &coop, &bpc);
  if (rc) return rc;
  if (!coop || bpc < 1) return fail(GC_EDEVICE, "cooperative persistent kernel unavailable");
  gc_server *s = new gc_server();
  s->teams = teams;
  s->launch_teams = wide_xcds(teams) ? 1 + teams : teams;
  s->grid = (unsigned int)cus;
  s->arena_bytes = round256(arena_bytes);
  const size_t off_dq = round256(sizeof(Bar));
  const size_t off_ws = off_dq + round256(sizeof(DevQueue));
  const size_t ws_bytes = off_ws + team_workspace_bytes() * (size_t)s->launch_teams;
  hipError_t e = hipMalloc((void **)&s->dev, ws_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&s->arena, s->arena_bytes);
  if (e == hipSuccess) e = hipMemset(s->dev, 0, ws_bytes);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&s->hq, sizeof(HostQueue), hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&s->jobs, sizeof(Job) * kServerSlots, hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&s->mirror, s->arena_bytes, hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&s->ring, sizeof(unsigned int) * kServerSlots, hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&s->ring_wide, sizeof(unsigned int) * kServerSlots,
                      hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&s->ring_dev, s->ring, 0);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&s->ring_wide_dev, s->ring_wide, 0);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&s->mirror_dev, s->mirror, 0);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&s->hq_dev, s->hq, 0);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&s->jobs_dev, s->jobs, 0);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->kernel_done, hipEventDisableTiming);
  if (e != hipSuccess) {
    gc_server_destroy(s);
    return fail(GC_ENOMEM, "server allocation failed: %s", hipGetErrorString(e));
  }
  memset(s->hq, 0, sizeof(HostQueue));
  memset(s->jobs, 0, sizeof(Job) * kServerSlots);
  s->bar = reinterpret_cast<Bar *>(s->dev);
  s->dq = reinterpret_cast<DevQueue *>(s->dev + off_dq);
  s->team_ws = s->dev + off_ws;
  s->free_ranges[0] = s->arena_bytes;
  s->slot_ticket.assign(kServerSlots, 0);
  *out = s;
  return GC_OK;
}

int gc_server_submit(gc_server *s, int n, int d, int ordering, uint64_t *ticket) {
  g_error.clear();
  if (!s || !ticket) return fail(GC_EINVAL, "NULL argument");
  if (n < 1 || n > 32 || d < 1 || ordering < GC_LEX || ordering > GC_GREVLEX)
    return fail(GC_EINVAL, "invalid job n=%d d=%d ordering=%d", n, d, ordering);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopped) return fail(GC_ETIMEOUT, "server stopped after a device-side wait expired");
  Ticket t;
  t.n = n;
  t.d = d;
  t.ord = ordering;
  t.bytes = round256(greedy_code_capacity(n, d) * sizeof(uint32_t));
  t.submitted = std::chrono::steady_clock::now();
  if (t.bytes > s->arena_bytes)
    return fail(GC_ENOMEM, "job needs %zu bytes, arena holds %zu", t.bytes, s->arena_bytes);
  const uint64_t id = s->next_ticket++;
  s->tickets[id] = t;
  s->waiting.push_back(id);
  *ticket = id;
  return pump(s);
}

int gc_server_poll(gc_server *s, uint64_t ticket, int *state, uint64_t *count) {
  g_error.clear();
  if (!s || !state) return fail(GC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(GC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  int rc = pump(s);
  if (rc) return rc;
  refresh(s, it->first, it->second);
  *state = it->second.state;
  if (count) *count = it->second.state == GC_JOB_DONE ? s->jobs[it->second.slot].out_count : 0;
  return GC_OK;
}

int gc_server_words(gc_server *s, uint64_t ticket, const uint32_t **d_words, uint64_t *count) {
  g_error.clear();
  if (!s || !d_words || !count) return fail(GC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(GC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  refresh(s, it->first, it->second);
  if (it->second.state == GC_JOB_FAILED)
    return fail(it->second.status, "job failed with status %d", it->second.status);
  if (it->second.state != GC_JOB_DONE) return fail(GC_EBUSY, "job not finished");
  *d_words = reinterpret_cast<const uint32_t *>(s->arena + it->second.offset);
  *count = s->jobs[it->second.slot].out_count;
  return GC_OK;
}

int gc_server_fetch(gc_server *s, uint64_t ticket, uint32_t *host_words, uint64_t cap, uint64_t *count) {
  const uint32_t *dw = nullptr;
  uint64_t m = 0;
  int rc = gc_server_words(s, ticket, &dw, &m);
  if (rc) return rc;
  if (count) *count = m;
  if (m > cap) return fail(GC_ECAPACITY, "code has %llu words, buffer %llu", (unsigned long long)m,
                           (unsigned long long)cap);
  if (!host_words && m) return fail(GC_EINVAL, "host_words is NULL");
  // The kernel wrote the words to the host mirror before publishing `done`
  // (observed with acquire by gc_server_words), so this is a host copy.
  std::lock_guard<std::mutex> lk(s->mu);
  const size_t off = reinterpret_cast<const char *>(dw) - s->arena;
  if (m) memcpy(host_words, s->mirror + off, m * sizeof(uint32_t));
  return GC_OK;
}

int gc_server_release(gc_server *s, uint64_t ticket) {
  g_error.clear();
  if (!s) return fail(GC_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(GC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  refresh(s, it->first, it->second);
  if (it->second.state == GC_JOB_WAITING || it->second.state == GC_JOB_ADMITTED)
    return fail(GC_EBUSY, "job not finished");
  if (it->second.has_space) arena_free(s, it->second.offset, it->second.bytes);
  s->tickets.erase(it);
  return pump(s);
}

int gc_server_stats(gc_server *s, uint64_t ticket, gc_stats *stats, double *device_ms) {
  g_error.clear();
  if (!s) return fail(GC_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(GC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  refresh(s, it->first, it->second);
  if (it->second.state != GC_JOB_DONE && it->second.state != GC_JOB_FAILED)
    return fail(GC_EBUSY, "job not finished");
  if (it->second.slot < 0) return fail(it->second.status, "job failed before it was admitted");
  const Job &J = s->jobs[it->second.slot];
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->count = J.out_count;
    stats->windows = J.windows;
    stats->resolve_rounds = J.rounds;
    stats->survivors = J.survivors;
    stats->checks_near = J.chk_near;
    stats->checks_deep = J.chk_deep;
    stats->checks_pairs = J.chk_pairs;
    stats->near_ms = J.ticks_near / 1e5;
    stats->survivors_ms = J.ticks_surv / 1e5;
    stats->resolve_ms = J.ticks_resolve / 1e5;
    stats->deep_ms = J.ticks_deep / 1e5;
  }
  if (device_ms) *device_ms = (double)(J.t_done - J.t_claim) / 1e5;
  return GC_OK;
}

int gc_server_drain(gc_server *s, int timeout_ms) {
  g_error.clear();
  if (!s) return fail(GC_EINVAL, "NULL server");
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      int rc = pump(s);
      if (rc) return rc;
      std::vector<uint64_t> ids(s->inflight.begin(), s->inflight.end());
      for (uint64_t id : ids) refresh(s, id, s->tickets[id]);
      if (s->waiting.empty() && s->inflight.empty()) return GC_OK;
    }
    const auto el = std::chrono::duration_cast<std::chrono::milliseconds>(std::chrono::steady_clock::now() - t0);
    if (timeout_ms >= 0 && el.count() > timeout_ms) return fail(GC_ETIMEOUT, "drain timed out");
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

int gc_server_destroy(gc_server *s) {
  if (!s) return GC_OK;
  if (s->hq) __atomic_store_n(&s->hq->shutdown, 1u, __ATOMIC_RELEASE);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->kernel_done) (void)hipEventDestroy(s->kernel_done);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->jobs) (void)hipHostFree(s->jobs);
  if (s->hq) (void)hipHostFree(s->hq);
  if (s->arena) (void)hipFree(s->arena);
  if (s->mirror) (void)hipHostFree(s->mirror);
  if (s->ring) (void)hipHostFree(s->ring);
  if (s->ring_wide) (void)hipHostFree(s->ring_wide);
  if (s->dev) (void)hipFree(s->dev);
  delete s;
  return GC_OK;
}

}  // extern "C"
