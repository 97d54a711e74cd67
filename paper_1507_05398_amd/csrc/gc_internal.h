// gc_internal.h -- structures shared by the persistent kernel and the host
// code of libgreedy_code.so (single code, batch and server entry points).
// Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "greedy_code.h"

namespace gcimpl {

constexpr int kBlock = 1024;   // threads per workgroup
constexpr int kMaxXcd = 16;    // XCD ids are taken modulo this
constexpr int kMaxTeams = 8;

// One code to build.  In batch mode the array lives in device memory, in
// server mode in pinned host memory (coherent, mapped): the device reads the
// inputs once and writes the outputs, `done` last.
struct Job {
  // inputs
  int n, d, ord, mode;            // mode: 0 by ordering, 1 tentative, 2 deep-scan all survivors
  unsigned long long near_depth;  // 0: default
  unsigned int target;            // 0: default
  unsigned int deep_tile;         // candidates per deep-scan tile (0: default)
  unsigned int valu_screen;       // 1: distance screens on the vector ALU instead of the matrix cores
  uint32_t *code;                 // device array of `capacity` words (16-byte aligned)
  unsigned long long capacity;
  unsigned long long *count;      // device counter written at completion (may be null)
  uint32_t *host_copy;            // device-visible pinned host array that receives the words
                                  // before `done` is set (may be null)
  int wclass;                     // 0: every weight is a candidate; w + 1: only weight w
  int so;                         // 1: self-orthogonal (even weights, even common ones)
  unsigned long long p_start;     // first position screened
  unsigned long long p_stop;      // end of the screened positions (0: the walk's end)
  unsigned long long m_start;     // words already in `code` (accepted before p_start)
  uint32_t basis[32];             // GC_BORDER: b_1 .. b_n
  // outputs
  unsigned long long out_count;
  unsigned long long windows, rounds, survivors, chk_near, chk_deep, chk_pairs;
  unsigned long long ticks_near, ticks_surv, ticks_resolve, ticks_deep;  // phase time (100 MHz)
  unsigned long long t_claim, t_done;  // device wall clock (100 MHz) at claim / completion
  int status;
  unsigned int done;              // 0 pending, 1 finished (written last)
  int wide;                       // server: queued on the wide ring
};

// Job queue.  `submitted` and `shutdown` may live in host memory (server);
// `claimed` and `abort` always live in device memory.
struct HostQueue {
  unsigned int submitted;   // batch: jobs visible to the device; server: entries of the narrow ring
  unsigned int shutdown;    // host sets 1: the kernel exits when idle
  unsigned int submitted_wide;  // server: entries of the wide ring
  unsigned int pad[61];
};

struct DevQueue {
  unsigned int claimed;     // next job (batch) or narrow-ring entry (server) to claim
  unsigned int completed;   // jobs finished
  int abort;                // a bounded wait expired: every team stops
  unsigned int launches;
  unsigned int claimed_wide;  // server: next wide-ring entry to claim
  unsigned int pad[59];
};

// Per-team instance state.
struct Ctl {
  unsigned long long m;   // committed words
  unsigned long long p;   // start of the next window
  unsigned long long w;   // length of the next window
  int status;
  int action;
  unsigned int ndeep;
  int job;                // job being built, -1 when the team stops
  unsigned long long stat_windows, stat_rounds, stat_surv, stat_near, stat_deep, stat_pairs;
  unsigned long long ticks[4];   // near screen, survivors+pairs, resolve, deep scan
  unsigned int resolved;          // generation: bumped by team rank 0 after each resolve
  unsigned int pad[23];
};

// Barrier state: per XCD a counter, a generation and the member count (each
// on its own 256-byte line); per team a counter and generation for the XCD
// leaders; a one-time join count.
struct Bar {
  unsigned int join_count;
  unsigned int pad0[63];
  unsigned int xcd[kMaxXcd][64];     // [0] count, [1] generation, [2] members
  unsigned int team[kMaxTeams][64];  // [0] count, [1] generation, [2] members, [3] xcds
};

struct Params {
  Job *jobs;
  HostQueue *hq;
  DevQueue *dq;
  Bar *bar;
  int njobs_fixed;               // batch: number of jobs; server: -1 (read hq->submitted)
  int nteams;
  // Server split: team 0 is the XCDs whose id mod 8 is below `split` and
  // claims from the wide ring first, then the narrow ring; each other XCD is
  // one of the teams 1 .. nteams-1, which claim from the narrow ring only.
  // 0: teams are XCD id mod nteams and claim one queue (batch, or a one-team
  // server).
  int split;
  unsigned int *ring;            // server: job indices in publication order (narrow jobs)
  unsigned int *ring_wide;       // server: job indices of the wide jobs
  unsigned int spin_limit;       // bounded waits inside a job
  unsigned int idle_limit;       // server: polls of an empty queue before the kernel exits
  char *team_ws;                 // per-team workspace, team_ws_stride bytes each
  unsigned long long team_ws_stride;
};

size_t team_workspace_bytes();
int device_info(int dev, int *cus, int *coop, int *blocks_per_cu);
// Which kernel symbol a persistent launch uses (same code; separate names in
// profiles).
enum class LaunchKind { kSingle, kSingleSO, kBatch, kServer };

hipError_t launch_persistent(const Params &P, unsigned int grid, hipStream_t stream, LaunchKind kind);
hipError_t launch_init(Bar *bar, DevQueue *dq, int reset_queue, hipStream_t stream);
int fail(int code, const char *fmt, ...);
// Tuning remembered by greedy_code_tune for (current device, n, d, ordering).
bool tuned_for(int n, int d, int ordering, gc_tuning *out);
// Helpers shared by the entry points.
int check_job_args(int n, int d, int ordering);
int pick_grid(unsigned int requested, unsigned int *grid);
unsigned int spin_limit_from_env();
void fill_job(Job *J, int n, int d, int ordering, uint32_t *words, uint64_t capacity, uint64_t *count,
              const gc_tuning *tuning);
// Validates a caller's job array and fills `J` (caller order) and `order`
// (queue position -> caller index, longest jobs first).
int prepare_batch(const gc_job *jobs, int njobs, Job *J, int *order);
extern thread_local std::string g_error;

}  // namespace gcimpl
