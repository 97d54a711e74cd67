// batch_graph.hip -- a batch launch captured once into a HIP graph and
// replayed: the upload of the job table (from pinned host memory), the reset
// kernel of the barrier block and job queue, the cooperative persistent
// launch and the download of the job outputs (into pinned host memory).  A
// replay costs one hipGraphLaunch; its buffers are allocated at creation.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <vector>

#include "gc_internal.h"
#include "greedy_code.h"

struct gc_batch_graph {
  int njobs = 0, teams = 0;
  std::vector<int> order;              // queue position -> caller's job index
  char *dev = nullptr;                 // Bar | DevQueue | job table | team workspaces
  gcimpl::Job *jobs_in = nullptr;      // pinned: job inputs, queue order
  gcimpl::Job *jobs_out = nullptr;     // pinned: job outputs, queue order
  gcimpl::DevQueue *dq_out = nullptr;  // pinned: queue state after the launch (abort flag)
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace gcimpl {
namespace {

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

void release(gc_batch_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->capture) (void)hipStreamDestroy(g->capture);
  if (g->jobs_in) (void)hipHostFree(g->jobs_in);
  if (g->jobs_out) (void)hipHostFree(g->jobs_out);
  if (g->dq_out) (void)hipHostFree(g->dq_out);
  if (g->dev) (void)hipFree(g->dev);
  delete g;
}

}  // namespace
}  // namespace gcimpl

using namespace gcimpl;

extern "C" {

int gc_batch_graph_create(const gc_job *jobs, int njobs, int teams, gc_batch_graph **out) {
  g_error.clear();
  if (!out) return fail(GC_EINVAL, "out is NULL");
  *out = nullptr;
  if (njobs <= 0 || !jobs) return fail(GC_EINVAL, "a graph needs at least one job");
  if (teams == 0) teams = njobs >= 4 ? 4 : (njobs >= 2 ? 2 : 1);
  if (teams != 1 && teams != 2 && teams != 4 && teams != 8)
    return fail(GC_EINVAL, "teams must be 1, 2, 4 or 8 (got %d)", teams);
  std::vector<Job> J((size_t)njobs);
  gc_batch_graph *g = new gc_batch_graph();
  g->njobs = njobs;
  g->teams = teams;
  g->order.resize((size_t)njobs);
  int rc = prepare_batch(jobs, njobs, J.data(), g->order.data());
  if (rc) {
    release(g);
    return rc;
  }
  unsigned int grid = 0;
  rc = pick_grid(0, &grid);
  if (rc) {
    release(g);
    return rc;
  }
  const size_t off_dq = up256(sizeof(Bar));
  const size_t off_jobs = off_dq + up256(sizeof(DevQueue));
  const size_t off_ws = off_jobs + up256(sizeof(Job) * (size_t)njobs);
  const size_t bytes = off_ws + team_workspace_bytes() * (size_t)teams;
  hipError_t e = hipMalloc((void **)&g->dev, bytes);
  if (e == hipSuccess) e = hipHostMalloc((void **)&g->jobs_in, sizeof(Job) * njobs, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&g->jobs_out, sizeof(Job) * njobs, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&g->dq_out, sizeof(DevQueue), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking);
  if (e != hipSuccess) {
    release(g);
    return fail(GC_ENOMEM, "graph buffers: %s", hipGetErrorString(e));
  }
  for (int k = 0; k < njobs; ++k) g->jobs_in[k] = J[g->order[k]];
  memset(g->jobs_out, 0, sizeof(Job) * njobs);
  memset(g->dq_out, 0, sizeof(DevQueue));

  Params P;
  memset(&P, 0, sizeof(P));
  P.jobs = reinterpret_cast<Job *>(g->dev + off_jobs);
  P.hq = nullptr;
  P.dq = reinterpret_cast<DevQueue *>(g->dev + off_dq);
  P.bar = reinterpret_cast<Bar *>(g->dev);
  P.njobs_fixed = njobs;
  P.nteams = teams;
  P.spin_limit = spin_limit_from_env();
  P.idle_limit = 0;
  P.team_ws = g->dev + off_ws;
  P.team_ws_stride = team_workspace_bytes();

  // Everything the replay needs is captured as nodes; the barrier block and
  // the queue are reset by a kernel (no memset node).
  e = hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal);
  hipError_t ec = hipSuccess;
  if (e == hipSuccess) {
    ec = hipMemcpyAsync(P.jobs, g->jobs_in, sizeof(Job) * njobs, hipMemcpyHostToDevice, g->capture);
    if (ec == hipSuccess) ec = launch_init(P.bar, P.dq, 1, g->capture);
    if (ec == hipSuccess) ec = launch_persistent(P, grid, g->capture, LaunchKind::kBatch);
    if (ec == hipSuccess)
      ec = hipMemcpyAsync(g->jobs_out, P.jobs, sizeof(Job) * njobs, hipMemcpyDeviceToHost, g->capture);
    if (ec == hipSuccess)
      ec = hipMemcpyAsync(g->dq_out, P.dq, sizeof(DevQueue), hipMemcpyDeviceToHost, g->capture);
    e = hipStreamEndCapture(g->capture, &g->graph);
  }
  if (ec != hipSuccess || e != hipSuccess || !g->graph) {
    const hipError_t shown = ec != hipSuccess ? ec : e;
    release(g);
    return fail(GC_EDEVICE, "capture of the batch launch failed: %s", hipGetErrorString(shown));
  }
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    release(g);
    return fail(GC_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
  }
  *out = g;
  return GC_OK;
}

int gc_batch_graph_launch(gc_batch_graph *g, void *hip_stream) {
  g_error.clear();
  if (!g) return fail(GC_EINVAL, "NULL graph");
  const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(GC_EDEVICE, "hipGraphLaunch failed: %s", hipGetErrorString(e));
  return GC_OK;
}

int gc_batch_graph_results(gc_batch_graph *g, gc_job *jobs) {
  g_error.clear();
  if (!g || !jobs) return fail(GC_EINVAL, "NULL argument");
  for (int k = 0; k < g->njobs; ++k) {
    const Job &J = g->jobs_out[k];
    gc_job &o = jobs[g->order[k]];
    o.count = J.out_count;
    o.status = J.done ? J.status : GC_ETIMEOUT;
    o.device_ms = J.done ? (double)(J.t_done - J.t_claim) / 1e5 : 0.0;
  }
  if (g->dq_out->abort) return fail(GC_ETIMEOUT, "a bounded device-side wait expired");
  for (int i = 0; i < g->njobs; ++i)
    if (jobs[i].status) return fail(jobs[i].status, "job %d failed with status %d", i, jobs[i].status);
  return GC_OK;
}

int gc_batch_graph_destroy(gc_batch_graph *g) {
  release(g);
  return GC_OK;
}

}  // extern "C"
