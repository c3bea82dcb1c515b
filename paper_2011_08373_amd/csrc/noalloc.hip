// rp_repair_noalloc: the repair loop of Alg. 1 with the device workspace taken
// from a fixed array the library holds on each GPU, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid allocation).
//
// The array lives in the code object as a file-scope device variable.  On
// the host its name is only a stand-in for the symbol: its device address is
// looked up once per device with hipGetSymbolAddress (with that device
// current) and only that address is handed to the engine.  Every call on a
// device shares that device's array; the engine initialises every part of it
// that it reads (descriptor tables and the zeroed error and counter words
// come with the upload), so a call never depends on what an earlier call left
// there.  Calls that overlap on one device race on the array.
//
// The call makes no device or page-locked allocation: the descriptor upload
// and the result readback go through ordinary host memory, every round is
// launched directly (no graph is instantiated) and no timing events are
// recorded.  Host-side planning still uses the heap.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"
#include "plan.h"

namespace rp {

constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;   // 64 MiB per device

static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the scratch array on the current device, looked up the
// first time a call runs on that device; nullptr on failure.
void* scratch_on_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace rp

using namespace rp;

extern "C" {

size_t rp_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

rp_status rp_repair_noalloc(const rp_kernel* k, const rp_repair_opts* opts, rp_repair_out* out,
                            uint64_t* trajectory, uint32_t traj_cap, void* stream) {
  if (validate_kernel(k) != RP_OK || !out || (traj_cap && !trajectory)) return RP_ERR_INVALID;
  rp_repair_opts op = opts ? *opts : rp_repair_opts{0, 1, 1, 0, 0};
  if (op.policy > 1 || op.solver > 1) return RP_ERR_INVALID;
  Plan pl;
  make_plan(k, pl);
  JobInput ji;
  ji.plan = &pl;
  ji.phi0 = option_units(pl, op);
  ji.policy = op.policy;
  ji.max_rounds = op.max_rounds;
  ji.solver = op.solver;
  EngineOpts o;
  o.op = OP_REPAIR;
  o.traj_cap = traj_cap;
  o.use_graph = false;
  o.no_alloc = true;
  std::vector<JobInput> v{ji};
  // too large for the fixed array: rejected before any device work
  if (engine_workspace(v, o) > NOALLOC_SCRATCH_BYTES) return RP_ERR_WORKSPACE;
  void* ws = scratch_on_current_device();
  if (!ws) return RP_ERR_DEVICE;
  std::vector<JobResult> res;
  int rc = engine_run(v, o, ws, NOALLOC_SCRATCH_BYTES, (hipStream_t)stream, res, nullptr);
  if (rc != RP_OK) return (rp_status)rc;
  fill_repair_out(res[0].st, pl, *out);
  if (traj_cap) {
    const size_t nt = std::min<size_t>(traj_cap, res[0].traj.size());
    std::memcpy(trajectory, res[0].traj.data(), nt * sizeof(uint64_t));
  }
  return (rp_status)out->status;
}

}  // extern "C"
