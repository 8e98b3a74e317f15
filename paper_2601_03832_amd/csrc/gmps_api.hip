// Host runtime of libgmps: argument checking, workspace carving, bundling of instances
// into workgroups (longest first), hipGraph capture of the iterate launches, and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <mutex>
#include <new>
#include <unordered_set>
#include <vector>

#include "../../include/gmps.h"
#include "gmps_internal.h"

namespace gmps {
hipError_t launch_group(int mode, const IterParams& P, int grid, size_t lds, hipStream_t st);
hipError_t group_occupancy(int mode, size_t lds, int* blocks_per_cu);
size_t group_lds_bytes(int mode, int cls);
int team_per_bundle(int cls);
size_t team_lds_bytes(bool mixed, bool pc, bool pipe, int cls);
hipError_t launch_team(bool mixed, bool pc, bool pipe, int cls, const IterParams& P, int grid, size_t lds, hipStream_t st);
hipError_t team_occupancy(bool mixed, bool pc, bool pipe, int cls, size_t lds, int* blocks_per_cu);
size_t team_circ_lds_bytes(int cls);
hipError_t launch_team_circ(int cls, const IterParams& P, int grid, size_t lds, hipStream_t st);
hipError_t team_circ_occupancy(int cls, size_t lds, int* blocks_per_cu);
hipError_t launch_queue_reset(QueueState* q, hipStream_t st);
hipError_t launch_init(bool mixed, InstDev* inst, int B, const int64_t* site_start, int32_t* bonds, void* arena,
                       int64_t total_sites, char* warm, void* edge, hipStream_t st);
hipError_t launch_prob(bool mixed, InstDev* inst, const uint64_t* marked, const int32_t* bonds, const void* arena,
                       const void* edge, int B, double* out, hipStream_t st);
hipError_t launch_overlap_uniform(bool mixed, const InstDev* inst, int which, const int32_t* bonds,
                                  const void* arena, const void* edge, double* out, hipStream_t st);
hipError_t launch_amplitudes(bool mixed, int maxc, const InstDev* inst, int which, const int32_t* bonds,
                             const void* arena, const void* edge, const uint64_t* xs, int64_t cnt, double* out,
                             double* norm2, hipStream_t st);
hipError_t launch_sample(bool mixed, int maxc, const InstDev* inst, const uint64_t* marked, const int32_t* bonds,
                         const void* arena, const void* edge, int B, int inst_base, const int64_t* shot_off,
                         int64_t total, uint64_t seed, uint64_t* bits, unsigned long long* hits, hipStream_t st);
}  // namespace gmps

using namespace gmps;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
// Staging region of the read-out calls in the workspace: amplitude queries and sampled bitstrings
// pass through it in chunks, so the library allocates no device memory after gmps_create.
constexpr size_t kStageBytes = size_t(16) << 20;

// Effective bond cap: the exact Schmidt rank of every intermediate state is at most M+1
// (the state stays a combination of the uniform superposition and M marked basis states),
// and a bond of a chain of n sites never exceeds 2^floor(n/2).
int effective_cap(int n, int M, int cap) {
  int64_t need = std::min<int64_t>(cap, (int64_t)M + 1);
  if (n / 2 < 30) need = std::min<int64_t>(need, int64_t(1) << (n / 2));
  return (int)need;
}

// Iterate kernels: the lane-group kernel (bond caps up to 6) and the team kernels.
enum { kPathAuto = 0, kPathGroup = 1, kPathTeam = 2 };
constexpr int kLaunchKinds = 1 + kNumWide;  // the lane-group kernel, then one per team class

// Smallest tile class of the requested kernel whose bond capacity holds the effective cap
// (the lane-group kernel hands caps beyond its classes to the team kernels); -1 if none.
int pick_class(int n, int M, int cap, int path) {
  const int need = effective_cap(n, M, cap);
  if (path != kPathTeam)
    for (int c = 0; c < kNumClasses; ++c)
      if (kClasses[c].CM >= need) return c;
  for (int w = 0; w < kNumWide; ++w)
    if (kWide[w].CM >= need) return kWideBase + w;
  return -1;
}

// The library's choice is the team kernel: a step of a long serial chain takes less time
// there for every class, and it holds every bond cap.
int resolve_path(int requested) { return requested == kPathGroup ? kPathGroup : kPathTeam; }

// Warm-start record bytes of one (reflection, site) for a class.
size_t warm_rec_bytes(int cls) {
  return is_wide(cls) ? sizeof(double) * (size_t)wide_warm_doubles(class_cm(cls)) : sizeof(WarmRec);
}

bool valid_instance(const gmps_instance& in) {
  return in.n >= 1 && in.n <= 63 && in.M >= 1 && (in.n >= 62 || in.M < (int64_t(1) << in.n)) && in.chi_cap >= 1 &&
         in.reserved == 0 && in.marked_off >= 0;
}

struct Layout {
  size_t inst, marked, bonds, bundles, queue, prob, hits, site_start, warm, edge, stage, arena, total;
  int64_t total_marked, total_sites;
};

bool compute_layout(const gmps_instance* inst, int B, gmps_prec prec, int path, Layout* L, std::vector<int>* cls_out,
                    std::vector<int64_t>* site_off_out, std::vector<int64_t>* warm_off_out = nullptr,
                    std::vector<int64_t>* edge_off_out = nullptr) {
  const size_t elem = prec == GMPS_FP64 ? 16 : 8;
  int64_t tm = 0, ts = 0;
  size_t arena_elems = 0;
  if (cls_out) cls_out->resize(B);
  if (site_off_out) site_off_out->resize(B);
  if (warm_off_out) warm_off_out->resize(B);
  if (edge_off_out) edge_off_out->resize(B);
  size_t warm_bytes = 0;
  int64_t edge_cd = 0;
  for (int i = 0; i < B; ++i) {
    if (!valid_instance(inst[i])) return false;
    const int c = pick_class(inst[i].n, inst[i].M, inst[i].chi_cap, path);
    if (c < 0) return false;
    if (cls_out) (*cls_out)[i] = c;
    if (site_off_out) (*site_off_out)[i] = (int64_t)arena_elems;
    arena_elems += (size_t)inst[i].n * slot_elems(class_cm(c));
    if (warm_off_out) (*warm_off_out)[i] = (int64_t)warm_bytes;
    warm_bytes += (size_t)(inst[i].M + 1) * inst[i].n * warm_rec_bytes(c);
    if (edge_off_out) (*edge_off_out)[i] = edge_cd;
    edge_cd += (int64_t)edge_count(inst[i].n, edge_width(inst[i].M)) * slot_elems(class_cm(c));
    tm += inst[i].M;
    ts += inst[i].n;
  }
  size_t off = 0;
  L->inst = off;       off = align_up(off + sizeof(InstDev) * B);
  L->marked = off;     off = align_up(off + sizeof(uint64_t) * std::max<int64_t>(tm, 1));
  L->bonds = off;      off = align_up(off + sizeof(int32_t) * kBondStride * B);
  L->bundles = off;    off = align_up(off + sizeof(Bundle) * B);
  L->queue = off;      off = align_up(off + sizeof(QueueState) * kLaunchKinds);
  L->prob = off;       off = align_up(off + sizeof(double) * B);
  L->hits = off;       off = align_up(off + sizeof(uint64_t) * B);
  L->site_start = off; off = align_up(off + sizeof(int64_t) * (B + 1));
  L->warm = off;       off = align_up(off + warm_bytes);
  L->edge = off;       off = align_up(off + 16 * (size_t)edge_cd);
  L->stage = off;      off = align_up(off + kStageBytes);
  L->arena = off;      off = align_up(off + elem * arena_elems);
  L->total = off;
  L->total_marked = tm;
  L->total_sites = ts;
  return true;
}

}  // namespace

struct gmps_batch {
  int B = 0;
  bool mixed = false;  // complex64 site tensors (GMPS_MIXED and GMPS_FP32)
  bool fp32 = false;   // GMPS_FP32: factorisations in FP32 too (lane-group kernel)
  hipStream_t stream = nullptr;
  int device = 0;
  char* ws = nullptr;
  Layout lay{};
  std::vector<InstDev> inst_h;
  std::vector<int64_t> k_done_h;
  IterParams params{};
  double trunc_tol = 1e-12;
  int max_sweeps = 16;
  int waves_per_cu = 0;
  bool use_graph = true;
  int round_mode = 0;  // 0: library default, 1: stochastic, -1: nearest
  int jacobi_warm = 0;  // 0: library default (mixed path only), 1 on, -1 off
  bool precontract = false;  // reflections as psi + product terms (team kernel only)
  bool pipeline = false;     // pipelined sweeps for the single-wave classes (team kernel default)
  int path = kPathGroup;
  int max_cm = 0;       // largest class bond of the batch (read-out register sizing)
  int num_cus = 0;
  // pinned staging for the per-call bundle table
  Bundle* bundles_pin = nullptr;
  QueueState* queue_pin = nullptr;
  hipEvent_t staging_done = nullptr;
  bool staging_pending = false;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  bool timed = false;
  // graph cache keyed by every launch's (grid, lds, first bundle)
  hipGraphExec_t graph = nullptr;
  std::vector<int64_t> graph_key;
  // side streams and events that run the kernels of several classes side by side
  hipStream_t side[kLaunchKinds] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kLaunchKinds] = {};
  // device address of this GPU's copy of the static sampling scratch (null if the lookup failed)
  char* scratch = nullptr;
  // launch plans the autotuner may choose: pipelined sweeps (team kernel, no lossy cap) and
  // pre-contracted reflections (team kernel, every bond cap <= 17)
  bool pipeline_ok = false;
  bool pc_ok = false;
  std::string device_name;
  // gate-level circuits (gmps_circuit_build): the caller's device buffer of gate streams and
  // the layers each instance's circuit holds
  const uint32_t* circuit = nullptr;
  std::vector<int64_t> circ_k;
};

// Scratch of sample_shots_noalloc: hit counters, shot offsets and bitstrings, in device memory
// that every GPU the library runs on holds from module load until the process ends. Host code
// reaches it only through the per-device address hipGetSymbolAddress returns (the array's own
// name is a host-side stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[GMPS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// This GPU's address of `scratch`, looked up once per device with that device current.
char* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
      std::fprintf(stderr, "gmps: hipGetSymbolAddress(scratch) failed: %s\n", hipGetErrorString(e));
      return nullptr;
    }
    g_scratch[dev] = static_cast<char*>(p);
  }
  return g_scratch[dev];
}

// Pre-contracted reflections: one reflection for the whole oracle when the cap keeps every
// exact Schmidt rank (so no state exceeds rank M+1) and chi + M columns fit the class tile.
bool whole_oracle(bool precontract, const InstDev& d) {
  return precontract && is_wide(d.cls) && team_pc_class(d.cls - kWideBase) &&
         d.cap == effective_cap(d.n, d.M, INT32_MAX) && d.M <= class_cm(d.cls);
}

__global__ void zero_u64_kernel(unsigned long long* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0ull;
}

// lane-group kernel instantiation: 0 FP64, 1 mixed, 2 all-FP32
int group_mode(const gmps_batch* b) { return b->fp32 ? 2 : b->mixed ? 1 : 0; }

// The team kernels keep the edge sites (the norm-carrying end site among them) in complex FP64 edge
// slots, which the read-out kernels then use in place of their site slots; the lane-group kernel
// does not maintain them.
const void* readout_edge(const gmps_batch* b) { return b->path == kPathTeam ? b->params.edge : nullptr; }

int hip_fail(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    std::fprintf(stderr, "gmps: %s failed: %s\n", what, hipGetErrorString(e));
    return GMPS_E_HIP;
  }
  return GMPS_OK;
}

#define GMPS_HIP(call)                                 \
  do {                                                 \
    int _rc = hip_fail((call), #call);                 \
    if (_rc != GMPS_OK) return _rc;                    \
  } while (0)

}  // namespace

extern "C" {

const char* gmps_strerror(int status) {
  switch (status) {
    case GMPS_OK: return "ok";
    case GMPS_E_ARG: return "invalid argument";
    case GMPS_E_WORKSPACE: return "workspace missing, misaligned or too small (or a request beyond the static sampling array)";
    case GMPS_E_HIP: return "HIP runtime error";
    case GMPS_E_UNSUPPORTED: return "unsupported configuration (bond cap beyond the compiled tile classes, or no GPU)";
    case GMPS_E_NUMERIC: return "numerical failure in some instance (NaN/Inf or norm drift)";
  }
  return "unknown status";
}

size_t gmps_workspace_bytes(const gmps_instance* inst, int32_t B, gmps_prec prec) {
  if (!inst || B <= 0 || (prec != GMPS_FP64 && prec != GMPS_MIXED && prec != GMPS_FP32)) return 0;
  // enough for either iterate kernel, so the choice can be made at gmps_create()
  Layout Lg, Lt;
  if (!compute_layout(inst, B, prec, kPathGroup, &Lg, nullptr, nullptr)) return 0;
  if (!compute_layout(inst, B, prec, kPathTeam, &Lt, nullptr, nullptr)) return 0;
  return std::max(Lg.total, Lt.total);
}

int gmps_create(gmps_batch** out, const gmps_instance* inst, int32_t B, const uint64_t* marked, gmps_prec prec,
                const gmps_options* opt, void* dev_workspace, size_t ws_bytes, void* hip_stream) {
  if (!out) return GMPS_E_ARG;
  *out = nullptr;
  if (!inst || B <= 0 || !marked || (prec != GMPS_FP64 && prec != GMPS_MIXED && prec != GMPS_FP32)) return GMPS_E_ARG;
  for (int i = 0; i < B; ++i)
    if (!valid_instance(inst[i])) return GMPS_E_ARG;
  if (opt && (opt->kernel < 0 || opt->kernel > kPathTeam)) return GMPS_E_ARG;
  const bool fp32 = prec == GMPS_FP32;
  // the all-FP32 path exists on the lane-group kernel only
  if (fp32 && opt && opt->kernel == kPathTeam) return GMPS_E_UNSUPPORTED;
  const int path = fp32 ? kPathGroup : resolve_path(opt ? opt->kernel : kPathAuto);
  const bool precontract = opt && opt->precontract > 0;
  // pre-contracted reflections run on the team kernel in FP64 only: on complex64 storage the
  // exact product terms meet bond spaces tilted by the rounding of the stored sites, and the
  // rotation angle drifts, faster with n (both sweep orders)
  if (precontract && (path != kPathTeam || prec != GMPS_FP64)) return GMPS_E_UNSUPPORTED;
  Layout L;
  std::vector<int> cls;
  std::vector<int64_t> site_off, warm_off, edge_off;
  for (int i = 0; i < B; ++i) {
    const int c = pick_class(inst[i].n, inst[i].M, inst[i].chi_cap, path);
    if (c < 0 || (fp32 && is_wide(c))) return GMPS_E_UNSUPPORTED;
    // the pre-contracted reflections are built for bond caps up to 17 only
    if (precontract && !(is_wide(c) && team_pc_class(c - kWideBase))) return GMPS_E_UNSUPPORTED;
  }
  if (!compute_layout(inst, B, prec, path, &L, &cls, &site_off, &warm_off, &edge_off)) return GMPS_E_ARG;
  // marked sets: in range and distinct within an instance
  int64_t tm = 0;
  for (int i = 0; i < B; ++i) tm = std::max<int64_t>(tm, inst[i].marked_off + inst[i].M);
  std::vector<uint64_t> packed;
  packed.reserve(L.total_marked);
  for (int i = 0; i < B; ++i) {
    std::unordered_set<uint64_t> seen;
    for (int j = 0; j < inst[i].M; ++j) {
      const uint64_t x = marked[inst[i].marked_off + j];
      if (inst[i].n < 64 && (x >> inst[i].n) != 0) return GMPS_E_ARG;
      if (!seen.insert(x).second) return GMPS_E_ARG;
      packed.push_back(x);
    }
  }
  // the documented requirement: what gmps_workspace_bytes() returns for this batch
  if (!dev_workspace || ws_bytes < gmps_workspace_bytes(inst, B, prec) ||
      (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) != 0)
    return GMPS_E_WORKSPACE;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return GMPS_E_UNSUPPORTED;

  gmps_batch* b = new (std::nothrow) gmps_batch();
  if (!b) return GMPS_E_ARG;
  b->B = B;
  b->mixed = prec != GMPS_FP64;
  b->fp32 = fp32;
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  b->ws = reinterpret_cast<char*>(dev_workspace);
  b->lay = L;
  b->path = path;
  for (int i = 0; i < B; ++i) b->max_cm = std::max(b->max_cm, class_cm(cls[i]));
  b->trunc_tol = fp32 ? 1e-6 : b->mixed ? 5e-7 : 1e-12;
  if (opt) {
    if (opt->trunc_tol > 0) b->trunc_tol = opt->trunc_tol;
    if (opt->max_sweeps > 0) b->max_sweeps = opt->max_sweeps;
    if (opt->waves_per_cu > 0) b->waves_per_cu = opt->waves_per_cu;
    if (opt->use_graph < 0) b->use_graph = false;
    b->round_mode = opt->round_mode > 0 ? 1 : opt->round_mode < 0 ? -1 : 0;
    b->jacobi_warm = opt->jacobi_warm;
  }
  b->precontract = precontract;
  b->pipeline = path == kPathTeam && !(opt && opt->pipeline < 0);
  // A cap below the exact rank drops weight, and what a truncation drops depends on the sweep
  // order: such a batch keeps the sequential sweeps, whose truncations run right to left as
  // in the CPU oracle's MPS.
  b->pipeline_ok = path == kPathTeam;
  for (int i = 0; i < B; ++i)
    if (effective_cap(inst[i].n, inst[i].M, inst[i].chi_cap) < effective_cap(inst[i].n, inst[i].M, INT32_MAX))
      b->pipeline_ok = false;
  b->pipeline = b->pipeline && b->pipeline_ok;
  b->pc_ok = path == kPathTeam && !b->mixed;
  for (int i = 0; i < B; ++i)
    if (!(is_wide(cls[i]) && team_pc_class(cls[i] - kWideBase))) b->pc_ok = false;
  hipGetDevice(&b->device);
  b->scratch = scratch_address(b->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) {
    delete b;
    return GMPS_E_HIP;
  }
  b->num_cus = prop.multiProcessorCount;
  b->device_name = std::string(prop.name) + "/" + prop.gcnArchName + "/" + std::to_string(b->num_cus);

  b->inst_h.resize(B);
  int64_t moff = 0;
  std::vector<int64_t> site_start(B + 1, 0);
  for (int i = 0; i < B; ++i) {
    InstDev& d = b->inst_h[i];
    std::memset(&d, 0, sizeof(d));
    d.n = inst[i].n;
    d.M = inst[i].M;
    d.cap = effective_cap(inst[i].n, inst[i].M, inst[i].chi_cap);
    d.cls = cls[i];
    d.whole = whole_oracle(precontract, d) ? 1 : 0;
    d.marked_off = moff;
    d.site_off = site_off[i];
    d.warm_off = warm_off[i];
    d.edge_off = edge_off[i];
    d.ew = edge_width(inst[i].M);
    moff += inst[i].M;
    site_start[i + 1] = site_start[i] + inst[i].n;
  }
  b->k_done_h.assign(B, 0);
  hipStream_t st = b->stream;
  int rc = GMPS_OK;
  auto fail = [&](int code) {
    gmps_destroy(b);
    return code;
  };
  if ((rc = hip_fail(hipMemcpyAsync(b->ws + L.inst, b->inst_h.data(), sizeof(InstDev) * B, hipMemcpyHostToDevice, st),
                     "copy instances")) != GMPS_OK)
    return fail(rc);
  if ((rc = hip_fail(hipMemcpyAsync(b->ws + L.marked, packed.data(), sizeof(uint64_t) * packed.size(),
                                    hipMemcpyHostToDevice, st),
                     "copy marked")) != GMPS_OK)
    return fail(rc);
  if ((rc = hip_fail(hipMemcpyAsync(b->ws + L.site_start, site_start.data(), sizeof(int64_t) * (B + 1),
                                    hipMemcpyHostToDevice, st),
                     "copy site table")) != GMPS_OK)
    return fail(rc);
  if ((rc = hip_fail(hipStreamSynchronize(st), "sync")) != GMPS_OK) return fail(rc);
  if ((rc = hip_fail(hipHostMalloc(reinterpret_cast<void**>(&b->bundles_pin), sizeof(Bundle) * B, hipHostMallocDefault),
                     "pinned bundles")) != GMPS_OK)
    return fail(rc);
  if ((rc = hip_fail(hipHostMalloc(reinterpret_cast<void**>(&b->queue_pin), sizeof(QueueState) * kLaunchKinds,
                                   hipHostMallocDefault),
                     "pinned queue")) != GMPS_OK)
    return fail(rc);
  if ((rc = hip_fail(hipEventCreateWithFlags(&b->staging_done, hipEventDisableTiming), "event")) != GMPS_OK)
    return fail(rc);
  if ((rc = hip_fail(hipEventCreate(&b->ev_start), "event")) != GMPS_OK) return fail(rc);
  if ((rc = hip_fail(hipEventCreate(&b->ev_stop), "event")) != GMPS_OK) return fail(rc);

  IterParams& P = b->params;
  P.inst = reinterpret_cast<InstDev*>(b->ws + L.inst);
  P.marked = reinterpret_cast<const uint64_t*>(b->ws + L.marked);
  P.bonds = reinterpret_cast<int32_t*>(b->ws + L.bonds);
  P.arena = b->ws + L.arena;
  P.bundles = reinterpret_cast<const Bundle*>(b->ws + L.bundles);
  P.queue = reinterpret_cast<QueueState*>(b->ws + L.queue);
  P.trunc_tol = b->trunc_tol;
  // rounding-noise floor of an SVD tile: FP64 contractions, or complex64 ones
  P.skip_tol = std::min(b->trunc_tol, b->mixed ? 1e-7 : 1e-15);
  P.rank_tol = b->trunc_tol;
  P.max_sweeps = b->max_sweeps;
  // stochastic rounding applies to FP64 results stored as complex64 (none on the all-FP32 path)
  // stochastic rounding of stored complex64 values: set per class kernel at launch
  P.stoch_round = 0;
  // warm starts by default only on the lane-group kernel's mixed path (complex64 arithmetic)
  const bool warm_on = b->jacobi_warm > 0 || (b->jacobi_warm == 0 && b->mixed && !b->fp32 && path == kPathGroup);
  P.warm = warm_on ? reinterpret_cast<void*>(b->ws + L.warm) : nullptr;
  P.edge = reinterpret_cast<void*>(b->ws + L.edge);
  *out = b;
  return GMPS_OK;
}

int mps_init_uniform(gmps_batch* b) {
  if (!b) return GMPS_E_ARG;
  GMPS_HIP(launch_init(b->mixed, b->params.inst, b->B, reinterpret_cast<const int64_t*>(b->ws + b->lay.site_start),
                       b->params.bonds, b->params.arena, b->lay.total_sites, b->ws + b->lay.warm, b->params.edge,
                       b->stream));
  std::fill(b->k_done_h.begin(), b->k_done_h.end(), 0);
  return GMPS_OK;
}

}  // extern "C"

namespace {

// Sampling appended to an iterate launch: hits only, every instance of the batch.
struct SampleReq {
  const int64_t* shot_off;  // device [B + 1], in the staging region
  int64_t total;
  uint64_t seed;
};

int iterate_impl(gmps_batch* b, const int64_t* k, int32_t k_len, const SampleReq* smp, bool circuit = false);

}  // namespace

extern "C" {

int grover_iterate(gmps_batch* b, const int64_t* k, int32_t k_len) {
  if (!b || !k || (k_len != 1 && k_len != b->B)) return GMPS_E_ARG;
  for (int i = 0; i < k_len; ++i)
    if (k[i] < 0) return GMPS_E_ARG;
  return iterate_impl(b, k, k_len, nullptr);
}

}  // extern "C"

namespace {

// Gates of one layer of Fig. 1(A) for instance (n, marked): per marked x, X on each qubit where
// x has a 0, the n-controlled Z, the same X gates; then the diffusion as H, X on every qubit,
// the n-controlled Z, X and H on every qubit.
int64_t layer_gates(int n, const uint64_t* x, int M) {
  int64_t g = 0;
  for (int t = 0; t < M; ++t) g += 2 * (n - __builtin_popcountll(x[t])) + 1;
  return g + 4 * (int64_t)n + 1;
}

void append_layer(std::vector<uint32_t>& out, int n, const uint64_t* x, int M) {
  for (int t = 0; t < M; ++t) {
    for (int q = 0; q < n; ++q)
      if (!((x[t] >> (n - 1 - q)) & 1ull)) out.push_back(gate_word(kGateX, q));
    out.push_back(gate_word(kGateMCZ, 0));
    for (int q = 0; q < n; ++q)
      if (!((x[t] >> (n - 1 - q)) & 1ull)) out.push_back(gate_word(kGateX, q));
  }
  for (int q = 0; q < n; ++q) out.push_back(gate_word(kGateH, q));
  for (int q = 0; q < n; ++q) out.push_back(gate_word(kGateX, q));
  out.push_back(gate_word(kGateMCZ, 0));
  for (int q = 0; q < n; ++q) out.push_back(gate_word(kGateX, q));
  for (int q = 0; q < n; ++q) out.push_back(gate_word(kGateH, q));
}

}  // namespace

extern "C" {

size_t gmps_circuit_bytes(const gmps_instance* inst, int32_t B, const uint64_t* marked, const int64_t* k,
                          int32_t k_len) {
  if (!inst || B <= 0 || !marked || !k || (k_len != 1 && k_len != B)) return 0;
  size_t total = 0;
  for (int i = 0; i < B; ++i) {
    const int64_t ki = k[k_len == 1 ? 0 : i];
    if (!valid_instance(inst[i]) || ki < 0) return 0;
    total += sizeof(uint32_t) * (size_t)(ki * layer_gates(inst[i].n, marked + inst[i].marked_off, inst[i].M));
  }
  return total;
}

int gmps_circuit_build(gmps_batch* b, const int64_t* k, int32_t k_len, void* dev_gates, size_t bytes) {
  if (!b || !k || (k_len != 1 && k_len != b->B)) return GMPS_E_ARG;
  if (b->path != kPathTeam || b->mixed) return GMPS_E_UNSUPPORTED;
  for (int i = 0; i < b->B; ++i) {
    const InstDev& d = b->inst_h[i];
    if (k[k_len == 1 ? 0 : i] < 0) return GMPS_E_ARG;
    if (d.n < 2 || !(is_wide(d.cls) && team_pc_class(d.cls - kWideBase))) return GMPS_E_UNSUPPORTED;
  }
  // the marked sets as the library holds them (packed per instance)
  std::vector<uint64_t> mk(b->lay.total_marked);
  GMPS_HIP(hipMemcpyAsync(mk.data(), b->params.marked, sizeof(uint64_t) * mk.size(), hipMemcpyDeviceToHost, b->stream));
  GMPS_HIP(hipStreamSynchronize(b->stream));
  size_t need = 0;
  for (int i = 0; i < b->B; ++i) {
    const InstDev& d = b->inst_h[i];
    need += sizeof(uint32_t) * (size_t)(k[k_len == 1 ? 0 : i] * layer_gates(d.n, mk.data() + d.marked_off, d.M));
  }
  if (need > 0 && (!dev_gates || bytes < need || (reinterpret_cast<uintptr_t>(dev_gates) % 4) != 0))
    return GMPS_E_WORKSPACE;
  // each instance's k layers, built on the host and copied in turn; the handle takes the new
  // offsets only once every copy has succeeded
  uint32_t* dst = static_cast<uint32_t*>(dev_gates);
  int64_t off = 0;
  std::vector<uint32_t> g;
  std::vector<InstDev> inst = b->inst_h;
  std::vector<int64_t> ks(b->B, 0);
  for (int i = 0; i < b->B; ++i) {
    InstDev& d = inst[i];
    const int64_t ki = k[k_len == 1 ? 0 : i];
    const uint64_t* x = mk.data() + d.marked_off;
    g.clear();
    g.reserve((size_t)(ki * layer_gates(d.n, x, d.M)));
    for (int64_t l = 0; l < ki; ++l) append_layer(g, d.n, x, d.M);
    if (!g.empty()) GMPS_HIP(hipMemcpy(dst + off, g.data(), sizeof(uint32_t) * g.size(), hipMemcpyHostToDevice));
    d.circ_off = off;
    d.circ_len = (int64_t)g.size();
    off += (int64_t)g.size();
    ks[i] = ki;
  }
  GMPS_HIP(hipMemcpyAsync(b->params.inst, inst.data(), sizeof(InstDev) * b->B, hipMemcpyHostToDevice, b->stream));
  GMPS_HIP(hipStreamSynchronize(b->stream));
  b->inst_h = inst;
  b->circ_k = ks;
  b->circuit = static_cast<const uint32_t*>(dev_gates);
  return GMPS_OK;
}

int grover_circuit_run(gmps_batch* b) {
  if (!b) return GMPS_E_ARG;
  if (b->circ_k.size() != (size_t)b->B) return GMPS_E_ARG;  // no circuit built
  return iterate_impl(b, b->circ_k.data(), b->B, nullptr, true);
}

int grover_iterate_sample(gmps_batch* b, const int64_t* k, int32_t k_len, const int64_t* shots, int32_t shots_len,
                          uint64_t seed, int64_t* out_hits) {
  if (!b || !k || (k_len != 1 && k_len != b->B) || !shots || (shots_len != 1 && shots_len != b->B)) return GMPS_E_ARG;
  for (int i = 0; i < k_len; ++i)
    if (k[i] < 0) return GMPS_E_ARG;
  for (int i = 0; i < shots_len; ++i)
    if (shots[i] < 0) return GMPS_E_ARG;
  if (align_up(sizeof(int64_t) * ((size_t)b->B + 1)) > kStageBytes) return GMPS_E_WORKSPACE;
  // the shot offsets go to the staging region ahead of the graph launch that reads them
  std::vector<int64_t> off(b->B + 1, 0);
  for (int i = 0; i < b->B; ++i) off[i + 1] = off[i] + shots[shots_len == 1 ? 0 : i];
  int64_t* doff = reinterpret_cast<int64_t*>(b->ws + b->lay.stage);
  GMPS_HIP(hipMemcpyAsync(doff, off.data(), sizeof(int64_t) * (b->B + 1), hipMemcpyHostToDevice, b->stream));
  SampleReq smp{doff, off[b->B], seed};
  int rc = iterate_impl(b, k, k_len, &smp);
  if (rc != GMPS_OK) return rc;
  if (out_hits)
    GMPS_HIP(hipMemcpyAsync(out_hits, b->ws + b->lay.hits, sizeof(int64_t) * b->B, hipMemcpyDeviceToHost, b->stream));
  GMPS_HIP(hipStreamSynchronize(b->stream));  // also keeps off alive until the copy has run
  return GMPS_OK;
}

}  // extern "C"

namespace {

int iterate_impl(gmps_batch* b, const int64_t* k, int32_t k_len, const SampleReq* smp, bool circuit) {
  // Bundle instances that share (class, n, M, k), then order each kernel's bundles by
  // estimated cost, longest first, so the persistent queue hands out the long serial
  // chains early.
  struct Key {
    int cls, n, M, whole;
    int64_t k;
    bool operator<(const Key& o) const {
      if (cls != o.cls) return cls < o.cls;
      if (whole != o.whole) return whole < o.whole;
      if (n != o.n) return n < o.n;
      if (M != o.M) return M < o.M;
      return k < o.k;
    }
  };
  std::map<Key, std::vector<int>> groups;
  for (int i = 0; i < b->B; ++i) {
    const int64_t ki = k[k_len == 1 ? 0 : i];
    if (ki == 0) continue;
    const InstDev& d = b->inst_h[i];
    groups[{d.cls, d.n, d.M, d.whole, ki}].push_back(i);
  }
  if (b->staging_pending) {
    GMPS_HIP(hipEventSynchronize(b->staging_done));
    b->staging_pending = false;
  }
  std::vector<std::pair<double, Bundle>> bundles[kLaunchKinds];
  size_t lds[kLaunchKinds] = {};
  double work[kLaunchKinds] = {};
  for (auto& g : groups) {
    const int cls = g.first.cls;
    const bool team = is_wide(cls);
    const int kind = team ? 1 + (cls - kWideBase) : 0;
    const int per = team ? team_per_bundle(cls) : 64 / kClasses[cls].G;
    // a site step of either kernel takes roughly (CM + 1) times a fixed latency
    const int refl = g.first.whole ? 2 : g.first.M + 1;  // reflections per iteration
    const double cost = (double)g.first.k * refl * std::max(1, g.first.n - 1) * (class_cm(cls) + 1.0);
    lds[kind] = std::max(lds[kind], team ? (circuit ? team_circ_lds_bytes(cls) : team_lds_bytes(b->mixed, b->precontract, b->pipeline, cls))
                                         : group_lds_bytes(group_mode(b), cls) * per);
    for (size_t s = 0; s < g.second.size(); s += per) {
      Bundle bd;
      std::memset(&bd, 0, sizeof(bd));
      bd.cls = cls;
      bd.k = g.first.k;
      bd.count = (int)std::min<size_t>(per, g.second.size() - s);
      for (int t = 0; t < bd.count; ++t) bd.inst[t] = g.second[s + t];
      bundles[kind].push_back({cost, bd});
      work[kind] += cost;
    }
  }
  for (int i = 0; i < b->B; ++i) b->k_done_h[i] += k[k_len == 1 ? 0 : i];
  b->timed = false;
  int first[kLaunchKinds], count[kLaunchKinds], grid[kLaunchKinds];
  int nb = 0;
  for (int kd = 0; kd < kLaunchKinds; ++kd) {
    std::stable_sort(bundles[kd].begin(), bundles[kd].end(),
                     [](const std::pair<double, Bundle>& a, const std::pair<double, Bundle>& c) { return a.first > c.first; });
    first[kd] = nb;
    count[kd] = (int)bundles[kd].size();
    for (auto& bp : bundles[kd]) b->bundles_pin[nb++] = bp.second;
    b->queue_pin[kd].next = 0;
    b->queue_pin[kd].nbundles = count[kd];
  }
  if (nb == 0 && !smp) return GMPS_OK;
  GMPS_HIP(hipMemcpyAsync(b->ws + b->lay.bundles, b->bundles_pin, sizeof(Bundle) * nb, hipMemcpyHostToDevice,
                          b->stream));
  GMPS_HIP(hipMemcpyAsync(b->ws + b->lay.queue, b->queue_pin, sizeof(QueueState) * kLaunchKinds, hipMemcpyHostToDevice,
                          b->stream));
  GMPS_HIP(hipEventRecord(b->staging_done, b->stream));
  b->staging_pending = true;

  // Persistent grids: each class kernel gets a workgroup per bundle up to what its occupancy
  // allows; when the kernels together would need more of the device than there is, each
  // keeps the share of it that its estimated work has, so that no class waits for another.
  std::vector<int64_t> key;
  int cap_wg[kLaunchKinds] = {};
  double fill = 0.0, work_total = 0.0;
  for (int kd = 0; kd < kLaunchKinds; ++kd) {
    grid[kd] = 0;
    if (count[kd] == 0) continue;
    int per_cu = 0;
    if (kd == 0) GMPS_HIP(group_occupancy(group_mode(b), lds[kd], &per_cu));
    else if (circuit) GMPS_HIP(team_circ_occupancy(kWideBase + kd - 1, lds[kd], &per_cu));
    else GMPS_HIP(team_occupancy(b->mixed, b->precontract, b->pipeline, kWideBase + kd - 1, lds[kd], &per_cu));
    if (b->waves_per_cu > 0) per_cu = std::min(per_cu, b->waves_per_cu);
    per_cu = std::max(per_cu, 1);
    cap_wg[kd] = per_cu * b->num_cus;
    grid[kd] = std::min(count[kd], cap_wg[kd]);
    fill += (double)grid[kd] / cap_wg[kd];
    work_total += work[kd];
  }
  for (int kd = 0; kd < kLaunchKinds; ++kd) {
    if (count[kd] == 0) continue;
    if (fill > 1.0 && work_total > 0.0)
      grid[kd] = std::max(1, std::min(grid[kd], (int)(cap_wg[kd] * work[kd] / work_total)));
    key.insert(key.end(), {kd, grid[kd], (int64_t)lds[kd], first[kd]});
  }
  // sampling appended to the launch: its total and seed are kernel arguments of the graph
  if (smp) key.insert(key.end(), {-1, smp->total, (int64_t)smp->seed});
  // the gate-level circuit kernels read the gate streams
  if (circuit) key.insert(key.end(), {-2, (int64_t)reinterpret_cast<uintptr_t>(b->circuit)});
  Bundle* dev_bundles = reinterpret_cast<Bundle*>(b->ws + b->lay.bundles);
  QueueState* dev_queue = reinterpret_cast<QueueState*>(b->ws + b->lay.queue);
  // the kernels of different classes run side by side: the first on st, the others on side
  // streams forked from st after the queue reset and joined back into st
  int nkinds = 0;
  for (int kd = 0; kd < kLaunchKinds; ++kd) nkinds += grid[kd] > 0 ? 1 : 0;
  if (nkinds > 1 && !b->fork_ev) {
    GMPS_HIP(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
    for (int kd = 0; kd < kLaunchKinds; ++kd) {
      GMPS_HIP(hipStreamCreateWithFlags(&b->side[kd], hipStreamNonBlocking));
      GMPS_HIP(hipEventCreateWithFlags(&b->join_ev[kd], hipEventDisableTiming));
    }
  }
  unsigned long long* dhits = reinterpret_cast<unsigned long long*>(b->ws + b->lay.hits);
  auto launch_all = [&](hipStream_t st) -> hipError_t {
    hipError_t e = hipSuccess;
    if (smp) {
      // hit counters cleared by a kernel: no memset node in the graph
      hipLaunchKernelGGL(zero_u64_kernel, dim3((b->B + 255) / 256), dim3(256), 0, st, dhits, (int64_t)b->B);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_queue_reset(dev_queue, st);
    if (e == hipSuccess && nkinds > 1) e = hipEventRecord(b->fork_ev, st);
    bool on_main = true;
    for (int kd = 0; kd < kLaunchKinds && e == hipSuccess; ++kd) {
      if (grid[kd] == 0) continue;
      hipStream_t ks = st;
      if (!on_main) {
        ks = b->side[kd];
        e = hipStreamWaitEvent(ks, b->fork_ev, 0);
        if (e != hipSuccess) break;
      }
      IterParams P = b->params;
      P.bundles = dev_bundles + first[kd];
      P.queue = dev_queue + kd;
      P.circuit = circuit ? b->circuit : nullptr;
      // The team kernels compute in FP64 and compensate their complex64 stores: they round to
      // nearest unless stochastic rounding is asked for, and their Jacobi rotates every column
      // above the FP64 floor. The lane-group kernel computes in the storage type on the mixed
      // path: it rounds stochastically unless nearest is asked for, and leaves columns at the
      // complex64 floor unrotated.
      const bool comp = kd > 0;
      P.stoch_round = (b->mixed && !b->fp32 && (comp ? b->round_mode == 1 : b->round_mode != -1)) ? 1 : 0;
      if (comp) P.skip_tol = std::min(b->trunc_tol, 1e-15);
      e = kd == 0   ? launch_group(group_mode(b), P, grid[kd], lds[kd], ks)
          : circuit ? launch_team_circ(kWideBase + kd - 1, P, grid[kd], lds[kd], ks)
                    : launch_team(b->mixed, b->precontract, b->pipeline, kWideBase + kd - 1, P, grid[kd], lds[kd], ks);
      if (e == hipSuccess && !on_main) {
        e = hipEventRecord(b->join_ev[kd], ks);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, b->join_ev[kd], 0);
      }
      on_main = false;
    }
    // perfect sampling of every final state, after the class kernels have joined
    if (e == hipSuccess && smp && smp->total > 0)
      e = launch_sample(b->mixed, b->max_cm, b->params.inst, b->params.marked, b->params.bonds, b->params.arena,
                        readout_edge(b), b->B, 0, smp->shot_off, smp->total, smp->seed, nullptr, dhits, st);
    return e;
  };

  GMPS_HIP(hipEventRecord(b->ev_start, b->stream));
  if (b->use_graph) {
    if (!b->graph || b->graph_key != key) {
      if (b->graph) {
        hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
      }
      hipStream_t cap;
      GMPS_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      hipGraph_t g;
      GMPS_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
      hipError_t le = launch_all(cap);
      hipError_t ce = hipStreamEndCapture(cap, &g);
      hipStreamDestroy(cap);
      GMPS_HIP(le);
      GMPS_HIP(ce);
      hipError_t ie = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      GMPS_HIP(ie);
      b->graph_key = key;
    }
    GMPS_HIP(hipGraphLaunch(b->graph, b->stream));
  } else {
    GMPS_HIP(launch_all(b->stream));
  }
  GMPS_HIP(hipEventRecord(b->ev_stop, b->stream));
  b->timed = true;
  return GMPS_OK;
}

}  // namespace

extern "C" {

int gmps_last_iterate_ms(gmps_batch* b, double* ms) {
  if (!b || !ms) return GMPS_E_ARG;
  if (!b->timed) {
    *ms = 0.0;
    return GMPS_OK;
  }
  GMPS_HIP(hipEventSynchronize(b->ev_stop));
  float f = 0.f;
  GMPS_HIP(hipEventElapsedTime(&f, b->ev_start, b->ev_stop));
  *ms = f;
  return GMPS_OK;
}

}  // extern "C"

namespace {

#ifndef GMPS_SOURCE_HASH
#define GMPS_SOURCE_HASH "unhashed"
#endif

uint64_t fnv1a(const std::string& t) {
  uint64_t h = 1469598103934665603ull;
  for (unsigned char c : t) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

// Switches the batch to a launch plan: the flags the kernels and the bundling read, the
// whole-oracle flag of every instance (device table rewritten; the caller re-initialises the
// chain), and the cached graph, whose kernels the plan changes.
int set_plan(gmps_batch* b, bool pipeline, bool precontract, int wpc) {
  if (precontract && !b->pc_ok) return GMPS_E_UNSUPPORTED;
  const bool pc_changed = precontract != b->precontract;
  b->pipeline = pipeline;
  b->precontract = precontract;
  b->waves_per_cu = wpc;
  if (pc_changed) {
    for (auto& d : b->inst_h) d.whole = whole_oracle(precontract, d) ? 1 : 0;
    GMPS_HIP(hipMemcpyAsync(b->params.inst, b->inst_h.data(), sizeof(InstDev) * b->B, hipMemcpyHostToDevice, b->stream));
    GMPS_HIP(hipStreamSynchronize(b->stream));
  }
  if (b->graph) {
    GMPS_HIP(hipStreamSynchronize(b->stream));
    hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_key.clear();
  }
  return GMPS_OK;
}

}  // namespace

extern "C" {

constexpr int kTuneTimedRuns = 3;  // timed probe runs per plan

int gmps_autotune(gmps_batch* b, const int64_t* k, int32_t k_len, int32_t probe_iters, const char* cache_path,
                  gmps_plan* out) {
  if (!b || !k || (k_len != 1 && k_len != b->B) || probe_iters < 1) return GMPS_E_ARG;
  int64_t kmax = 0;
  for (int i = 0; i < k_len; ++i) {
    if (k[i] < 0) return GMPS_E_ARG;
    kmax = std::max(kmax, k[i]);
  }
  // the probe keeps the proportions of the run: the longest chain takes probe_iters iterations
  std::vector<int64_t> kp(b->B);
  for (int i = 0; i < b->B; ++i) {
    const int64_t ki = k[k_len == 1 ? 0 : i];
    kp[i] = ki == 0 ? 0 : std::max<int64_t>(1, (int64_t)std::llround((double)ki * probe_iters / (double)std::max<int64_t>(kmax, 1)));
  }
  // plans that keep the batch's parity: pipelined or sequential sweeps where the pipeline is
  // allowed; pre-contracted reflections on FP64 with lossless caps only (on complex64 storage
  // their angle drifts, and a lossy truncation is checked against the oracle on the
  // per-projector reflections); the library's occupancy or one or two workgroups per CU and
  // class kernel
  struct Plan {
    bool pipe, pc;
    int wpc;
  };
  std::vector<Plan> plans;
  const bool team = b->path == kPathTeam;
  for (int pipe = 0; pipe < 2; ++pipe) {
    if (pipe && !(team && b->pipeline_ok)) continue;
    for (int pc = 0; pc < 2; ++pc) {
      if (pc && !(team && b->pc_ok && b->pipeline_ok)) continue;
      for (int wpc : {0, 1, 2}) plans.push_back({pipe != 0, pc != 0, wpc});
    }
  }
  // cache key: device, device sources, precision and the batch's (class, n, M, k) multiset
  std::vector<std::string> items;
  for (int i = 0; i < b->B; ++i) {
    const InstDev& d = b->inst_h[i];
    items.push_back(std::to_string(d.cls) + ":" + std::to_string(d.n) + ":" + std::to_string(d.M) + ":" +
                    std::to_string(kp[i]));
  }
  std::sort(items.begin(), items.end());
  std::string sig = b->device_name + "|" GMPS_SOURCE_HASH "|" + (b->fp32 ? "fp32" : b->mixed ? "mixed" : "fp64") +
                    "|" + std::to_string(b->path) + "|" + std::to_string(probe_iters);
  for (auto& t : items) sig += "|" + t;
  char key[17];
  std::snprintf(key, sizeof(key), "%016llx", (unsigned long long)fnv1a(sig));
  gmps_plan best{};
  bool found = false;
  if (cache_path && *cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[256];
      while (std::fgets(line, sizeof(line), f)) {
        char kk[64];
        int pp = 0, cc = 0, ww = 0;
        double ms = 0.0;
        if (std::sscanf(line, "%63s %d %d %d %lf", kk, &pp, &cc, &ww, &ms) == 5 && std::strcmp(kk, key) == 0) {
          // a cached plan is used only if it is still one of this batch's candidates
          for (auto& pl : plans)
            if (pl.pipe == (pp > 0) && pl.pc == (cc > 0) && pl.wpc == ww) {
              best.pipeline = pp > 0 ? 1 : -1;
              best.precontract = cc > 0 ? 1 : -1;
              best.waves_per_cu = ww;
              best.ms = ms;
              found = true;
            }
        }
      }
      std::fclose(f);
    }
  }
  int rc;
  if (!found) {
    double best_ms = 1e300;
    for (auto& pl : plans) {
      if ((rc = set_plan(b, pl.pipe, pl.pc, pl.wpc)) != GMPS_OK) return rc;
      // the first run also captures the plan's graph and is not timed; a plan's time is the
      // minimum of the timed runs: one run spreads by ~3%, more than the gap between the
      // closest plans (the occupancy limit against two workgroups per CU)
      double ms = 1e300;
      for (int rep = 0; rep <= kTuneTimedRuns; ++rep) {
        if ((rc = mps_init_uniform(b)) != GMPS_OK) return rc;
        if ((rc = grover_iterate(b, kp.data(), b->B)) != GMPS_OK) return rc;
        double t = 0.0;
        if ((rc = gmps_last_iterate_ms(b, &t)) != GMPS_OK) return rc;
        if (rep > 0) ms = std::min(ms, t);
      }
      if (ms < best_ms) {
        best_ms = ms;
        best.pipeline = pl.pipe ? 1 : -1;
        best.precontract = pl.pc ? 1 : -1;
        best.waves_per_cu = pl.wpc;
        best.ms = ms;
      }
    }
    if (cache_path && *cache_path) {
      if (FILE* f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "%s %d %d %d %.6f\n", key, best.pipeline, best.precontract, best.waves_per_cu, best.ms);
        std::fclose(f);
      }
    }
  }
  if ((rc = set_plan(b, best.pipeline > 0, best.precontract > 0, best.waves_per_cu)) != GMPS_OK) return rc;
  if ((rc = mps_init_uniform(b)) != GMPS_OK) return rc;
  best.cached = found ? 1 : 0;
  best.candidates = (int32_t)plans.size();
  if (out) *out = best;
  return GMPS_OK;
}

static int any_bad_status(gmps_batch* b, bool* bad) {
  std::vector<InstDev> h(b->B);
  GMPS_HIP(hipMemcpyAsync(h.data(), b->params.inst, sizeof(InstDev) * b->B, hipMemcpyDeviceToHost, b->stream));
  GMPS_HIP(hipStreamSynchronize(b->stream));
  *bad = false;
  for (auto& d : h)
    if (d.status & (GMPS_ST_NAN | GMPS_ST_DRIFT)) *bad = true;
  return GMPS_OK;
}

int marked_prob(gmps_batch* b, double* out_p) {
  if (!b || !out_p) return GMPS_E_ARG;
  double* dprob = reinterpret_cast<double*>(b->ws + b->lay.prob);
  GMPS_HIP(launch_prob(b->mixed, b->params.inst, b->params.marked, b->params.bonds, b->params.arena, readout_edge(b),
                       b->B, dprob, b->stream));
  GMPS_HIP(hipMemcpyAsync(out_p, dprob, sizeof(double) * b->B, hipMemcpyDeviceToHost, b->stream));
  bool bad = false;
  int rc = any_bad_status(b, &bad);
  if (rc != GMPS_OK) return rc;
  return bad ? GMPS_E_NUMERIC : GMPS_OK;
}

}  // extern "C"

namespace {

// Sampling shared by sample_shots and sample_shots_noalloc: the instances are sampled in
// chunks of at most kChunkInst whose offset table and bitstrings fit the staging area st;
// a chunk's bits are copied out before the next chunk reuses the area. dhits: B counters.
constexpr int kChunkInst = 512;

int sample_staged(gmps_batch* b, const int64_t* shots, int32_t shots_len, uint64_t seed, uint64_t* out_bits,
                  int64_t* out_hits, char* st, size_t st_bytes, unsigned long long* dhits) {
  int64_t off[kChunkInst + 1];
  const size_t head = align_up(sizeof(int64_t) * (kChunkInst + 1));
  int64_t done = 0;  // shots of the instances before the current chunk
  for (int i0 = 0; i0 < b->B;) {
    off[0] = 0;
    int i1 = i0;
    for (; i1 < b->B && i1 - i0 < kChunkInst; ++i1) {
      const int64_t s = shots[shots_len == 1 ? 0 : i1];
      if (head + sizeof(uint64_t) * (size_t)(off[i1 - i0] + s) > st_bytes) break;
      off[i1 - i0 + 1] = off[i1 - i0] + s;
    }
    if (i1 == i0) return GMPS_E_WORKSPACE;  // one instance's shots exceed the staging area
    const int nb = i1 - i0;
    const int64_t total = off[nb];
    int64_t* doff = reinterpret_cast<int64_t*>(st);
    uint64_t* dbits = reinterpret_cast<uint64_t*>(st + head);
    GMPS_HIP(hipMemcpyAsync(doff, off, sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, b->stream));
    GMPS_HIP(launch_sample(b->mixed, b->max_cm, b->params.inst + i0, b->params.marked, b->params.bonds + (int64_t)i0 * kBondStride,
                           b->params.arena, readout_edge(b), nb, i0, doff, total, seed, dbits, dhits + i0, b->stream));
    if (out_bits && total > 0)
      GMPS_HIP(hipMemcpyAsync(out_bits + done, dbits, sizeof(uint64_t) * total, hipMemcpyDeviceToHost, b->stream));
    // the offsets were read from host memory that changes before the next chunk, and the
    // staging area is reused by it
    GMPS_HIP(hipStreamSynchronize(b->stream));
    done += total;
    i0 = i1;
  }
  if (out_hits) GMPS_HIP(hipMemcpyAsync(out_hits, dhits, sizeof(int64_t) * b->B, hipMemcpyDeviceToHost, b->stream));
  GMPS_HIP(hipStreamSynchronize(b->stream));
  return GMPS_OK;
}

}  // namespace

extern "C" {

int sample_shots(gmps_batch* b, const int64_t* shots, int32_t shots_len, uint64_t seed, uint64_t* out_bits,
                 int64_t* out_hits) {
  if (!b || !shots || (shots_len != 1 && shots_len != b->B)) return GMPS_E_ARG;
  for (int i = 0; i < shots_len; ++i)
    if (shots[i] < 0) return GMPS_E_ARG;
  unsigned long long* dhits = reinterpret_cast<unsigned long long*>(b->ws + b->lay.hits);
  GMPS_HIP(hipMemsetAsync(dhits, 0, sizeof(uint64_t) * b->B, b->stream));
  return sample_staged(b, shots, shots_len, seed, out_bits, out_hits, b->ws + b->lay.stage, kStageBytes, dhits);
}

int sample_shots_noalloc(gmps_batch* b, const int64_t* shots, int32_t shots_len, uint64_t seed, uint64_t* out_bits,
                         int64_t* out_hits) {
  if (!b || !shots || (shots_len != 1 && shots_len != b->B)) return GMPS_E_ARG;
  for (int i = 0; i < shots_len; ++i)
    if (shots[i] < 0) return GMPS_E_ARG;
  if (!b->scratch) return GMPS_E_HIP;
  // layout of the scratch: B hit counters, then the staging area of the chunks; every size is
  // checked here, before anything is enqueued
  const size_t hits_bytes = align_up(sizeof(uint64_t) * (size_t)b->B);
  const size_t head = align_up(sizeof(int64_t) * (kChunkInst + 1));
  if (hits_bytes + head >= (size_t)GMPS_NOALLOC_SCRATCH_BYTES) return GMPS_E_WORKSPACE;
  const size_t st_bytes = (size_t)GMPS_NOALLOC_SCRATCH_BYTES - hits_bytes;
  const int64_t max_shots = (int64_t)((st_bytes - head) / sizeof(uint64_t));
  for (int i = 0; i < shots_len; ++i)
    if (shots[i] > max_shots) return GMPS_E_WORKSPACE;
  unsigned long long* dhits = reinterpret_cast<unsigned long long*>(b->scratch);
  // the counters keep the previous call's values: cleared by a kernel (no memset node if the
  // caller captures the stream)
  hipLaunchKernelGGL(zero_u64_kernel, dim3((b->B + 255) / 256), dim3(256), 0, b->stream, dhits, (int64_t)b->B);
  GMPS_HIP(hipGetLastError());
  return sample_staged(b, shots, shots_len, seed, out_bits, out_hits, b->scratch + hits_bytes, st_bytes, dhits);
}

int gmps_amplitudes(gmps_batch* b, int32_t inst, const uint64_t* xs, int64_t cnt, double* out_reim) {
  if (!b || inst < 0 || inst >= b->B || cnt < 0 || (cnt > 0 && (!xs || !out_reim))) return GMPS_E_ARG;
  if (cnt == 0) return GMPS_OK;
  const int n = b->inst_h[inst].n;
  for (int64_t t = 0; t < cnt; ++t)
    if (n < 64 && (xs[t] >> n) != 0) return GMPS_E_ARG;
  // queries pass through the staging region in chunks; each amplitude is divided by the norm
  // of the state (the chain's norm differs from 1 by the rounding of its stored tensors)
  char* st = b->ws + b->lay.stage;
  double* dnorm = reinterpret_cast<double*>(st);
  const int64_t chunk = (int64_t)((kStageBytes - kAlign) / (sizeof(uint64_t) + 2 * sizeof(double)));
  double norm2 = 0.0;
  for (int64_t t0 = 0; t0 < cnt; t0 += chunk) {
    const int64_t c = std::min(chunk, cnt - t0);
    uint64_t* dxs = reinterpret_cast<uint64_t*>(st + kAlign);
    double* dout = reinterpret_cast<double*>(st + kAlign + align_up(sizeof(uint64_t) * c));
    GMPS_HIP(hipMemcpyAsync(dxs, xs + t0, sizeof(uint64_t) * c, hipMemcpyHostToDevice, b->stream));
    GMPS_HIP(launch_amplitudes(b->mixed, b->max_cm, b->params.inst, inst, b->params.bonds, b->params.arena,
                               readout_edge(b), dxs, c, dout, dnorm, b->stream));
    GMPS_HIP(hipMemcpyAsync(out_reim + 2 * t0, dout, sizeof(double) * 2 * c, hipMemcpyDeviceToHost, b->stream));
    if (t0 == 0) GMPS_HIP(hipMemcpyAsync(&norm2, dnorm, sizeof(double), hipMemcpyDeviceToHost, b->stream));
    GMPS_HIP(hipStreamSynchronize(b->stream));
  }
  if (!(norm2 > 0.0) || !std::isfinite(norm2)) return GMPS_E_NUMERIC;
  const double inv = 1.0 / std::sqrt(norm2);
  for (int64_t t = 0; t < 2 * cnt; ++t) out_reim[t] *= inv;
  return GMPS_OK;
}

int gmps_overlap_uniform(gmps_batch* b, int32_t inst, double* out_reim) {
  if (!b || inst < 0 || inst >= b->B || !out_reim) return GMPS_E_ARG;
  char* st = b->ws + b->lay.stage;
  double* dnorm = reinterpret_cast<double*>(st);
  double* dov = reinterpret_cast<double*>(st + kAlign);
  const uint64_t x0 = 0;
  uint64_t* dxs = reinterpret_cast<uint64_t*>(st + 2 * kAlign);
  double* damp = reinterpret_cast<double*>(st + 3 * kAlign);
  // the norm comes with an amplitude query (any index) through the same launch
  GMPS_HIP(hipMemcpyAsync(dxs, &x0, sizeof(uint64_t), hipMemcpyHostToDevice, b->stream));
  GMPS_HIP(launch_amplitudes(b->mixed, b->max_cm, b->params.inst, inst, b->params.bonds, b->params.arena,
                             readout_edge(b), dxs, 1, damp, dnorm, b->stream));
  GMPS_HIP(launch_overlap_uniform(b->mixed, b->params.inst, inst, b->params.bonds, b->params.arena, readout_edge(b),
                                  dov, b->stream));
  double h[3];
  GMPS_HIP(hipMemcpyAsync(h, dov, sizeof(double) * 2, hipMemcpyDeviceToHost, b->stream));
  GMPS_HIP(hipMemcpyAsync(h + 2, dnorm, sizeof(double), hipMemcpyDeviceToHost, b->stream));
  GMPS_HIP(hipStreamSynchronize(b->stream));
  if (!(h[2] > 0.0) || !std::isfinite(h[2])) return GMPS_E_NUMERIC;
  const double inv = 1.0 / std::sqrt(h[2]);
  out_reim[0] = h[0] * inv;
  out_reim[1] = h[1] * inv;
  return GMPS_OK;
}

}  // extern "C"

namespace {

// Checkpoint format: a header, one record per instance (its shape, to check the handle that
// imports it, and its counters), the bond table, then the device regions that hold the chains
// as they are: warm-start records and edge slots, and the site arena.
constexpr uint64_t kStateMagic = 0x31657461745347ull;  // a fixed tag
struct StateHeader {
  uint64_t magic;
  int32_t B, mixed, fp32, path;
  uint64_t regions_bytes, arena_bytes;
};
struct StateInst {
  int32_t n, M, cap, cls;
  int64_t k_done;
  int32_t status, pad;
  double drift, trunc_w, flops64, flops32;
};

// the device regions beyond the arena that a checkpoint holds: the edge slots, and the
// warm-start records in front of them when the batch's kernels read them
size_t region_start(const gmps_batch* b) { return b->params.warm ? b->lay.warm : b->lay.edge; }

size_t state_bytes(const gmps_batch* b) {
  return sizeof(StateHeader) + sizeof(StateInst) * (size_t)b->B + sizeof(int32_t) * kBondStride * (size_t)b->B +
         (b->lay.stage - region_start(b)) + (b->lay.total - b->lay.arena);
}

}  // namespace

extern "C" {

size_t gmps_state_bytes(const gmps_batch* b) { return b ? state_bytes(b) : 0; }

int gmps_state_export(gmps_batch* b, void* host, size_t bytes) {
  if (!b || !host || bytes < state_bytes(b)) return GMPS_E_ARG;
  char* p = static_cast<char*>(host);
  StateHeader h{kStateMagic, b->B, b->mixed ? 1 : 0, b->fp32 ? 1 : 0, b->path, b->lay.stage - region_start(b),
                b->lay.total - b->lay.arena};
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  std::vector<InstDev> d(b->B);
  GMPS_HIP(hipMemcpyAsync(d.data(), b->params.inst, sizeof(InstDev) * b->B, hipMemcpyDeviceToHost, b->stream));
  GMPS_HIP(hipStreamSynchronize(b->stream));
  for (int i = 0; i < b->B; ++i) {
    StateInst r{d[i].n, d[i].M, d[i].cap, d[i].cls, d[i].k_done, d[i].status, 0, d[i].drift, d[i].trunc_w,
                d[i].flops64, d[i].flops32};
    std::memcpy(p, &r, sizeof(r));
    p += sizeof(r);
  }
  GMPS_HIP(hipMemcpy(p, b->params.bonds, sizeof(int32_t) * kBondStride * b->B, hipMemcpyDeviceToHost));
  p += sizeof(int32_t) * kBondStride * b->B;
  GMPS_HIP(hipMemcpy(p, b->ws + region_start(b), h.regions_bytes, hipMemcpyDeviceToHost));
  p += h.regions_bytes;
  GMPS_HIP(hipMemcpy(p, b->ws + b->lay.arena, h.arena_bytes, hipMemcpyDeviceToHost));
  return GMPS_OK;
}

int gmps_state_import(gmps_batch* b, const void* host, size_t bytes) {
  if (!b || !host || bytes < sizeof(StateHeader)) return GMPS_E_ARG;
  const char* p = static_cast<const char*>(host);
  StateHeader h;
  std::memcpy(&h, p, sizeof(h));
  p += sizeof(h);
  // a checkpoint of this batch only: same instances, precision, kernel and layout
  if (h.magic != kStateMagic || h.B != b->B || h.mixed != (b->mixed ? 1 : 0) || h.fp32 != (b->fp32 ? 1 : 0) ||
      h.path != b->path || h.regions_bytes != b->lay.stage - region_start(b) || h.arena_bytes != b->lay.total - b->lay.arena ||
      bytes < state_bytes(b))
    return GMPS_E_ARG;
  std::vector<InstDev> d = b->inst_h;
  for (int i = 0; i < b->B; ++i) {
    StateInst r;
    std::memcpy(&r, p, sizeof(r));
    p += sizeof(r);
    if (r.n != d[i].n || r.M != d[i].M || r.cap != d[i].cap || r.cls != d[i].cls) return GMPS_E_ARG;
    d[i].k_done = r.k_done;
    d[i].status = r.status;
    d[i].drift = r.drift;
    d[i].trunc_w = r.trunc_w;
    d[i].flops64 = r.flops64;
    d[i].flops32 = r.flops32;
  }
  GMPS_HIP(hipStreamSynchronize(b->stream));
  GMPS_HIP(hipMemcpy(b->params.inst, d.data(), sizeof(InstDev) * b->B, hipMemcpyHostToDevice));
  GMPS_HIP(hipMemcpy(b->params.bonds, p, sizeof(int32_t) * kBondStride * b->B, hipMemcpyHostToDevice));
  p += sizeof(int32_t) * kBondStride * b->B;
  GMPS_HIP(hipMemcpy(b->ws + region_start(b), p, h.regions_bytes, hipMemcpyHostToDevice));
  p += h.regions_bytes;
  GMPS_HIP(hipMemcpy(b->ws + b->lay.arena, p, h.arena_bytes, hipMemcpyHostToDevice));
  for (int i = 0; i < b->B; ++i) b->k_done_h[i] = d[i].k_done;
  return GMPS_OK;
}

int gmps_diagnostics(gmps_batch* b, double* norm_drift, double* trunc_weight, int32_t* bond_dims, int32_t* status,
                     int64_t* k_done, double* flops) {
  if (!b) return GMPS_E_ARG;
  std::vector<InstDev> h(b->B);
  GMPS_HIP(hipMemcpyAsync(h.data(), b->params.inst, sizeof(InstDev) * b->B, hipMemcpyDeviceToHost, b->stream));
  if (bond_dims)
    GMPS_HIP(hipMemcpyAsync(bond_dims, b->params.bonds, sizeof(int32_t) * kBondStride * b->B, hipMemcpyDeviceToHost,
                            b->stream));
  GMPS_HIP(hipStreamSynchronize(b->stream));
  for (int i = 0; i < b->B; ++i) {
    if (norm_drift) norm_drift[i] = h[i].drift;
    if (trunc_weight) trunc_weight[i] = h[i].trunc_w;
    if (status) status[i] = h[i].status;
    if (k_done) k_done[i] = h[i].k_done;
    if (flops) {
      flops[2 * i] = h[i].flops64;
      flops[2 * i + 1] = h[i].flops32;
    }
  }
  return GMPS_OK;
}

int gmps_destroy(gmps_batch* b) {
  if (!b) return GMPS_OK;
  if (b->stream || true) hipStreamSynchronize(b->stream);
  if (b->graph) hipGraphExecDestroy(b->graph);
  if (b->bundles_pin) hipHostFree(b->bundles_pin);
  if (b->queue_pin) hipHostFree(b->queue_pin);
  if (b->staging_done) hipEventDestroy(b->staging_done);
  if (b->ev_start) hipEventDestroy(b->ev_start);
  if (b->ev_stop) hipEventDestroy(b->ev_stop);
  for (int kd = 0; kd < kLaunchKinds; ++kd) {
    if (b->side[kd]) hipStreamDestroy(b->side[kd]);
    if (b->join_ev[kd]) hipEventDestroy(b->join_ev[kd]);
  }
  if (b->fork_ev) hipEventDestroy(b->fork_ev);
  delete b;
  return GMPS_OK;
}

}  // extern "C"
