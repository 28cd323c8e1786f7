// abi.hip -- the extern "C" boundary declared in include/lbm.h: argument
// validation on the host, context bookkeeping (which lattice holds f*(t)),
// and dispatch to the kernel launchers.  Nothing here allocates device
// memory, and the stepping, field and adjoint calls only enqueue work.  Two
// calls wait on the host: lbm_use_graphs (which also captures and
// instantiates the replayed step graphs) and lbm_destroy, both for the
// latest graph replay, through an event recorded after it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/lbm.h"
#include "d3q19.h"
#include "kernels.h"

static_assert(sizeof(lbm_params) == 96 && offsetof(lbm_params, steps_per_pass) == 88,
              "lbm_params layout changed: update the bindings");
static_assert(lbm::Storage<lbm::ST_F32>::kRest == LBM_MARK_F32_REST &&
                  lbm::Storage<lbm::ST_F32>::kMoving == LBM_MARK_F32_MOVING &&
                  lbm::Storage<lbm::ST_F32X>::kRest == LBM_MARK_F32_REST &&
                  lbm::Storage<lbm::ST_F32X>::kMoving == LBM_MARK_F32_MOVING &&
                  lbm::Storage<lbm::ST_F64>::kRest == LBM_MARK_F64_REST &&
                  lbm::Storage<lbm::ST_F64>::kMoving == LBM_MARK_F64_MOVING &&
                  lbm::Storage<lbm::ST_F16>::kRest == LBM_MARK_F16_REST &&
                  lbm::Storage<lbm::ST_F16>::kMoving == LBM_MARK_F16_MOVING &&
                  lbm::Storage<lbm::ST_BF16>::kRest == LBM_MARK_BF16_REST &&
                  lbm::Storage<lbm::ST_BF16>::kMoving == LBM_MARK_BF16_MOVING,
              "solid markers of the kernels and of lbm.h differ");

namespace {

thread_local char g_err[512] = "";

lbm_status fail(lbm_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

lbm_status hip_fail(hipError_t e, const char* what) {
  return fail(LBM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t elem_size(int32_t storage) {
  switch (storage) {
    case LBM_F32: return 4;
    case LBM_F16: return 2;
    case LBM_BF16: return 2;
    case LBM_F64: return 8;
    case LBM_F32X: return 4;
    default: return 0;
  }
}

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

// Padding between consecutive direction arrays: at the power-of-two sizes
// of cubic boxes the 19 arrays would otherwise sit at multiples of a large
// power of two from each other, and a wave's 19 concurrent streams at the
// same offset could contend for the same memory channels.  (Measured 1-2%
// slower at 512^3 without it, which is within the few per cent by which
// separate allocations of the same grids differ; the padding costs 4.75 KB.)
constexpr size_t kDirPadBytes = 256;

struct Sizes {
  int64_t xs;
  uint64_t plane;       // elements of one direction array (nz * ny * xs)
  uint64_t dir;         // elements from one direction array to the next
  size_t grid_bytes;
  size_t scratch_bytes;
  size_t adj_bytes;
  size_t mask_off;      // scratch byte offset of the two-step link mask (0: none)
};

lbm_status check_params(const lbm_params* p, Sizes* sz) {
  if (!p) return fail(LBM_E_ARG, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(LBM_E_ARG, "grid dimensions must be >= 1 (got %d x %d x %d)", p->nx, p->ny, p->nz);
  const size_t es = elem_size(p->storage);
  if (!es) return fail(LBM_E_ARG, "unknown storage type %d", p->storage);
  if (!(p->tau > 0.5) || std::isnan(p->tau) || (std::isinf(p->tau) && p->tau < 0))
    return fail(LBM_E_ARG, "tau must be > 1/2 or +infinity (got %g)", p->tau);
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(p->force[d])) return fail(LBM_E_ARG, "force[%d] is not finite", d);
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(p->wall_u[d])) return fail(LBM_E_ARG, "wall_u[%d] is not finite", d);
  if (p->equilibrium != LBM_EQ_QIAN && p->equilibrium != LBM_EQ_INCOMPRESSIBLE)
    return fail(LBM_E_ARG, "unknown equilibrium %d", p->equilibrium);
  if (p->obstacle_kernel != 0 && p->obstacle_kernel != 1)
    return fail(LBM_E_ARG, "obstacle_kernel must be 0 or 1 (got %d)", p->obstacle_kernel);
  if (p->steps_per_pass < LBM_STEPS_AUTO || p->steps_per_pass > 2)
    return fail(LBM_E_ARG, "steps_per_pass must be -1 (automatic), 0, 1 or 2 (got %d)",
                p->steps_per_pass);
  if (p->steps_per_pass == 2 && p->obstacle_kernel == 1)
    return fail(LBM_E_UNSUPPORTED, "two steps per pass are not available with the obstacle kernel");
  if (p->storage == LBM_F16 && (p->f16_scale_log2 < -24 || p->f16_scale_log2 > 24))
    return fail(LBM_E_ARG, "f16_scale_log2 must be in [-24, 24] (got %d)", p->f16_scale_log2);
  if (p->x_align < 0 || p->x_align > 4096)
    return fail(LBM_E_ARG, "x_align must be in [0, 4096] (got %d)", p->x_align);
  const int64_t align = p->x_align ? p->x_align : 64;
  const int64_t xs = (int64_t(p->nx) + align - 1) / align * align;
  const uint64_t plane = uint64_t(xs) * uint64_t(p->ny) * uint64_t(p->nz);
  const uint64_t cells = uint64_t(p->nx) * uint64_t(p->ny) * uint64_t(p->nz);
  if (plane * es > 0xFFFFFFFFull || cells >= (1ull << 31) || uint64_t(p->ny) * p->nz >= (1ull << 31))
    return fail(LBM_E_UNSUPPORTED,
                "grid too large: one direction array needs %llu bytes (limit 4 GiB - 1)",
                (unsigned long long)(plane * es));
  const uint64_t dir = plane + kDirPadBytes / es;
  const lbm::Geo g = lbm::make_geo(p->nx, p->ny, p->nz, int(xs), dir);
  if (sz) {
    sz->xs = xs;
    sz->plane = plane;
    sz->dir = dir;
    sz->grid_bytes = (size_t(19) * dir * es + 255) / 256 * 256;
    sz->scratch_bytes = size_t(lbm::kReduceBlocks) * 5 * sizeof(double);
    // the two-step pass's link mask follows the reduction partials, when two
    // steps per pass may run and the pass can address a pair of direction
    // arrays with 32-bit offsets
    sz->mask_off = 0;
    if ((p->steps_per_pass == 2 || p->steps_per_pass == LBM_STEPS_AUTO) &&
        p->obstacle_kernel == 0 && 2 * dir * es < (uint64_t(1) << 32)) {
      sz->mask_off = (sz->scratch_bytes + 255) / 256 * 256;
      sz->scratch_bytes = sz->mask_off + (size_t(cells) * sizeof(uint32_t) + 255) / 256 * 256;
    }
    sz->adj_bytes = size_t(g.nblocks) * 3 * sizeof(double);
  }
  return LBM_OK;
}

}  // namespace

// Partial sums of lbm_reduce_noalloc: one record of 5 doubles per reduction
// block, in a file-scope device array (each GPU the library runs on holds
// its own copy until the process ends).  Host code never hands the array's
// name to a kernel -- in host code that name is a stand-in, not a device
// address -- but the address hipGetSymbolAddress returns on each device,
// taken once per device by lbm_init with that device current.
constexpr size_t kNoallocScratchDoubles = size_t(lbm::kReduceBlocks) * 5;
static __device__ __align__(256) double noalloc_scratch[kNoallocScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[kMaxDevices] = {};

// Device address of noalloc_scratch on the current device (looked up once
// per device).
lbm_status noalloc_scratch_here(int* dev_out, double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(LBM_E_UNSUPPORTED, "device %d is beyond the %d devices the library tracks", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess) return hip_fail(e, "address of the static reduction scratch");
    g_noalloc_ptr[dev] = static_cast<double*>(p);
  }
  *dev_out = dev;
  *out = g_noalloc_ptr[dev];
  return LBM_OK;
}

}  // namespace

struct lbm_ctx {
  lbm_params p;
  Sizes sz;
  lbm::Geo geo;
  lbm::PhysParams ph;
  void* grid[2];
  const uint8_t* flags;
  double* scratch;
  uint32_t* lmask;  // the two-step link mask in scratch (resting walls), or NULL
  hipStream_t stream;
  int32_t cur;
  int64_t t;
  bool force;
  int32_t graph_steps;         // 0: one launch per step; else replay graphs of this many steps
  int graph_end[2];            // grid that holds the latest level after a replay from grid p
  hipGraphExec_t graph[2];     // per starting grid, captured by lbm_use_graphs
  hipStream_t capture_stream;  // library-owned, used only to capture the graphs
  hipEvent_t replay_done;      // recorded after the latest graph replay
  bool replayed;               // replay_done has been recorded
  int device;                  // current device at lbm_init
  double* noalloc;             // that device's address of noalloc_scratch
};

namespace {

lbm_status check_ctx(const lbm_ctx* c) {
  if (!c) return fail(LBM_E_ARG, "context is NULL");
  return LBM_OK;
}

lbm_status launch_steps_on(lbm_ctx* c, const void* src, void* dst, hipStream_t s) {
  if (c->flags && c->ph.split) {
    // the split design: bounce-back values into the solid slots of src first
    hipError_t e = lbm::launch_obstacle(c->p.storage, c->geo, c->ph, const_cast<void*>(src),
                                        c->flags, s);
    if (e != hipSuccess) return hip_fail(e, "obstacle kernel launch");
  }
  hipError_t e = lbm::launch_step(c->p.storage, c->flags != nullptr, c->force, c->geo, c->ph, src,
                                  dst, c->flags, s);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "stream-collide launch");
}

lbm_status launch_steps(lbm_ctx* c, const void* src, void* dst) {
  return launch_steps_on(c, src, dst, c->stream);
}

// Enqueues n steps from grid *cur on stream s, two fused steps per pass when
// the context asks for it (each pass writes the other grid, like one single
// step); *cur becomes the grid that holds the latest enqueued level and
// *done the number of steps enqueued (all n unless a launch failed).
lbm_status enqueue_steps(lbm_ctx* c, int32_t n, int* cur, hipStream_t s, int32_t* done) {
  *done = 0;
  // 2: always fused pairs; automatic: pairs where the fused pass fills the
  // GPU, single steps elsewhere and with the split design (the same bits)
  const bool pairs =
      c->p.steps_per_pass == 2 ||
      (c->p.steps_per_pass == LBM_STEPS_AUTO && c->p.obstacle_kernel == 0 &&
       lbm::step2_blocks(c->p.storage, c->geo) >= lbm::kStep2MinBlocks);
  while (n > 0) {
    const int k = *cur;
    if (pairs && n >= 2) {
      hipError_t e = lbm::launch_step2(c->p.storage, c->flags != nullptr, c->force, c->geo, c->ph,
                                       c->grid[k], c->grid[k ^ 1], c->flags, c->lmask, s);
      if (e != hipSuccess) return hip_fail(e, "two-step launch");
      n -= 2;
      *done += 2;
    } else {
      lbm_status st = launch_steps_on(c, c->grid[k], c->grid[k ^ 1], s);
      if (st != LBM_OK) return st;
      n -= 1;
      *done += 1;
    }
    *cur = k ^ 1;
  }
  return LBM_OK;
}

// Waits for the latest replay (through its event, valid whatever became of
// the stream it was queued on), then destroys the executable graphs.
hipError_t drop_graphs(lbm_ctx* c) {
  hipError_t e = hipSuccess;
  if (c->replayed) {
    e = hipEventSynchronize(c->replay_done);
    c->replayed = false;
  }
  for (int p = 0; p < 2; ++p)
    if (c->graph[p]) {
      (void)hipGraphExecDestroy(c->graph[p]);
      c->graph[p] = nullptr;
    }
  return e;
}

// Captures graph_steps steps starting from grid `parity` and records which
// grid a replay ends on (graph_end).  Only kernel launches are recorded.
lbm_status build_graph(lbm_ctx* c, int parity) {
  hipError_t e = hipSuccess;
  if (!c->capture_stream) {
    e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
  }
  e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "begin capture");
  int cur = parity;
  int32_t done = 0;
  lbm_status st = enqueue_steps(c, c->graph_steps, &cur, c->capture_stream, &done);
  c->graph_end[parity] = cur;
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->capture_stream, &g);
  if (st != LBM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  e = hipGraphInstantiate(&c->graph[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->graph[parity] = nullptr;
    return hip_fail(e, "graph instantiation");
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_query(const lbm_params* p, int64_t* x_stride, int64_t* dir_stride,
                     size_t* grid_bytes, size_t* scratch_bytes, size_t* adj_partials_bytes) {
  Sizes sz;
  lbm_status st = check_params(p, &sz);
  if (st != LBM_OK) return st;
  if (x_stride) *x_stride = sz.xs;
  if (dir_stride) *dir_stride = int64_t(sz.dir);
  if (grid_bytes) *grid_bytes = sz.grid_bytes;
  if (scratch_bytes) *scratch_bytes = sz.scratch_bytes;
  if (adj_partials_bytes) *adj_partials_bytes = sz.adj_bytes;
  return LBM_OK;
}

int32_t lbm_bytes_per_update(int32_t storage) {
  return int32_t(19 * 2 * elem_size(storage));
}

void lbm_lattice(int32_t* e, double* w, int32_t* opp) {
  using lbm::D3Q19;
  for (int i = 0; i < lbm::Q; ++i) {
    if (e) {
      e[3 * i + 0] = D3Q19::cx[i];
      e[3 * i + 1] = D3Q19::cy[i];
      e[3 * i + 2] = D3Q19::cz[i];
    }
    if (w) w[i] = lbm::weight<double>(i);
    if (opp) opp[i] = D3Q19::opp[i];
  }
}

lbm_status lbm_solid_markers(int32_t storage, uint64_t* rest, uint64_t* moving) {
  if (!rest || !moving) return fail(LBM_E_ARG, "rest and moving must not be NULL");
  switch (storage) {
    case LBM_F32:
    case LBM_F32X: *rest = LBM_MARK_F32_REST; *moving = LBM_MARK_F32_MOVING; break;
    case LBM_F64: *rest = LBM_MARK_F64_REST; *moving = LBM_MARK_F64_MOVING; break;
    case LBM_F16: *rest = LBM_MARK_F16_REST; *moving = LBM_MARK_F16_MOVING; break;
    case LBM_BF16: *rest = LBM_MARK_BF16_REST; *moving = LBM_MARK_BF16_MOVING; break;
    default: return fail(LBM_E_ARG, "unknown storage type %d", storage);
  }
  return LBM_OK;
}

lbm_status lbm_init(lbm_ctx** out, const lbm_params* p, void* grid_a, void* grid_b,
                    const uint8_t* flags, void* scratch, const float* rho0, const float* u0,
                    void* stream) {
  if (!out) return fail(LBM_E_ARG, "out is NULL");
  *out = nullptr;
  Sizes sz;
  lbm_status st = check_params(p, &sz);
  if (st != LBM_OK) return st;
  if (!grid_a || !grid_b) return fail(LBM_E_ARG, "grid pointers must not be NULL");
  if (grid_a == grid_b) return fail(LBM_E_ARG, "grid_a and grid_b must differ");
  if (!scratch) return fail(LBM_E_ARG, "scratch must not be NULL");
  if (!aligned256(grid_a) || !aligned256(grid_b) || !aligned256(scratch))
    return fail(LBM_E_ARG, "grids and scratch must be 256-byte aligned");
  if ((rho0 && (reinterpret_cast<uintptr_t>(rho0) & 3u)) ||
      (u0 && (reinterpret_cast<uintptr_t>(u0) & 3u)))
    return fail(LBM_E_ARG, "rho0 and u0 must be 4-byte aligned");
  int dev = 0;
  double* noalloc = nullptr;
  st = noalloc_scratch_here(&dev, &noalloc);
  if (st != LBM_OK) return st;
  lbm_ctx* c = new (std::nothrow) lbm_ctx;
  if (!c) return fail(LBM_E_ARG, "out of host memory");
  c->device = dev;
  c->noalloc = noalloc;
  c->p = *p;
  c->sz = sz;
  c->geo = lbm::make_geo(p->nx, p->ny, p->nz, int(sz.xs), sz.dir);
  c->ph.omega = std::isinf(p->tau) ? 0.0 : 1.0 / p->tau;
  for (int d = 0; d < 3; ++d) c->ph.F[d] = p->force[d];
  c->ph.scale = p->storage == LBM_F16 ? std::ldexp(1.0, p->f16_scale_log2) : 1.0;
  for (int d = 0; d < 3; ++d) c->ph.wall_u[d] = p->wall_u[d];
  c->ph.moving =
      flags != nullptr && (p->wall_u[0] != 0.0 || p->wall_u[1] != 0.0 || p->wall_u[2] != 0.0);
  c->ph.incomp = p->equilibrium == LBM_EQ_INCOMPRESSIBLE;
  c->ph.split = p->obstacle_kernel == 1;
  c->grid[0] = grid_a;
  c->grid[1] = grid_b;
  c->flags = flags;
  c->scratch = static_cast<double*>(scratch);
  c->lmask = (flags && sz.mask_off && !c->ph.moving)
                 ? reinterpret_cast<uint32_t*>(static_cast<char*>(scratch) + sz.mask_off)
                 : nullptr;
  c->stream = static_cast<hipStream_t>(stream);
  c->cur = 0;
  c->t = 0;
  c->force = p->force[0] != 0.0 || p->force[1] != 0.0 || p->force[2] != 0.0;
  c->graph_steps = 0;
  c->graph[0] = c->graph[1] = nullptr;
  c->capture_stream = nullptr;
  c->replay_done = nullptr;
  c->replayed = false;
  hipError_t e = lbm::launch_fill_zero(grid_a, sz.grid_bytes, c->stream);
  if (e == hipSuccess) e = lbm::launch_fill_zero(grid_b, sz.grid_bytes, c->stream);
  if (e == hipSuccess)
    e = lbm::launch_init(p->storage, c->geo, c->ph, grid_a, flags, rho0, u0, c->stream);
  if (e == hipSuccess && c->lmask) e = lbm::launch_link_mask(c->geo, flags, c->lmask, c->stream);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "initialisation launch");
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int32_t n) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (n < 0) return fail(LBM_E_ARG, "step count must be >= 0 (got %d)", n);
  bool replay = false;
  while (c->graph_steps && n >= c->graph_steps) {
    hipError_t e = hipGraphLaunch(c->graph[c->cur], c->stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    replay = true;
    n -= c->graph_steps;
    c->t += c->graph_steps;
    c->cur = c->graph_end[c->cur];
  }
  if (replay) {
    hipError_t e = hipEventRecord(c->replay_done, c->stream);
    if (e != hipSuccess) return hip_fail(e, "replay event");
    c->replayed = true;
  }
  int cur = c->cur;
  int32_t done = 0;
  st = enqueue_steps(c, n, &cur, c->stream, &done);
  c->t += done;  // the steps enqueued before a failed launch still count
  c->cur = cur;
  return st;
}

lbm_status lbm_step_from(lbm_ctx* c, const void* src, void* dst) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!src || !dst) return fail(LBM_E_ARG, "src and dst must not be NULL");
  if (src == dst) return fail(LBM_E_ARG, "src and dst must differ");
  if (!aligned256(src) || !aligned256(dst)) return fail(LBM_E_ARG, "src/dst must be 256-byte aligned");
  return launch_steps(c, src, dst);
}

lbm_status lbm_step2_from(lbm_ctx* c, const void* src, void* mid, void* dst) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!src || !mid || !dst) return fail(LBM_E_ARG, "src, mid and dst must not be NULL");
  if (src == mid || src == dst || mid == dst) return fail(LBM_E_ARG, "src, mid and dst must differ");
  if (!aligned256(src) || !aligned256(mid) || !aligned256(dst))
    return fail(LBM_E_ARG, "src/mid/dst must be 256-byte aligned");
  if (c->p.storage != LBM_F32)
    return fail(LBM_E_UNSUPPORTED, "lbm_step2_from needs FP32 storage");
  if (c->p.obstacle_kernel)
    return fail(LBM_E_UNSUPPORTED, "lbm_step2_from is not available with obstacle_kernel = 1");
  hipError_t e = lbm::launch_step2_mid(c->p.storage, c->flags != nullptr, c->force, c->geo, c->ph,
                                       src, mid, dst, c->flags, c->lmask, c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "two-step launch");
}

static lbm_status macro_any(lbm_ctx* c, void* rho, void* u, bool f64) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!rho && !u) return LBM_OK;
  hipError_t e = lbm::launch_macro(c->p.storage, f64, c->geo, c->ph, c->grid[c->cur], c->flags,
                                   rho, u, c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "macroscopics launch");
}

lbm_status lbm_macroscopics(lbm_ctx* c, float* rho, float* u) { return macro_any(c, rho, u, false); }

lbm_status lbm_macroscopics_f64(lbm_ctx* c, double* rho, double* u) {
  return macro_any(c, rho, u, true);
}

lbm_status lbm_reduce(lbm_ctx* c, double* out5) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!out5) return fail(LBM_E_ARG, "out5 is NULL");
  hipError_t e = lbm::launch_reduce(c->p.storage, c->geo, c->ph, c->grid[c->cur], c->flags,
                                    c->scratch, out5, c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "reduction launch");
}

lbm_status lbm_reduce_noalloc(lbm_ctx* c, double* out5) {
  static_assert(kNoallocScratchDoubles >= size_t(lbm::kReduceBlocks) * 5,
                "the static scratch must hold every partial record of the reduction");
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!out5) return fail(LBM_E_ARG, "out5 is NULL");
  // The reduction writes exactly kReduceBlocks partial records for any grid
  // size (its blocks stride over the cells), which is the array's capacity;
  // a launcher that asked for more would be rejected here.
  if (size_t(lbm::kReduceBlocks) * 5 > kNoallocScratchDoubles)
    return fail(LBM_E_UNSUPPORTED, "reduction needs more than the %zu static partial sums",
                kNoallocScratchDoubles);
  hipError_t e = lbm::launch_reduce(c->p.storage, c->geo, c->ph, c->grid[c->cur], c->flags,
                                    c->noalloc, out5, c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "reduction launch");
}

lbm_status lbm_refresh_solids(lbm_ctx* c) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!c->flags) return LBM_OK;
  hipError_t e =
      lbm::launch_mark_solids(c->p.storage, c->geo, c->ph, c->grid[c->cur], c->flags, c->stream);
  if (e == hipSuccess && c->lmask) e = lbm::launch_link_mask(c->geo, c->flags, c->lmask, c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "solid marker launch");
}

int32_t lbm_current(const lbm_ctx* c) { return c ? c->cur : -1; }
int64_t lbm_time(const lbm_ctx* c) { return c ? c->t : -1; }

lbm_status lbm_set_current(lbm_ctx* c, int32_t parity, int64_t t) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (parity != 0 && parity != 1) return fail(LBM_E_ARG, "parity must be 0 or 1");
  if (t < 0) return fail(LBM_E_ARG, "time must be >= 0");
  c->cur = parity;
  c->t = t;
  return LBM_OK;
}

lbm_status lbm_set_stream(lbm_ctx* c, void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  c->stream = static_cast<hipStream_t>(stream);
  return LBM_OK;
}

lbm_status lbm_save(lbm_ctx* c, void* dst) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!dst) return fail(LBM_E_ARG, "dst is NULL");
  hipError_t e = hipMemcpyAsync(dst, c->grid[c->cur], c->sz.grid_bytes, hipMemcpyDeviceToDevice,
                                c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "save copy");
}

lbm_status lbm_restore(lbm_ctx* c, const void* src, int64_t t) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!src) return fail(LBM_E_ARG, "src is NULL");
  if (t < 0) return fail(LBM_E_ARG, "time must be >= 0");
  hipError_t e = hipMemcpyAsync(c->grid[c->cur], src, c->sz.grid_bytes, hipMemcpyDeviceToDevice,
                                c->stream);
  if (e != hipSuccess) return hip_fail(e, "restore copy");
  c->t = t;
  return LBM_OK;
}

static lbm_status adj_check(lbm_ctx* c) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (c->p.storage != LBM_F32 && c->p.storage != LBM_F32X)
    return fail(LBM_E_UNSUPPORTED, "the adjoint supports FP32 storage only");
  return LBM_OK;
}

lbm_status lbm_adjoint_seed(lbm_ctx* c, const void* fstar_prev, const float* dL_drho,
                            const float* dL_du, float* nu_T, double* partials) {
  lbm_status st = adj_check(c);
  if (st != LBM_OK) return st;
  if (!fstar_prev || !nu_T || !partials)
    return fail(LBM_E_ARG, "fstar_prev, nu_T and partials must not be NULL");
  if (fstar_prev == nu_T) return fail(LBM_E_ARG, "fstar_prev and nu_T must differ");
  if (!aligned256(fstar_prev) || !aligned256(nu_T))
    return fail(LBM_E_ARG, "fstar_prev and nu_T must be 256-byte aligned");
  hipError_t e = lbm::launch_adj_seed(c->flags != nullptr, c->geo, c->ph,
                                      static_cast<const float*>(fstar_prev), c->flags, dL_drho,
                                      dL_du, nu_T, partials, c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "adjoint seed launch");
}

lbm_status lbm_adjoint_step(lbm_ctx* c, const void* fstar_prev, const float* nu_np1, float* nu_n,
                            double* partials) {
  lbm_status st = adj_check(c);
  if (st != LBM_OK) return st;
  if (!fstar_prev || !nu_np1 || !nu_n || !partials)
    return fail(LBM_E_ARG, "adjoint step pointers must not be NULL");
  if (nu_np1 == nu_n || fstar_prev == nu_n) return fail(LBM_E_ARG, "nu_n must differ from the inputs");
  if (!aligned256(fstar_prev) || !aligned256(nu_np1) || !aligned256(nu_n))
    return fail(LBM_E_ARG, "adjoint grids must be 256-byte aligned");
  hipError_t e = lbm::launch_adj_step(c->flags != nullptr, c->geo, c->ph,
                                      static_cast<const float*>(fstar_prev), c->flags, nu_np1, nu_n,
                                      partials, c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "adjoint step launch");
}

lbm_status lbm_adjoint_init(lbm_ctx* c, const float* nu_1, const float* rho0, const float* u0,
                            float* dL_du0) {
  lbm_status st = adj_check(c);
  if (st != LBM_OK) return st;
  if (!nu_1 || !dL_du0) return fail(LBM_E_ARG, "nu_1 and dL_du0 must not be NULL");
  if (!aligned256(nu_1)) return fail(LBM_E_ARG, "nu_1 must be 256-byte aligned");
  hipError_t e = lbm::launch_adj_init(c->flags != nullptr, c->geo, c->ph, c->flags, nu_1, rho0, u0,
                                      dL_du0, c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "adjoint init launch");
}

lbm_status lbm_adjoint_finish_dF(lbm_ctx* c, const double* partials, double* dLdF3) {
  lbm_status st = adj_check(c);
  if (st != LBM_OK) return st;
  if (!partials || !dLdF3) return fail(LBM_E_ARG, "partials and dLdF3 must not be NULL");
  hipError_t e = lbm::launch_adj_finish(c->geo, partials, dLdF3, c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "adjoint finish launch");
}

lbm_status lbm_stream_copy(void* dst, const void* src, size_t n_bytes, void* stream) {
  if (!dst || !src) return fail(LBM_E_ARG, "copy pointers must not be NULL");
  if (!aligned256(dst) || !aligned256(src)) return fail(LBM_E_ARG, "copy pointers must be 256-byte aligned");
  if (n_bytes % 16) return fail(LBM_E_ARG, "n_bytes must be a multiple of 16");
  if (!n_bytes) return LBM_OK;
  hipError_t e = lbm::launch_copy(dst, src, n_bytes / 16, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "copy launch");
}

lbm_status lbm_copy_probe(void* dst, const void* src, size_t n_bytes, int32_t vec_per_thread,
                          int32_t nontemporal, int32_t blocks, void* stream) {
  if (!dst || !src) return fail(LBM_E_ARG, "copy pointers must not be NULL");
  if (!aligned256(dst) || !aligned256(src)) return fail(LBM_E_ARG, "copy pointers must be 256-byte aligned");
  if (n_bytes % 16) return fail(LBM_E_ARG, "n_bytes must be a multiple of 16");
  if (vec_per_thread != 1 && vec_per_thread != 2 && vec_per_thread != 4)
    return fail(LBM_E_ARG, "vec_per_thread must be 1, 2 or 4 (got %d)", vec_per_thread);
  if (nontemporal != 0 && nontemporal != 1) return fail(LBM_E_ARG, "nontemporal must be 0 or 1");
  if (blocks < 0) return fail(LBM_E_ARG, "blocks must be >= 0 (got %d)", blocks);
  if (!n_bytes) return LBM_OK;
  hipError_t e = lbm::launch_copy_variant(dst, src, n_bytes / 16, vec_per_thread, nontemporal != 0,
                                          size_t(blocks), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "copy probe launch");
}

lbm_status lbm_pull_copy(lbm_ctx* c, const void* src, void* dst) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!src || !dst) return fail(LBM_E_ARG, "src and dst must not be NULL");
  if (src == dst) return fail(LBM_E_ARG, "src and dst must differ");
  if (!aligned256(src) || !aligned256(dst)) return fail(LBM_E_ARG, "src/dst must be 256-byte aligned");
  hipError_t e = lbm::launch_pull_copy(c->p.storage, c->geo, src, dst, c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "pull-copy launch");
}

lbm_status lbm_use_graphs(lbm_ctx* c, int32_t steps_per_graph) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (steps_per_graph != 0 && (steps_per_graph < 2 || steps_per_graph > 4096 || steps_per_graph % 2))
    return fail(LBM_E_ARG, "steps_per_graph must be 0 or an even count in [2, 4096] (got %d)",
                steps_per_graph);
  if (steps_per_graph == c->graph_steps) return LBM_OK;
  hipError_t e = drop_graphs(c);  // no replay of the old graphs left in flight
  if (e != hipSuccess) return hip_fail(e, "waiting for the latest graph replay");
  c->graph_steps = 0;
  if (!steps_per_graph) return LBM_OK;
  if (!c->capture_stream) {
    e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
  }
  if (!c->replay_done) {
    e = hipEventCreateWithFlags(&c->replay_done, hipEventDisableTiming);
    if (e != hipSuccess) {
      c->replay_done = nullptr;
      return hip_fail(e, "replay event");
    }
  }
  c->graph_steps = steps_per_graph;
  for (int p = 0; p < 2 && st == LBM_OK; ++p) st = build_graph(c, p);
  if (st != LBM_OK) {
    (void)drop_graphs(c);
    c->graph_steps = 0;
  }
  return st;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  (void)drop_graphs(c);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  if (c->replay_done) (void)hipEventDestroy(c->replay_done);
  delete c;
}

const char* lbm_last_error(void) { return g_err; }

}  // extern "C"
