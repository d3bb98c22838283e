// rr_api.hip -- host runtime behind the C-ABI declared in include/rrmhd.h:
// handle, A/B population buffers, stream ordering, error mapping.
#include <hip/hip_runtime.h>

#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/rrmhd.h"
#include "rr_closure.h"
#include "rr_internal.h"
#include "rr_kernels.h"
#include "rr_node.h"

namespace {

thread_local char g_detail[512] = "";

int dev_err(hipError_t e, const char *what) {
  std::snprintf(g_detail, sizeof g_detail, "%s: %s", what, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? RRMHD_ENOMEM : RRMHD_EDEVICE;
}

}  // namespace

// shared with the three-dimensional handle (rr_3d.hip)
int rr_device_error(hipError_t e, const char *what) { return dev_err(e, what); }

namespace {

#define HIP_OR_RETURN(expr)                          \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return dev_err(e_, #expr); \
  } while (0)

bool finite_pos(double v) { return std::isfinite(v); }

// ---- workspace of the allocation-free diagnostics ---------------------------
// rrmhd_diagnostics_noalloc keeps the partial sums of the diagnostics pass and
// its eight results in this file-scope device array instead of the handle's
// lazily allocated workspace.  Every GPU the library runs on holds its own
// copy until the process ends.  In host code the name `scratch` only stands
// for the symbol: its device address is looked up once per device with
// hipGetSymbolAddress (at rrmhd_create, with that device current) and only
// that address is ever passed to kernels or copies.
constexpr size_t kScratchBytes = 72 * 1024;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use).
int scratch_address(int *dev_out, void **out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dev_err(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) {
    std::snprintf(g_detail, sizeof g_detail, "device %d beyond the scratch table", dev);
    return RRMHD_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return dev_err(e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = p;
  }
  *dev_out = dev;
  *out = g_scratch_dev[dev];
  return RRMHD_OK;
}

}  // namespace

struct rrmhd {
  rr::Domain D{};
  int storage = 0;
  int64_t elem = 4;  // bytes per stored value
  double tau_f = 0, tau_m = 0;
  rrmhd_bc bc{};
  hipStream_t stream = nullptr;
  void *buf[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t steps = 0;
  bool inplace = false;  // one population buffer (alternating step phases)
  size_t bytes = 0;      // bytes of one population buffer
  int phase = 0;         // in-place: 0 pull layout, 1 swapped layout
  bool ready = false;
  rr::LaunchShape shape{};
  void *diag_work = nullptr;
  void *fields_work = nullptr;  // 2 nx ny doubles for the j_z / w_z fields
  double *diag_out = nullptr;   // device, 8 doubles
  double *diag_host = nullptr;  // pinned, 8 doubles
  void *scratch = nullptr;      // device address of this device's `scratch`
  void *mlp = nullptr;          // prepared closure parameters (device)
  bool closure_on = false;
  int closure_grid = 0;         // persistent blocks of the closure kernel
  // graph replay of runs of graph_chunk steps (0: plain launches); one graph
  // per starting buffer (or in-place phase), on an internal stream ordered
  // after the caller's stream with events
  int graph_chunk = 0;
  bool poison = false;  // debug: NaN-fill the destination buffer before each step
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  hipStream_t own = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

// Debug fill of a population buffer with a NaN pattern (32-bit words).
__global__ void k_poison(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static hipError_t poison_buffer(const rrmhd *h, void *buf, hipStream_t st) {
  const int64_t words = (int64_t)(h->bytes / 4);
  const uint32_t nan = h->elem == 4 ? 0x7fc00000u : 0x7e007e00u;
  hipLaunchKernelGGL(k_poison, dim3(2048), dim3(256), 0, st, (uint32_t *)buf, words, nan);
  return hipGetLastError();
}

static void free_graphs(rrmhd *h) {
  for (auto &g : h->graph)
    if (g) (void)hipGraphExecDestroy(g), g = nullptr;
}

extern "C" {

const char *rrmhd_strerror(int code) {
  switch (code) {
    case RRMHD_OK: return "ok";
    case RRMHD_EINVAL: return "invalid argument";
    case RRMHD_ENOMEM: return "out of device memory";
    case RRMHD_EDEVICE: return "HIP device error";
    case RRMHD_ENONFINITE: return "non-finite diagnostic";
    case RRMHD_ESTATE: return "invalid state (not initialised)";
    case RRMHD_EIO: return "checkpoint file I/O error";
    default: return "unknown error";
  }
}

const char *rrmhd_last_error_detail(void) { return g_detail; }

int rrmhd_destroy(rrmhd *h) {
  if (!h) return RRMHD_OK;
  int rc = RRMHD_OK;
  if (h->stream || h->buf[0]) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = dev_err(e, "hipStreamSynchronize");
  }
  for (void *&p : h->buf)
    if (p) (void)hipFree(p), p = nullptr;
  if (h->diag_work) (void)hipFree(h->diag_work);
  if (h->fields_work) (void)hipFree(h->fields_work);
  if (h->diag_out) (void)hipFree(h->diag_out);
  if (h->diag_host) (void)hipHostFree(h->diag_host);
  if (h->mlp) (void)hipFree(h->mlp);
  free_graphs(h);
  if (h->ev_in) (void)hipEventDestroy(h->ev_in);
  if (h->ev_out) (void)hipEventDestroy(h->ev_out);
  if (h->own) (void)hipStreamDestroy(h->own);
  delete h;
  return rc;
}

int rrmhd_create(const rrmhd_grid *grid, double tau_f, double tau_m,
                 const rrmhd_bc *bc, void *hip_stream, rrmhd **out) {
  if (!out) return RRMHD_EINVAL;
  *out = nullptr;
  if (!grid) return RRMHD_EINVAL;
  if (grid->nx < 1 || grid->ny < 1) return RRMHD_EINVAL;
  const int kind = grid->storage & 0xff, flags = grid->storage & ~0xff;
  if (kind != RRMHD_STORE_F32 && kind != RRMHD_STORE_F16 && kind != RRMHD_STORE_F16_SR)
    return RRMHD_EINVAL;
  if ((flags & ~(RRMHD_STORE_INPLACE | RRMHD_STORE_PLANAR)) != 0) return RRMHD_EINVAL;
  if (!(std::isfinite(tau_f) && std::isfinite(tau_m)) || tau_f <= 0.5 || tau_m <= 0.5)
    return RRMHD_EINVAL;
  rrmhd_bc b{};
  b.kind = RRMHD_BC_PERIODIC;
  if (bc) b = *bc;
  if (b.kind != RRMHD_BC_PERIODIC && b.kind != RRMHD_BC_WALLS_Y) return RRMHD_EINVAL;
  if (b.kind == RRMHD_BC_WALLS_Y && grid->ny < 2) return RRMHD_EINVAL;
  for (int k = 0; k < 2; ++k)
    if (!finite_pos(b.force[k]) || !finite_pos(b.b_wall[k])) return RRMHD_EINVAL;
  const int64_t N = (int64_t)grid->nx * grid->ny;
  // in-plane offsets are 32-bit byte offsets: a plane stays below 4 GiB
  if (N * (kind == RRMHD_STORE_F32 ? 4 : 2) >= ((int64_t)1 << 32)) return RRMHD_EINVAL;
  float S = grid->codec_scale;
  if (S == 0.0f) S = 1.0f;
  int ex = 0;
  if (!(S > 0.0f) || std::frexp(S, &ex) != 0.5f) return RRMHD_EINVAL;  // power of two

  rrmhd *h = new (std::nothrow) rrmhd();
  if (!h) return RRMHD_ENOMEM;
  // the stochastic-rounding variant is FP16 storage for every read path
  h->storage = kind == RRMHD_STORE_F16_SR ? RRMHD_STORE_F16 : kind;
  h->inplace = (flags & RRMHD_STORE_INPLACE) != 0;
  h->elem = kind == RRMHD_STORE_F32 ? 4 : 2;
  h->tau_f = tau_f;
  h->tau_m = tau_m;
  h->bc = b;
  h->stream = (hipStream_t)hip_stream;
  rr::Domain &D = h->D;
  D.nx = grid->nx;
  D.ny = grid->ny;
  // planes start on 256-byte boundaries; an optional extra gap between
  // planes (RRMHD_PLANE_PAD_BYTES, a multiple of 256) staggers the plane
  // starts across HBM channels
  const int64_t align = 256 / h->elem;
  D.walls = b.kind == RRMHD_BC_WALLS_Y;
  // Layout: periodic handles keep the 19 planes row-interleaved (each grid
  // row holds its 19 plane rows side by side, each starting on a 256-byte
  // boundary), which streams faster than whole planes; walls, or
  // RRMHD_STORE_PLANAR (or RRMHD_LAYOUT=planar), keep planes of [ny][nx].
  bool rows = !D.walls && !(flags & RRMHD_STORE_PLANAR);
  if (const char *e = std::getenv("RRMHD_LAYOUT"))
    if (std::strcmp(e, "planar") == 0) rows = false;
  if (rows) {
    int64_t pad = 0;  // extra gap between row groups
    if (const char *e = std::getenv("RRMHD_ROW_PAD_BYTES")) {
      long long v = std::atoll(e);
      if (v >= 0 && v % 256 == 0) pad = v / h->elem;
    }
    D.plane = ((int64_t)grid->nx + align - 1) / align * align;
    D.row = rr::kStatePlanes * D.plane + pad;
    h->bytes = (size_t)D.row * grid->ny * h->elem;
  } else {
    int64_t pad = 256 / h->elem;  // measured best default: 256 B between planes
    if (const char *e = std::getenv("RRMHD_PLANE_PAD_BYTES")) {
      long long v = std::atoll(e);
      if (v >= 0 && v % 256 == 0) pad = v / h->elem;
    }
    D.plane = (N + align - 1) / align * align + pad;
    D.row = grid->nx;
    h->bytes = (size_t)D.plane * rr::kStatePlanes * h->elem;
  }
  const double om = 1.0 / tau_f, omm = 1.0 / tau_m;
  D.om_c = (float)(1.0 - om);
  D.omm_c = (float)(1.0 - omm);
  D.src_c = (float)(1.0 - 0.5 * om);
  D.Gx = (float)b.force[0];
  D.Gy = (float)b.force[1];
  D.bw2x = (float)(b.b_wall[0] / 3.0);
  D.bw2y = (float)(b.b_wall[1] / 3.0);
  D.s = kind != RRMHD_STORE_F32 ? S : 1.0f;
  D.sr = kind == RRMHD_STORE_F16_SR;
  D.inv_s = 1.0f / D.s;
  D.elem = (int)h->elem;
  h->shape = rr::default_shape(D);
  if (h->inplace) {
    // measured best for the alternating single-buffer steps at 8192^2, with
    // eight neighbouring tiles per XCD and non-temporal stores: FP16 storage
    // (round to nearest) on row-interleaved planes 64 x 2 threads with two
    // nodes per thread; otherwise one node per thread and one row per
    // workgroup, 128 wide (FP16 storage, or FP32 on row-interleaved planes)
    // or 64 wide (FP32 on planes of [ny][nx])
    const bool rows_wide = D.row != D.nx && D.nx >= 512;
    h->shape.ry = 1;
    h->shape.xcd = 2;
    if (rows_wide && h->elem == 2 && D.nx % 2 == 0 && !D.sr) {
      h->shape.bx = 64;
      h->shape.by = 2;
      h->shape.nt = 5;
    } else {
      h->shape.bx = (h->elem == 2 || rows_wide) ? 128 : 64;
      h->shape.by = 1;
      h->shape.nt = 1;
    }
  }

  // environment overrides of the launch shape ("BXxBY" or "BXxBYxRY") and of
  // the debug poison mode (two-buffer handles), for runs driven from outside
  if (const char *e = std::getenv("RRMHD_TILE")) {
    int bx = 0, by = 0, ry = 1;
    const int k = std::sscanf(e, "%dx%dx%d", &bx, &by, &ry);
    if (k >= 2 && bx >= 1 && by >= 1 && bx * by <= 256 && ry >= 1) {
      h->shape.bx = bx;
      h->shape.by = by;
      h->shape.ry = ry;
      h->shape.nt &= 1;  // a tile given this way is for the one-node update
    }
  }
  if (const char *e = std::getenv("RRMHD_DEBUG_POISON"))
    h->poison = !h->inplace && std::atoi(e) != 0;
  const size_t bytes = h->bytes;
  int rc = RRMHD_OK;
  for (int k = 0; k < (h->inplace ? 1 : 2) && rc == RRMHD_OK; ++k) {
    hipError_t e = hipMalloc(&h->buf[k], bytes);
    if (e != hipSuccess) rc = dev_err(e, "hipMalloc(populations)");
  }
  if (rc == RRMHD_OK) {
    hipError_t e = hipMalloc((void **)&h->diag_out, 8 * sizeof(double));
    if (e != hipSuccess) rc = dev_err(e, "hipMalloc(diag)");
  }
  if (rc == RRMHD_OK) {
    hipError_t e = hipHostMalloc((void **)&h->diag_host, 8 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) rc = dev_err(e, "hipHostMalloc(diag)");
  }
  if (rc == RRMHD_OK) {
    int dev = -1;
    rc = scratch_address(&dev, &h->scratch);
  }
  if (rc != RRMHD_OK) {
    rrmhd_destroy(h);
    return rc;
  }
  *out = h;
  return RRMHD_OK;
}

int rrmhd_set_launch(rrmhd *h, int bx, int by, int ry, int xcd, int nt) {
  if (!h || bx < 1 || by < 1 || bx * by > 256 || ry < 1) return RRMHD_EINVAL;
  free_graphs(h);
  h->shape.bx = bx;
  h->shape.by = by;
  h->shape.ry = ry;
  h->shape.xcd = (xcd >= 0 && xcd <= 2) ? xcd : 0;
  h->shape.nt = nt & 15;
  return RRMHD_OK;
}

int rrmhd_get_launch(const rrmhd *h, int *bx, int *by, int *ry, int *xcd, int *nt) {
  if (!h) return RRMHD_EINVAL;
  if (bx) *bx = h->shape.bx;
  if (by) *by = h->shape.by;
  if (ry) *ry = h->shape.ry;
  if (xcd) *xcd = h->shape.xcd;
  if (nt) *nt = h->shape.nt;
  return RRMHD_OK;
}

int rrmhd_set_stream(rrmhd *h, void *hip_stream) {
  if (!h) return RRMHD_EINVAL;
  h->stream = (hipStream_t)hip_stream;
  return RRMHD_OK;
}

int rrmhd_set_equilibrium(rrmhd *h, int kind) {
  if (!h || (kind != RRMHD_FEQ_ALGORITHM && kind != RRMHD_FEQ_FULL_MAXWELL)) return RRMHD_EINVAL;
  if (kind == RRMHD_FEQ_FULL_MAXWELL && (h->closure_on || h->inplace || h->D.sr))
    return RRMHD_EINVAL;
  free_graphs(h);
  h->D.feq = kind;
  return RRMHD_OK;
}

int rrmhd_init(rrmhd *h, const double *u, const double *b) {
  if (!h || !u || !b) return RRMHD_EINVAL;
  HIP_OR_RETURN(rr::launch_init(h->storage, h->D, u, b, h->bc.b_wall[0],
                                h->bc.b_wall[1], h->buf[0], h->stream));
  h->cur = 0;
  h->phase = 0;
  h->steps = 0;
  h->ready = true;
  return RRMHD_OK;
}

static int plain_steps(rrmhd *h, int64_t n, hipStream_t st) {
  for (int64_t k = 0; k < n; ++k) {
    // random bits of the stochastic-rounding codec: keyed by the step count
    h->D.sr_key = rr::mix32((uint32_t)h->steps * 0x27d4eb2fu + 0x165667b1u);
    if (h->inplace) {
      HIP_OR_RETURN(rr::launch_step_inplace(h->storage, h->D, h->buf[0], h->phase, h->shape, st));
      h->phase ^= 1;
    } else {
      if (h->poison) HIP_OR_RETURN(poison_buffer(h, h->buf[h->cur ^ 1], st));
      if (h->closure_on)
        HIP_OR_RETURN(rr::launch_step_closure(h->storage, h->D, (const rr::MlpDev *)h->mlp,
                                              h->buf[h->cur], h->buf[h->cur ^ 1],
                                              h->closure_grid, st));
      else
        HIP_OR_RETURN(rr::launch_step(h->storage, h->D, h->buf[h->cur], h->buf[h->cur ^ 1],
                                      h->shape, st));
      h->cur ^= 1;
    }
    h->steps++;
  }
  return RRMHD_OK;
}

int rrmhd_step(rrmhd *h, int64_t n) {
  if (!h || n < 0) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  const int64_t chunk = h->graph_chunk;
  if (chunk <= 0 || n < chunk) return plain_steps(h, n, h->stream);
  HIP_OR_RETURN(hipEventRecord(h->ev_in, h->stream));
  HIP_OR_RETURN(hipStreamWaitEvent(h->own, h->ev_in, 0));
  int64_t left = n;
  while (left >= chunk) {
    const int state = h->inplace ? h->phase : h->cur;
    hipGraphExec_t &g = h->graph[state];
    if (!g) {
      hipGraph_t graph = nullptr;
      const int c0 = h->cur, p0 = h->phase;
      const int64_t s0 = h->steps;
      HIP_OR_RETURN(hipStreamBeginCapture(h->own, hipStreamCaptureModeThreadLocal));
      int rc = plain_steps(h, chunk, h->own);
      hipError_t ee = hipStreamEndCapture(h->own, &graph);
      h->cur = c0;  // the capture recorded the launches; nothing ran yet
      h->phase = p0;
      h->steps = s0;
      if (rc != RRMHD_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ee != hipSuccess) return dev_err(ee, "hipStreamEndCapture");
      hipError_t ei = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return dev_err(ei, "hipGraphInstantiate");
    }
    HIP_OR_RETURN(hipGraphLaunch(g, h->own));
    if (chunk & 1) {
      h->cur ^= h->inplace ? 0 : 1;
      h->phase ^= h->inplace ? 1 : 0;
    }
    h->steps += chunk;
    left -= chunk;
  }
  int rc = plain_steps(h, left, h->own);
  if (rc != RRMHD_OK) return rc;
  HIP_OR_RETURN(hipEventRecord(h->ev_out, h->own));
  HIP_OR_RETURN(hipStreamWaitEvent(h->stream, h->ev_out, 0));
  return RRMHD_OK;
}

int rrmhd_set_debug_poison(rrmhd *h, int on) {
  if (!h || (on && h->inplace)) return RRMHD_EINVAL;
  if (h->poison != (on != 0)) free_graphs(h);
  h->poison = on != 0;
  return RRMHD_OK;
}

int rrmhd_set_graph_chunk(rrmhd *h, int chunk) {
  if (!h || chunk < 0) return RRMHD_EINVAL;
  if (chunk > 0 && h->D.sr) return RRMHD_EINVAL;  // a graph would freeze the step key
  free_graphs(h);
  if (chunk > 0 && !h->own) {
    HIP_OR_RETURN(hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking));
    HIP_OR_RETURN(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
    HIP_OR_RETURN(hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming));
  }
  h->graph_chunk = chunk;
  return RRMHD_OK;
}

int rrmhd_moments(rrmhd *h, double *rho, double *u, double *b) {
  if (!h) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  if (!rho && !u && !b) return RRMHD_OK;
  HIP_OR_RETURN(rr::launch_moments(h->storage, h->D, h->buf[h->cur], rho, u, b,
                                   h->stream, h->inplace ? h->phase : 0));
  return RRMHD_OK;
}

// One diagnostics pass with the given workspace (diag_work_bytes) and
// device output (8 doubles); the results land in the pinned diag_host.
static int run_diag_with(rrmhd *h, void *work, double *out_dev) {
  HIP_OR_RETURN(rr::launch_diagnostics(h->storage, h->D, h->buf[h->cur], work, out_dev,
                                       h->stream, h->inplace ? h->phase : 0));
  HIP_OR_RETURN(hipMemcpyAsync(h->diag_host, out_dev, 8 * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
  HIP_OR_RETURN(hipStreamSynchronize(h->stream));
  return RRMHD_OK;
}

static int run_diag(rrmhd *h) {
  if (!h->diag_work) {
    HIP_OR_RETURN(hipMalloc(&h->diag_work, rr::diag_work_bytes(h->D)));
  }
  return run_diag_with(h, h->diag_work, h->diag_out);
}

static int diag_results(const rrmhd *h, double *E_kin, double *E_mag, double *max_div_b) {
  const double *r = h->diag_host;
  const bool bad = !(std::isfinite(r[0]) && std::isfinite(r[1]) && std::isfinite(r[2]));
  const double nan = std::nan("");
  if (E_kin) *E_kin = bad ? nan : r[0];
  if (E_mag) *E_mag = bad ? nan : r[1];
  if (max_div_b) *max_div_b = bad ? nan : r[2];
  return bad ? RRMHD_ENONFINITE : RRMHD_OK;
}

int rrmhd_diagnostics(rrmhd *h, double *E_kin, double *E_mag, double *max_div_b) {
  if (!h) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  int rc = run_diag(h);
  if (rc != RRMHD_OK) return rc;
  return diag_results(h, E_kin, E_mag, max_div_b);
}

int rrmhd_diagnostics_noalloc(rrmhd *h, double *E_kin, double *E_mag, double *max_div_b) {
  if (!h) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  // the workspace holds the pass's partial sums, then its eight results
  const size_t work = rr::diag_work_bytes(h->D);
  const size_t need = (work + 255) / 256 * 256 + 8 * sizeof(double);
  if (need > kScratchBytes) {
    std::snprintf(g_detail, sizeof g_detail,
                  "diagnostics workspace of %zu bytes exceeds the static %zu", need,
                  kScratchBytes);
    return RRMHD_EINVAL;
  }
  if (!h->scratch) return RRMHD_ESTATE;
  // every partial sum the final reduction reads is written by the same pass
  // first, so nothing in the workspace needs clearing between calls
  char *base = (char *)h->scratch;
  int rc = run_diag_with(h, base, (double *)(base + (work + 255) / 256 * 256));
  if (rc != RRMHD_OK) return rc;
  return diag_results(h, E_kin, E_mag, max_div_b);
}

int rrmhd_invariants(rrmhd *h, double out[5]) {
  if (!h || !out) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  int rc = run_diag(h);
  if (rc != RRMHD_OK) return rc;
  for (int k = 0; k < 5; ++k) out[k] = h->diag_host[3 + k];
  return RRMHD_OK;
}

int rrmhd_step_count(const rrmhd *h, int64_t *out) {
  if (!h || !out) return RRMHD_EINVAL;
  *out = h->steps;
  return RRMHD_OK;
}

}  // extern "C"

// Copy between a population buffer and the dense state of 19 planes of
// [ny][nx] (device to device, on the handle's stream); to_buf selects the
// direction.
static hipError_t copy_planes(const rrmhd *h, void *dense, const void *buf_in, bool to_buf) {
  // to_buf: dense -> buf_in (the buffer is then written); else buf_in -> dense
  const size_t plane_bytes = (size_t)h->D.nx * h->D.ny * h->elem;
  const size_t width = (size_t)h->D.nx * h->elem, rstride = (size_t)h->D.row * h->elem;
  if (h->D.row == h->D.nx) {
    const size_t pitch = (size_t)h->D.plane * h->elem;
    return to_buf ? hipMemcpy2DAsync((void *)buf_in, pitch, dense, plane_bytes, plane_bytes,
                                     rr::kStatePlanes, hipMemcpyDeviceToDevice, h->stream)
                  : hipMemcpy2DAsync(dense, plane_bytes, buf_in, pitch, plane_bytes,
                                     rr::kStatePlanes, hipMemcpyDeviceToDevice, h->stream);
  }
  for (int p = 0; p < rr::kStatePlanes; ++p) {
    char *d = (char *)dense + p * plane_bytes;
    char *b = (char *)buf_in + (size_t)p * h->D.plane * h->elem;
    hipError_t e = to_buf ? hipMemcpy2DAsync(b, rstride, d, width, width, h->D.ny,
                                             hipMemcpyDeviceToDevice, h->stream)
                          : hipMemcpy2DAsync(d, width, b, rstride, width, h->D.ny,
                                             hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

extern "C" {

int64_t rrmhd_state_bytes(const rrmhd *h) {
  if (!h) return RRMHD_EINVAL;
  return (int64_t)h->D.nx * h->D.ny * rr::kStatePlanes * h->elem;
}

int rrmhd_save_state(rrmhd *h, void *dst, int64_t bytes) {
  if (!h || !dst || bytes < rrmhd_state_bytes(h)) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  if (h->inplace && h->phase) {
    HIP_OR_RETURN(rr::launch_swapped_to_pull(h->storage, h->D, h->buf[0], dst, h->stream));
    return RRMHD_OK;
  }
  HIP_OR_RETURN(copy_planes(h, dst, (const char *)h->buf[h->cur], false));
  return RRMHD_OK;
}

int rrmhd_load_state(rrmhd *h, const void *src, int64_t bytes, int64_t step_count) {
  if (!h || !src || bytes < rrmhd_state_bytes(h) || step_count < 0) return RRMHD_EINVAL;
  HIP_OR_RETURN(copy_planes(h, const_cast<void *>(src), h->buf[0], true));
  h->cur = 0;
  h->phase = 0;
  h->steps = step_count;
  h->ready = true;
  return RRMHD_OK;
}

}  // extern "C"

namespace {

// Checkpoint file header (little-endian, as written by x86 and read back on
// the same platform).
struct CkHeader {
  char magic[8];
  int32_t version, nx, ny, storage;
  float codec_scale;
  int32_t bc_kind, equilibrium, zero;
  double tau_f, tau_m, force[2], b_wall[2];
  int64_t steps, payload;
};
static_assert(sizeof(CkHeader) == 104, "checkpoint header layout");
constexpr char kCkMagic[8] = {'R', 'R', 'M', 'H', 'D', 'C', 'K', '1'};

CkHeader ck_header(const rrmhd *h) {
  CkHeader c{};
  std::memcpy(c.magic, kCkMagic, 8);
  c.version = 1;
  c.nx = h->D.nx;
  c.ny = h->D.ny;
  c.storage = h->storage == RRMHD_STORE_F32 ? RRMHD_STORE_F32
                                            : (h->D.sr ? RRMHD_STORE_F16_SR : RRMHD_STORE_F16);
  c.codec_scale = h->D.s;
  c.bc_kind = h->bc.kind;
  c.equilibrium = h->D.feq;
  c.tau_f = h->tau_f;
  c.tau_m = h->tau_m;
  for (int k = 0; k < 2; ++k) {
    c.force[k] = h->bc.force[k];
    c.b_wall[k] = h->bc.b_wall[k];
  }
  c.steps = h->steps;
  c.payload = (int64_t)h->D.nx * h->D.ny * h->elem * rr::kStatePlanes;
  return c;
}

int io_err(const char *what, const char *path) {
  std::snprintf(g_detail, sizeof g_detail, "%s %s: %s", what, path, std::strerror(errno));
  return RRMHD_EIO;
}

// Bitwise comparison of doubles: the file must carry exactly the handle's
// parameters.
bool same(double a, double b) { return std::memcmp(&a, &b, sizeof a) == 0; }

}  // namespace

int rr_ck_mismatch(const char *field) {
  std::snprintf(g_detail, sizeof g_detail, "checkpoint does not match the handle: %s", field);
  return RRMHD_EINVAL;
}

int rr_ck_write(const char *path, const void *hdr, size_t hdr_bytes, const char *base,
                size_t pitch, size_t row, int planes, size_t rstride, int nrows) {
  char *host = new (std::nothrow) char[row];
  if (!host) return RRMHD_ENOMEM;
  int rc = RRMHD_OK;
  FILE *f = std::fopen(path, "wb");
  if (!f) rc = io_err("cannot open", path);
  if (rc == RRMHD_OK && std::fwrite(hdr, hdr_bytes, 1, f) != 1) rc = io_err("cannot write", path);
  for (int p = 0; p < planes && rc == RRMHD_OK; ++p) {
    hipError_t e =
        nrows > 1 ? hipMemcpy2D(host, row / nrows, base + (size_t)p * pitch, rstride, row / nrows,
                                nrows, hipMemcpyDeviceToHost)
                  : hipMemcpy(host, base + (size_t)p * pitch, row, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = dev_err(e, "hipMemcpy(checkpoint plane)");
    else if (std::fwrite(host, 1, row, f) != row) rc = io_err("cannot write", path);
  }
  if (f && std::fclose(f) != 0 && rc == RRMHD_OK) rc = io_err("cannot close", path);
  delete[] host;
  return rc;
}

int rr_ck_open(const char *path, void *hdr, size_t hdr_bytes, FILE **out) {
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) return io_err("cannot open", path);
  if (std::fread(hdr, hdr_bytes, 1, f) != 1) {
    std::fclose(f);
    return rr_ck_mismatch("file shorter than the header");
  }
  *out = f;
  return RRMHD_OK;
}

int rr_ck_read_planes(FILE *f, const char *path, size_t hdr_bytes, char *base, size_t pitch,
                      size_t row, int planes, bool *touched, size_t rstride, int nrows) {
  *touched = false;
  // the whole payload must be in the file before the device state is
  // touched, so a short file leaves the handle unchanged
  if (std::fseek(f, 0, SEEK_END) != 0) return io_err("cannot seek", path);
  const long end = std::ftell(f);
  if (end < 0) return io_err("cannot seek", path);
  if ((uint64_t)end != hdr_bytes + (uint64_t)row * planes) return rr_ck_mismatch("file size");
  if (std::fseek(f, (long)hdr_bytes, SEEK_SET) != 0) return io_err("cannot seek", path);
  char *host = new (std::nothrow) char[row];
  if (!host) return RRMHD_ENOMEM;
  int rc = RRMHD_OK;
  for (int p = 0; p < planes && rc == RRMHD_OK; ++p) {
    if (std::fread(host, 1, row, f) != row) {
      rc = io_err("cannot read", path);
      break;
    }
    *touched = true;
    hipError_t e =
        nrows > 1 ? hipMemcpy2D(base + (size_t)p * pitch, rstride, host, row / nrows, row / nrows,
                                nrows, hipMemcpyHostToDevice)
                  : hipMemcpy(base + (size_t)p * pitch, host, row, hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = dev_err(e, "hipMemcpy(checkpoint plane)");
  }
  delete[] host;
  return rc;
}

extern "C" {

int rrmhd_save(rrmhd *h, const char *path) {
  if (!h || !path) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  const CkHeader hd = ck_header(h);
  const size_t row = (size_t)h->D.nx * h->D.ny * h->elem;
  void *tmp = nullptr;
  const char *base = (const char *)h->buf[h->cur];
  size_t pitch = (size_t)h->D.plane * h->elem;
  size_t rstride = 0;
  int nrows = 1;
  if (h->D.row != h->D.nx) {  // row-interleaved: each plane gathered row by row
    rstride = (size_t)h->D.row * h->elem;
    nrows = h->D.ny;
  }
  if (h->inplace && h->phase) {
    // between the two step forms: gather the swapped layout first
    HIP_OR_RETURN(hipMalloc(&tmp, row * rr::kStatePlanes));
    hipError_t e = rr::launch_swapped_to_pull(h->storage, h->D, h->buf[0], tmp, h->stream);
    if (e != hipSuccess) {
      (void)hipFree(tmp);
      return dev_err(e, "launch_swapped_to_pull");
    }
    base = (const char *)tmp;
    pitch = row;
    rstride = 0;  // the gathered copy is dense
    nrows = 1;
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  int rc = e != hipSuccess ? dev_err(e, "hipStreamSynchronize")
                           : rr_ck_write(path, &hd, sizeof hd, base, pitch, row, rr::kStatePlanes,
                                         rstride, nrows);
  if (tmp) (void)hipFree(tmp);
  return rc;
}

int rrmhd_load(rrmhd *h, const char *path) {
  if (!h || !path) return RRMHD_EINVAL;
  CkHeader hd{};
  FILE *f = nullptr;
  int rc = rr_ck_open(path, &hd, sizeof hd, &f);
  if (rc != RRMHD_OK) return rc;
  const CkHeader me = ck_header(h);
  const bool mine16 = me.storage != RRMHD_STORE_F32, file16 = hd.storage != RRMHD_STORE_F32;
  if (std::memcmp(hd.magic, kCkMagic, 8) != 0 || hd.version != 1) rc = rr_ck_mismatch("magic/version");
  else if (hd.nx != me.nx || hd.ny != me.ny) rc = rr_ck_mismatch("grid size");
  else if (hd.storage < RRMHD_STORE_F32 || hd.storage > RRMHD_STORE_F16_SR || mine16 != file16)
    rc = rr_ck_mismatch("storage");
  else if (hd.codec_scale != me.codec_scale) rc = rr_ck_mismatch("codec scale");
  else if (!same(hd.tau_f, me.tau_f) || !same(hd.tau_m, me.tau_m)) rc = rr_ck_mismatch("tau");
  else if (hd.bc_kind != me.bc_kind || !same(hd.force[0], me.force[0]) ||
           !same(hd.force[1], me.force[1]) || !same(hd.b_wall[0], me.b_wall[0]) ||
           !same(hd.b_wall[1], me.b_wall[1]))
    rc = rr_ck_mismatch("boundary conditions");
  else if (hd.equilibrium != me.equilibrium) rc = rr_ck_mismatch("equilibrium");
  else if (hd.payload != me.payload || hd.steps < 0) rc = rr_ck_mismatch("payload size / step count");
  if (rc == RRMHD_OK) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = dev_err(e, "hipStreamSynchronize");
  }
  bool touched = false;
  if (rc == RRMHD_OK)
    rc = rr_ck_read_planes(f, path, sizeof hd, (char *)h->buf[0], (size_t)h->D.plane * h->elem,
                           (size_t)h->D.nx * h->D.ny * h->elem, rr::kStatePlanes, &touched,
                           h->D.row != h->D.nx ? (size_t)h->D.row * h->elem : 0,
                           h->D.row != h->D.nx ? h->D.ny : 1);
  std::fclose(f);
  if (rc != RRMHD_OK) {
    if (touched) h->ready = false;  // part of the state was overwritten
    return rc;
  }
  h->cur = 0;
  h->phase = 0;
  h->steps = hd.steps;
  h->ready = true;
  return RRMHD_OK;
}

int rr_handle_info(const rrmhd *h, int *nx, int *ny, int *storage, hipStream_t *stream,
                   int *ready) {
  if (!h) return RRMHD_EINVAL;
  if (nx) *nx = h->D.nx;
  if (ny) *ny = h->D.ny;
  if (storage) *storage = h->storage;
  if (stream) *stream = h->stream;
  if (ready) *ready = h->ready ? 1 : 0;
  return RRMHD_OK;
}

int rr_handle_walls(const rrmhd *h) { return h && h->D.walls ? 1 : 0; }

int rr_handle_inplace(const rrmhd *h) { return h && h->inplace ? 1 : 0; }

int rr_handle_rows(const rrmhd *h) { return h && h->D.row != h->D.nx ? 1 : 0; }

void rr_handle_set_ready(rrmhd *h, int ready) {
  if (h) h->ready = ready != 0;
}

int rrmhd_closure_set(rrmhd *h, const float *params, const float *norm) {
  if (!h) return RRMHD_EINVAL;
  if (!params) {
    if (h->closure_on) free_graphs(h);
    h->closure_on = false;
    return RRMHD_OK;
  }
  if (!norm) return RRMHD_EINVAL;
  if (!h->mlp) HIP_OR_RETURN(hipMalloc(&h->mlp, rr::mlp_dev_bytes()));
  HIP_OR_RETURN(rr::launch_mlp_prepare(params, norm, (rr::MlpDev *)h->mlp, h->stream));
  if (!h->closure_grid) {
    int dev = 0, cus = 256;
    HIP_OR_RETURN(hipGetDevice(&dev));
    HIP_OR_RETURN(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    h->closure_grid = cus;  // one 1024-thread block per CU (LDS-bound)
  }
  return RRMHD_OK;
}

int rrmhd_closure_enable(rrmhd *h, int on) {
  if (!h) return RRMHD_EINVAL;
  if (on && (!h->mlp || h->D.walls || h->D.Gx != 0.0f || h->D.Gy != 0.0f || h->D.feq ||
             h->inplace || h->D.sr))
    return RRMHD_EINVAL;
  if (h->closure_on != (on != 0)) free_graphs(h);
  h->closure_on = on != 0;
  return RRMHD_OK;
}

int rrmhd_closure_eval(const float *params, const float *norm, const float *x, int64_t n,
                       float *y, void *hip_stream) {
  if (!params || !norm || n < 0 || (n > 0 && (!x || !y))) return RRMHD_EINVAL;
  const hipStream_t st = (hipStream_t)hip_stream;
  void *mlp = nullptr;
  HIP_OR_RETURN(hipMalloc(&mlp, rr::mlp_dev_bytes()));
  hipError_t e = rr::launch_mlp_prepare(params, norm, (rr::MlpDev *)mlp, st);
  if (e == hipSuccess) e = rr::launch_mlp_eval((const rr::MlpDev *)mlp, x, y, n, st);
  hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(mlp);
  if (e != hipSuccess) return dev_err(e, "closure eval");
  if (e2 != hipSuccess) return dev_err(e2, "hipStreamSynchronize");
  return RRMHD_OK;
}

int rrmhd_closure_gelu_table(uint16_t *out, void *hip_stream) {
  if (!out) return RRMHD_EINVAL;
  HIP_OR_RETURN(rr::launch_gelu_table(out, (hipStream_t)hip_stream));
  return RRMHD_OK;
}

int rrmhd_train_impose_fluid(rrmhd *h, const double *rho, const double *j, const double *b) {
  if (!h || !rho || !j || !b || h->D.walls || h->inplace) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  const int rc = rr_launch_impose_fluid(h->storage, &h->D, h->buf[h->cur], rho, j, b, h->stream);
  if (rc != RRMHD_OK) return rr_device_error(hipGetLastError(), "rrmhd_train_impose_fluid");
  return RRMHD_OK;
}

int rrmhd_current_vorticity(rrmhd *h, double *jz, double *wz) {
  if (!h) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  if (h->D.walls) return RRMHD_EINVAL;
  if (!jz && !wz) return RRMHD_OK;
  if (!h->fields_work)
    HIP_OR_RETURN(hipMalloc(&h->fields_work, sizeof(double) * 2 * (size_t)h->D.nx * h->D.ny));
  // velocity planes for the vorticity's gradient
  int rc = rr_launch_current_vorticity(h->storage, &h->D, h->buf[h->cur], 1.0 / h->tau_m, jz, wz,
                                       (double *)h->fields_work, h->stream,
                                       h->inplace ? h->phase : 0);
  if (rc != RRMHD_OK) return dev_err(hipGetLastError(), "current/vorticity kernels");
  return RRMHD_OK;
}

}  // extern "C"
