// rr_batch.hip -- ensemble of independent periodic domains of uneven sizes
// and relaxation times advanced by one persistent kernel launch per step.
//
// All domains live in one pair of buffers; domain d's 19 planes start at
// element offset base[d].  The work list is flat: domain d owns tiles
// [tile_first[d], tile_first[d] + ntiles[d]) of 256 threads (bx x by, its own
// tile shape), and the workgroups of one launch share out the whole list
// (statically by stride, one tile per workgroup, or by dynamic fetches from a
// device counter), so the load is balanced tile by tile whatever the mix of
// sizes.  The node
// update is the same device function as the single-domain kernel, so each
// domain evolves bitwise as a standalone run would.  n steps are captured
// into one hipGraph and launched at once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/rrmhd.h"
#include "rr_internal.h"
#include "rr_kernels.h"
#include "rr_node.h"
#include "rr_pull.h"

namespace rr {

struct BatchDom {
  int64_t base;   // element offset of plane 0 in each buffer
  int64_t plane;  // elements between planes
  int nx, ny;
  float om_c, omm_c;
  int bx, by;  // tile shape, bx * by = 256
  int tiles_x;
  int tile_first;
};

// One step of the whole ensemble.  Static schedule (per_fetch = 0): workgroup
// w takes tiles w, w + G, w + 2G, ... (G = grid size; G = ntiles is one tile
// per workgroup).  Dynamic schedule (per_fetch = k > 0): the list is cut into
// kSeg contiguous segments, one per XCD (workgroups are dispatched to the
// XCDs round-robin, so workgroup w runs on XCD w % kSeg); a workgroup starts
// with its own first chunk of k tiles of its segment and then takes chunk
// numbers from the segment's device counter, so each XCD works through a
// contiguous window of its segment and the counters are not shared across
// XCDs.  Per segment, ctr[kCtrStride s] counts fetched chunks and
// ctr[kCtrStride s + 1] finished workgroups; the segment's last workgroup to
// finish sets both back to zero, so every launch starts from zero without a
// memset node.  A workgroup leaves its loop once a fetched chunk lies past
// its segment, so no workgroup waits on another.
constexpr int kSeg = 8, kCtrStride = 64;  // counters 256 B apart

template <class C, bool NT>
__device__ __forceinline__ void batch_tile(const BatchDom *__restrict__ doms,
                                           const int *__restrict__ tile_dom, int t, float s,
                                           float inv_s, const typename C::T *__restrict__ src,
                                           typename C::T *__restrict__ dst) {
  const int d = __builtin_amdgcn_readfirstlane(tile_dom[t]);
  const BatchDom D = doms[d];
  const int lt = t - D.tile_first;
  const int ty = lt / D.tiles_x, tx = lt - ty * D.tiles_x;
  const int ly = threadIdx.x / D.bx, lx = threadIdx.x - ly * D.bx;
  const int x = tx * D.bx + lx, y = ty * D.by + ly;
  if (x < D.nx && y < D.ny) {
    CollideParams P;
    P.om_c = D.om_c;
    P.omm_c = D.omm_c;
    P.Gx = 0.0f;
    P.Gy = 0.0f;
    P.src_c = 0.0f;
    const PlaneGeom G{D.plane, D.nx, D.ny, s, inv_s, 0u, (int64_t)D.nx};  // planes of [ny][nx]
    update_periodic<C, false, NT, false>(G, src + D.base, dst + D.base, x, y, P);
  }
}

template <class C, bool NT, bool DYN>
__global__ __launch_bounds__(256) void k_batch_step(const BatchDom *__restrict__ doms,
                                                    const int *__restrict__ tile_dom,
                                                    int ntiles, int per_fetch, float s,
                                                    float inv_s,
                                                    const typename C::T *__restrict__ src,
                                                    typename C::T *__restrict__ dst,
                                                    int *__restrict__ ctr) {
  if (!DYN) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x)
      batch_tile<C, NT>(doms, tile_dom, t, s, inv_s, src, dst);
    return;
  }
  __shared__ int next[2];
  const int seg = blockIdx.x % kSeg;
  const int wl = blockIdx.x / kSeg;
  const int nwg = ((int)gridDim.x - seg + kSeg - 1) / kSeg;  // workgroups of this segment
  const int lo = (int)((int64_t)ntiles * seg / kSeg);
  const int hi = (int)((int64_t)ntiles * (seg + 1) / kSeg);
  int *c = ctr + kCtrStride * seg;
  int k = 0;
  for (int t0 = lo + wl * per_fetch; t0 < hi;) {
    const int t1 = min(t0 + per_fetch, hi);
    for (int t = t0; t < t1; ++t) batch_tile<C, NT>(doms, tile_dom, t, s, inv_s, src, dst);
    if (threadIdx.x == 0) next[k] = lo + (atomicAdd(&c[0], 1) + nwg) * per_fetch;
    __syncthreads();
    t0 = next[k];
    k ^= 1;  // the other slot: thread 0 may write it before slower waves read this one
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&c[1], 1) == nwg - 1) {
      __threadfence();
      atomicExch(&c[0], 0);
      atomicExch(&c[1], 0);
    }
  }
}

}  // namespace rr

namespace {

thread_local char g_bdetail[512] = "";

int bdev_err(hipError_t e, const char *what) {
  std::snprintf(g_bdetail, sizeof g_bdetail, "%s: %s", what, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? RRMHD_ENOMEM : RRMHD_EDEVICE;
}

#define BHIP(expr)                                     \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return bdev_err(e_, #expr);  \
  } while (0)

}  // namespace

struct rrmhd_batch {
  int n = 0;
  int storage = 0;
  int64_t elem = 4;
  float s = 1.0f, inv_s = 1.0f;
  std::vector<rr::BatchDom> doms;
  std::vector<int> tile_dom;
  std::vector<double> tau_f, tau_m;
  std::vector<int64_t> init_step;  // batch step at which domain d was initialised
  int ntiles = 0;
  int grid = 0;      // workgroups per launch (-1: one per tile)
  int per_fetch = 0;  // tiles per dynamic fetch (0: static stride)
  int nt = 1;
  int *d_ctr = nullptr;  // dynamic-schedule counters (zero between launches)
  rr::BatchDom *d_doms = nullptr;
  int *d_tile_dom = nullptr;
  void *buf[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t steps = 0;
  hipStream_t user = nullptr;  // caller's stream
  hipStream_t own = nullptr;   // internal stream for graph launches
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int graph_chunk = 0;
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // by starting parity
  void *diag_work = nullptr;
  size_t diag_bytes = 0;
  double *diag_out = nullptr, *diag_host = nullptr;
};

static void free_graphs(rrmhd_batch *b) {
  for (auto &g : b->graph)
    if (g) (void)hipGraphExecDestroy(g), g = nullptr;
}

static int upload_tiles(rrmhd_batch *b) {
  // rebuild the flat tile list from the per-domain shapes
  b->tile_dom.clear();
  int first = 0;
  for (int d = 0; d < b->n; ++d) {
    rr::BatchDom &D = b->doms[d];
    D.tiles_x = (D.nx + D.bx - 1) / D.bx;
    const int tiles_y = (D.ny + D.by - 1) / D.by;
    D.tile_first = first;
    for (int k = 0; k < D.tiles_x * tiles_y; ++k) b->tile_dom.push_back(d);
    first += D.tiles_x * tiles_y;
  }
  b->ntiles = first;
  if (b->d_tile_dom) (void)hipFree(b->d_tile_dom), b->d_tile_dom = nullptr;
  BHIP(hipMalloc((void **)&b->d_tile_dom, sizeof(int) * b->tile_dom.size()));
  BHIP(hipMemcpy(b->d_tile_dom, b->tile_dom.data(), sizeof(int) * b->tile_dom.size(),
                 hipMemcpyHostToDevice));
  BHIP(hipMemcpy(b->d_doms, b->doms.data(), sizeof(rr::BatchDom) * b->n,
                 hipMemcpyHostToDevice));
  free_graphs(b);
  return RRMHD_OK;
}

template <class C, bool NT>
static void launch_sched(const rrmhd_batch *b, dim3 grid, hipStream_t st, const void *src,
                         void *dst) {
  using T = typename C::T;
  const dim3 block(256);
  if (b->per_fetch > 0)
    hipLaunchKernelGGL((rr::k_batch_step<C, NT, true>), grid, block, 0, st, b->d_doms,
                       b->d_tile_dom, b->ntiles, b->per_fetch, b->s, b->inv_s,
                       (const T *)src, (T *)dst, b->d_ctr);
  else
    hipLaunchKernelGGL((rr::k_batch_step<C, NT, false>), grid, block, 0, st, b->d_doms,
                       b->d_tile_dom, b->ntiles, 0, b->s, b->inv_s, (const T *)src, (T *)dst,
                       b->d_ctr);
}

static int launch_grid(const rrmhd_batch *b) {
  if (b->per_fetch > 0) {
    // at least one workgroup per segment; never more than the chunks need
    const int chunks = (b->ntiles + b->per_fetch - 1) / b->per_fetch + rr::kSeg;
    int g = (b->grid < 0 || b->grid > chunks) ? chunks : b->grid;
    return g < rr::kSeg ? rr::kSeg : g;
  }
  return b->grid < 0 ? b->ntiles : b->grid;
}

static hipError_t launch_one(rrmhd_batch *b, hipStream_t st) {
  const void *src = b->buf[b->cur];
  void *dst = b->buf[b->cur ^ 1];
  const dim3 grid(launch_grid(b));
  if (b->storage == RRMHD_STORE_F16) {
    if (b->nt)
      launch_sched<rr::CodecF16U, true>(b, grid, st, src, dst);  // ensemble storage scale is 1
    else
      launch_sched<rr::CodecF16U, false>(b, grid, st, src, dst);
  } else {
    if (b->nt)
      launch_sched<rr::CodecF32, true>(b, grid, st, src, dst);
    else
      launch_sched<rr::CodecF32, false>(b, grid, st, src, dst);
  }
  return hipGetLastError();
}

static rr::Domain domain_of(const rrmhd_batch *b, int d) {
  const rr::BatchDom &B = b->doms[d];
  rr::Domain D{};
  D.nx = B.nx;
  D.ny = B.ny;
  D.plane = B.plane;
  D.row = B.nx;  // planes of [ny][nx]
  D.walls = 0;
  D.om_c = B.om_c;
  D.omm_c = B.omm_c;
  D.s = b->s;
  D.inv_s = b->inv_s;
  D.elem = (int)b->elem;
  return D;
}

extern "C" {

int rrmhd_batch_destroy(rrmhd_batch *b) {
  if (!b) return RRMHD_OK;
  if (b->user || b->buf[0]) (void)hipStreamSynchronize(b->user);
  if (b->own) (void)hipStreamSynchronize(b->own);
  free_graphs(b);
  for (void *&p : b->buf)
    if (p) (void)hipFree(p), p = nullptr;
  if (b->d_doms) (void)hipFree(b->d_doms);
  if (b->d_tile_dom) (void)hipFree(b->d_tile_dom);
  if (b->d_ctr) (void)hipFree(b->d_ctr);
  if (b->diag_work) (void)hipFree(b->diag_work);
  if (b->diag_out) (void)hipFree(b->diag_out);
  if (b->diag_host) (void)hipHostFree(b->diag_host);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->own) (void)hipStreamDestroy(b->own);
  delete b;
  return RRMHD_OK;
}

int rrmhd_batch_create(int n, const rrmhd_grid *grids, const double *tau_f,
                       const double *tau_m, int storage, void *hip_stream,
                       rrmhd_batch **out) {
  if (!out) return RRMHD_EINVAL;
  *out = nullptr;
  if (n < 1 || !grids || !tau_f || !tau_m) return RRMHD_EINVAL;
  if (storage != RRMHD_STORE_F32 && storage != RRMHD_STORE_F16) return RRMHD_EINVAL;
  for (int d = 0; d < n; ++d) {
    if (grids[d].nx < 1 || grids[d].ny < 1) return RRMHD_EINVAL;
    if ((int64_t)grids[d].nx * grids[d].ny * 4 >= ((int64_t)1 << 32)) return RRMHD_EINVAL;
    if (!(std::isfinite(tau_f[d]) && std::isfinite(tau_m[d])) || tau_f[d] <= 0.5 ||
        tau_m[d] <= 0.5)
      return RRMHD_EINVAL;
  }
  rrmhd_batch *b = new (std::nothrow) rrmhd_batch();
  if (!b) return RRMHD_ENOMEM;
  b->n = n;
  b->storage = storage;
  b->elem = storage == RRMHD_STORE_F16 ? 2 : 4;
  b->user = (hipStream_t)hip_stream;
  b->doms.resize(n);
  b->tau_f.assign(tau_f, tau_f + n);
  b->tau_m.assign(tau_m, tau_m + n);
  b->init_step.assign(n, -1);
  const int64_t align = 256 / b->elem;
  int64_t off = 0;
  size_t diag = 0;
  for (int d = 0; d < n; ++d) {
    rr::BatchDom &D = b->doms[d];
    D.nx = grids[d].nx;
    D.ny = grids[d].ny;
    const int64_t N = (int64_t)D.nx * D.ny;
    D.plane = (N + align - 1) / align * align + align;  // 256 B gap as single domains
    D.base = off;
    off += D.plane * rr::kStatePlanes;
    D.om_c = (float)(1.0 - 1.0 / tau_f[d]);
    D.omm_c = (float)(1.0 - 1.0 / tau_m[d]);
    // 32 x 8 tiles, one workgroup per tile: the fastest measured default on
    // the uneven 64..1024 mix (hardware dispatch keeps the tiles in flight a
    // contiguous window of the list)
    D.bx = 32;
    D.by = 256 / D.bx;
    rr::Domain dd = domain_of(b, d);
    diag = std::max(diag, rr::diag_work_bytes(dd));
  }
  b->diag_bytes = diag;
  int rc = RRMHD_OK;
  auto chk = [&](hipError_t e, const char *w) {
    if (rc == RRMHD_OK && e != hipSuccess) rc = bdev_err(e, w);
  };
  for (int k = 0; k < 2; ++k) chk(hipMalloc(&b->buf[k], (size_t)off * b->elem), "hipMalloc(batch)");
  chk(hipMalloc((void **)&b->d_doms, sizeof(rr::BatchDom) * n), "hipMalloc(doms)");
  chk(hipMalloc((void **)&b->diag_out, 8 * sizeof(double)), "hipMalloc(diag)");
  chk(hipHostMalloc((void **)&b->diag_host, 8 * sizeof(double), hipHostMallocDefault),
      "hipHostMalloc(diag)");
  const size_t ctr_bytes = sizeof(int) * rr::kSeg * rr::kCtrStride;
  chk(hipMalloc((void **)&b->d_ctr, ctr_bytes), "hipMalloc(counters)");
  if (rc == RRMHD_OK) chk(hipMemset(b->d_ctr, 0, ctr_bytes), "hipMemset(counters)");
  chk(hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking), "hipStreamCreate");
  chk(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming), "hipEventCreate");
  chk(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming), "hipEventCreate");
  b->grid = -1;  // one workgroup per tile
  if (rc == RRMHD_OK) rc = upload_tiles(b);
  if (rc != RRMHD_OK) {
    rrmhd_batch_destroy(b);
    return rc;
  }
  *out = b;
  return RRMHD_OK;
}

int rrmhd_batch_init(rrmhd_batch *b, int d, const double *u, const double *bf) {
  if (!b || d < 0 || d >= b->n || !u || !bf) return RRMHD_EINVAL;
  rr::Domain D = domain_of(b, d);
  char *dst = (char *)b->buf[b->cur] + b->doms[d].base * b->elem;
  BHIP(rr::launch_init(b->storage, D, u, bf, 0.0, 0.0, dst, b->user));
  b->init_step[d] = b->steps;
  return RRMHD_OK;
}

int rrmhd_batch_set_shape(rrmhd_batch *b, int d, int bx, int grid, int nt) {
  if (!b || d < -1 || d >= b->n) return RRMHD_EINVAL;
  if (bx != 0 && (bx < 1 || bx > 256 || 256 % bx != 0)) return RRMHD_EINVAL;
  if (grid < -1) return RRMHD_EINVAL;
  if (bx) {
    for (int k = (d < 0 ? 0 : d); k < (d < 0 ? b->n : d + 1); ++k) {
      b->doms[k].bx = bx;
      b->doms[k].by = 256 / bx;
    }
  }
  if (grid) b->grid = grid;
  if (nt >= 0) b->nt = nt ? 1 : 0;
  return upload_tiles(b);
}

int rrmhd_batch_set_fetch(rrmhd_batch *b, int tiles_per_fetch) {
  if (!b || tiles_per_fetch < 0 || tiles_per_fetch > 64) return RRMHD_EINVAL;
  b->per_fetch = tiles_per_fetch;
  free_graphs(b);
  return RRMHD_OK;
}

static int plain_steps(rrmhd_batch *b, int64_t n, hipStream_t st) {
  for (int64_t k = 0; k < n; ++k) {
    BHIP(launch_one(b, st));
    b->cur ^= 1;
    b->steps++;
  }
  return RRMHD_OK;
}

int rrmhd_batch_step(rrmhd_batch *b, int64_t n) {
  if (!b || n < 0) return RRMHD_EINVAL;
  for (int d = 0; d < b->n; ++d)
    if (b->init_step[d] < 0) return RRMHD_ESTATE;
  const int64_t chunk = b->graph_chunk;
  if (chunk <= 0 || n < chunk) return plain_steps(b, n, b->user);
  // graph path: order the internal stream after the caller's work
  BHIP(hipEventRecord(b->ev_in, b->user));
  BHIP(hipStreamWaitEvent(b->own, b->ev_in, 0));
  int64_t left = n;
  while (left >= chunk) {
    hipGraphExec_t &g = b->graph[b->cur];
    if (!g) {
      hipGraph_t graph = nullptr;
      const int c0 = b->cur;
      const int64_t s0 = b->steps;
      BHIP(hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal));
      int rc = plain_steps(b, chunk, b->own);
      hipError_t ee = hipStreamEndCapture(b->own, &graph);
      b->cur = c0;  // capture recorded the launches; nothing ran yet
      b->steps = s0;
      if (rc != RRMHD_OK) return rc;
      if (ee != hipSuccess) return bdev_err(ee, "hipStreamEndCapture");
      hipError_t ei = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return bdev_err(ei, "hipGraphInstantiate");
    }
    BHIP(hipGraphLaunch(g, b->own));
    if (chunk & 1) b->cur ^= 1;
    b->steps += chunk;
    left -= chunk;
  }
  int rc = plain_steps(b, left, b->own);
  if (rc != RRMHD_OK) return rc;
  BHIP(hipEventRecord(b->ev_out, b->own));
  BHIP(hipStreamWaitEvent(b->user, b->ev_out, 0));
  return RRMHD_OK;
}

int rrmhd_batch_set_graph_chunk(rrmhd_batch *b, int chunk) {
  if (!b || chunk < 0) return RRMHD_EINVAL;
  free_graphs(b);
  b->graph_chunk = chunk;
  return RRMHD_OK;
}

int rrmhd_batch_moments(rrmhd_batch *b, int d, double *rho, double *u, double *bf) {
  if (!b || d < 0 || d >= b->n) return RRMHD_EINVAL;
  if (b->init_step[d] < 0) return RRMHD_ESTATE;
  rr::Domain D = domain_of(b, d);
  const char *src = (const char *)b->buf[b->cur] + b->doms[d].base * b->elem;
  BHIP(rr::launch_moments(b->storage, D, src, rho, u, bf, b->user));
  return RRMHD_OK;
}

int rrmhd_batch_diagnostics(rrmhd_batch *b, int d, double *E_kin, double *E_mag,
                            double *max_div_b) {
  if (!b || d < 0 || d >= b->n) return RRMHD_EINVAL;
  if (b->init_step[d] < 0) return RRMHD_ESTATE;
  if (!b->diag_work) BHIP(hipMalloc(&b->diag_work, b->diag_bytes));
  rr::Domain D = domain_of(b, d);
  const char *src = (const char *)b->buf[b->cur] + b->doms[d].base * b->elem;
  BHIP(rr::launch_diagnostics(b->storage, D, src, b->diag_work, b->diag_out, b->user));
  BHIP(hipMemcpyAsync(b->diag_host, b->diag_out, 8 * sizeof(double), hipMemcpyDeviceToHost,
                      b->user));
  BHIP(hipStreamSynchronize(b->user));
  const double *r = b->diag_host;
  const bool bad = !(std::isfinite(r[0]) && std::isfinite(r[1]) && std::isfinite(r[2]));
  const double nan = std::nan("");
  if (E_kin) *E_kin = bad ? nan : r[0];
  if (E_mag) *E_mag = bad ? nan : r[1];
  if (max_div_b) *max_div_b = bad ? nan : r[2];
  return bad ? RRMHD_ENONFINITE : RRMHD_OK;
}

int rrmhd_batch_info(const rrmhd_batch *b, int64_t *nodes, int64_t *steps, int *ntiles,
                     int *grid) {
  if (!b) return RRMHD_EINVAL;
  int64_t s = 0;
  for (const auto &D : b->doms) s += (int64_t)D.nx * D.ny;
  if (nodes) *nodes = s;
  if (steps) *steps = b->steps;
  if (ntiles) *ntiles = b->ntiles;
  if (grid) *grid = launch_grid(b);
  return RRMHD_OK;
}

const char *rrmhd_batch_last_error_detail(void) { return g_bdetail; }

int rr_batch_domains(const rrmhd_batch *b, int *n, int *storage, int *nx, int *ny) {
  if (!b) return RRMHD_EINVAL;
  if (n) *n = b->n;
  if (storage) *storage = b->storage;
  for (int d = 0; d < b->n; ++d) {
    if (nx) nx[d] = b->doms[d].nx;
    if (ny) ny[d] = b->doms[d].ny;
  }
  return RRMHD_OK;
}

static size_t batch_bytes(const rrmhd_batch *b) {
  const rr::BatchDom &L = b->doms.back();
  return (size_t)(L.base + L.plane * rr::kStatePlanes) * b->elem;
}

int rr_batch_save(rrmhd_batch *b, void **copy) {
  if (!b || !copy) return RRMHD_EINVAL;
  *copy = nullptr;
  const size_t nb = batch_bytes(b);
  BHIP(hipMalloc(copy, nb));
  BHIP(hipMemcpyAsync(*copy, b->buf[b->cur], nb, hipMemcpyDeviceToDevice, b->user));
  BHIP(hipStreamSynchronize(b->user));
  return RRMHD_OK;
}

int rr_batch_restore(rrmhd_batch *b, void *copy, int64_t steps) {
  if (!b || !copy) return RRMHD_EINVAL;
  BHIP(hipStreamSynchronize(b->own));
  BHIP(hipMemcpyAsync(b->buf[0], copy, batch_bytes(b), hipMemcpyDeviceToDevice, b->user));
  BHIP(hipStreamSynchronize(b->user));
  (void)hipFree(copy);
  b->cur = 0;
  b->steps = steps;
  return RRMHD_OK;
}

hipStream_t rr_batch_stream(const rrmhd_batch *b) { return b ? b->user : nullptr; }

}  // extern "C"
