// lbm_api.hip -- host side of the C ABI declared in include/lbm.h:
// parameter validation, context state (ping-pong index, time), kernel
// arguments, error reporting.  Kernels live in lbm_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "lbm.h"
#include "lbm_launch.h"

struct lbm_ctx {
  lbm_params p;
  lbm::KArgsAny args;
  void* lat[2];
  int cur;            // index of the lattice holding the current state
  int64_t t;          // steps since the state was set
  bool has_state;
  bool has_force_field;
  hipStream_t stream;
  double* diag_scratch;  // device: partial sums (diag_blocks * 4) + result (4); first diagnostics call
  int diag_blocks;
  int64_t pitch, lattice_bytes;
  char err[512];
};

namespace {

thread_local char g_create_err[512] = "";

int storage_size(int32_t s) {
  switch (s) {
    case LBM_FP64: return 8;
    case LBM_FP32: return 4;
    case LBM_FP16_DEV: return 2;
    case LBM_BF16_DEV: return 2;
    default: return 0;
  }
}

int real_size(int32_t s) { return s == LBM_FP64 ? 8 : 4; }

void set_err(char* buf, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, 512, fmt, ap);
  va_end(ap);
}

// Validate a parameter set; message into buf.
bool validate(const lbm_params* p, char* buf) {
  if (!p) { set_err(buf, "params is NULL"); return false; }
  if (p->nx < 2 || p->ny < 2) { set_err(buf, "grid %d x %d: need nx, ny >= 2", p->nx, p->ny); return false; }
  if (storage_size(p->storage) == 0) { set_err(buf, "unknown storage mode %d", p->storage); return false; }
  const double om[5] = {p->omega_nu, p->omega3, p->omega6, p->omega7, p->omega8};
  const char* nm[5] = {"omega_nu", "omega3", "omega6", "omega7", "omega8"};
  for (int i = 0; i < 5; ++i)
    if (!(om[i] > 0.0 && om[i] < 2.0)) { set_err(buf, "%s = %g outside (0, 2)", nm[i], om[i]); return false; }
  if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) { set_err(buf, "rho0 = %g must be > 0", p->rho0); return false; }
  if (!std::isfinite(p->fx) || !std::isfinite(p->fy)) { set_err(buf, "body force is not finite"); return false; }
  for (int s = 0; s < 4; ++s) {
    if (p->bc[s] != LBM_PERIODIC && p->bc[s] != LBM_WALL) { set_err(buf, "bc[%d] = %d unknown", s, p->bc[s]); return false; }
    if (!std::isfinite(p->wall_u[s])) { set_err(buf, "wall_u[%d] not finite", s); return false; }
    if (p->bc[s] == LBM_PERIODIC && p->wall_u[s] != 0.0) {
      set_err(buf, "wall_u[%d] = %g on a periodic side", s, p->wall_u[s]);
      return false;
    }
  }
  if (p->rounding != LBM_ROUND_NEAREST && p->rounding != LBM_ROUND_STOCHASTIC) {
    set_err(buf, "rounding = %d unknown", p->rounding);
    return false;
  }
  if (p->rounding == LBM_ROUND_STOCHASTIC && p->storage != LBM_FP16_DEV && p->storage != LBM_BF16_DEV) {
    set_err(buf, "stochastic rounding needs FP16 or BF16 storage");
    return false;
  }
  if ((p->bc[0] == LBM_PERIODIC) != (p->bc[1] == LBM_PERIODIC)) { set_err(buf, "x sides: periodic on one side only"); return false; }
  if ((p->bc[2] == LBM_PERIODIC) != (p->bc[3] == LBM_PERIODIC)) { set_err(buf, "y sides: periodic on one side only"); return false; }
  const int64_t pitch = ((int64_t)p->nx + 63) / 64 * 64;
  // Kernels address a plane with 32-bit byte offsets.
  if ((int64_t)p->ny * pitch * storage_size(p->storage) >= ((int64_t)1 << 32)) {
    set_err(buf, "lattice plane of %lld elements x %d B exceeds 4 GiB", (long long)(p->ny * pitch),
            storage_size(p->storage));
    return false;
  }
  return true;
}

template <typename R>
void fill_args(const lbm_params* p, int64_t pitch, const void* force, lbm::KArgs<R>& a) {
  lbm::Geom& g = a.g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.pitch = (int32_t)pitch;
  g.plane = (int64_t)p->ny * pitch;
  // Tile width: the widest power of two in {64, 128, 256} not beyond the
  // padded row, so narrow lattices still fill whole wavefronts.
  g.tx_shift = pitch >= 256 ? 8 : (pitch >= 128 ? 7 : 6);
  const int tx = 1 << g.tx_shift, ty = 256 / tx;
  g.tiles_x = (int32_t)((p->nx + tx - 1) / tx);
  g.tiles_y = (int32_t)((p->ny + ty - 1) / ty);
  for (int s = 0; s < 4; ++s) g.wall[s] = p->bc[s] == LBM_WALL;
  static const int GX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static const int GY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const int64_t esz = storage_size(p->storage);
  const int64_t total = 9 * g.plane * esz;
  // 32-bit byte offsets, and rows short enough (in bytes) for 24-bit multiplies
  g.fast = total < ((int64_t)1 << 32) && g.pitch * esz < (1 << 24);
  g.wb_stores = 2 * total <= lbm::kWriteBackMaxBytes;
  g.lattice_bytes = g.fast ? (uint32_t)total : 0u;
  for (int k = 0; k < 9; ++k) {
    // plane k read at (x - e_x, y - e_y): offset k*plane - e_y*pitch - e_x, >= 0
    // for k >= 1 because plane >= 2*pitch; k = 0 has no shift.
    const int64_t ld = (k * g.plane - (int64_t)GY[k] * pitch - GX[k]) * esz;
    const int64_t st = k * g.plane * esz;
    g.ld_soff[k] = g.fast ? (uint32_t)ld : 0u;
    g.st_soff[k] = g.fast ? (uint32_t)st : 0u;
  }
  // 64 x 16 tiles, or 64 x 8 where 64 x 16 would leave the chip short of
  // workgroups (measured: 16-bit 512^2 49 -> 64 GLUPS, 1024^2 120 -> 135)
  g.t2_ty = storage_size(p->storage) == 8 || (int64_t)p->nx * p->ny <= lbm::kStep2SmallMaxNodes ? 8 : 16;
  g.t2_tiles_x = (int32_t)((p->nx + 63) / 64);
  g.t2_tiles_y = (int32_t)((p->ny + g.t2_ty - 1) / g.t2_ty);
  const int64_t nodes = (int64_t)p->nx * p->ny;
  g.t4_ty = storage_size(p->storage) == 8 ? lbm::kStep4TyF64
            : nodes <= lbm::kStep4SmallMaxNodes ? lbm::kStep4TyF32Small
            : nodes <= lbm::kStep4MidMaxNodes ? lbm::kStep4TyF32Mid
                                              : lbm::kStep4TyF32;
  if (storage_size(p->storage) != 8) {
    g.t3_ty = lbm::kStep3TyF32;
    g.t3_threads = lbm::kStep3ThreadsF32;
  } else if ((int64_t)p->nx * p->ny >= lbm::kStep3LargeMinNodes) {
    g.t3_ty = lbm::kStep3TyF64Large;
    g.t3_threads = lbm::kStep3ThreadsF64Large;
  } else {
    g.t3_ty = lbm::kStep3TyF64;
    g.t3_threads = lbm::kStep3ThreadsF64;
  }
  g.t3_tiles_x = g.t2_tiles_x;
  g.t3_tiles_y = (int32_t)((p->ny + g.t3_ty - 1) / g.t3_ty);
  a.w[0] = (R)p->omega3;
  a.w[1] = (R)p->omega_nu;
  a.w[2] = (R)p->omega_nu;
  a.w[3] = (R)p->omega6;
  a.w[4] = (R)p->omega7;
  a.w[5] = (R)p->omega8;
  a.rho0 = (R)p->rho0;
  a.fx = (R)p->fx;
  a.fy = (R)p->fy;
  a.force = (const R*)force;
  // Moving-wall term 6 rho0 w_a (e_a . U_wall) per side: x walls move in y,
  // y walls move in x.
  static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  for (int s = 0; s < 4; ++s)
    for (int k = 0; k < 9; ++k) {
      const double tang = s < 2 ? EY[k] : EX[k];
      a.wadd[s * 9 + k] = (R)(6.0 * p->rho0 * W[k] * tang * p->wall_u[s]);
    }
}

// Steps fused per launch: four on the 64 x TY tiles in FP64 and FP32, two in
// 16-bit storage.
int steps_per_launch(int32_t storage) { return (storage == LBM_FP32 || storage == LBM_FP64) ? 4 : 2; }

bool aligned(const void* ptr) { return ((uintptr_t)ptr & 255u) == 0; }

// Key of the stochastic-rounding hash for the step from time t: mixes the
// seed and t so every step draws fresh bits (same key scheme for every node;
// the node index is mixed in on the device).
uint32_t step_key(const lbm_params& p, int64_t t) {
  if (p.rounding != LBM_ROUND_STOCHASTIC) return 0u;
  const uint32_t a = lbm::pcg_hash((uint32_t)p.seed ^ lbm::pcg_hash((uint32_t)(p.seed >> 32)));
  return lbm::pcg_hash(a ^ lbm::pcg_hash((uint32_t)t ^ lbm::pcg_hash((uint32_t)((uint64_t)t >> 32))));
}

lbm_status dev_err(lbm_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return LBM_OK;
  set_err(c->err, "%s: %s", what, hipGetErrorString(e));
  return LBM_EDEVICE;
}

lbm_status inval(lbm_ctx* c, const char* msg) {
  set_err(c->err, "%s", msg);
  return LBM_EINVAL;
}

}  // namespace

// Reduction scratch of lbm_diagnostics_noalloc: the per-block partial sums
// (four doubles per block) of the fixed diagnostics grid.  A file-scope
// device array, so the call never allocates; each GPU holds its own copy, at
// its own address, until the process ends.
constexpr int kDiagScratchBlocks = 1024;
static __device__ __align__(256) double scratch[kDiagScratchBlocks * 4];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the device of the context's stream.  The
// host-side name is only a stand-in for the symbol; its device address comes
// from hipGetSymbolAddress, taken once per device with that device current.
lbm_status scratch_of(lbm_ctx* c, double** out) {
  int dev = -1;
  hipError_t e = c->stream ? hipStreamGetDevice(c->stream, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return dev_err(c, e, "device of the context's stream");
  if (dev < 0 || dev >= kMaxDevices) {
    set_err(c->err, "device %d beyond the %d devices the static scratch tracks", dev, kMaxDevices);
    return LBM_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    e = hipGetDevice(&cur);
    if (e != hipSuccess) return dev_err(c, e, "current device");
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return dev_err(c, e, "select the stream's device");
    void* p = nullptr;
    const hipError_t es = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev && (e = hipSetDevice(cur)) != hipSuccess) return dev_err(c, e, "restore the current device");
    if (es != hipSuccess) return dev_err(c, es, "address of the diagnostics scratch");
    if (!p) {
      set_err(c->err, "address of the diagnostics scratch: null");
      return LBM_EDEVICE;
    }
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_lattice_layout(const lbm_params* p, int64_t* pitch, int64_t* bytes) {
  char buf[512];
  if (!validate(p, buf)) { set_err(g_create_err, "%s", buf); return LBM_EINVAL; }
  const int64_t pt = ((int64_t)p->nx + 63) / 64 * 64;
  if (pitch) *pitch = pt;
  if (bytes) *bytes = 9 * (int64_t)p->ny * pt * storage_size(p->storage);
  return LBM_OK;
}

lbm_status lbm_create(const lbm_params* p, void* lat0, void* lat1, const void* force_field,
                      void* stream, lbm_ctx** out) {
  if (!out) { set_err(g_create_err, "out is NULL"); return LBM_EINVAL; }
  *out = nullptr;
  if (!validate(p, g_create_err)) return LBM_EINVAL;
  if (!lat0 || !lat1 || lat0 == lat1) { set_err(g_create_err, "need two distinct lattice buffers"); return LBM_EINVAL; }
  if (!aligned(lat0) || !aligned(lat1) || (force_field && !aligned(force_field))) {
    set_err(g_create_err, "device buffers must be 256-byte aligned");
    return LBM_EINVAL;
  }
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) { set_err(g_create_err, "out of host memory"); return LBM_EDEVICE; }
  c->p = *p;
  c->pitch = ((int64_t)p->nx + 63) / 64 * 64;
  c->lattice_bytes = 9 * (int64_t)p->ny * c->pitch * storage_size(p->storage);
  c->lat[0] = lat0;
  c->lat[1] = lat1;
  c->cur = 0;
  c->t = 0;
  c->has_state = false;
  c->has_force_field = force_field != nullptr;
  c->stream = (hipStream_t)stream;
  c->args.storage = p->storage;
  c->args.stochastic = p->rounding == LBM_ROUND_STOCHASTIC;
  if (p->storage == LBM_FP64) fill_args<double>(p, c->pitch, force_field, c->args.d);
  else fill_args<float>(p, c->pitch, force_field, c->args.f);
  // Diagnostics: a fixed number of blocks (enough to fill 256 CUs), so the
  // reduction order does not depend on the grid size.
  c->diag_blocks = kDiagScratchBlocks;
  c->diag_scratch = nullptr;  // allocated by the first lbm_diagnostics call
  c->err[0] = 0;
  *out = c;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->diag_scratch) (void)hipFree(c->diag_scratch);
  delete c;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err : g_create_err; }

lbm_status lbm_set_stream(lbm_ctx* c, void* stream) {
  if (!c) return LBM_EINVAL;
  c->stream = (hipStream_t)stream;
  return LBM_OK;
}

int64_t lbm_time(const lbm_ctx* c) { return c ? c->t : -1; }

void* lbm_current_lattice(const lbm_ctx* c) { return c ? c->lat[c->cur] : nullptr; }

lbm_status lbm_init_equilibrium(lbm_ctx* c, const void* rho, const void* ux, const void* uy) {
  if (!c) return LBM_EINVAL;
  if (!rho || !ux || !uy) return inval(c, "init_equilibrium: rho, ux, uy must be non-NULL");
  lbm_status s = dev_err(c, lbm::launch_init(c->args, rho, ux, uy, c->lat[0], c->stream), "init kernel");
  if (s != LBM_OK) return s;
  c->cur = 0;
  c->t = 0;
  c->has_state = true;
  return LBM_OK;
}

lbm_status lbm_set_populations(lbm_ctx* c, const void* f) {
  if (!c) return LBM_EINVAL;
  if (!f) return inval(c, "set_populations: f is NULL");
  lbm_status s = dev_err(c, lbm::launch_set(c->args, f, c->lat[0], c->stream), "set kernel");
  if (s != LBM_OK) return s;
  c->cur = 0;
  c->t = 0;
  c->has_state = true;
  return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx* c, void* f) {
  if (!c) return LBM_EINVAL;
  if (!f) return inval(c, "get_populations: f is NULL");
  if (!c->has_state) { set_err(c->err, "get_populations before the state was set"); return LBM_ESTATE; }
  return dev_err(c, lbm::launch_get(c->args, c->lat[c->cur], f, c->stream), "get kernel");
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return LBM_EINVAL;
  if (n < 0) return inval(c, "step: n < 0");
  if (!c->has_state) { set_err(c->err, "step before the state was set"); return LBM_ESTATE; }
  // Steps run in groups of steps_per_launch fused in one launch
  // (intermediate states stay in LDS); the remainder runs as a three-step,
  // a two-step and/or a single-step launch.
  const int group = steps_per_launch(c->p.storage);
  int64_t left = n;
  for (; group == 4 && left >= 4; left -= 4) {
    lbm_status s = dev_err(c, lbm::launch_step4(c->args, c->lat[c->cur], c->lat[c->cur ^ 1], step_key(c->p, c->t),
                                                step_key(c->p, c->t + 1), step_key(c->p, c->t + 2),
                                                step_key(c->p, c->t + 3), c->stream),
                           "four-step kernel");
    if (s != LBM_OK) return s;
    c->cur ^= 1;
    c->t += 4;
  }
  for (; group >= 3 && left >= 3; left -= 3) {
    lbm_status s = dev_err(c, lbm::launch_step3(c->args, c->lat[c->cur], c->lat[c->cur ^ 1], step_key(c->p, c->t),
                                                step_key(c->p, c->t + 1), step_key(c->p, c->t + 2), c->stream),
                           "three-step kernel");
    if (s != LBM_OK) return s;
    c->cur ^= 1;
    c->t += 3;
  }
  for (; left >= 2; left -= 2) {
    lbm_status s = dev_err(c, lbm::launch_step2(c->args, c->lat[c->cur], c->lat[c->cur ^ 1],
                                                step_key(c->p, c->t), step_key(c->p, c->t + 1), c->stream),
                           "two-step kernel");
    if (s != LBM_OK) return s;
    c->cur ^= 1;
    c->t += 2;
  }
  if (left == 1) {
    lbm_status s = dev_err(c, lbm::launch_step(c->args, c->lat[c->cur], c->lat[c->cur ^ 1],
                                               step_key(c->p, c->t), c->stream),
                           "step kernel");
    if (s != LBM_OK) return s;
    c->cur ^= 1;
    c->t += 1;
  }
  return LBM_OK;
}

// The explicit-buffer calls carry no step index, so they cannot draw fresh
// stochastic-rounding bits per step: they refuse that rounding.
static lbm_status no_stochastic(lbm_ctx* c, const char* what) {
  set_err(c->err, "%s: stochastic rounding is supported by lbm_step only (no step index here)", what);
  return LBM_EUNSUPPORTED;
}

lbm_status lbm_step_between(lbm_ctx* c, const void* src, void* dst) {
  if (!c) return LBM_EINVAL;
  if (c->p.rounding == LBM_ROUND_STOCHASTIC) return no_stochastic(c, "step_between");
  if (!src || !dst || src == dst) return inval(c, "step_between: need distinct non-NULL src, dst");
  if (!aligned(src) || !aligned(dst)) return inval(c, "step_between: buffers must be 256-byte aligned");
  return dev_err(c, lbm::launch_step(c->args, src, dst, 0u, c->stream), "step kernel");
}

lbm_status lbm_step_sequence(lbm_ctx* c, const void* src, void* const* states, int64_t n) {
  if (!c) return LBM_EINVAL;
  if (c->p.rounding == LBM_ROUND_STOCHASTIC) return no_stochastic(c, "step_sequence");
  if (n < 0) return inval(c, "step_sequence: n < 0");
  if (n > 0 && (!src || !states)) return inval(c, "step_sequence: need src and states");
  if (n > 0 && !aligned(src)) return inval(c, "step_sequence: buffers must be 256-byte aligned");
  for (int64_t i = 0; i < n; ++i) {
    const void* prev = i == 0 ? src : states[i - 1];
    if (!states[i] || states[i] == prev) return inval(c, "step_sequence: states[i] NULL or equal to its input");
    if (!aligned(states[i])) return inval(c, "step_sequence: buffers must be 256-byte aligned");
  }
  // FP32 lattices run groups of four steps as one four-step launch that also
  // stores the three intermediate states, as long as the group's five
  // buffers are distinct, and a remainder of three or two steps as one launch
  // of that form cut short; the rest runs as single steps.
  const uint32_t key = 0u;  // nearest rounding: the key is not used
  int64_t i = 0;
  const bool tiles4 = c->p.storage == LBM_FP32;
  for (; tiles4 && i + 4 <= n; i += 4) {
    const void* in = i == 0 ? src : states[i - 1];
    void *k0 = states[i], *k1 = states[i + 1], *k2 = states[i + 2], *out = states[i + 3];
    const void* b[5] = {in, k0, k1, k2, out};
    bool distinct = true;
    for (int p = 0; p < 5; ++p)
      for (int q = p + 1; q < 5; ++q) distinct = distinct && b[p] != b[q];
    if (!distinct) break;
    lbm_status s = dev_err(c, lbm::launch_step4_keep(c->args, in, k0, k1, k2, out, key, key, key, key, c->stream),
                           "four-step kernel");
    if (s != LBM_OK) return s;
  }
  if (tiles4 && (n - i == 3 || n - i == 2)) {
    const int r = (int)(n - i);
    const void* in = i == 0 ? src : states[i - 1];
    void* k0 = states[i];
    void* k1 = states[i + 1];
    void* k2 = r == 3 ? states[i + 2] : nullptr;
    const bool distinct = in != k1 && k0 != k1 && (!k2 || (in != k2 && k0 != k2 && k1 != k2));  // in != k0 checked
    if (distinct) {
      lbm_status s = dev_err(c, lbm::launch_step4_keep(c->args, in, k0, k1, k2, nullptr, key, key, key, key,
                                                       c->stream),
                             "four-step kernel");
      if (s != LBM_OK) return s;
      i = n;
    }
  }
  for (; i < n; ++i) {
    lbm_status s = dev_err(c, lbm::launch_step(c->args, i == 0 ? src : states[i - 1], states[i], key, c->stream),
                           "step kernel");
    if (s != LBM_OK) return s;
  }
  return LBM_OK;
}

lbm_status lbm_snapshot(lbm_ctx* c, void* dst) {
  if (!c) return LBM_EINVAL;
  if (!dst) return inval(c, "snapshot: dst is NULL");
  if (!c->has_state) { set_err(c->err, "snapshot before the state was set"); return LBM_ESTATE; }
  return dev_err(c, hipMemcpyAsync(dst, c->lat[c->cur], (size_t)c->lattice_bytes, hipMemcpyDeviceToDevice, c->stream),
                 "snapshot copy");
}

lbm_status lbm_restore(lbm_ctx* c, const void* src, int64_t t) {
  if (!c) return LBM_EINVAL;
  if (!src) return inval(c, "restore: src is NULL");
  if (t < 0) return inval(c, "restore: t < 0");
  lbm_status s = dev_err(c, hipMemcpyAsync(c->lat[c->cur], src, (size_t)c->lattice_bytes, hipMemcpyDeviceToDevice,
                                           c->stream), "restore copy");
  if (s != LBM_OK) return s;
  c->t = t;
  c->has_state = true;
  return LBM_OK;
}

lbm_status lbm_macroscopic(lbm_ctx* c, void* rho, void* ux, void* uy, void* sxx, void* syy, void* sxy) {
  if (!c) return LBM_EINVAL;
  if (!c->has_state) { set_err(c->err, "macroscopic before the state was set"); return LBM_ESTATE; }
  if (!rho && !ux && !uy && !sxx && !syy && !sxy) return LBM_OK;
  return dev_err(c, lbm::launch_macro(c->args, c->lat[c->cur], rho, ux, uy, sxx, syy, sxy, c->stream),
                 "macroscopic kernel");
}

lbm_status lbm_diagnostics(lbm_ctx* c, double out[4]) {
  if (!c) return LBM_EINVAL;
  if (!out) return inval(c, "diagnostics: out is NULL");
  if (!c->has_state) { set_err(c->err, "diagnostics before the state was set"); return LBM_ESTATE; }
  if (!c->diag_scratch) {
    const hipError_t e = hipMalloc((void**)&c->diag_scratch, sizeof(double) * (c->diag_blocks * 4 + 4));
    if (e != hipSuccess) {
      c->diag_scratch = nullptr;
      set_err(c->err, "hipMalloc(diagnostics scratch): %s", hipGetErrorString(e));
      return LBM_EDEVICE;
    }
  }
  double* res = c->diag_scratch + 4 * c->diag_blocks;
  const double base = (double)c->p.nx * (double)c->p.ny * c->p.rho0;
  lbm_status s = dev_err(c, lbm::launch_diag(c->args, c->lat[c->cur], c->diag_scratch, c->diag_blocks, base, res,
                                             c->stream), "diagnostics kernel");
  if (s != LBM_OK) return s;
  s = dev_err(c, hipMemcpyAsync(out, res, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "diagnostics copy");
  if (s != LBM_OK) return s;
  s = dev_err(c, hipStreamSynchronize(c->stream), "diagnostics sync");
  if (s != LBM_OK) return s;
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(out[k])) {
      set_err(c->err, "diagnostics: sum %d is not finite (unstable run)", k);
      return LBM_EUNSTABLE;
    }
  return LBM_OK;
}

lbm_status lbm_diagnostics_noalloc(lbm_ctx* c, void* out) {
  if (!c) return LBM_EINVAL;
  if (!out) return inval(c, "diagnostics_noalloc: out is NULL");
  if (((uintptr_t)out & 7u) != 0) return inval(c, "diagnostics_noalloc: out must be 8-byte aligned");
  if (!c->has_state) { set_err(c->err, "diagnostics before the state was set"); return LBM_ESTATE; }
  if (c->diag_blocks > kDiagScratchBlocks) {
    set_err(c->err, "diagnostics_noalloc: %d partial sums exceed the static scratch (%d)", c->diag_blocks,
            kDiagScratchBlocks);
    return LBM_EINVAL;
  }
  double* scr = nullptr;
  lbm_status s = scratch_of(c, &scr);
  if (s != LBM_OK) return s;
  // Every partial sum is written before the final kernel reads it (same
  // stream), so nothing in the scratch needs clearing.
  const double base = (double)c->p.nx * (double)c->p.ny * c->p.rho0;
  return dev_err(c, lbm::launch_diag(c->args, c->lat[c->cur], scr, c->diag_blocks, base, (double*)out, c->stream),
                 "diagnostics kernel");
}

lbm_status lbm_adjoint_step(lbm_ctx* c, const void* lat_prev, const void* mu_in, void* mu_out, void* grad_force) {
  if (!c) return LBM_EINVAL;
  if (c->p.storage != LBM_FP64 && c->p.storage != LBM_FP32) {
    set_err(c->err, "adjoint needs FP64 or FP32 storage");
    return LBM_EUNSUPPORTED;
  }
  if (!lat_prev || !mu_in || !mu_out || mu_in == mu_out) return inval(c, "adjoint_step: need lat_prev and distinct mu_in, mu_out");
  if (grad_force && !c->has_force_field) return inval(c, "adjoint_step: grad_force needs a bound force field");
  return dev_err(c, lbm::launch_adjoint_step(c->args, lat_prev, mu_in, mu_out, grad_force, c->stream),
                 "adjoint step kernel");
}

lbm_status lbm_adjoint_sequence(lbm_ctx* c, const void* const* states, int64_t n, void* mu_a, void* mu_b,
                                void* grad_force, int* result_in_b) {
  if (!c) return LBM_EINVAL;
  if (c->p.storage != LBM_FP64 && c->p.storage != LBM_FP32) {
    set_err(c->err, "adjoint needs FP64 or FP32 storage");
    return LBM_EUNSUPPORTED;
  }
  if (n < 0) return inval(c, "adjoint_sequence: n < 0");
  if (!mu_a || !mu_b || mu_a == mu_b) return inval(c, "adjoint_sequence: need distinct mu_a, mu_b");
  if (!result_in_b) return inval(c, "adjoint_sequence: result_in_b is NULL");
  if (n > 0 && !states) return inval(c, "adjoint_sequence: need states");
  for (int64_t i = 0; i < n; ++i)
    if (!states[i]) return inval(c, "adjoint_sequence: states[i] is NULL");
  if (grad_force && !c->has_force_field) return inval(c, "adjoint_sequence: grad_force needs a bound force field");
  // On large FP32 lattices groups of four steps run as one four-step adjoint
  // launch; then pairs of steps as one two-step launch; an odd one alone.
  void* mu[2] = {mu_a, mu_b};
  int k = 0;
  int64_t i = n - 1;
  const bool quads = c->p.storage == LBM_FP32 && c->p.nx >= 128 && c->p.ny >= 64 &&
                     (int64_t)c->p.nx * c->p.ny >= lbm::kAdjoint4MinNodes;
  for (; quads && i >= 3; i -= 4, k ^= 1) {
    lbm_status s = dev_err(c, lbm::launch_adjoint_step4(c->args, states[i], states[i - 1], states[i - 2],
                                                        states[i - 3], mu[k], mu[k ^ 1], grad_force, c->stream),
                           "four-step adjoint kernel");
    if (s != LBM_OK) return s;
  }
  for (; i >= 1; i -= 2, k ^= 1) {
    lbm_status s = dev_err(c, lbm::launch_adjoint_step2(c->args, states[i], states[i - 1], mu[k], mu[k ^ 1],
                                                        grad_force, c->stream),
                           "two-step adjoint kernel");
    if (s != LBM_OK) return s;
  }
  if (i == 0) {
    lbm_status s = dev_err(c, lbm::launch_adjoint_step(c->args, states[0], mu[k], mu[k ^ 1], grad_force, c->stream),
                           "adjoint step kernel");
    if (s != LBM_OK) return s;
    k ^= 1;
  }
  *result_in_b = k;
  return LBM_OK;
}

lbm_status lbm_adjoint_macroscopic(lbm_ctx* c, const void* lat, const void* g_rho, const void* g_ux,
                                   const void* g_uy, void* mu_out, void* grad_force) {
  if (!c) return LBM_EINVAL;
  if (c->p.storage != LBM_FP64 && c->p.storage != LBM_FP32) {
    set_err(c->err, "adjoint needs FP64 or FP32 storage");
    return LBM_EUNSUPPORTED;
  }
  if (!lat || !mu_out) return inval(c, "adjoint_macroscopic: need lat and mu_out");
  if (grad_force && !c->has_force_field) return inval(c, "adjoint_macroscopic: grad_force needs a bound force field");
  return dev_err(c, lbm::launch_adjoint_macro(c->args, lat, g_rho, g_ux, g_uy, mu_out, grad_force, c->stream),
                 "adjoint macroscopic kernel");
}

lbm_status lbm_adjoint_init(lbm_ctx* c, const void* rho, const void* ux, const void* uy, const void* mu0,
                            void* g_rho, void* g_ux, void* g_uy, void* grad_force) {
  if (!c) return LBM_EINVAL;
  if (c->p.storage != LBM_FP64 && c->p.storage != LBM_FP32) {
    set_err(c->err, "adjoint needs FP64 or FP32 storage");
    return LBM_EUNSUPPORTED;
  }
  if (!rho || !ux || !uy || !mu0) return inval(c, "adjoint_init: need rho, ux, uy, mu0");
  if (grad_force && !c->has_force_field) return inval(c, "adjoint_init: grad_force needs a bound force field");
  return dev_err(c, lbm::launch_adjoint_init(c->args, rho, ux, uy, mu0, g_rho, g_ux, g_uy, grad_force, c->stream),
                 "adjoint init kernel");
}

}  // extern "C"
