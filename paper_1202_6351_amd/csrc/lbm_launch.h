// lbm_launch.h -- internal interface between the host API (lbm_api.hip) and
// the kernels (lbm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Lattice geometry and launch tiling.
struct Geom {
  int32_t nx, ny;
  int32_t pitch;     // elements per row (multiple of 64)
  int64_t plane;     // ny * pitch
  int32_t tx_shift;  // log2 of the tile width TX (tiles are TX x 256/TX nodes)
  int32_t tiles_x, tiles_y;
  int32_t wall[4];   // x_lo, x_hi, y_lo, y_hi: 1 = wall, 0 = periodic
  // Interior fast path (whole lattice below 4 GiB): byte offset of plane a
  // from the lattice base, for the pull read (shifted by -e_a) and for the
  // store (unshifted).
  int32_t fast;            // 1 if the byte offsets below fit in 32 bits and a row's bytes in 24
  int32_t wb_stores;       // 1: write-back stores (the lattice pair fits kWriteBackMaxBytes)
  uint32_t lattice_bytes;  // 9 * plane * sizeof(storage) (when fast)
  uint32_t ld_soff[9];
  uint32_t st_soff[9];
  // Two- and three-step kernel tilings: 64 x t2_ty (t3_ty) output nodes per
  // workgroup.
  int32_t t2_ty, t2_tiles_x, t2_tiles_y;
  int32_t t3_ty, t3_tiles_x, t3_tiles_y, t3_threads;
  int32_t t4_ty;  // four-step kernel tile height (FP32: by lattice size)
};

// Three-step kernel shapes: output tile 64 x TY, NT threads per workgroup
// (both at four workgroups' or two large workgroups' worth of LDS per CU).
// FP64 takes the large shape, whose ring costs fewer recomputed nodes, once
// the lattice has enough tiles of it to fill the chip.
constexpr int kStep3TyF32 = 12, kStep3ThreadsF32 = 256;
constexpr int kStep3TyF64 = 4, kStep3ThreadsF64 = 256;
constexpr int kStep3TyF64Large = 10, kStep3ThreadsF64Large = 512;
constexpr int64_t kStep3LargeMinNodes = 1 << 20;

// Step kernels write a lattice back through the caches (instead of
// streaming it past them) when both lattices together take at most this many
// bytes, so that the next launch finds the state in the last-level cache.
constexpr int64_t kWriteBackMaxBytes = (int64_t)192 << 20;

// Four-step kernel: 64 x TY tiles, NT threads per workgroup.  FP32 takes the
// tile height by lattice size, so that smaller lattices still give the chip
// enough workgroups: 64 x 8 (512 threads) up to kStep4SmallMaxNodes, 64 x 12
// (768) up to kStep4MidMaxNodes, 64 x 24 (768) above.  Measured on one
// MI355X, GLUPS at 512^2 / 724^2 / 1024^2 / 2048^2: 78.9 / 103.0 / 140.0 /
// 179.9 with 64 x 8, 72.3 / 101.5 / 146.5 / 174.9 with 64 x 12, 67.5 / 99.9
// / 141.7 / 189.4 with 64 x 24.
constexpr int kStep4TyF32 = 24, kStep4ThreadsF32 = 768;
constexpr int kStep4TyF32Mid = 12, kStep4ThreadsF32Mid = 768;
constexpr int kStep4TyF32Small = 8, kStep4ThreadsF32Small = 512;
constexpr int64_t kStep4SmallMaxNodes = 600000, kStep4MidMaxNodes = 1200000;
constexpr int kStep4TyF64 = 8, kStep4ThreadsF64 = 512;

// Two-step kernel: 64 x 8 tiles (instead of 64 x 16) for lattices of up to
// this many nodes.
constexpr int64_t kStep2SmallMaxNodes = (int64_t)1 << 21;

// Two-step adjoint tiles: 64 x TY nodes, NT threads (a multiple of 64).
constexpr int kAdjoint2TyF32 = 8, kAdjoint2ThreadsF32 = 256;
constexpr int kAdjoint2TyF64 = 4, kAdjoint2ThreadsF64 = 256;
// FP32 lattices of up to kAdjoint2SmallMaxNodes nodes take 512-thread
// workgroups, so that a thread has at most two cells in the first stage and
// one node in the second (three and two with 256 threads on 64 x 8 tiles; two
// and one on 64 x 4, but with 27 % ring cells against 14 %).  Measured at
// 512^2: 64 x 8 / 256 threads 7.2 us per adjoint step, 64 x 4 / 256 6.9,
// 64 x 8 / 512 6.7; the FP32 rollout (T = 2000, checkpoint 100) 26.0 ->
// 24.8 ms against 64 x 4.  From 1024^2 up 256 threads are as fast.
constexpr int kAdjoint2TyF32Small = 8, kAdjoint2ThreadsF32Small = 512;
constexpr int64_t kAdjoint2SmallMaxNodes = 600000;
// Four-step adjoint (FP32 only): 64 x TY tiles, NT threads, used for groups
// of four steps on lattices of at least kAdjoint4MinNodes nodes that are at
// least 128 x 64; 64 x 8 tiles up to kAdjoint2SmallMaxNodes nodes, 64 x 16
// above.  Measured against pairs: 2048^2, 296.5 us per launch against two
// pair launches of 167.8 us; 512^2 (64 x 8), the FP32 rollout (T = 2000,
// checkpoint 100) 24.0 -> 22.4 ms.  Smaller lattices keep the pairs, whose
// latency chain is shorter (not measured below 512^2).
constexpr int kAdjoint4Ty = 16, kAdjoint4TySmall = 8, kAdjoint4Threads = 512;
constexpr int64_t kAdjoint4MinNodes = 200000;

// Kernel arguments in the compute real R.
template <typename R>
struct KArgs {
  Geom g;
  R w[6];          // omega_3 .. omega_8
  R rho0, fx, fy;
  const R* force;  // [2][ny][nx] or nullptr
  R wadd[4 * 9];   // moving-wall term per side and direction
};

struct KArgsAny {
  int32_t storage;  // lbm_storage
  int32_t stochastic;  // 1: stochastic rounding of 16-bit stores
  KArgs<double> d;  // used when the compute real is double (FP64)
  KArgs<float> f;   // used otherwise
  const Geom& g() const { return storage == 0 ? d.g : f.g; }
};

// PCG hash (O'Neill's permuted congruential output applied to one LCG step,
// as tabulated by Jarzynski and Olano, "Hash Functions for GPU Rendering",
// JCGT 2020): a counter-based generator, key -> 32 well-mixed bits.
__host__ __device__ inline uint32_t pcg_hash(uint32_t v) {
  const uint32_t state = v * 747796405u + 2891336453u;
  const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}

// key: stochastic-rounding key of this step (ignored unless stochastic).
hipError_t launch_step(const KArgsAny& a, const void* src, void* dst, uint32_t key, hipStream_t st);
// Two steps in one launch: src (state n) -> dst (state n+2); key_a, key_b are
// the stochastic-rounding keys of steps n and n+1.  Same result as two
// launch_step calls.
hipError_t launch_step2(const KArgsAny& a, const void* src, void* dst, uint32_t key_a, uint32_t key_b,
                        hipStream_t st);
// Three steps in one launch (FP64 and FP32 storage): src (state n) -> dst
// (state n+3), keys of steps n, n+1, n+2.  Same result as three launch_step
// calls.
hipError_t launch_step3(const KArgsAny& a, const void* src, void* dst, uint32_t key_a, uint32_t key_b,
                        uint32_t key_c, hipStream_t st);
// Four steps in one launch (FP32, FP64): src (state n) -> dst (state n+4), keys of
// steps n .. n+3.  Same result as four launch_step calls.
hipError_t launch_step4(const KArgsAny& a, const void* src, void* dst, uint32_t key_a, uint32_t key_b,
                        uint32_t key_c, uint32_t key_d, hipStream_t st);
// The same, also storing the intermediate states n+1, n+2, n+3 to keep0,
// keep1, keep2 (src, keep0..2, dst pairwise distinct): the same result as
// four launch_step calls src -> keep0 -> keep1 -> keep2 -> dst.  dst null:
// three steps, up to keep2; keep2 and dst null: two steps, up to keep1.
// FP32 only (else hipErrorInvalidValue).
hipError_t launch_step4_keep(const KArgsAny& a, const void* src, void* keep0, void* keep1, void* keep2, void* dst,
                             uint32_t key_a, uint32_t key_b, uint32_t key_c, uint32_t key_d, hipStream_t st);
hipError_t launch_init(const KArgsAny& a, const void* rho, const void* ux, const void* uy, void* dst,
                       hipStream_t st);
hipError_t launch_set(const KArgsAny& a, const void* f, void* dst, hipStream_t st);
hipError_t launch_get(const KArgsAny& a, const void* src, void* f, hipStream_t st);
hipError_t launch_macro(const KArgsAny& a, const void* src, void* rho, void* ux, void* uy, void* sxx,
                        void* syy, void* sxy, hipStream_t st);
hipError_t launch_diag(const KArgsAny& a, const void* src, double* partial, int nblocks, double base_mass,
                       double* out, hipStream_t st);
hipError_t launch_adjoint_step(const KArgsAny& a, const void* prev, const void* mu_in, void* mu_out,
                               void* grad_force, hipStream_t st);
// Two adjoint steps in one launch: mu_in (cotangent of state n+1) back
// through step n (state n in prev_a) and step n-1 (state n-1 in prev_b) to
// mu_out.  Same result as two launch_adjoint_step calls.
hipError_t launch_adjoint_step2(const KArgsAny& a, const void* prev_a, const void* prev_b, const void* mu_in,
                                void* mu_out, void* grad_force, hipStream_t st);
// Four adjoint steps in one launch (FP32): mu_in (cotangent of state n+1)
// back through steps n, n-1, n-2, n-3 (states in prev_a .. prev_d) to mu_out.
// Same result as four launch_adjoint_step calls.
hipError_t launch_adjoint_step4(const KArgsAny& a, const void* prev_a, const void* prev_b, const void* prev_c,
                                const void* prev_d, const void* mu_in, void* mu_out, void* grad_force,
                                hipStream_t st);
hipError_t launch_adjoint_macro(const KArgsAny& a, const void* lat, const void* g_rho, const void* g_ux,
                                const void* g_uy, void* mu_out, void* grad_force, hipStream_t st);
hipError_t launch_adjoint_init(const KArgsAny& a, const void* rho, const void* ux, const void* uy,
                               const void* mu0, void* g_rho, void* g_ux, void* g_uy, void* grad_force,
                               hipStream_t st);

}  // namespace lbm
