// lbm_kernels.hip -- gfx950 kernels of the cascaded D2Q9 lattice Boltzmann
// step (Ning & Premnath, Section II) with periodic, halfway bounce-back and
// moving-wall boundaries (Section III), its diagnostics and its adjoint.
//
// Data layout in HBM: a lattice is nine planes [9][ny][pitch] of the storage
// type S (double, float, _Float16 or __bf16), x fastest, each row 64-element
// aligned; the stored value is the deviation d = f - w rho0 (w the D2Q9 rest
// weights) of the post-collision populations of the previous step (pull
// scheme).  One thread owns one node.  A step gathers the nine populations
// streaming into the node (plane a at x - e_a: coalesced, misaligned by one
// element for e_x != 0), collides in registers (cascade.h) and writes the
// nine results to the other lattice at the node itself (aligned, coalesced;
// non-temporal, or write-back when both lattices fit in the last-level
// cache).  A link whose source lies beyond a wall reads the reversed
// population of the node itself (halfway bounce-back) plus the moving-wall
// term; walls are resolved per thread from (x, y) with selects, so there is
// no mask array and the wall rows do not diverge from the interior.
//
// Launch shape of the single step: 256-thread blocks covering TX x (256/TX)
// nodes, TX in {64, 128, 256} (a 64-wide wavefront spans one row segment).
// The fused launches keep intermediate steps in LDS, so the state crosses
// HBM once per two, three or four steps.  k_step2, k_step3 and k_step4 give
// each workgroup a 64 x TY tile plus a recompute ring (two, three or four
// steps); k_step4 can also store its intermediate states (the state-keeping
// recompute of the adjoint).  In every kernel the 1-D block index is remapped so that each of
// the 8 XCDs (blocks are dealt to XCDs round-robin) processes one contiguous
// band of tiles, keeping the lines shared between horizontally and
// vertically adjacent tiles in one L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cascade.h"
#include "lbm_launch.h"

namespace lbm {

// ------------------------------------------------------------ storage codec
template <typename S> struct Codec;
template <> struct Codec<double> {
  using R = double;
  __device__ static R load(double v) { return v; }
  __device__ static double store(R v) { return v; }
};
template <> struct Codec<float> {
  using R = float;
  __device__ static R load(float v) { return v; }
  __device__ static float store(R v) { return v; }
};
// 16-bit codecs.  store() rounds to nearest even.  store_sr() rounds
// stochastically: r supplies uniform random bits in its low 13 (binary16) or
// 16 (bfloat16) bits, and the magnitude is rounded up with probability equal
// to the discarded fraction (unbiased).  bfloat16: the bits are added to the
// FP32 bit pattern below the kept significand and the sum is truncated; the
// store takes the upper half as it is.  binary16: gfx950's v_cvt_sr_f16_f32,
// which reads its random word's top 13 bits.  Measured on the GPU over 4 M
// (value, word) pairs, it equals that add-and-truncate rule for normal
// results, and for results in binary16's subnormal range (|x| < 2^-14) it
// adds the bits as a fraction of the subnormal step 2^-24 and truncates
// toward zero, so those round stochastically too.  (The bfloat16 conversion
// instruction equals the rule above with the word's top 16 bits; it would
// cost a shift and a register pack more per population than the add.)
typedef _Float16 lbm_f16x2 __attribute__((ext_vector_type(2)));
template <> struct Codec<_Float16> {
  using R = float;
  __device__ static R load(_Float16 v) { return (float)v; }
  __device__ static _Float16 store(R v) { return (_Float16)v; }
  __device__ static _Float16 store_sr(R v, uint32_t r) {
    lbm_f16x2 h = {};
    h = __builtin_amdgcn_cvt_sr_f16_f32(h, v, r << 19, false);
    return h[0];
  }
};
template <> struct Codec<__bf16> {
  using R = float;
  __device__ static R load(__bf16 v) { return (float)v; }
  __device__ static __bf16 store(R v) { return (__bf16)v; }
  __device__ static __bf16 store_sr(R v, uint32_t r) {
    const uint32_t b = __builtin_bit_cast(uint32_t, v) + (r & 0xFFFFu);
    return __builtin_bit_cast(__bf16, (uint16_t)(b >> 16));
  }
};

// D2Q9 rest weights.
template <typename R>
__device__ __forceinline__ R weight(int a) {
  return a == 0 ? R(4.0 / 9.0) : (a < 5 ? R(1.0 / 9.0) : R(1.0 / 36.0));
}

// ------------------------------------------------------------- node index
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  // Blocks are dealt to the 8 XCDs round-robin; give XCD k the contiguous
  // range of logical tiles [start_k, start_k + count_k).
  const int q = nblocks >> 3, rem = nblocks & 7;
  const int xcd = b & 7, local = b >> 3;
  const int start = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
  return start + local;
}

struct NodePos {
  int x, y;
  bool valid;
};

__device__ __forceinline__ NodePos node_pos(const Geom& g) {
  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int tx = tile % g.tiles_x, ty = tile / g.tiles_x;
  const int lx = (int)threadIdx.x & ((1 << g.tx_shift) - 1);
  const int ly = (int)threadIdx.x >> g.tx_shift;
  NodePos p;
  p.x = (tx << g.tx_shift) + lx;
  p.y = ty * (256 >> g.tx_shift) + ly;
  p.valid = p.x < g.nx && p.y < g.ny;
  return p;
}

// Buffer-resource access for the interior fast path.  One descriptor covers
// a whole lattice; plane a is reached through a scalar offset (soffset) that
// already includes its streaming shift, so a wavefront addresses all nine
// loads and nine stores with one 32-bit VGPR byte offset (buffer_load/store
// ... offen) and no per-plane address arithmetic.
constexpr int kBufferWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format
constexpr int kNonTemporal = 2;           // cache policy: nt (no reuse expected)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferWord3);
}

template <typename S> struct BufIO;
template <> struct BufIO<float> {
  __device__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, 0));
  }
  template <int CP = kNonTemporal>
  __device__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)off, (int)soff,
                                          CP);
  }
};
template <> struct BufIO<double> {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  __device__ static double load(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, 0));
  }
  template <int CP = kNonTemporal>
  __device__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)off, (int)soff, CP);
  }
};
template <> struct BufIO<_Float16> {
  __device__ static _Float16 load(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, (int)soff, 0));
  }
  template <int CP = kNonTemporal>
  __device__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, _Float16 v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)off, (int)soff,
                                          CP);
  }
};
template <> struct BufIO<__bf16> {
  __device__ static __bf16 load(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, (int)soff, 0));
  }
  template <int CP = kNonTemporal>
  __device__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, __bf16 v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)off, (int)soff,
                                          CP);
  }
};

// Neighbour coordinates with periodic wrap and the wall flags of a node.
struct Edges {
  int xm, xp, ym, yp;      // x-1, x+1, y-1, y+1 wrapped
  bool wxl, wxh, wyl, wyh;  // node touches the x_lo / x_hi / y_lo / y_hi wall
};

__device__ __forceinline__ Edges edges(const Geom& g, int x, int y) {
  Edges e;
  e.xm = x == 0 ? g.nx - 1 : x - 1;
  e.xp = x == g.nx - 1 ? 0 : x + 1;
  e.ym = y == 0 ? g.ny - 1 : y - 1;
  e.yp = y == g.ny - 1 ? 0 : y + 1;
  e.wxl = (x == 0) && g.wall[0];
  e.wxh = (x == g.nx - 1) && g.wall[1];
  e.wyl = (y == 0) && g.wall[2];
  e.wyh = (y == g.ny - 1) && g.wall[3];
  return e;
}

// Where the population streaming into (x, y) along direction A comes from:
// element offset into the lattice and the moving-wall term.  Fluid or
// periodic link: plane A at (x - e_x, y - e_y).  Link crossing a wall
// (halfway bounce-back): plane opp(A) at (x, y), plus 6 rho0 w_A (e_A .
// U_wall) of that wall (precomputed per side and direction in wadd).  A link
// crossing two walls passes through their corner point, which is at rest:
// plain bounce-back, no wall term.
template <int A, typename R>
__device__ __forceinline__ int64_t link_src(const Geom& g, const Edges& e, int x, int y,
                                            const R* wadd, R& add) {
  constexpr int ex = EX[A], ey = EY[A];
  const bool hx = (ex == 1 && e.wxl) || (ex == -1 && e.wxh);
  const bool hy = (ey == 1 && e.wyl) || (ey == -1 && e.wyh);
  const int sx = ex == 1 ? e.xm : (ex == -1 ? e.xp : x);
  const int sy = ey == 1 ? e.ym : (ey == -1 ? e.yp : y);
  add = hx == hy ? R(0) : (hx ? wadd[(ex == 1 ? 0 : 1) * 9 + A] : wadd[(ey == 1 ? 2 : 3) * 9 + A]);
  const bool hit = hx || hy;
  const int plane = hit ? OPP[A] : A;
  const int off = hit ? y * g.pitch + x : sy * g.pitch + sx;
  return (int64_t)plane * g.plane + off;
}

// BUF: on a lattice below 4 GiB, read the same sources through a buffer
// descriptor (32-bit element offsets from three row offsets, no 64-bit
// address arithmetic per link): the forward step's edge nodes and window
// cells.  (The adjoint's gathers measured slower that way and keep the flat
// loads.)
template <typename S, typename R, bool BUF = false>
__device__ __forceinline__ void gather(const Geom& g, const R* wadd, const S* __restrict__ src,
                                       int x, int y, R d[9]) {
  const Edges e = edges(g, x, y);
  if (BUF && g.fast) {
    const __amdgpu_buffer_rsrc_t rs = rsrc(src, g.lattice_bytes);
    const uint32_t rm = (uint32_t)(e.ym * g.pitch), r0 = (uint32_t)(y * g.pitch), rp = (uint32_t)(e.yp * g.pitch);
#define LBM_GATHER_B(A)                                                                                     \
    {                                                                                                       \
      constexpr int ex = EX[A], ey = EY[A];                                                                 \
      const bool hx = (ex == 1 && e.wxl) || (ex == -1 && e.wxh);                                            \
      const bool hy = (ey == 1 && e.wyl) || (ey == -1 && e.wyh);                                            \
      const R add = hx == hy ? R(0)                                                                         \
                             : (hx ? wadd[(ex == 1 ? 0 : 1) * 9 + A] : wadd[(ey == 1 ? 2 : 3) * 9 + A]);    \
      const uint32_t sx = (uint32_t)(ex == 1 ? e.xm : (ex == -1 ? e.xp : x));                               \
      const uint32_t sr = ey == 1 ? rm : (ey == -1 ? rp : r0);                                              \
      const uint32_t off = (hx || hy) ? r0 + (uint32_t)x + (uint32_t)(OPP[A] * g.plane)                     \
                                      : sr + sx + (uint32_t)(A * g.plane);                                  \
      d[A] = Codec<S>::load(BufIO<S>::load(rs, off * (uint32_t)sizeof(S), 0)) + add;                        \
    }
    LBM_GATHER_B(0) LBM_GATHER_B(1) LBM_GATHER_B(2) LBM_GATHER_B(3) LBM_GATHER_B(4)
    LBM_GATHER_B(5) LBM_GATHER_B(6) LBM_GATHER_B(7) LBM_GATHER_B(8)
#undef LBM_GATHER_B
    return;
  }
#define LBM_GATHER(A)                                          \
  {                                                            \
    R add;                                                     \
    const int64_t i = link_src<A, R>(g, e, x, y, wadd, add);   \
    d[A] = Codec<S>::load(src[i]) + add;                       \
  }
  LBM_GATHER(0) LBM_GATHER(1) LBM_GATHER(2) LBM_GATHER(3) LBM_GATHER(4)
  LBM_GATHER(5) LBM_GATHER(6) LBM_GATHER(7) LBM_GATHER(8)
#undef LBM_GATHER
}

// Inverse of gather(): write the pre-collision value v[a] of (x, y) to the
// place the next gather reads it from (minus the wall term).  Every lattice
// element is written exactly once over all nodes (streaming is a
// permutation).
template <typename S, typename R>
__device__ __forceinline__ void scatter(const Geom& g, const R* wadd, S* __restrict__ dst, int x,
                                        int y, const R v[9], bool subtract_wall) {
  const Edges e = edges(g, x, y);
#define LBM_SCATTER(A)                                          \
  {                                                             \
    R add;                                                      \
    const int64_t i = link_src<A, R>(g, e, x, y, wadd, add);    \
    dst[i] = Codec<S>::store(subtract_wall ? v[A] - add : v[A]); \
  }
  LBM_SCATTER(0) LBM_SCATTER(1) LBM_SCATTER(2) LBM_SCATTER(3) LBM_SCATTER(4)
  LBM_SCATTER(5) LBM_SCATTER(6) LBM_SCATTER(7) LBM_SCATTER(8)
#undef LBM_SCATTER
}

template <typename R>
__device__ __forceinline__ void node_force(const KArgs<R>& a, int x, int y, R& Fx, R& Fy) {
  if (a.force) {
    const int64_t c = (int64_t)y * a.g.nx + x;
    Fx = a.force[c];
    Fy = a.force[(int64_t)a.g.nx * a.g.ny + c];
  } else {
    Fx = a.fx;
    Fy = a.fy;
  }
}

template <typename R>
__device__ __forceinline__ Rates<R> rates(const KArgs<R>& a) {
  return make_rates<R>(a.w, a.rho0);
}

// ------------------------------------------------------------------ kernels

// The nine stored values of node (x, y) into lattice dst.  Non-temporal
// stores stream a large lattice past the caches; a lattice whose pair fits in
// the last-level cache (g.wb_stores) is written back through them, so the next
// launch reads it from there.
template <typename S>
__device__ __forceinline__ void store_node(const Geom& g, S* __restrict__ dst, int x, int y, const S o[9]) {
  if (g.fast) {
    const __amdgpu_buffer_rsrc_t w = rsrc(dst, g.lattice_bytes);
    const uint32_t off = (uint32_t)(y * g.pitch + x) * (uint32_t)sizeof(S);
    if (g.wb_stores) {
#pragma unroll
      for (int k = 0; k < 9; ++k) BufIO<S>::template store<0>(w, off, g.st_soff[k], o[k]);
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) BufIO<S>::store(w, off, g.st_soff[k], o[k]);
    }
  } else {
    const int64_t c = (int64_t)y * g.pitch + x;
    if (g.wb_stores) {
#pragma unroll
      for (int k = 0; k < 9; ++k) dst[(int64_t)k * g.plane + c] = o[k];
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) __builtin_nontemporal_store(o[k], dst + (int64_t)k * g.plane + c);
    }
  }
}

// The nine values of node (x, y) into a kept intermediate state, streamed
// past the caches like a large lattice: a segment's kept states outgrow the
// last-level cache, and the adjoint reads each one only after the recompute
// has written many others (the FP32 rollout at 512^2, T = 2000, checkpoint
// 100: 25.0 -> 23.9 ms against write-back stores; no change at 2048^2).  The
// interior path's kept stores take the same non-temporal policy.
template <typename S>
__device__ __forceinline__ void store_kept(const Geom& g, S* __restrict__ dst, int x, int y, const S o[9]) {
  const int64_t c = (int64_t)y * g.pitch + x;
#pragma unroll
  for (int k = 0; k < 9; ++k) __builtin_nontemporal_store(o[k], dst + (int64_t)k * g.plane + c);
}

// Stores of one node's nine post-collision values as the storage type, with
// the step's rounding: nearest even, or stochastic with 16 random bits per
// population.  The bits of populations 0 and 1 are the PCG hash of the node
// and the step's key; those of populations 2..8 come from Marsaglia's
// xorshift32 (shifts 13, 17, 5; "Xorshift RNGs", J. Stat. Softw. 2003)
// seeded from that hash with its low bit set (xorshift32 never leaves 0).
// Each of its states is uniform over the non-zero 32-bit words, so every
// population's rounding stays unbiased, without the integer multiplies of
// a hash per pair.
template <typename S, bool SR>
__device__ __forceinline__ void round_out(const typename Codec<S>::R out[9], uint32_t node, uint32_t key,
                                          S o[9]) {
  if constexpr (SR) {
    const uint32_t h = pcg_hash(node ^ key);
    o[0] = Codec<S>::store_sr(out[0], h >> 16);
    o[1] = Codec<S>::store_sr(out[1], h);
    uint32_t x = (h ^ 0x9E3779B9u) | 1u;
#pragma unroll
    for (int k = 2; k < 9; k += 2) {
      x ^= x << 13;
      x ^= x >> 17;
      x ^= x << 5;
      o[k] = Codec<S>::store_sr(out[k], x >> 16);
      if (k + 1 < 9) o[k + 1] = Codec<S>::store_sr(out[k + 1], x);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) o[k] = Codec<S>::store(out[k]);
  }
}

// One fused stream-and-collide step: src (state n) -> dst (state n+1).
// FM: 0 = no body force, 1 = uniform force, 2 = per-node force field.
// A wavefront whose 64 nodes are all interior (no wrap, no wall link) pulls
// plane a through a descriptor based at src + a*plane - e_ay*pitch - e_ax
// with the node's own offset; wavefronts touching the domain edge take the
// general gather with wrap and bounce-back selects.
template <typename S, int FM, bool SR>
__global__ __launch_bounds__(256) void k_step(KArgs<typename Codec<S>::R> a, const S* __restrict__ src,
                                              S* __restrict__ dst, uint32_t key) {
  using R = typename Codec<S>::R;
  const NodePos p = node_pos(a.g);
  if (!p.valid) return;
  const Geom& g = a.g;
  const uint32_t off = (uint32_t)(p.y * g.pitch + p.x) * (uint32_t)sizeof(S);
  const bool inner = p.x >= 1 && p.x <= g.nx - 2 && p.y >= 1 && p.y <= g.ny - 2;
  const bool fast = g.fast && __all(inner);
  R d[9];
  if (fast) {
    const __amdgpu_buffer_rsrc_t r = rsrc(src, g.lattice_bytes);
#pragma unroll
    for (int k = 0; k < 9; ++k) d[k] = Codec<S>::load(BufIO<S>::load(r, off, g.ld_soff[k]));
  } else {
    gather<S, R, true>(g, a.wadd, src, p.x, p.y, d);
  }
  R Fx = R(0), Fy = R(0);
  if (FM == 1) {
    Fx = a.fx;
    Fy = a.fy;
  } else if (FM == 2) {
    node_force(a, p.x, p.y, Fx, Fy);
  }
  R out[9];
  collide_step<R, FM != 0>(rates(a), Fx, Fy, d, out);
  S o[9];
  round_out<S, SR>(out, (uint32_t)(p.y * g.nx + p.x), key, o);
  store_node<S>(g, dst, p.x, p.y, o);
}

// ---- multi-step launches (temporal blocking) ----------------------------
//
// A workgroup owns a 64 x TY tile of output nodes and keeps a window of the
// tile plus an H-node ring in LDS.  Every intermediate value is rounded to the
// storage type exactly as a stored step would round it (stochastic keys
// included), so a K-step launch is bit-for-bit K single steps.  Window cells
// hold nodes at their wrapped position on periodic sides; cells beyond a wall
// are never computed or read (links across a wall bounce back from the
// node's own cell).

// Global node of window cell (wx, wy) in unwrapped coordinates: false if it
// lies beyond a wall, else its wrapped position.
// gx and gy are assigned on every path, the false one included, and callers
// call it whether or not they will use the cell: with an output left
// unassigned on some path, the compiler (ROCm 7.2, gfx950) has zeroed gx for
// all lanes of the y-wrap branch, the lanes that wrapped among them, when the
// results went into per-thread arrays of three cells.
// A coordinate wrapped into [0, n): one period off in all but windows wider
// than the lattice, so the remainder (an integer division) is the rare case.
__device__ __forceinline__ int wrap_coord(int w, int n) {
  w += w < 0 ? n : (w >= n ? -n : 0);
  if (w < 0 || w >= n) w = ((w % n) + n) % n;
  return w;
}

__device__ __forceinline__ bool window_node(const Geom& g, int wx, int wy, int& gx, int& gy) {
  bool ok = true;
  if (wx < 0 || wx >= g.nx) {
    ok = g.wall[wx < 0 ? 0 : 1] == 0;
    wx = wrap_coord(wx, g.nx);
  }
  if (wy < 0 || wy >= g.ny) {
    ok = ok & (g.wall[wy < 0 ? 2 : 3] == 0);
    wy = wrap_coord(wy, g.ny);
  }
  gx = wx;
  gy = wy;
  return ok;
}

// The nine populations streaming into node (gx, gy), held in window cell
// (cx, cy) whose neighbours hold the previous step's post-collision values.
// WALLS = false: the caller knows that no link of the node crosses a wall.
template <bool WALLS, typename S, typename R, int EH, int EW, int EHP>
__device__ __forceinline__ void pull_window(const KArgs<R>& a, int gx, int gy, const S (&mid)[9][EHP][EW],
                                            int cx, int cy, R d[9]) {
  if constexpr (!WALLS) {
#pragma unroll
    for (int k = 0; k < 9; ++k) d[k] = Codec<S>::load(mid[k][cy - EY[k]][cx - EX[k]]);
    return;
  }
  const Edges e = edges(a.g, gx, gy);
#define LBM_PULL_WIN(A)                                                                        \
  {                                                                                            \
    constexpr int ax = EX[A], ay = EY[A];                                                      \
    const bool hx = (ax == 1 && e.wxl) || (ax == -1 && e.wxh);                                 \
    const bool hy = (ay == 1 && e.wyl) || (ay == -1 && e.wyh);                                 \
    const R add = hx == hy ? R(0)                                                              \
                           : (hx ? a.wadd[(ax == 1 ? 0 : 1) * 9 + A]                           \
                                 : a.wadd[(ay == 1 ? 2 : 3) * 9 + A]);                         \
    d[A] = (hx || hy) ? Codec<S>::load(mid[OPP[A]][cy][cx]) + add                              \
                      : Codec<S>::load(mid[A][cy - ay][cx - ax]);                              \
  }
  LBM_PULL_WIN(0) LBM_PULL_WIN(1) LBM_PULL_WIN(2) LBM_PULL_WIN(3) LBM_PULL_WIN(4)
  LBM_PULL_WIN(5) LBM_PULL_WIN(6) LBM_PULL_WIN(7) LBM_PULL_WIN(8)
#undef LBM_PULL_WIN
}

template <int FM, typename R>
__device__ __forceinline__ void force_at(const KArgs<R>& a, int gx, int gy, R& Fx, R& Fy) {
  Fx = R(0);
  Fy = R(0);
  if (FM == 1) {
    Fx = a.fx;
    Fy = a.fy;
  } else if (FM == 2) {
    node_force(a, gx, gy, Fx, Fy);
  }
}

// Step n for one window cell from its nine pulled populations d, rounded and
// kept in LDS.
// FW: also keep the cell's force in the LDS array fw ([2][EH][EW]) for the
// later stages.  keep (not null): also store the result there, at (gx, gy).
template <typename S, int FM, bool SR, int EH, int EW, bool U = false, bool FW = false, int EHP>
__device__ __forceinline__ void collide_into_window(const KArgs<typename Codec<S>::R>& a,
                                                    const Rates<typename Codec<S>::R>& rt, int gx, int gy,
                                                    const typename Codec<S>::R d[9], uint32_t key,
                                                    S (&mid)[9][EHP][EW], int cx, int cy,
                                                    typename Codec<S>::R* fw = nullptr,
                                                    S* __restrict__ keep = nullptr) {
  using R = typename Codec<S>::R;
  R Fx, Fy;
  force_at<FM>(a, gx, gy, Fx, Fy);
  if constexpr (FW) {
    fw[cy * EW + cx] = Fx;
    fw[EH * EW + cy * EW + cx] = Fy;
  }
  R out[9];
  collide_step<R, FM != 0, U>(rt, Fx, Fy, d, out);
  S o[9];
  round_out<S, SR>(out, (uint32_t)(gy * a.g.nx + gx), key, o);
#pragma unroll
  for (int k = 0; k < 9; ++k) mid[k][cy][cx] = o[k];
  if (keep) store_kept<S>(a.g, keep, gx, gy, o);
}

// Pull of window cell (gx, gy) for the first stage: from HBM, through the
// buffer fast path when the whole window allows it.
template <typename S>
__device__ __forceinline__ void pull_hbm(const KArgs<typename Codec<S>::R>& a, __amdgpu_buffer_rsrc_t rs,
                                         const S* __restrict__ src, bool fast, int gx, int gy,
                                         typename Codec<S>::R d[9]) {
  using R = typename Codec<S>::R;
  const Geom& g = a.g;
  if (fast) {
    const uint32_t off = (uint32_t)(gy * g.pitch + gx) * (uint32_t)sizeof(S);
#pragma unroll
    for (int k = 0; k < 9; ++k) d[k] = Codec<S>::load(BufIO<S>::load(rs, off, g.ld_soff[k]));
  } else {
    gather<S, R, true>(g, a.wadd, src, gx, gy, d);
  }
}

// First stage: step n on every cell of the window (origin (wx0, wy0) in
// unwrapped coordinates) from HBM into LDS, one cell at a time.  fast: no
// cell of the window pulls across a wall or a wrap, and the lattice is below
// 4 GiB.
template <typename S, int FM, bool SR, int EH, int EW, bool U = false, int EHP>
__device__ __forceinline__ void stage_from_hbm(const KArgs<typename Codec<S>::R>& a,
                                               const Rates<typename Codec<S>::R>& rt, const S* __restrict__ src,
                                               int wx0, int wy0, bool fast, uint32_t key, S (&mid)[9][EHP][EW]) {
  using R = typename Codec<S>::R;
  const __amdgpu_buffer_rsrc_t rs = rsrc(src, a.g.lattice_bytes);
  for (int i = (int)threadIdx.x; i < EW * EH; i += 256) {
    const int cx = i % EW, cy = i / EW;
    int gx, gy;
    if (!window_node(a.g, wx0 + cx, wy0 + cy, gx, gy)) continue;
    R d[9];
    pull_hbm<S>(a, rs, src, fast, gx, gy, d);
    collide_into_window<S, FM, SR, EH, EW, U>(a, rt, gx, gy, d, key, mid, cx, cy);
  }
}

// The same with every load of the thread's cells issued before the first
// collision, so that HBM latency is paid once per stage rather than once per
// cell.
// FW: keep the window's force in fw (see collide_into_window).  KEEP: store
// the step's result for the tile's nodes (window cells [H, EW - H) x
// [H, EH - H) inside the domain) to keep.
template <typename S, int FM, bool SR, int EH, int EW, int NT, bool U = false, bool FW = false, bool KEEP = false, int EHP>
__device__ __forceinline__ void stage_from_hbm_prefetch(const KArgs<typename Codec<S>::R>& a,
                                                        const Rates<typename Codec<S>::R>& rt,
                                                        const S* __restrict__ src, int wx0, int wy0, bool fast,
                                                        uint32_t key, S (&mid)[9][EHP][EW],
                                                        typename Codec<S>::R* fw = nullptr,
                                                        S* __restrict__ keep = nullptr) {
  constexpr int H = (EW - 64) / 2;
  using R = typename Codec<S>::R;
  constexpr int NPT = (EW * EH + NT - 1) / NT;
  const __amdgpu_buffer_rsrc_t rs = rsrc(src, a.g.lattice_bytes);
  R d[NPT][9];
  int gx[NPT], gy[NPT];
  bool live[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int i = (int)threadIdx.x + NT * j;
    const bool in = window_node(a.g, wx0 + i % EW, wy0 + i / EW, gx[j], gy[j]);
    live[j] = i < EW * EH && in;
    if (live[j]) pull_hbm<S>(a, rs, src, fast, gx[j], gy[j], d[j]);
  }
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int i = (int)threadIdx.x + NT * j;
    const int cx = i % EW, cy = i / EW;
    S* kp = nullptr;
    if constexpr (KEEP) {
      const bool tile = cx >= H && cx < EW - H && cy >= H && cy < EH - H && wx0 + cx < a.g.nx &&
                        wy0 + cy < a.g.ny;
      kp = tile ? keep : nullptr;
    }
    if (live[j]) collide_into_window<S, FM, SR, EH, EW, U, FW>(a, rt, gx[j], gy[j], d[j], key, mid, cx, cy, fw, kp);
  }
}

// Middle stage, in place: one step on the window cells at most RING nodes
// outside the tile (the window has an H-node ring).  Every thread pulls and
// collides its cells into registers; after a barrier it writes them back.
// WALLS = false: the window lies inside the domain and no cell's link
// crosses a wall.
// FW: forces from fw instead of the force field.  KEEP: store the results of
// the tile's nodes to keep.
template <bool WALLS, typename S, int FM, bool SR, int EH, int EW, int H, int RING, int NT, bool U = false,
          bool FW = false, bool KEEP = false, int EHP>
__device__ __forceinline__ void stage_in_lds(const KArgs<typename Codec<S>::R>& a,
                                             const Rates<typename Codec<S>::R>& rt, int wx0, int wy0,
                                             uint32_t key, S (&mid)[9][EHP][EW],
                                             const typename Codec<S>::R* fw = nullptr,
                                             S* __restrict__ keep = nullptr) {
  using R = typename Codec<S>::R;
  constexpr int RW = EW - 2 * (H - RING), RH = EH - 2 * (H - RING), NPT = (RW * RH + NT - 1) / NT;
  const Geom& g = a.g;
  S o[NPT][9];
  bool live[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int i = (int)threadIdx.x + NT * j;
    const int cx = H - RING + i % RW, cy = H - RING + i / RW;
    int gx = wx0 + cx, gy = wy0 + cy;
    live[j] = i < RW * RH && (!WALLS || window_node(g, wx0 + cx, wy0 + cy, gx, gy));
    if (!live[j]) continue;
    R d[9];
    pull_window<WALLS, S, R, EH, EW>(a, gx, gy, mid, cx, cy, d);
    R Fx, Fy;
    if constexpr (FW) {
      Fx = fw[cy * EW + cx];
      Fy = fw[EH * EW + cy * EW + cx];
    } else {
      force_at<FM>(a, gx, gy, Fx, Fy);
    }
    R out[9];
    collide_step<R, FM != 0, U>(rt, Fx, Fy, d, out);
    round_out<S, SR>(out, (uint32_t)(gy * g.nx + gx), key, o[j]);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    if (!live[j]) continue;
    const int i = (int)threadIdx.x + NT * j;
    const int cx = H - RING + i % RW, cy = H - RING + i / RW;
#pragma unroll
    for (int k = 0; k < 9; ++k) mid[k][cy][cx] = o[j][k];
    if constexpr (KEEP) {
      const int ux = wx0 + cx, uy = wy0 + cy;  // a tile node is its own position
      if (cx >= H && cx < EW - H && cy >= H && cy < EH - H && ux < g.nx && uy < g.ny)
        store_kept<S>(g, keep, ux, uy, o[j]);
    }
  }
  __syncthreads();
}

// Last stage: one step on the 64 x TY tile from LDS to HBM.
// FW: forces from fw instead of the force field.
template <bool WALLS, typename S, int FM, bool SR, int TY, int EH, int EW, int H, int NT, bool U = false,
          bool FW = false, int EHP>
__device__ __forceinline__ void stage_to_hbm(const KArgs<typename Codec<S>::R>& a,
                                             const Rates<typename Codec<S>::R>& rt, int x0, int y0,
                                             uint32_t key, const S (&mid)[9][EHP][EW], S* __restrict__ dst,
                                             const typename Codec<S>::R* fw = nullptr) {
  using R = typename Codec<S>::R;
  const Geom& g = a.g;
  const int lx = (int)threadIdx.x & 63;
  for (int ly = (int)threadIdx.x >> 6; ly < TY; ly += NT / 64) {
    const int gx = x0 + lx, gy = y0 + ly;
    if (gx >= g.nx || gy >= g.ny) continue;
    R d[9];
    pull_window<WALLS, S, R, EH, EW>(a, gx, gy, mid, lx + H, ly + H, d);
    R Fx, Fy;
    if constexpr (FW) {
      Fx = fw[(ly + H) * EW + lx + H];
      Fy = fw[EH * EW + (ly + H) * EW + lx + H];
    } else {
      force_at<FM>(a, gx, gy, Fx, Fy);
    }
    R out[9];
    collide_step<R, FM != 0, U>(rt, Fx, Fy, d, out);
    S o[9];
    round_out<S, SR>(out, (uint32_t)(gy * g.nx + gx), key, o);
    store_node<S>(g, dst, gx, gy, o);
  }
}

// ---- interior tiles ------------------------------------------------------
//
// A tile whose window and the window's own pulls stay inside the domain (no
// wall link, no wrap), on a lattice below 4 GiB.  A stage's region is a
// rectangle of RW x RH window cells, numbered row-major; cell i lies at
// window index i + (i / RW) (EW - RW) + c0.  Every HBM address of the stage
// is the window origin's plus that cell's element offset (one scalar base,
// one per-cell offset), every LDS access a per-cell index plus a
// compile-time offset, and no cell takes a wall or wrap decision.

// Pointer to cell w of the first plane of an LDS window array, opaque to
// the optimiser: it neither folds part of the cell index into the access
// offsets nor derives one cell's address from another's, so each cell keeps
// one base register and its accesses are that base plus an immediate offset.
template <typename S>
using LdsPtr = __attribute__((address_space(3))) S*;
template <typename S>
__device__ __forceinline__ LdsPtr<S> lds_opaque(LdsPtr<S> p) {
  uint32_t a = (uint32_t)(uintptr_t)p;
  asm("" : "+v"(a));
  return (LdsPtr<S>)(uintptr_t)a;
}
template <typename S>
__device__ __forceinline__ LdsPtr<S> lds_cell(const S* lds, int w) {
  return lds_opaque((LdsPtr<S>)(lds + w));
}

// Force of a window cell: none, the uniform one, or the field's.  The
// field ([2][ny][nx], 8 or 16 B per node, so below 4 GiB whenever the
// lattice is) is read through a buffer descriptor with one 32-bit offset.
template <int FM, typename R>
__device__ __forceinline__ void core_force(const KArgs<R>& a, int gx, int gy, R& Fx, R& Fy) {
  Fx = R(0);
  Fy = R(0);
  if constexpr (FM == 1) {
    Fx = a.fx;
    Fy = a.fy;
  } else if constexpr (FM == 2) {
    const uint32_t plane = (uint32_t)(a.g.nx * a.g.ny) * (uint32_t)sizeof(R);
    const __amdgpu_buffer_rsrc_t rf = rsrc(a.force, 2 * plane);
    const uint32_t off = (uint32_t)(gy * a.g.nx + gx) * (uint32_t)sizeof(R);
    Fx = BufIO<R>::load(rf, off, 0);
    Fy = BufIO<R>::load(rf, off, plane);
  }
}

// First stage: step n on every window cell, from HBM into LDS.  A thread's
// cells go in batches of B: the loads of a whole batch are issued before its
// first collision.  FW: also keep each cell's force in fw ([2][EH][EW]) for
// the later stages.  KEEP: also store the result of the tile's nodes to keep.
// PRIO: the waves issue a batch's loads at raised priority, so that on a SIMD
// they go out ahead of another workgroup's arithmetic (four-step launches:
// FP32 cavity 4096^2, 284.7 -> 280.0 us per launch, A/B twice on one box;
// the two-step 16-bit launch got 2.5 % slower with it and does without).
template <typename S, int FM, bool SR, int EH, int EW, int NT, bool U, int B, bool FW = false, bool KEEP = false,
          bool PRIO = false, int EHP>
__device__ __forceinline__ void core_stage_hbm(const KArgs<typename Codec<S>::R>& a,
                                               const Rates<typename Codec<S>::R>& rt, const S* __restrict__ src,
                                               int wx0, int wy0, uint32_t key, S (&mid)[9][EHP][EW],
                                               typename Codec<S>::R* fw = nullptr, S* __restrict__ keep = nullptr) {
  using R = typename Codec<S>::R;
  constexpr int NC = EW * EH, NPT = (NC + NT - 1) / NT, PL = EHP * EW, H = (EW - 64) / 2;
  const Geom& g = a.g;
  const __amdgpu_buffer_rsrc_t rs = rsrc(src, g.lattice_bytes);
  // byte offset of this thread's first cell were it in row 0; a cell in
  // window row cy lies cy (pitch - EW) elements further
  const uint32_t t0 = (uint32_t)(wy0 * g.pitch + wx0 + (int)threadIdx.x) * (uint32_t)sizeof(S);
  const uint32_t skip = (uint32_t)(g.pitch - EW) * (uint32_t)sizeof(S);
  S* lds = &mid[0][0][0];
  const int t = (int)threadIdx.x;
#pragma unroll
  for (int j0 = 0; j0 < NPT; j0 += B) {
    R d[B][9];
    uint32_t off[B];
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(3);
#pragma unroll
    for (int jb = 0; jb < B; ++jb) {
      const int j = j0 + jb, i = t + NT * j;
      if (j < NPT && (NC % NT == 0 || j + 1 < NPT || i < NC)) {
        const uint32_t cy = (uint32_t)i / (uint32_t)EW;
        off[jb] = t0 + (uint32_t)(NT * j * sizeof(S)) + __umul24(cy, skip);
#pragma unroll
        for (int k = 0; k < 9; ++k) d[jb][k] = Codec<S>::load(BufIO<S>::load(rs, off[jb], g.ld_soff[k]));
      }
    }
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int jb = 0; jb < B; ++jb) {
      const int j = j0 + jb, i = t + NT * j;
      if (j < NPT && (NC % NT == 0 || j + 1 < NPT || i < NC)) {
        const int cy = i / EW, cx = i - cy * EW, gx = wx0 + cx, gy = wy0 + cy;
        R Fx, Fy;
        core_force<FM>(a, gx, gy, Fx, Fy);
        if constexpr (FW) {
          fw[i] = Fx;
          fw[EH * EW + i] = Fy;
        }
        R out[9];
        collide_step<R, FM != 0, U>(rt, Fx, Fy, d[jb], out);
        S o[9];
        round_out<S, SR>(out, SR ? (uint32_t)(gy * g.nx + gx) : 0u, key, o);
#pragma unroll
        for (int k = 0; k < 9; ++k) lds[k * PL + i] = o[k];
        if constexpr (KEEP) {
          if (cx >= H && cx < EW - H && cy >= H && cy < EH - H) {
            const __amdgpu_buffer_rsrc_t rk = rsrc(keep, g.lattice_bytes);
#pragma unroll
            for (int k = 0; k < 9; ++k) BufIO<S>::store(rk, off[jb], g.st_soff[k], o[k]);
          }
        }
      }
    }
  }
}

// Middle stage, in place: one step on the window cells at most RING nodes
// outside the tile (the window has an H-node ring).  Every thread pulls and
// collides its cells into registers; after a barrier it writes them back.
// FW: forces from fw.  KEEP: also store the result of the tile's nodes to
// keep (after the write-back; no load follows in the launch but LDS ones).
template <typename S, int FM, bool SR, int EH, int EW, int H, int RING, int NT, bool U, bool FW = false,
          bool KEEP = false, int EHP>
__device__ __forceinline__ void core_stage_lds(const KArgs<typename Codec<S>::R>& a,
                                               const Rates<typename Codec<S>::R>& rt, int wx0, int wy0,
                                               uint32_t key, S (&mid)[9][EHP][EW],
                                               const typename Codec<S>::R* fw = nullptr,
                                               S* __restrict__ keep = nullptr) {
  using R = typename Codec<S>::R;
  constexpr int M = H - RING, RW = EW - 2 * M, RH = EH - 2 * M, NC = RW * RH, NPT = (NC + NT - 1) / NT;
  constexpr int PL = EHP * EW;
  S* lds = &mid[0][0][0];
  const int t = (int)threadIdx.x;
  S o[NPT][9];
  // the cell in the first eight planes and in the last one (beyond the reach
  // of an immediate offset), shared by the pulls and the write-back
  LdsPtr<S> w[NPT], w8[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int i = t + NT * j;
    if (NC % NT == 0 || j + 1 < NPT || i < NC) {
      const int ry = (int)((uint32_t)i / (uint32_t)RW), c = i + ry * (EW - RW) + M * (EW + 1);
      w[j] = lds_cell(lds, c);
      w8[j] = lds_opaque(w[j] + 8 * PL);
      R d[9];
#pragma unroll
      for (int k = 0; k < 8; ++k) d[k] = Codec<S>::load(w[j][k * PL - EY[k] * EW - EX[k]]);
      d[8] = Codec<S>::load(w8[j][-EY[8] * EW - EX[8]]);
      const int gx = wx0 + M + (i - ry * RW), gy = wy0 + M + ry;
      R Fx, Fy;
      if constexpr (FW) {
        Fx = fw[c];
        Fy = fw[EH * EW + c];
      } else {
        core_force<FM>(a, gx, gy, Fx, Fy);
      }
      R out[9];
      collide_step<R, FM != 0, U>(rt, Fx, Fy, d, out);
      round_out<S, SR>(out, SR ? (uint32_t)(gy * a.g.nx + gx) : 0u, key, o[j]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int i = t + NT * j;
    if (NC % NT == 0 || j + 1 < NPT || i < NC) {
#pragma unroll
      for (int k = 0; k < 8; ++k) w[j][k * PL] = o[j][k];
      *w8[j] = o[j][8];
      if constexpr (KEEP) {
        const int ry = (int)((uint32_t)i / (uint32_t)RW), cx = M + (i - ry * RW), cy = M + ry;
        if (cx >= H && cx < EW - H && cy >= H && cy < EH - H) {
          const __amdgpu_buffer_rsrc_t rk = rsrc(keep, a.g.lattice_bytes);
          const uint32_t off = (uint32_t)((wy0 + cy) * a.g.pitch + wx0 + cx) * (uint32_t)sizeof(S);
#pragma unroll
          for (int k = 0; k < 9; ++k) BufIO<S>::store(rk, off, a.g.st_soff[k], o[j][k]);
        }
      }
    }
  }
  __syncthreads();
}

// Last stage: one step on the 64 x TY tile from LDS to HBM.
// EDGE: the tile may reach beyond the domain; such nodes are not stored.
// FW: forces from fw.
template <typename S, int FM, bool SR, int TY, int EH, int EW, int H, int NT, bool U, bool EDGE, bool FW = false,
          int EHP>
__device__ __forceinline__ void core_stage_out(const KArgs<typename Codec<S>::R>& a,
                                               const Rates<typename Codec<S>::R>& rt, int x0, int y0,
                                               uint32_t key, const S (&mid)[9][EHP][EW], S* __restrict__ dst,
                                               const typename Codec<S>::R* fw = nullptr) {
  using R = typename Codec<S>::R;
  constexpr int PL = EHP * EW;
  const Geom& g = a.g;
  const S* lds = &mid[0][0][0];
  const __amdgpu_buffer_rsrc_t wr = rsrc(dst, g.lattice_bytes);
  const int lx = (int)threadIdx.x & 63;
  // byte offset of this thread's first node; each further node lies NT / 64
  // rows below (a workgroup-uniform stride)
  uint32_t off = ((uint32_t)(y0 * g.pitch + x0 + lx) + __umul24(threadIdx.x >> 6, (uint32_t)g.pitch)) *
                 (uint32_t)sizeof(S);
  const uint32_t stride = (uint32_t)(NT / 64) * (uint32_t)g.pitch * (uint32_t)sizeof(S);
  // TY / (NT / 64) full passes over the tile rows, then a partial one
  constexpr int RP = NT / 64, NP = (TY + RP - 1) / RP;
#pragma unroll
  for (int p = 0; p < NP; ++p, off += stride) {
    const int ly = (int)(threadIdx.x >> 6) + RP * p;
    if (TY % RP != 0 && p + 1 == NP && ly >= TY) break;
    const int c = (ly + H) * EW + lx + H;
    const LdsPtr<S> w = lds_cell(lds, c);
    R d[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) d[k] = Codec<S>::load(w[k * PL - EY[k] * EW - EX[k]]);
    R Fx, Fy;
    if constexpr (FW) {
      Fx = fw[c];
      Fy = fw[EH * EW + c];
    } else {
      core_force<FM>(a, x0 + lx, y0 + ly, Fx, Fy);
    }
    R out[9];
    collide_step<R, FM != 0, U>(rt, Fx, Fy, d, out);
    S o[9];
    round_out<S, SR>(out, SR ? (uint32_t)((y0 + ly) * g.nx + x0 + lx) : 0u, key, o);
    if (EDGE && (x0 + lx >= g.nx || y0 + ly >= g.ny)) continue;
    if (g.wb_stores) {
#pragma unroll
      for (int k = 0; k < 9; ++k) BufIO<S>::template store<0>(wr, off, g.st_soff[k], o[k]);
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) BufIO<S>::store(wr, off, g.st_soff[k], o[k]);
    }
  }
}

// Edge tiles in LDS: every window cell c beyond a wall that a node n = c +
// e_k of the window pulls from gets, in plane k, the value n's bounce-back
// takes there (its own opposite population plus the wall term, zero where
// the link crosses two walls), so that the next stage pulls every node as
// an interior node does.  Storage types of at least 32 bits only: the value
// is kept exactly as the pull computes it.  One thread per cell of the (at
// most four) lines of cells just beyond a wall: x_lo, x_hi columns, y_lo,
// y_hi rows.
template <typename S, int EH, int EW, int NT, int EHP>
__device__ __forceinline__ void fill_wall_links(const KArgs<typename Codec<S>::R>& a, int wx0, int wy0,
                                                S (&mid)[9][EHP][EW]) {
  static_assert(sizeof(S) >= 4, "the fill keeps the pulled value in the storage type");
  static_assert(2 * EH + 2 * EW <= NT, "one thread per wall-line cell");
  using R = typename Codec<S>::R;
  const Geom& g = a.g;
  const int t = (int)threadIdx.x;
  if (t >= 2 * EH + 2 * EW) return;
  const int line = t < 2 * EH ? t / EH : 2 + (t - 2 * EH) / EW;
  const int j = t < 2 * EH ? t % EH : (t - 2 * EH) % EW;
  if (!g.wall[line]) return;
  const int cx = line < 2 ? (line == 0 ? -1 : g.nx) - wx0 : j;
  const int cy = line < 2 ? j : (line == 2 ? -1 : g.ny) - wy0;
  if (cx < 0 || cx >= EW || cy < 0 || cy >= EH) return;
#pragma unroll
  for (int k = 1; k < 9; ++k) {
    // the directions that point from the line into the domain
    const bool in = line == 0 ? EX[k] == 1 : line == 1 ? EX[k] == -1 : line == 2 ? EY[k] == 1 : EY[k] == -1;
    const int ncx = cx + EX[k], ncy = cy + EY[k];
    if (!in || ncx < 0 || ncx >= EW || ncy < 0 || ncy >= EH) continue;
    int gx, gy;
    if (!window_node(g, wx0 + ncx, wy0 + ncy, gx, gy)) continue;
    const Edges e = edges(g, gx, gy);
    const bool hx = (EX[k] == 1 && e.wxl) || (EX[k] == -1 && e.wxh);
    const bool hy = (EY[k] == 1 && e.wyl) || (EY[k] == -1 && e.wyh);
    if (!hx && !hy) continue;
    const R add = hx == hy ? R(0)
                           : (hx ? a.wadd[(EX[k] == 1 ? 0 : 1) * 9 + k] : a.wadd[(EY[k] == 1 ? 2 : 3) * 9 + k]);
    mid[k][cy][cx] = Codec<S>::store(Codec<S>::load(mid[OPP[k]][ncy][ncx]) + add);
  }
}

// Rows of a window array in LDS: EH, or up to two more, so that each of the
// nine planes spans a whole number of 256-byte units, if the array still
// fits in 80 KB (two workgroups per CU).  Then no two pulls of a cell lie a
// multiple of 256 bytes apart (none is paired into one two-address LDS read,
// which costs an address add), while a cell's writes to eight planes pair
// up from a single address.
template <typename S, int EH, int EW>
constexpr int lds_rows() {
  for (int r = EH; r <= EH + 2; ++r)
    if (r * EW * (int)sizeof(S) % 256 == 0) return 9 * r * EW * (int)sizeof(S) <= 80 * 1024 ? r : EH;
  return EH;
}

// Tile origin of this workgroup; interior: every pull of the window with an
// H-node ring stays inside the domain (no wall link, no wrap); fast: interior
// and the lattice takes the buffer path.
template <int TY, int H>
__device__ __forceinline__ void tile_origin(const Geom& g, int tiles_x, int& x0, int& y0, bool& interior,
                                            bool& fast) {
  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  x0 = (tile % tiles_x) * 64;
  y0 = (tile / tiles_x) * TY;
  interior = x0 - H - 1 >= 0 && x0 + 64 + H <= g.nx - 1 && y0 - H - 1 >= 0 && y0 + TY + H <= g.ny - 1;
  fast = g.fast && interior;
}

// Two fused steps per launch.  Step n on the tile plus a one-node ring
// (66 x (TY+2) nodes) from HBM into LDS, then step n+1 on the tile from LDS
// to HBM.  HBM traffic per update is halved; the ring costs
// (66 (TY+2)) / (64 TY) - 1 = 16 % (TY = 16) extra collisions, and its loads
// hit L2 (neighbouring tiles run on the same XCD).
template <typename S, int FM, bool SR, int TY, bool U>
__global__ __launch_bounds__(256) void k_step2(KArgs<typename Codec<S>::R> a, const S* __restrict__ src,
                                               S* __restrict__ dst, uint32_t key_a, uint32_t key_b) {
  constexpr int H = 1, EW = 64 + 2 * H, EH = TY + 2 * H;
  __shared__ S mid[9][EH][EW];
  const auto rt = rates(a);
  int x0, y0;
  bool interior, fast;
  tile_origin<TY, H>(a.g, a.g.t2_tiles_x, x0, y0, interior, fast);
  if (fast) {  // workgroup-uniform: an interior tile of a lattice below 4 GiB
    core_stage_hbm<S, FM, SR, EH, EW, 256, U, 2>(a, rt, src, x0 - H, y0 - H, key_a, mid);
    __syncthreads();
    core_stage_out<S, FM, SR, TY, EH, EW, H, 256, U, false>(a, rt, x0, y0, key_b, mid, dst);
    return;
  }
  stage_from_hbm<S, FM, SR, EH, EW, U>(a, rt, src, x0 - H, y0 - H, fast, key_a, mid);
  __syncthreads();
  if (interior)  // workgroup-uniform
    stage_to_hbm<false, S, FM, SR, TY, EH, EW, H, 256, U>(a, rt, x0, y0, key_b, mid, dst);
  else
    stage_to_hbm<true, S, FM, SR, TY, EH, EW, H, 256, U>(a, rt, x0, y0, key_b, mid, dst);
}

// Three fused steps per launch.  Step n on the tile plus a two-node ring
// (68 x (TY+4)) from HBM into LDS, all loads issued up front; step n+1 on the
// tile plus a one-node ring in place in LDS; step n+2 on the tile to HBM.
// HBM traffic per update is a third of a single step's; the rings cost
// (68 (TY+4) + 66 (TY+2) + 64 TY) / (3 * 64 TY) - 1 = 21 % extra collisions
// at TY = 12 (FP32: 39 KB of LDS, four workgroups per CU) and 56 % at TY = 4
// (FP64: 39 KB).
template <typename S, int FM, bool SR, int TY, int NT>
__global__ __launch_bounds__(NT) void k_step3(KArgs<typename Codec<S>::R> a, const S* __restrict__ src,
                                               S* __restrict__ dst, uint32_t key_a, uint32_t key_b,
                                               uint32_t key_c) {
  constexpr int H = 2, EW = 64 + 2 * H, EH = TY + 2 * H;
  __shared__ S mid[9][EH][EW];
  const auto rt = rates(a);
  int x0, y0;
  bool interior, fast;
  tile_origin<TY, H>(a.g, a.g.t3_tiles_x, x0, y0, interior, fast);
  if (fast) {  // workgroup-uniform: an interior tile of a lattice below 4 GiB
    core_stage_hbm<S, FM, SR, EH, EW, NT, false, 3>(a, rt, src, x0 - H, y0 - H, key_a, mid);
    __syncthreads();
    core_stage_lds<S, FM, SR, EH, EW, H, 1, NT, false>(a, rt, x0 - H, y0 - H, key_b, mid);
    core_stage_out<S, FM, SR, TY, EH, EW, H, NT, false, false>(a, rt, x0, y0, key_c, mid, dst);
    return;
  }
  stage_from_hbm_prefetch<S, FM, SR, EH, EW, NT>(a, rt, src, x0 - H, y0 - H, fast, key_a, mid);
  __syncthreads();
  if (interior) {  // workgroup-uniform: every thread meets the same barriers
    stage_in_lds<false, S, FM, SR, EH, EW, H, 1, NT>(a, rt, x0 - H, y0 - H, key_b, mid);
    stage_to_hbm<false, S, FM, SR, TY, EH, EW, H, NT>(a, rt, x0, y0, key_c, mid, dst);
  } else {
    stage_in_lds<true, S, FM, SR, EH, EW, H, 1, NT>(a, rt, x0 - H, y0 - H, key_b, mid);
    stage_to_hbm<true, S, FM, SR, TY, EH, EW, H, NT>(a, rt, x0, y0, key_c, mid, dst);
  }
}

// Four fused steps per launch (FP32 and FP64, every lattice size).  Step n
// on the tile plus a three-node ring (70 x (TY+6)) from HBM into LDS; steps
// n+1 and n+2 in place in LDS on the tile plus a two- and a one-node ring;
// step n+3 on the tile to HBM.  HBM traffic per update is a quarter of a
// single step's; the rings cost
// (70 (TY+6) + 68 (TY+4) + 66 (TY+2) + 64 TY) / (4 * 64 TY) - 1 extra
// collisions: 18 % at TY = 24 (FP32 on large lattices, 74 KB of LDS, 768
// threads), 31 % at TY = 12 and 45 % at TY = 8 (FP64: 69 KB, 512 threads).
// With a force field (FM = 2) on FP32 tiles of up to 12 rows, the first stage
// also keeps the window's force in LDS (fw, 8-10 KB more, still two
// workgroups per CU), so that the later stages load nothing from memory.
// KEEP: the intermediate states n+1, n+2, n+3 of the tile's nodes are also
// stored to keep0, keep1, keep2 (the state-keeping recompute); the later
// stages then issue no load after those stores, which would otherwise wait
// for them (loads and stores share one completion counter).  A KEEP launch
// with dst null stops after keep2, and with keep2 (and dst) null after
// keep1: three or two kept steps (the decision is uniform over the grid).
template <typename S, int FM, bool SR, int TY, int NT, bool U, bool KEEP>
__global__ __launch_bounds__(NT) void k_step4(KArgs<typename Codec<S>::R> a, const S* __restrict__ src,
                                               S* __restrict__ dst, S* __restrict__ keep0, S* __restrict__ keep1,
                                               S* __restrict__ keep2, uint32_t key_a, uint32_t key_b,
                                               uint32_t key_c, uint32_t key_d) {
  using R = typename Codec<S>::R;
  constexpr int H = 3, EW = 64 + 2 * H, EH = TY + 2 * H;
  constexpr bool FW = FM == 2 && sizeof(S) == 4 && TY <= 12;
  __shared__ S mid[9][lds_rows<S, EH, EW>()][EW];
  __shared__ R fwin[FW ? 2 * EH * EW : 1];
  R* fw = FW ? fwin : nullptr;
  const auto rt = rates(a);
  int x0, y0;
  bool interior, fast;
  tile_origin<TY, H>(a.g, a.g.t3_tiles_x, x0, y0, interior, fast);
  // State-keeping launches take the interior path only where no later stage
  // loads from memory after the first kept store: no force field, or its
  // window held in LDS.
  if constexpr (!KEEP || FM != 2 || FW) {
    if (fast) {  // workgroup-uniform: an interior tile of a lattice below 4 GiB
      // (a force field is read at the cells' own, unwrapped nodes: in every
      // stage, or once into fw)
      core_stage_hbm<S, FM, SR, EH, EW, NT, U, 3, FW, KEEP, true>(a, rt, src, x0 - H, y0 - H, key_a, mid, fw,
                                                                  keep0);
      __syncthreads();
      core_stage_lds<S, FM, SR, EH, EW, H, 2, NT, U, FW, KEEP>(a, rt, x0 - H, y0 - H, key_b, mid, fw, keep1);
      if (KEEP && !keep2) return;
      core_stage_lds<S, FM, SR, EH, EW, H, 1, NT, U, FW, KEEP>(a, rt, x0 - H, y0 - H, key_c, mid, fw, keep2);
      if (KEEP && !dst) return;
      core_stage_out<S, FM, SR, TY, EH, EW, H, NT, U, false, FW>(a, rt, x0, y0, key_d, mid, dst, fw);
      return;
    }
  }
  if constexpr (!KEEP && FM != 2) {
    if (TY >= 24 && a.g.fast) {  // workgroup-uniform: an edge tile of a lattice below 4 GiB
      // The first stage pulls through the general gather (walls, wraps);
      // the later ones run as on interior tiles once the cells beyond each
      // wall hold the bounce-back values.  Window cells beyond a wall are
      // computed too (garbage, never pulled by a node: the fill overwrites
      // what a node pulls from them).  Tall tiles only: with 8 or 12 rows
      // (the small lattices, a few workgroups per CU) the three extra
      // barriers cost more than the interior stages save.
      stage_from_hbm_prefetch<S, FM, SR, EH, EW, NT, U>(a, rt, src, x0 - H, y0 - H, false, key_a, mid);
      __syncthreads();
      fill_wall_links<S, EH, EW, NT>(a, x0 - H, y0 - H, mid);
      __syncthreads();
      core_stage_lds<S, FM, SR, EH, EW, H, 2, NT, U>(a, rt, x0 - H, y0 - H, key_b, mid);
      fill_wall_links<S, EH, EW, NT>(a, x0 - H, y0 - H, mid);
      __syncthreads();
      core_stage_lds<S, FM, SR, EH, EW, H, 1, NT, U>(a, rt, x0 - H, y0 - H, key_c, mid);
      fill_wall_links<S, EH, EW, NT>(a, x0 - H, y0 - H, mid);
      __syncthreads();
      core_stage_out<S, FM, SR, TY, EH, EW, H, NT, U, true>(a, rt, x0, y0, key_d, mid, dst);
      return;
    }
  }
  stage_from_hbm_prefetch<S, FM, SR, EH, EW, NT, U, FW, KEEP>(a, rt, src, x0 - H, y0 - H, fast, key_a, mid, fw,
                                                               keep0);
  __syncthreads();
  if (interior) {  // workgroup-uniform: every thread meets the same barriers
    stage_in_lds<false, S, FM, SR, EH, EW, H, 2, NT, U, FW, KEEP>(a, rt, x0 - H, y0 - H, key_b, mid, fw, keep1);
    if (KEEP && !keep2) return;
    stage_in_lds<false, S, FM, SR, EH, EW, H, 1, NT, U, FW, KEEP>(a, rt, x0 - H, y0 - H, key_c, mid, fw, keep2);
    if (KEEP && !dst) return;
    stage_to_hbm<false, S, FM, SR, TY, EH, EW, H, NT, U, FW>(a, rt, x0, y0, key_d, mid, dst, fw);
  } else {
    stage_in_lds<true, S, FM, SR, EH, EW, H, 2, NT, U, FW, KEEP>(a, rt, x0 - H, y0 - H, key_b, mid, fw, keep1);
    if (KEEP && !keep2) return;
    stage_in_lds<true, S, FM, SR, EH, EW, H, 1, NT, U, FW, KEEP>(a, rt, x0 - H, y0 - H, key_c, mid, fw, keep2);
    if (KEEP && !dst) return;
    stage_to_hbm<true, S, FM, SR, TY, EH, EW, H, NT, U, FW>(a, rt, x0, y0, key_d, mid, dst, fw);
  }
}

// Initial state f-bar = f^eq - S/2 (transformed equilibrium with hF = -F/2).
// The FP64 fields are turned into deviations before narrowing to R.
template <typename S>
__global__ __launch_bounds__(256) void k_init(KArgs<typename Codec<S>::R> a, const double* rho,
                                              const double* ux, const double* uy, S* __restrict__ dst) {
  using R = typename Codec<S>::R;
  const NodePos p = node_pos(a.g);
  if (!p.valid) return;
  const int64_t c = (int64_t)p.y * a.g.nx + p.x;
  R Fx, Fy;
  node_force(a, p.x, p.y, Fx, Fy);
  const R drho = (R)(rho[c] - (double)a.rho0);
  const R vx = (R)ux[c], vy = (R)uy[c];
  R Cs[3][3], Y[3][3], v[9];
  equilibrium_cm(a.rho0, drho, vx, vy, R(-0.5) * Fx, R(-0.5) * Fy, Cs);
  populations(vx, vy, Cs, Y, v);
  scatter<S, R>(a.g, a.wadd, dst, p.x, p.y, v, true);
}

// Arbitrary populations f-bar [9][ny][nx] (FP64) -> state.
template <typename S>
__global__ __launch_bounds__(256) void k_set(KArgs<typename Codec<S>::R> a, const double* f,
                                             S* __restrict__ dst) {
  using R = typename Codec<S>::R;
  const NodePos p = node_pos(a.g);
  if (!p.valid) return;
  const int64_t c = (int64_t)p.y * a.g.nx + p.x, n = (int64_t)a.g.nx * a.g.ny;
  R v[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) v[k] = (R)(f[k * n + c] - weight<double>(k) * (double)a.rho0);
  scatter<S, R>(a.g, a.wadd, dst, p.x, p.y, v, true);
}

// State -> pre-collision populations f-bar [9][ny][nx] (FP64).
template <typename S>
__global__ __launch_bounds__(256) void k_get(KArgs<typename Codec<S>::R> a, const S* __restrict__ src,
                                             double* f) {
  using R = typename Codec<S>::R;
  const NodePos p = node_pos(a.g);
  if (!p.valid) return;
  R d[9];
  gather<S, R>(a.g, a.wadd, src, p.x, p.y, d);
  const int64_t c = (int64_t)p.y * a.g.nx + p.x, n = (int64_t)a.g.nx * a.g.ny;
#pragma unroll
  for (int k = 0; k < 9; ++k) f[k * n + c] = (double)d[k] + weight<double>(k) * (double)a.rho0;
}

// Hydrodynamic fields and strain rate of the current state.
template <typename S>
__global__ __launch_bounds__(256) void k_macro(KArgs<typename Codec<S>::R> a, const S* __restrict__ src,
                                               double* rho, double* ux, double* uy, double* sxx,
                                               double* syy, double* sxy) {
  using R = typename Codec<S>::R;
  const NodePos p = node_pos(a.g);
  if (!p.valid) return;
  R d[9];
  gather<S, R>(a.g, a.wadd, src, p.x, p.y, d);
  R Fx, Fy;
  node_force(a, p.x, p.y, Fx, Fy);
  const Rates<R> r = rates(a);
  R M[3][3], X[3][3], C[3][3], drho, inv, vx, vy;
  raw_moments(d, M);
  node_fields(r, M, Fx, Fy, drho, inv, vx, vy);
  const int64_t c = (int64_t)p.y * a.g.nx + p.x;
  if (rho) rho[c] = (double)a.rho0 + (double)drho;
  if (ux) ux[c] = vx;
  if (uy) uy[c] = vy;
  if (sxx || syy || sxy) {
    central(vx, vy, M, X, C);
    // Non-equilibrium second moments of f = f-bar + S/2 (the source has no
    // second-order central moments): f3neq = C_20 + C_02 - 2 rho/3,
    // f4neq = C_20 - C_02, f5neq = C_11, written in deviation form.
    const R u2x = vx * vx, u2y = vy * vy;
    const R f3 = (C[2][0] + C[0][2]) + a.rho0 * (u2x + u2y) - R(2.0 / 3.0) * drho;
    const R f4 = (C[2][0] - C[0][2]) + a.rho0 * (u2x - u2y);
    const R f5 = C[1][1] + a.rho0 * vx * vy;
    const R dxjx = R(-0.75) * (r.w3 * f3 + r.w4 * f4);
    const R dyjy = R(-0.75) * (r.w3 * f3 - r.w4 * f4);
    const R shear = R(-3) * r.w5 * f5;
    if (sxx) sxx[c] = dxjx * inv;
    if (syy) syy[c] = dyjy * inv;
    if (sxy) sxy[c] = R(0.5) * shear * inv;
  }
}

// Sum of v over the 64 lanes of a wavefront: a butterfly over lane distances
// 32, 16, ..., 1 (cross-lane permutes, no LDS, no barrier).  The order is
// fixed, and both partners of each exchange add the same two values, so
// every lane ends with the same, timing-independent sum.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Sums of acc[0..3] over a 256-thread block, in a fixed order: each
// wavefront reduces its lanes, then thread k (< 4) adds the four wavefront
// sums of quantity k.  Returns the block sum of quantity threadIdx.x in
// threads 0..3.
__device__ __forceinline__ double block_sum4(const double acc[4]) {
  __shared__ double wsum[4][4];  // [wavefront][quantity]
  const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) wsum[wave][k] = s;
  }
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x < 4) r = ((wsum[0][threadIdx.x] + wsum[1][threadIdx.x]) + wsum[2][threadIdx.x]) + wsum[3][threadIdx.x];
  return r;
}

// Per-block FP64 partial sums of (rho - rho0, rho ux, rho uy, rho |u|^2 / 2).
// Fixed grid and fixed reduction order: the result does not depend on timing.
template <typename S>
__global__ __launch_bounds__(256) void k_diag_partial(KArgs<typename Codec<S>::R> a, const S* __restrict__ src,
                                                      double* __restrict__ partial) {
  using R = typename Codec<S>::R;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t n = (int64_t)a.g.nx * a.g.ny;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256) {
    const int y = (int)(c / a.g.nx), x = (int)(c - (int64_t)y * a.g.nx);
    R d[9];
    gather<S, R>(a.g, a.wadd, src, x, y, d);
    R Fx, Fy;
    node_force(a, x, y, Fx, Fy);
    R M[3][3], drho, inv, vx, vy;
    raw_moments(d, M);
    node_fields(rates(a), M, Fx, Fy, drho, inv, vx, vy);
    const double rh = (double)a.rho0 + (double)drho;
    acc[0] += (double)drho;
    acc[1] += rh * (double)vx;
    acc[2] += rh * (double)vy;
    acc[3] += 0.5 * rh * ((double)vx * (double)vx + (double)vy * (double)vy);
  }
  const double s = block_sum4(acc);
  if (threadIdx.x < 4) partial[(int64_t)blockIdx.x * 4 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_diag_final(const double* __restrict__ partial, int nblocks,
                                                    double base_mass, double* __restrict__ out) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = (int)threadIdx.x; b < nblocks; b += 256)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += partial[(int64_t)b * 4 + k];
  const double s = block_sum4(acc);
  if (threadIdx.x < 4) out[threadIdx.x] = threadIdx.x == 0 ? base_mass + s : s;
}

// Pull and its transpose for a node whose links all stay inside the domain
// (no wall, no wrap): plane A at (x - e_x, y - e_y).
template <typename S, typename R>
__device__ __forceinline__ void gather_inner(const Geom& g, const S* __restrict__ src, int x, int y, R d[9]) {
  const int64_t c = (int64_t)y * g.pitch + x;
#pragma unroll
  for (int k = 0; k < 9; ++k) d[k] = Codec<S>::load(src[(int64_t)k * g.plane + c - EY[k] * g.pitch - EX[k]]);
}

template <typename R>
__device__ __forceinline__ void scatter_inner(const Geom& g, R* __restrict__ dst, int x, int y, const R v[9]) {
  const int64_t c = (int64_t)y * g.pitch + x;
#pragma unroll
  for (int k = 0; k < 9; ++k) dst[(int64_t)k * g.plane + c - EY[k] * g.pitch - EX[k]] = v[k];
}

// Adjoint of one step: mu_out = J^T mu_in, grad_force += dL/dF.
template <typename S>
__global__ __launch_bounds__(256) void k_adjoint_step(KArgs<typename Codec<S>::R> a, const S* __restrict__ prev,
                                                      const typename Codec<S>::R* __restrict__ mu_in,
                                                      typename Codec<S>::R* __restrict__ mu_out,
                                                      typename Codec<S>::R* __restrict__ grad_force) {
  using R = typename Codec<S>::R;
  const NodePos p = node_pos(a.g);
  if (!p.valid) return;
  // a node off the domain's edge rows and columns has no wall link and no
  // wrap: plain offsets (only edge wavefronts diverge)
  const bool inner = p.x >= 1 && p.x <= a.g.nx - 2 && p.y >= 1 && p.y <= a.g.ny - 2;
  R d[9];
  if (inner) gather_inner<S, R>(a.g, prev, p.x, p.y, d);
  else gather<S, R>(a.g, a.wadd, prev, p.x, p.y, d);
  R Fx, Fy;
  node_force(a, p.x, p.y, Fx, Fy);
  const int64_t c = (int64_t)p.y * a.g.pitch + p.x;
  R mu[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) mu[k] = mu_in[(int64_t)k * a.g.plane + c];
  R nu[9], aFx = R(0), aFy = R(0);
  collide_adj(rates(a), Fx, Fy, d, mu, nu, aFx, aFy);
  // Reverse streaming: the transpose of the gather permutation.
  if (inner) scatter_inner<R>(a.g, mu_out, p.x, p.y, nu);
  else scatter<R, R>(a.g, a.wadd, mu_out, p.x, p.y, nu, false);
  if (grad_force) {
    const int64_t cf = (int64_t)p.y * a.g.nx + p.x;
    grad_force[cf] += aFx;
    grad_force[(int64_t)a.g.nx * a.g.ny + cf] += aFy;
  }
}

// One workgroup's two adjoint steps (see k_adjoint_step2).  WALLS = false:
// every node the tile touches and its neighbours lie inside the domain, so
// the pulls, the reverse streaming and the window lookups need no wall or
// wrap handling.
template <bool WALLS, typename S, int TY, int NT>
__device__ __forceinline__ void adjoint_pair_tile(const KArgs<typename Codec<S>::R>& a, int x0, int y0,
                                                  const S* __restrict__ prev_a, const S* __restrict__ prev_b,
                                                  const typename Codec<S>::R* __restrict__ mu_in,
                                                  typename Codec<S>::R* __restrict__ mu_out,
                                                  typename Codec<S>::R* __restrict__ grad_force,
                                                  typename Codec<S>::R (&mid)[9][TY + 4][68],
                                                  typename Codec<S>::R (&aF1)[2][TY][64]) {
  using R = typename Codec<S>::R;
  constexpr int H = 2, EW = 64 + 2 * H, EH = TY + 2 * H;
  const Geom& g = a.g;
  const Rates<R> r = rates(a);
  const int wx0 = x0 - H, wy0 = y0 - H;
  // ---- stage 1: adjoint of step n on the tile and a one-node ring
  constexpr int RW = EW - 2, RH = EH - 2;
  for (int i = (int)threadIdx.x; i < RW * RH; i += NT) {
    const int cx = 1 + i % RW, cy = 1 + i / RW;
    int gx = wx0 + cx, gy = wy0 + cy;
    if (WALLS && !window_node(g, wx0 + cx, wy0 + cy, gx, gy)) continue;
    R d[9];
    if constexpr (WALLS) gather<S, R>(g, a.wadd, prev_a, gx, gy, d);
    else gather_inner<S, R>(g, prev_a, gx, gy, d);
    R Fx, Fy;
    node_force(a, gx, gy, Fx, Fy);
    const int64_t c = (int64_t)gy * g.pitch + gx;
    R mu[9], nu[9], ax = R(0), ay = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) mu[k] = mu_in[(int64_t)k * g.plane + c];
    collide_adj(r, Fx, Fy, d, mu, nu, ax, ay);
    if constexpr (WALLS) {
      const Edges e = edges(g, gx, gy);
#define LBM_SCATTER_WIN(A)                                                        \
      {                                                                           \
        constexpr int sx = EX[A], sy = EY[A];                                     \
        const bool hx = (sx == 1 && e.wxl) || (sx == -1 && e.wxh);                \
        const bool hy = (sy == 1 && e.wyl) || (sy == -1 && e.wyh);                \
        if (hx || hy) mid[OPP[A]][cy][cx] = nu[A];                                \
        else mid[A][cy - sy][cx - sx] = nu[A];                                    \
      }
      LBM_SCATTER_WIN(0) LBM_SCATTER_WIN(1) LBM_SCATTER_WIN(2) LBM_SCATTER_WIN(3) LBM_SCATTER_WIN(4)
      LBM_SCATTER_WIN(5) LBM_SCATTER_WIN(6) LBM_SCATTER_WIN(7) LBM_SCATTER_WIN(8)
#undef LBM_SCATTER_WIN
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) mid[k][cy - EY[k]][cx - EX[k]] = nu[k];
    }
    if (cx >= H && cx < H + 64 && cy >= H && cy < H + TY) {
      aF1[0][cy - H][cx - H] = ax;
      aF1[1][cy - H][cx - H] = ay;
    }
  }
  __syncthreads();
  // ---- stage 2: adjoint of step n-1 on the tile
  const int lx = (int)threadIdx.x & 63;
  for (int ly = (int)threadIdx.x >> 6; ly < TY; ly += NT / 64) {
    const int gx = x0 + lx, gy = y0 + ly;
    if (gx >= g.nx || gy >= g.ny) continue;
    R d[9];
    if constexpr (WALLS) gather<S, R>(g, a.wadd, prev_b, gx, gy, d);
    else gather_inner<S, R>(g, prev_b, gx, gy, d);
    R Fx, Fy;
    node_force(a, gx, gy, Fx, Fy);
    R mu[9], nu[9], ax = R(0), ay = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) mu[k] = mid[k][ly + H][lx + H];
    collide_adj(r, Fx, Fy, d, mu, nu, ax, ay);
    if constexpr (WALLS) scatter<R, R>(g, a.wadd, mu_out, gx, gy, nu, false);
    else scatter_inner<R>(g, mu_out, gx, gy, nu);
    if (grad_force) {
      const int64_t cf = (int64_t)gy * g.nx + gx;
      grad_force[cf] = (grad_force[cf] + aF1[0][ly][lx]) + ax;
      const int64_t cg = (int64_t)g.nx * g.ny + cf;
      grad_force[cg] = (grad_force[cg] + aF1[1][ly][lx]) + ay;
    }
  }
}

// Two adjoint steps per launch, newest first: the cotangent mu_in of state
// n+1 goes back through step n (state n in prev_a) and then step n-1 (state
// n-1 in prev_b) to the cotangent mu_out of state n-1.  A workgroup owns a
// 64 x TY tile.  Stage 1 runs the adjoint of step n on the tile and a one-node
// ring and scatters its reverse-streamed result into an LDS window (the
// cotangent of state n, which each window position receives from exactly one
// cell).  Stage 2 runs the adjoint of step n-1 on the tile from that window
// and scatters to mu_out.  grad_force receives (g + aF_n) + aF_(n-1): the
// same sums in the same order as two single adjoint steps, so the result is
// bit-for-bit theirs.  HBM per node and two steps: mu in and out, both
// states, force and gradient once -- 168 B (FP32) against 264.
template <typename S, int TY, int NT>
__global__ __launch_bounds__(NT) void k_adjoint_step2(KArgs<typename Codec<S>::R> a, const S* __restrict__ prev_a,
                                                       const S* __restrict__ prev_b,
                                                       const typename Codec<S>::R* __restrict__ mu_in,
                                                       typename Codec<S>::R* __restrict__ mu_out,
                                                       typename Codec<S>::R* __restrict__ grad_force) {
  static_assert(NT % 64 == 0 && NT <= 1024, "whole wavefronts");
  using R = typename Codec<S>::R;
  __shared__ R mid[9][TY + 4][68];  // cotangent of state n on the window (two-node ring)
  __shared__ R aF1[2][TY][64];      // stage 1 force cotangents of the tile
  const Geom& g = a.g;
  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int x0 = (tile % g.t2_tiles_x) * 64, y0 = (tile / g.t2_tiles_x) * TY;
  // stage 1 nodes span [x0 - 1, x0 + 64] x [y0 - 1, y0 + TY]; none on the
  // domain's edge rows or columns means no wall link and no wrap anywhere
  const bool inner = x0 >= 2 && x0 + 66 <= g.nx && y0 >= 2 && y0 + TY + 2 <= g.ny;
  if (inner)  // workgroup-uniform
    adjoint_pair_tile<false, S, TY, NT>(a, x0, y0, prev_a, prev_b, mu_in, mu_out, grad_force, mid, aF1);
  else
    adjoint_pair_tile<true, S, TY, NT>(a, x0, y0, prev_a, prev_b, mu_in, mu_out, grad_force, mid, aF1);
}

// Four adjoint steps per launch (FP32 lattices of kAdjoint4MinNodes nodes or
// more, 64 x TY tiles with TY = 8 or 16).  The window array holds the cotangents of a 64 x TY tile and a
// four-node ring.  Stage 1 runs the adjoint of step n on the cells within
// three nodes of the tile (mu_in from HBM) and scatters its reverse-streamed
// result into the window, as the pair's first stage does.  Stages 2 and 3
// run the adjoints of steps n-1 and n-2 on the cells within two and one
// nodes, in place: every thread reads its cells' nine cotangents and
// computes, then after a barrier scatters.  A window position receives each
// plane from exactly one cell, and the positions a stage reads get all nine
// planes from the stage before.  Stage 4 runs the adjoint of step n-3 on the
// tile and scatters to mu_out.  The force gradient of a tile node is carried
// in acc as ((g + a_n) + a_(n-1)) + a_(n-2), then + a_(n-3): the sums of four
// single adjoint steps in their order, so the launch equals them bit for
// bit.  HBM per node and four steps: four states 144 B, cotangent in and out
// 72, force 8, gradient read and written 16 -- 240 B against 336 for two
// pair launches.

// Reverse streaming of cell (cx, cy) of node (gx, gy) into the window.
template <bool WALLS, typename R, int EH, int EW>
__device__ __forceinline__ void adjoint_win_scatter(const Geom& g, R (&win)[9][EH][EW], int cx, int cy, int gx,
                                                    int gy, const R nu[9]) {
  if constexpr (WALLS) {
    const Edges e = edges(g, gx, gy);
#define LBM_SCATTER_WIN4(A)                                                       \
    {                                                                             \
      constexpr int sx = EX[A], sy = EY[A];                                       \
      const bool hx = (sx == 1 && e.wxl) || (sx == -1 && e.wxh);                  \
      const bool hy = (sy == 1 && e.wyl) || (sy == -1 && e.wyh);                  \
      if (hx || hy) win[OPP[A]][cy][cx] = nu[A];                                  \
      else win[A][cy - sy][cx - sx] = nu[A];                                      \
    }
    LBM_SCATTER_WIN4(0) LBM_SCATTER_WIN4(1) LBM_SCATTER_WIN4(2) LBM_SCATTER_WIN4(3) LBM_SCATTER_WIN4(4)
    LBM_SCATTER_WIN4(5) LBM_SCATTER_WIN4(6) LBM_SCATTER_WIN4(7) LBM_SCATTER_WIN4(8)
#undef LBM_SCATTER_WIN4
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) win[k][cy - EY[k]][cx - EX[k]] = nu[k];
  }
}

// One in-place middle stage of the four-step adjoint: the cells at least M
// cells inside the window (M = 2: within two nodes of the tile; M = 3: one).
template <bool WALLS, typename S, int TY, int NT, int M>
__device__ __forceinline__ void adjoint_quad_mid(const KArgs<typename Codec<S>::R>& a,
                                                 const Rates<typename Codec<S>::R>& r, int x0, int y0,
                                                 const S* __restrict__ prev, bool grad,
                                                 typename Codec<S>::R (&win)[9][TY + 8][72],
                                                 typename Codec<S>::R (&acc)[2][TY][64]) {
  using R = typename Codec<S>::R;
  constexpr int H = 4, EW = 72, EH = TY + 8, RW = EW - 2 * M, RH = EH - 2 * M, NC = RW * RH;
  constexpr int NPT = (NC + NT - 1) / NT;
  const Geom& g = a.g;
  const int wx0 = x0 - H, wy0 = y0 - H;
  R nu[NPT][9];
  int gxs[NPT], gys[NPT];
  bool live[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int i = (int)threadIdx.x + NT * j;
    const int cx = M + i % RW, cy = M + i / RW;
    int gx = wx0 + cx, gy = wy0 + cy;
    live[j] = i < NC;
    if (WALLS && live[j]) live[j] = window_node(g, wx0 + cx, wy0 + cy, gx, gy);
    gxs[j] = gx;
    gys[j] = gy;
    if (!live[j]) continue;
    R d[9];
    if constexpr (WALLS) gather<S, R>(g, a.wadd, prev, gx, gy, d);
    else gather_inner<S, R>(g, prev, gx, gy, d);
    R Fx, Fy;
    node_force(a, gx, gy, Fx, Fy);
    R mu[9], ax = R(0), ay = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) mu[k] = win[k][cy][cx];
    collide_adj(r, Fx, Fy, d, mu, nu[j], ax, ay);
    const int lx = cx - H, ly = cy - H;
    if (grad && lx >= 0 && lx < 64 && ly >= 0 && ly < TY) {
      acc[0][ly][lx] = acc[0][ly][lx] + ax;
      acc[1][ly][lx] = acc[1][ly][lx] + ay;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    if (!live[j]) continue;
    const int i = (int)threadIdx.x + NT * j;
    const int cx = M + i % RW, cy = M + i / RW;
    adjoint_win_scatter<WALLS, R, EH, EW>(g, win, cx, cy, gxs[j], gys[j], nu[j]);
  }
  __syncthreads();
}

template <bool WALLS, typename S, int TY, int NT>
__device__ __forceinline__ void adjoint_quad_tile(const KArgs<typename Codec<S>::R>& a, int x0, int y0,
                                                  const S* __restrict__ prev_a, const S* __restrict__ prev_b,
                                                  const S* __restrict__ prev_c, const S* __restrict__ prev_d,
                                                  const typename Codec<S>::R* __restrict__ mu_in,
                                                  typename Codec<S>::R* __restrict__ mu_out,
                                                  typename Codec<S>::R* __restrict__ grad_force,
                                                  typename Codec<S>::R (&win)[9][TY + 8][72],
                                                  typename Codec<S>::R (&acc)[2][TY][64]) {
  using R = typename Codec<S>::R;
  constexpr int H = 4, EW = 72, EH = TY + 8;
  const Geom& g = a.g;
  const Rates<R> r = rates(a);
  const int wx0 = x0 - H, wy0 = y0 - H;
  const bool grad = grad_force != nullptr;
  // ---- stage 1: adjoint of step n on the cells within three nodes of the tile
  {
    constexpr int RW = EW - 2, RH = EH - 2;
    for (int i = (int)threadIdx.x; i < RW * RH; i += NT) {
      const int cx = 1 + i % RW, cy = 1 + i / RW;
      int gx = wx0 + cx, gy = wy0 + cy;
      if (WALLS && !window_node(g, wx0 + cx, wy0 + cy, gx, gy)) continue;
      R d[9];
      if constexpr (WALLS) gather<S, R>(g, a.wadd, prev_a, gx, gy, d);
      else gather_inner<S, R>(g, prev_a, gx, gy, d);
      R Fx, Fy;
      node_force(a, gx, gy, Fx, Fy);
      const int64_t c = (int64_t)gy * g.pitch + gx;
      R mu[9], nu[9], ax = R(0), ay = R(0);
#pragma unroll
      for (int k = 0; k < 9; ++k) mu[k] = mu_in[(int64_t)k * g.plane + c];
      collide_adj(r, Fx, Fy, d, mu, nu, ax, ay);
      adjoint_win_scatter<WALLS, R, EH, EW>(g, win, cx, cy, gx, gy, nu);
      const int lx = cx - H, ly = cy - H;
      if (grad && lx >= 0 && lx < 64 && ly >= 0 && ly < TY && x0 + lx < g.nx && y0 + ly < g.ny) {
        const int64_t cf = (int64_t)gy * g.nx + gx;
        acc[0][ly][lx] = grad_force[cf] + ax;
        acc[1][ly][lx] = grad_force[(int64_t)g.nx * g.ny + cf] + ay;
      }
    }
  }
  __syncthreads();
  // ---- stages 2 and 3, in place
  adjoint_quad_mid<WALLS, S, TY, NT, 2>(a, r, x0, y0, prev_b, grad, win, acc);
  adjoint_quad_mid<WALLS, S, TY, NT, 3>(a, r, x0, y0, prev_c, grad, win, acc);
  // ---- stage 4: adjoint of step n-3 on the tile, to mu_out
  const int lx = (int)threadIdx.x & 63;
  for (int ly = (int)threadIdx.x >> 6; ly < TY; ly += NT / 64) {
    const int gx = x0 + lx, gy = y0 + ly;
    if (gx >= g.nx || gy >= g.ny) continue;
    R d[9];
    if constexpr (WALLS) gather<S, R>(g, a.wadd, prev_d, gx, gy, d);
    else gather_inner<S, R>(g, prev_d, gx, gy, d);
    R Fx, Fy;
    node_force(a, gx, gy, Fx, Fy);
    R mu[9], nu[9], ax = R(0), ay = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) mu[k] = win[k][ly + H][lx + H];
    collide_adj(r, Fx, Fy, d, mu, nu, ax, ay);
    if constexpr (WALLS) scatter<R, R>(g, a.wadd, mu_out, gx, gy, nu, false);
    else scatter_inner<R>(g, mu_out, gx, gy, nu);
    if (grad) {
      const int64_t cf = (int64_t)gy * g.nx + gx;
      grad_force[cf] = acc[0][ly][lx] + ax;
      grad_force[(int64_t)g.nx * g.ny + cf] = acc[1][ly][lx] + ay;
    }
  }
}

template <typename S, int TY, int NT>
__global__ __launch_bounds__(NT) void k_adjoint_step4(KArgs<typename Codec<S>::R> a, const S* __restrict__ prev_a,
                                                      const S* __restrict__ prev_b, const S* __restrict__ prev_c,
                                                      const S* __restrict__ prev_d,
                                                      const typename Codec<S>::R* __restrict__ mu_in,
                                                      typename Codec<S>::R* __restrict__ mu_out,
                                                      typename Codec<S>::R* __restrict__ grad_force) {
  static_assert(NT % 64 == 0 && NT <= 1024, "whole wavefronts");
  using R = typename Codec<S>::R;
  __shared__ R win[9][TY + 8][72];  // cotangents on the window (four-node ring)
  __shared__ R acc[2][TY][64];      // running force gradient of the tile's nodes
  const Geom& g = a.g;
  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int x0 = (tile % g.t2_tiles_x) * 64, y0 = (tile / g.t2_tiles_x) * TY;
  // stage 1 nodes span [x0 - 3, x0 + 66] x [y0 - 3, y0 + TY + 2]; none on the
  // domain's edge rows or columns means no wall link and no wrap anywhere
  const bool inner = x0 >= 4 && x0 + 68 <= g.nx && y0 >= 4 && y0 + TY + 4 <= g.ny;
  if (inner)  // workgroup-uniform
    adjoint_quad_tile<false, S, TY, NT>(a, x0, y0, prev_a, prev_b, prev_c, prev_d, mu_in, mu_out, grad_force, win,
                                        acc);
  else
    adjoint_quad_tile<true, S, TY, NT>(a, x0, y0, prev_a, prev_b, prev_c, prev_d, mu_in, mu_out, grad_force, win,
                                       acc);
}

// Adjoint of the macroscopic map rho, u at lattice lat.
template <typename S>
__global__ __launch_bounds__(256) void k_adjoint_macro(KArgs<typename Codec<S>::R> a, const S* __restrict__ lat,
                                                       const typename Codec<S>::R* g_rho,
                                                       const typename Codec<S>::R* g_ux,
                                                       const typename Codec<S>::R* g_uy,
                                                       typename Codec<S>::R* __restrict__ mu_out,
                                                       typename Codec<S>::R* __restrict__ grad_force) {
  using R = typename Codec<S>::R;
  const NodePos p = node_pos(a.g);
  if (!p.valid) return;
  R d[9];
  gather<S, R>(a.g, a.wadd, lat, p.x, p.y, d);
  R Fx, Fy;
  node_force(a, p.x, p.y, Fx, Fy);
  R M[3][3], drho, inv, vx, vy;
  raw_moments(d, M);
  node_fields(rates(a), M, Fx, Fy, drho, inv, vx, vy);
  const int64_t cf = (int64_t)p.y * a.g.nx + p.x;
  const R gr = g_rho ? g_rho[cf] : R(0);
  const R gx = g_ux ? g_ux[cf] : R(0);
  const R gy = g_uy ? g_uy[cf] : R(0);
  // d rho / d f_a = 1;  d u / d f_a = (e_a - u)/rho;  d u / d F = 1/(2 rho).
  R nu[9];
#pragma unroll
  for (int k = 0; k < 9; ++k)
    nu[k] = gr + (gx * (R(EX[k]) - vx) + gy * (R(EY[k]) - vy)) * inv;
  scatter<R, R>(a.g, a.wadd, mu_out, p.x, p.y, nu, false);
  if (grad_force) {
    grad_force[cf] += R(0.5) * gx * inv;
    grad_force[(int64_t)a.g.nx * a.g.ny + cf] += R(0.5) * gy * inv;
  }
}

// Adjoint of the initial state map (rho, u, F) -> lattice.
template <typename S>
__global__ __launch_bounds__(256) void k_adjoint_init(KArgs<typename Codec<S>::R> a,
                                                      const double* rho, const double* ux,
                                                      const double* uy,
                                                      const typename Codec<S>::R* __restrict__ mu0,
                                                      typename Codec<S>::R* g_rho,
                                                      typename Codec<S>::R* g_ux,
                                                      typename Codec<S>::R* g_uy,
                                                      typename Codec<S>::R* __restrict__ grad_force) {
  using R = typename Codec<S>::R;
  const NodePos p = node_pos(a.g);
  if (!p.valid) return;
  const int64_t cf = (int64_t)p.y * a.g.nx + p.x;
  // The initial lattice is the scatter of v(x); its cotangent w.r.t. v is the
  // gather of mu0 (no wall term: it is additive).
  R av[9];
  {
    const Edges e = edges(a.g, p.x, p.y);
    R add;
#define LBM_GATHER_MU(A) av[A] = mu0[link_src<A, R>(a.g, e, p.x, p.y, a.wadd, add)];
    LBM_GATHER_MU(0) LBM_GATHER_MU(1) LBM_GATHER_MU(2) LBM_GATHER_MU(3) LBM_GATHER_MU(4)
    LBM_GATHER_MU(5) LBM_GATHER_MU(6) LBM_GATHER_MU(7) LBM_GATHER_MU(8)
#undef LBM_GATHER_MU
  }
  R Fx, Fy;
  node_force(a, p.x, p.y, Fx, Fy);
  const R vx = (R)ux[cf], vy = (R)uy[cf];
  R Cs[3][3], Y[3][3], v[9];
  equilibrium_cm(a.rho0, (R)(rho[cf] - (double)a.rho0), vx, vy, R(-0.5) * Fx, R(-0.5) * Fy, Cs);
  populations(vx, vy, Cs, Y, v);
  R aCs[3][3], aux = R(0), auy = R(0), adrho = R(0), ahx = R(0), ahy = R(0);
  populations_T(vx, vy, Cs, Y, av, aCs, aux, auy);
  equilibrium_cm_T(a.rho0, vx, vy, aCs, adrho, aux, auy, ahx, ahy);
  if (g_rho) g_rho[cf] = adrho;
  if (g_ux) g_ux[cf] = aux;
  if (g_uy) g_uy[cf] = auy;
  if (grad_force) {
    grad_force[cf] += R(-0.5) * ahx;
    grad_force[(int64_t)a.g.nx * a.g.ny + cf] += R(-0.5) * ahy;
  }
}

// ---------------------------------------------------------------- launchers

static dim3 grid_of(const Geom& g) { return dim3((unsigned)(g.tiles_x * g.tiles_y)); }

#define LBM_DISPATCH(storage, CALL)                                 \
  switch (storage) {                                                \
    case 0: { using S = double; CALL; }                             \
    case 1: { using S = float; CALL; }                              \
    case 2: { using S = _Float16; CALL; }                           \
    case 3: { using S = __bf16; CALL; }                             \
    default: return hipErrorInvalidValue;                           \
  }

// The KArgs arrive as the double or float instantiation; the dispatcher
// picks the one matching the storage mode's compute real.
template <typename S>
static const KArgs<typename Codec<S>::R>& args_of(const KArgsAny& a) {
  if constexpr (sizeof(typename Codec<S>::R) == 8) return a.d; else return a.f;
}

template <typename S, bool SR>
static hipError_t launch_step_fm(const KArgs<typename Codec<S>::R>& k, const void* src, void* dst, uint32_t key,
                                 hipStream_t st) {
  const int fm = k.force ? 2 : ((k.fx != 0 || k.fy != 0) ? 1 : 0);
  const dim3 grid = grid_of(k.g);
  if (fm == 0) hipLaunchKernelGGL((k_step<S, 0, SR>), grid, dim3(256), 0, st, k, (const S*)src, (S*)dst, key);
  else if (fm == 1) hipLaunchKernelGGL((k_step<S, 1, SR>), grid, dim3(256), 0, st, k, (const S*)src, (S*)dst, key);
  else hipLaunchKernelGGL((k_step<S, 2, SR>), grid, dim3(256), 0, st, k, (const S*)src, (S*)dst, key);
  return hipGetLastError();
}

// omega_6 = omega_7 = omega_8 = 1 (the paper's default): the collision leaves
// out their multiplies (exact identities), same results bit for bit.
template <typename R>
static bool unit678(const KArgs<R>& k) {
  return k.w[3] == R(1) && k.w[4] == R(1) && k.w[5] == R(1);
}

template <typename S, bool SR, int TY, bool U>
static void launch_step2_tyu(const KArgs<typename Codec<S>::R>& k, const void* src, void* dst, uint32_t ka,
                             uint32_t kb, hipStream_t st) {
  const int fm = k.force ? 2 : ((k.fx != 0 || k.fy != 0) ? 1 : 0);
  const dim3 grid((unsigned)(k.g.t2_tiles_x * k.g.t2_tiles_y));
  if (fm == 0)
    hipLaunchKernelGGL((k_step2<S, 0, SR, TY, U>), grid, dim3(256), 0, st, k, (const S*)src, (S*)dst, ka, kb);
  else if (fm == 1)
    hipLaunchKernelGGL((k_step2<S, 1, SR, TY, U>), grid, dim3(256), 0, st, k, (const S*)src, (S*)dst, ka, kb);
  else
    hipLaunchKernelGGL((k_step2<S, 2, SR, TY, U>), grid, dim3(256), 0, st, k, (const S*)src, (S*)dst, ka, kb);
}

template <typename S, bool SR, int TY>
static void launch_step2_ty(const KArgs<typename Codec<S>::R>& k, const void* src, void* dst, uint32_t ka,
                            uint32_t kb, hipStream_t st) {
  if (unit678(k))
    launch_step2_tyu<S, SR, TY, true>(k, src, dst, ka, kb, st);
  else
    launch_step2_tyu<S, SR, TY, false>(k, src, dst, ka, kb, st);
}

// Tile height 8 (FP64 always, the other storages on small lattices) or 16.
template <typename S, bool SR>
static hipError_t launch_step2_fm(const KArgs<typename Codec<S>::R>& k, const void* src, void* dst, uint32_t ka,
                                  uint32_t kb, hipStream_t st) {
  if (k.g.t2_ty == 8)
    launch_step2_ty<S, SR, 8>(k, src, dst, ka, kb, st);
  else if (sizeof(S) != 8 && k.g.t2_ty == 16)
    launch_step2_ty<S, SR, sizeof(S) == 8 ? 8 : 16>(k, src, dst, ka, kb, st);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_step2(const KArgsAny& a, const void* src, void* dst, uint32_t key_a, uint32_t key_b,
                        hipStream_t st) {
  switch (a.storage) {
    case 0: return launch_step2_fm<double, false>(a.d, src, dst, key_a, key_b, st);
    case 1: return launch_step2_fm<float, false>(a.f, src, dst, key_a, key_b, st);
    case 2:
      return a.stochastic ? launch_step2_fm<_Float16, true>(a.f, src, dst, key_a, key_b, st)
                          : launch_step2_fm<_Float16, false>(a.f, src, dst, key_a, key_b, st);
    case 3:
      return a.stochastic ? launch_step2_fm<__bf16, true>(a.f, src, dst, key_a, key_b, st)
                          : launch_step2_fm<__bf16, false>(a.f, src, dst, key_a, key_b, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename S, bool SR, int TY, int NT>
static hipError_t launch_step3_fm(const KArgs<typename Codec<S>::R>& k, const void* src, void* dst, uint32_t ka,
                                  uint32_t kb, uint32_t kc, hipStream_t st) {
  const int fm = k.force ? 2 : ((k.fx != 0 || k.fy != 0) ? 1 : 0);
  const dim3 grid((unsigned)(k.g.t3_tiles_x * k.g.t3_tiles_y));
  if (k.g.t3_ty != TY || k.g.t3_threads != NT) return hipErrorInvalidValue;
  if (fm == 0)
    hipLaunchKernelGGL((k_step3<S, 0, SR, TY, NT>), grid, dim3(NT), 0, st, k, (const S*)src, (S*)dst, ka, kb, kc);
  else if (fm == 1)
    hipLaunchKernelGGL((k_step3<S, 1, SR, TY, NT>), grid, dim3(NT), 0, st, k, (const S*)src, (S*)dst, ka, kb, kc);
  else
    hipLaunchKernelGGL((k_step3<S, 2, SR, TY, NT>), grid, dim3(NT), 0, st, k, (const S*)src, (S*)dst, ka, kb, kc);
  return hipGetLastError();
}

hipError_t launch_step3(const KArgsAny& a, const void* src, void* dst, uint32_t key_a, uint32_t key_b,
                        uint32_t key_c, hipStream_t st) {
  // FP64 and FP32 only: the 16-bit modes run two steps per launch.
  switch (a.storage) {
    case 0:
      return a.d.g.t3_threads == kStep3ThreadsF64Large
                 ? launch_step3_fm<double, false, kStep3TyF64Large, kStep3ThreadsF64Large>(a.d, src, dst, key_a,
                                                                                          key_b, key_c, st)
                 : launch_step3_fm<double, false, kStep3TyF64, kStep3ThreadsF64>(a.d, src, dst, key_a, key_b,
                                                                                key_c, st);
    case 1:
      return launch_step3_fm<float, false, kStep3TyF32, kStep3ThreadsF32>(a.f, src, dst, key_a, key_b, key_c, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename S, int TY, int NT, bool U, bool KEEP>
static hipError_t launch_step4_fmu(const KArgs<typename Codec<S>::R>& k, const void* src, void* dst, void* k0,
                                   void* k1, void* k2, uint32_t ka, uint32_t kb, uint32_t kc, uint32_t kd,
                                   hipStream_t st) {
  const int fm = k.force ? 2 : ((k.fx != 0 || k.fy != 0) ? 1 : 0);
  const dim3 grid((unsigned)(k.g.t3_tiles_x * ((k.g.ny + TY - 1) / TY)));
  if (fm == 0)
    hipLaunchKernelGGL((k_step4<S, 0, false, TY, NT, U, KEEP>), grid, dim3(NT), 0, st, k, (const S*)src, (S*)dst,
                       (S*)k0, (S*)k1, (S*)k2, ka, kb, kc, kd);
  else if (fm == 1)
    hipLaunchKernelGGL((k_step4<S, 1, false, TY, NT, U, KEEP>), grid, dim3(NT), 0, st, k, (const S*)src, (S*)dst,
                       (S*)k0, (S*)k1, (S*)k2, ka, kb, kc, kd);
  else
    hipLaunchKernelGGL((k_step4<S, 2, false, TY, NT, U, KEEP>), grid, dim3(NT), 0, st, k, (const S*)src, (S*)dst,
                       (S*)k0, (S*)k1, (S*)k2, ka, kb, kc, kd);
  return hipGetLastError();
}

template <typename S, int TY, int NT, bool KEEP = false>
static hipError_t launch_step4_fm(const KArgs<typename Codec<S>::R>& k, const void* src, void* dst, void* k0,
                                  void* k1, void* k2, uint32_t ka, uint32_t kb, uint32_t kc, uint32_t kd,
                                  hipStream_t st) {
  return unit678(k) ? launch_step4_fmu<S, TY, NT, true, KEEP>(k, src, dst, k0, k1, k2, ka, kb, kc, kd, st)
                    : launch_step4_fmu<S, TY, NT, false, KEEP>(k, src, dst, k0, k1, k2, ka, kb, kc, kd, st);
}

hipError_t launch_step4(const KArgsAny& a, const void* src, void* dst, uint32_t key_a, uint32_t key_b,
                        uint32_t key_c, uint32_t key_d, hipStream_t st) {
  switch (a.storage) {
    case 0:
      return launch_step4_fm<double, kStep4TyF64, kStep4ThreadsF64>(a.d, src, dst, nullptr, nullptr, nullptr, key_a,
                                                                    key_b, key_c, key_d, st);
    case 1:
      if (a.f.g.t4_ty == kStep4TyF32Small)
        return launch_step4_fm<float, kStep4TyF32Small, kStep4ThreadsF32Small>(a.f, src, dst, nullptr, nullptr,
                                                                               nullptr, key_a, key_b, key_c, key_d,
                                                                               st);
      if (a.f.g.t4_ty == kStep4TyF32Mid)
        return launch_step4_fm<float, kStep4TyF32Mid, kStep4ThreadsF32Mid>(a.f, src, dst, nullptr, nullptr, nullptr,
                                                                           key_a, key_b, key_c, key_d, st);
      return launch_step4_fm<float, kStep4TyF32, kStep4ThreadsF32>(a.f, src, dst, nullptr, nullptr, nullptr, key_a,
                                                                   key_b, key_c, key_d, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step4_keep(const KArgsAny& a, const void* src, void* keep0, void* keep1, void* keep2, void* dst,
                             uint32_t key_a, uint32_t key_b, uint32_t key_c, uint32_t key_d, hipStream_t st) {
  if (a.storage != 1 || !keep0 || !keep1 || (!keep2 && dst)) return hipErrorInvalidValue;
  if (a.f.g.t4_ty == kStep4TyF32Small)
    return launch_step4_fm<float, kStep4TyF32Small, kStep4ThreadsF32Small, true>(a.f, src, dst, keep0, keep1, keep2,
                                                                                 key_a, key_b, key_c, key_d, st);
  if (a.f.g.t4_ty == kStep4TyF32Mid)
    return launch_step4_fm<float, kStep4TyF32Mid, kStep4ThreadsF32Mid, true>(a.f, src, dst, keep0, keep1, keep2,
                                                                             key_a, key_b, key_c, key_d, st);
  return launch_step4_fm<float, kStep4TyF32, kStep4ThreadsF32, true>(a.f, src, dst, keep0, keep1, keep2, key_a, key_b,
                                                                     key_c, key_d, st);
}

hipError_t launch_step(const KArgsAny& a, const void* src, void* dst, uint32_t key, hipStream_t st) {
  switch (a.storage) {
    case 0: return launch_step_fm<double, false>(a.d, src, dst, key, st);
    case 1: return launch_step_fm<float, false>(a.f, src, dst, key, st);
    case 2:
      return a.stochastic ? launch_step_fm<_Float16, true>(a.f, src, dst, key, st)
                          : launch_step_fm<_Float16, false>(a.f, src, dst, key, st);
    case 3:
      return a.stochastic ? launch_step_fm<__bf16, true>(a.f, src, dst, key, st)
                          : launch_step_fm<__bf16, false>(a.f, src, dst, key, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init(const KArgsAny& a, const void* rho, const void* ux, const void* uy, void* dst,
                       hipStream_t st) {
  LBM_DISPATCH(a.storage, {
    hipLaunchKernelGGL(k_init<S>, grid_of(a.g()), dim3(256), 0, st, args_of<S>(a), (const double*)rho,
                       (const double*)ux, (const double*)uy, (S*)dst);
    return hipGetLastError();
  })
}

hipError_t launch_set(const KArgsAny& a, const void* f, void* dst, hipStream_t st) {
  LBM_DISPATCH(a.storage, {
    hipLaunchKernelGGL(k_set<S>, grid_of(a.g()), dim3(256), 0, st, args_of<S>(a), (const double*)f, (S*)dst);
    return hipGetLastError();
  })
}

hipError_t launch_get(const KArgsAny& a, const void* src, void* f, hipStream_t st) {
  LBM_DISPATCH(a.storage, {
    hipLaunchKernelGGL(k_get<S>, grid_of(a.g()), dim3(256), 0, st, args_of<S>(a), (const S*)src, (double*)f);
    return hipGetLastError();
  })
}

hipError_t launch_macro(const KArgsAny& a, const void* src, void* rho, void* ux, void* uy, void* sxx,
                        void* syy, void* sxy, hipStream_t st) {
  LBM_DISPATCH(a.storage, {
    hipLaunchKernelGGL(k_macro<S>, grid_of(a.g()), dim3(256), 0, st, args_of<S>(a), (const S*)src,
                       (double*)rho, (double*)ux, (double*)uy, (double*)sxx, (double*)syy, (double*)sxy);
    return hipGetLastError();
  })
}

hipError_t launch_diag(const KArgsAny& a, const void* src, double* partial, int nblocks, double base_mass,
                       double* out, hipStream_t st) {
  LBM_DISPATCH(a.storage, {
    hipLaunchKernelGGL(k_diag_partial<S>, dim3((unsigned)nblocks), dim3(256), 0, st, args_of<S>(a),
                       (const S*)src, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, st, (const double*)partial, nblocks,
                       base_mass, out);
    return hipGetLastError();
  })
}

hipError_t launch_adjoint_step2(const KArgsAny& a, const void* prev_a, const void* prev_b, const void* mu_in,
                                void* mu_out, void* grad_force, hipStream_t st) {
  const Geom& g = a.g();
  switch (a.storage) {
    case 0: {
      constexpr int TY = kAdjoint2TyF64, NT = kAdjoint2ThreadsF64;
      const dim3 grid((unsigned)(g.t2_tiles_x * ((g.ny + TY - 1) / TY)));
      hipLaunchKernelGGL((k_adjoint_step2<double, TY, NT>), grid, dim3(NT), 0, st, a.d, (const double*)prev_a,
                         (const double*)prev_b, (const double*)mu_in, (double*)mu_out, (double*)grad_force);
      return hipGetLastError();
    }
    case 1: {
      if ((int64_t)g.nx * g.ny <= kAdjoint2SmallMaxNodes) {
        constexpr int TY = kAdjoint2TyF32Small, NT = kAdjoint2ThreadsF32Small;
        const dim3 grid((unsigned)(g.t2_tiles_x * ((g.ny + TY - 1) / TY)));
        hipLaunchKernelGGL((k_adjoint_step2<float, TY, NT>), grid, dim3(NT), 0, st, a.f, (const float*)prev_a,
                           (const float*)prev_b, (const float*)mu_in, (float*)mu_out, (float*)grad_force);
        return hipGetLastError();
      }
      constexpr int TY = kAdjoint2TyF32, NT = kAdjoint2ThreadsF32;
      const dim3 grid((unsigned)(g.t2_tiles_x * ((g.ny + TY - 1) / TY)));
      hipLaunchKernelGGL((k_adjoint_step2<float, TY, NT>), grid, dim3(NT), 0, st, a.f, (const float*)prev_a,
                         (const float*)prev_b, (const float*)mu_in, (float*)mu_out, (float*)grad_force);
      return hipGetLastError();
    }
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint_step4(const KArgsAny& a, const void* prev_a, const void* prev_b, const void* prev_c,
                                const void* prev_d, const void* mu_in, void* mu_out, void* grad_force,
                                hipStream_t st) {
  const Geom& g = a.g();
  if (a.storage != 1) return hipErrorInvalidValue;
  if ((int64_t)g.nx * g.ny <= kAdjoint2SmallMaxNodes) {
    constexpr int TY = kAdjoint4TySmall, NT = kAdjoint4Threads;
    const dim3 grid((unsigned)(g.t2_tiles_x * ((g.ny + TY - 1) / TY)));
    hipLaunchKernelGGL((k_adjoint_step4<float, TY, NT>), grid, dim3(NT), 0, st, a.f, (const float*)prev_a,
                       (const float*)prev_b, (const float*)prev_c, (const float*)prev_d, (const float*)mu_in,
                       (float*)mu_out, (float*)grad_force);
    return hipGetLastError();
  }
  constexpr int TY = kAdjoint4Ty, NT = kAdjoint4Threads;
  const dim3 grid((unsigned)(g.t2_tiles_x * ((g.ny + TY - 1) / TY)));
  hipLaunchKernelGGL((k_adjoint_step4<float, TY, NT>), grid, dim3(NT), 0, st, a.f, (const float*)prev_a,
                     (const float*)prev_b, (const float*)prev_c, (const float*)prev_d, (const float*)mu_in,
                     (float*)mu_out, (float*)grad_force);
  return hipGetLastError();
}

hipError_t launch_adjoint_step(const KArgsAny& a, const void* prev, const void* mu_in, void* mu_out,
                               void* grad_force, hipStream_t st) {
  switch (a.storage) {
    case 0:
      hipLaunchKernelGGL(k_adjoint_step<double>, grid_of(a.g()), dim3(256), 0, st, a.d, (const double*)prev,
                         (const double*)mu_in, (double*)mu_out, (double*)grad_force);
      return hipGetLastError();
    case 1:
      hipLaunchKernelGGL(k_adjoint_step<float>, grid_of(a.g()), dim3(256), 0, st, a.f, (const float*)prev,
                         (const float*)mu_in, (float*)mu_out, (float*)grad_force);
      return hipGetLastError();
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint_macro(const KArgsAny& a, const void* lat, const void* g_rho, const void* g_ux,
                                const void* g_uy, void* mu_out, void* grad_force, hipStream_t st) {
  switch (a.storage) {
    case 0:
      hipLaunchKernelGGL(k_adjoint_macro<double>, grid_of(a.g()), dim3(256), 0, st, a.d, (const double*)lat,
                         (const double*)g_rho, (const double*)g_ux, (const double*)g_uy, (double*)mu_out,
                         (double*)grad_force);
      return hipGetLastError();
    case 1:
      hipLaunchKernelGGL(k_adjoint_macro<float>, grid_of(a.g()), dim3(256), 0, st, a.f, (const float*)lat,
                         (const float*)g_rho, (const float*)g_ux, (const float*)g_uy, (float*)mu_out,
                         (float*)grad_force);
      return hipGetLastError();
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint_init(const KArgsAny& a, const void* rho, const void* ux, const void* uy,
                               const void* mu0, void* g_rho, void* g_ux, void* g_uy, void* grad_force,
                               hipStream_t st) {
  switch (a.storage) {
    case 0:
      hipLaunchKernelGGL(k_adjoint_init<double>, grid_of(a.g()), dim3(256), 0, st, a.d, (const double*)rho,
                         (const double*)ux, (const double*)uy, (const double*)mu0, (double*)g_rho,
                         (double*)g_ux, (double*)g_uy, (double*)grad_force);
      return hipGetLastError();
    case 1:
      hipLaunchKernelGGL(k_adjoint_init<float>, grid_of(a.g()), dim3(256), 0, st, a.f, (const double*)rho,
                         (const double*)ux, (const double*)uy, (const float*)mu0, (float*)g_rho,
                         (float*)g_ux, (float*)g_uy, (float*)grad_force);
      return hipGetLastError();
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace lbm
