// Input gradient of the T-MLP output by reverse accumulation (gfx950):
// kernel templates, instantiated once per activation (adjoint_sine.hip,
// adjoint_finer.hip).
//
// For a point with exit depth d the output is y_d = t_1 + ... + t_d (Eq. 2),
// t_j the tail of layer j (linear, or the product form of Eq. 3), and
// h_j = sigma(z_j), z_j = W_j h_{j-1} + b_j, with sigma the SIREN sine
// sin(omega_j z) or the FINER sine sin(omega_j (|z| + 1) z). With
// g_j = dy/dh_j and delta_j = (sigma'(z_j) / omega_j) * g_j (the cosine
// cos(omega_j z_j), or (2|z_j| + 1) cos(omega_j (|z_j| + 1) z_j)):
//     g_d     = dt_d/dh_d,
//     g_{j-1} = (omega_j W_j)^T delta_j + dt_{j-1}/dh_{j-1},
//     dy/dx   = (omega_1 W_1)^T delta_1,
// with dt/dh = u1 a0 + u0 a1 for a tail (a0.h + c0)(a1.h + c1), u0 and u1 its
// two factors (a linear tail is stored with a1 = 0, c1 = 1).
//
// One workgroup handles a tile of points of equal depth, as the forward
// kernel does:
//  * forward recompute: the same MFMA chain, and each block's epilogue also
//    writes sigma'(z) / omega of its units to a per-workgroup global stash (in
//    the lanes' own accumulator layout, 16-bit for BF16/FP16, FP32 for
//    FP32) and each layer's tail factors u0, u1 to LDS;
//  * backward: g_{j-1} is one MFMA product per output block with the
//    transposed weights (packed with the same permuted K order, so the
//    packed delta_j registers are the B operand as they stand); the
//    epilogue adds the tail term, multiplies by the stashed cosine and packs
//    delta_{j-1}; at layer 1 it accumulates dy/dx on the vector ALU instead.
//    The tile's exit layer keeps its cosines in registers and layer 1's are
//    recomputed from the point, so only layers 2..d-1 use the stash; at
//    widths >= 256 each block's cosines are copied into LDS one block ahead,
//    with the next weight chunk.

#pragma once

#include "mfma_common.h"

namespace sand {

namespace {

using namespace mfma;

// Bytes of stashed cosines per lane per output block.
template <int PREC>
constexpr int stash_lane_bytes() {
  return PREC == PREC_FP32 ? 16 : 32;
}

// MFMA chain over NS K steps: step s multiplies A tile tile(s) of an LDS
// slot (64 lanes x VB bytes per tile) by the B operand b(s). The A operands
// are read PF steps ahead of their MFMA; the scheduling groups keep the
// compiler from hoisting more reads (each holds registers) or sinking each
// read to its MFMA (which would make every MFMA wait a full LDS round trip).
template <int PREC, int NS, int PF, class Tile, class BOp>
__device__ __forceinline__ typename Tr<PREC>::Acc mma_chain(const char* slot, int lane, Tile tile,
                                                            BOp b) {
  using T = Tr<PREC>;
  using V = typename T::V;
  constexpr int P = NS < PF ? NS : PF;
  auto a_of = [&](int s) -> V { return *(const V*)(slot + (tile(s) * 64 + lane) * T::VB); };
  V a[P];
#pragma unroll
  for (int s = 0; s < P; ++s) a[s] = a_of(s);
  typename T::Acc acc = {};
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const V cur = a[s % P];
    if (s + P < NS) a[s % P] = a_of(s + P);
    acc = T::mma(cur, b(s), acc);
  }
  __builtin_amdgcn_sched_group_barrier(0x100, P, 0);
#pragma unroll
  for (int s = 0; s < NS - P; ++s) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  }
  __builtin_amdgcn_sched_group_barrier(0x008, P, 0);
  return acc;
}

// This lane's position in its wavefront, computed afresh at each use (an asm
// statement is neither merged with another nor hoisted out of a loop), so
// that neither it nor the thread index is kept live, or spilled, across the
// tile loop.
__device__ __forceinline__ int lane_now() {
  int l;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
  return l;
}

// load_chunk from byte src_off (uniform) of a buffer resource: each lane's
// source is a 32-bit offset, so no 64-bit per-lane address stays live
// between chunks (this kernel's register budget is tighter than the forward
// kernel's). FRESH: a piece's offset is split into its uniform part
// (src_off + q KB, a scalar register) and the lane's 16 bytes from
// lane_now(), so that nothing lane-derived stays live at all; it costs a few
// vector instructions per copy and pays only where the kernel spills (the
// FINER 16-bit forms: their per-piece offsets were spilled and reloaded,
// with a full wait, right after the copy was issued).
template <int BYTES, int NW, bool FRESH>
__device__ __forceinline__ void load_chunk_buf(__amdgpu_buffer_rsrc_t src, int src_off, char* dst,
                                               int wave, int lane) {
  constexpr int NP = BYTES / 16;
  constexpr int WL = (NP + 64 * NW - 1) / (64 * NW);
  if constexpr (FRESH) lane = lane_now();
#pragma unroll
  for (int k = 0; k < WL; ++k) {
    const int q = k * NW + wave;
    const int piece = q * 64 + lane;
    if (q * 64 < NP && piece < NP) {
      if constexpr (FRESH)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(src, lds_ptr(dst + q * 1024), 16, lane * 16,
                                                 src_off + q * 1024, 0, 0);
      else
        __builtin_amdgcn_raw_ptr_buffer_load_lds(src, lds_ptr(dst + q * 1024), 16, piece * 16,
                                                 src_off, 0, 0);
    }
  }
}

// Whether an instantiation's weight copies use load_chunk_buf's FRESH form.
template <int PREC, int ACT>
constexpr bool kFreshCopy = ACT == ACT_FINER && PREC != PREC_FP32;

// Fourth word of a raw buffer resource on gfx9 (32-bit data format).
constexpr int kBufferWord3 = 0x00020000;

// A operands read ahead of their MFMA in the adjoint's product chains.
constexpr int kAdjPF = 4;

// Workgroup barrier without the release fence of __syncthreads, which waits
// for every global store of the wavefront (here: the block's stash stores,
// which no other wavefront reads). Callers have awaited what other
// wavefronts read after it (a weight chunk's LDS copy, with wait_chunk); the
// memory clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void barrier_no_fence() { asm volatile("s_barrier" ::: "memory"); }

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Tr<PREC>::lane_sum with the exchange addresses formed from lane_now()
// (ds_bpermute reads lane address / 4).
template <int PREC>
__device__ __forceinline__ float adj_lane_sum(float v) {
  const int a = lane_now() << 2;
  if constexpr (PREC == PREC_FP32)
    v += __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(a ^ 64, __builtin_bit_cast(int, v)));
  return v + __builtin_bit_cast(float,
                                __builtin_amdgcn_ds_bpermute(a ^ 128, __builtin_bit_cast(int, v)));
}

// A 64-bit value that is the same in every lane, in scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A wavefront's stash: cosines of (layer j, block rb) at byte offset
// ((j - 1) RB + rb) 64 LB + lane LB of its region (LB bytes per lane). It is
// addressed as a buffer (uniform base and block offset in scalar registers,
// the lane's offset in one vector register) so that no per-lane 64-bit
// address of any block has to stay live across the tile loop.
struct Stash {
  __amdgpu_buffer_rsrc_t rsrc;
  int voff;   // lane * LB
};

template <int PREC>
__device__ __forceinline__ void stash_put(const Stash& st, int soff,
                                          const float (&c)[Tr<PREC>::NR]) {
  if constexpr (PREC == PREC_FP32) {
    const f32x4 v = f32x4{c[0], c[1], c[2], c[3]};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, v), st.rsrc, st.voff, soff, 0);
  } else {
    using V = typename Tr<PREC>::V;
    V lo, hi;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      lo[k] = (typename Tr<PREC>::E)c[k];
      hi[k] = (typename Tr<PREC>::E)c[8 + k];
    }
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, lo), st.rsrc, st.voff, soff, 0);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, hi), st.rsrc, st.voff + 16,
                                           soff, 0);
  }
}

template <int PREC>
__device__ __forceinline__ void stash_get(const Stash& st, int soff, float (&c)[Tr<PREC>::NR]) {
  if constexpr (PREC == PREC_FP32) {
    const f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(st.rsrc, st.voff,
                                                                                    soff, 0));
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = v[k];
  } else {
    using V = typename Tr<PREC>::V;
    const V lo = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(st.rsrc, st.voff, soff, 0));
    const V hi =
        __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(st.rsrc, st.voff + 16, soff, 0));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      c[k] = (float)lo[k];
      c[8 + k] = (float)hi[k];
    }
  }
}

// Copy a wavefront's stashed cosines of one block (64 LB bytes from byte
// soff of its stash) into LDS at dst, without passing through registers,
// as the weight chunks are copied: the backward requests the next block's
// cosines with the next weight chunk and reads them from LDS (stash_lds),
// so their global-memory latency is covered by a block of work.
template <int PREC>
__device__ __forceinline__ void stash_fetch(const Stash& st, int soff, char* dst, int lane) {
  constexpr int SB = 64 * stash_lane_bytes<PREC>();
#pragma unroll
  for (int k = 0; k < SB / 1024; ++k)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(st.rsrc, lds_ptr(dst + k * 1024), 16, lane * 16,
                                             soff + k * 1024, 0, 0);
}

// The lane's cosines of a block copied by stash_fetch (the stash's own
// layout: the lane's LB bytes at lane LB).
template <int PREC>
__device__ __forceinline__ void stash_lds(const char* src, int lane, float (&c)[Tr<PREC>::NR]) {
  if constexpr (PREC == PREC_FP32) {
    const f32x4 v = *(const f32x4*)(src + lane * 16);
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = v[k];
  } else {
    using V = typename Tr<PREC>::V;
    const V lo = *(const V*)(src + lane * 32), hi = *(const V*)(src + lane * 32 + 16);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      c[k] = (float)lo[k];
      c[8 + k] = (float)hi[k];
    }
  }
}

template <int PREC, int KS>
__device__ __forceinline__ void pin_out(const typename Tr<PREC>::V (&out)[KS], int rb) {
  using T = Tr<PREC>;
  if constexpr (T::VB == 16) {
    asm volatile("" ::"v"(out[2 * rb]), "v"(out[2 * rb + 1]));
  } else {
#pragma unroll
    for (int e = 0; e < T::NR; ++e) asm volatile("" ::"v"(out[4 * rb + e]));
  }
}

// What a forward epilogue keeps of cos of the sine argument: FE_STASH
// writes it to the stash (and the packed activations to out); FE_NONE keeps
// nothing (layer 1 of a deeper tile: the backward recomputes it); FE_REGS
// packs the cosines into out instead of the activations (the tile's last
// layer, whose activations feed nothing and whose cosines the backward
// needs first).
// FE_F32 hands the cosines back in FP32 (cs_out) and packs nothing (layer 1
// of a depth-1 tile in the 16-bit precisions: its cosines are the whole
// gradient, so they are kept unrounded).
enum FwdKeep { FE_STASH, FE_NONE, FE_REGS, FE_F32 };

// Forward epilogue: sine, tail partial sums, and the slopes sigma'(z) / omega
// ("cosines") as FwdKeep says.
template <int PREC, int KS, int KEEP, int ACT>
__device__ __forceinline__ void fwd_epilogue(float kf, const char* tails, int g, int rb,
                                             const typename Tr<PREC>::Acc& acc,
                                             typename Tr<PREC>::V (&out)[KS], float& s0,
                                             float& s1, const Stash& stash, int soff,
                                             float* cs_out = nullptr) {
  using T = Tr<PREC>;
  float h[T::NR], cs[T::NR];
#pragma unroll
  for (int i = 0; i < T::NR / 4; ++i) {
    const f32x4 ta = T::tail_vec(tails, 0, i, g);
    const f32x4 tb = T::tail_vec(tails, 1, i, g);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = 4 * i + k;
      const float arg = act_arg<ACT>(acc[e], kf);
      h[e] = __builtin_amdgcn_sinf(arg);
      if constexpr (KEEP != FE_NONE) cs[e] = act_slope<ACT>(acc[e], arg, kf);
      s0 = fmaf(ta[k], h[e], s0);
      s1 = fmaf(tb[k], h[e], s1);
    }
    // one group of four at a time: computing every element's factors first
    // would hold them all in registers at once
    if constexpr (ACT == ACT_FINER) __builtin_amdgcn_sched_barrier(0);
  }
  if constexpr (KEEP == FE_F32) {
#pragma unroll
    for (int e = 0; e < T::NR; ++e) cs_out[e] = cs[e];
    asm volatile("" ::"v"(s0), "v"(s1));
    return;
  } else if constexpr (KEEP == FE_REGS) {
    T::template store<KS>(out, rb, cs);
  } else {
    T::template store<KS>(out, rb, h);
    if constexpr (KEEP == FE_STASH) stash_put<PREC>(stash, soff, cs);
  }
  asm volatile("" ::"v"(s0), "v"(s1));
  pin_out<PREC, KS>(out, rb);
}

// The NR cosines of output block rb that fwd_epilogue<FE_REGS> packed into
// act, as FP32 (the same 16-bit rounding as the stash).
template <int PREC, int KS>
__device__ __forceinline__ void cos_from_regs(const typename Tr<PREC>::V (&act)[KS], int rb,
                                              float (&cs)[Tr<PREC>::NR]) {
  using T = Tr<PREC>;
  if constexpr (T::VB == 16) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cs[k] = (float)act[2 * rb][k];
      cs[8 + k] = (float)act[2 * rb + 1][k];
    }
  } else {
#pragma unroll
    for (int e = 0; e < T::NR; ++e) cs[e] = act[4 * rb + e];
  }
}

// Backward epilogue of one block: delta' = cos * (acc + u1 a0 + u0 a1).
// Packs it for the next backward product, or (at layer 1) accumulates the
// input gradient with the (omega_1 W_1) rows from w1t.
template <int PREC, int KS>
__device__ __forceinline__ void bwd_epilogue(const float* tails, int tstride, int g, int rb,
                                             const typename Tr<PREC>::Acc& acc, float u0,
                                             float u1, const float (&cs)[Tr<PREC>::NR],
                                             typename Tr<PREC>::V (&out)[KS], bool last,
                                             const char* w1t, float (&gx)[3]) {
  using T = Tr<PREC>;
  float dl[T::NR];
#pragma unroll
  for (int i = 0; i < T::NR / 4; ++i) {
    const int row = T::tail_row(i, g);
    const f32x4 ta = *(const f32x4*)(tails + row);
    const f32x4 tb = *(const f32x4*)(tails + tstride + row);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = 4 * i + k;
      dl[e] = cs[e] * fmaf(u1, ta[k], fmaf(u0, tb[k], acc[e]));
    }
  }
  if (last) {
#pragma unroll
    for (int i = 0; i < T::NR / 4; ++i) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int e = 4 * i + k;
        const int u = T::BM * rb + T::tail_row(i, g) + k;
        const f32x4 w = *(const f32x4*)(w1t + u * 16);
        gx[0] = fmaf(dl[e], w[0], gx[0]);
        gx[1] = fmaf(dl[e], w[1], gx[1]);
        gx[2] = fmaf(dl[e], w[2], gx[2]);
      }
    }
    asm volatile("" ::"v"(gx[0]), "v"(gx[1]), "v"(gx[2]));
  } else {
    T::template store<KS>(out, rb, dl);
    pin_out<PREC, KS>(out, rb);
  }
}

template <int PREC, int WP>
struct AdjCfg {
  using C = Cfg<PREC, WP>;
  static constexpr int SLOT = C::CH > C::CH_B ? C::CH : C::CH_B;
  static constexpr int W1T = WP * 16;
  static constexpr int UST = C::NW * kMaxLayers * Tr<PREC>::NQ * 2 * 4;   // tail factors
  // backward: two blocks of each wavefront's stashed cosines (stash_fetch),
  // at widths >= 256 only, where one workgroup per CU is the limit anyway
  // (narrower layers keep two or more workgroups per CU and read the stash
  // directly)
  static constexpr bool LSTASH = WP >= 256;
  static constexpr int SB = 64 * stash_lane_bytes<PREC>();
  static constexpr int SST = LSTASH ? 2 * C::NW * SB : 0;
  static constexpr int LDS = 2 * SLOT + C::L1B + W1T + UST + SST;
  // stash bytes per wavefront and layer
  static constexpr int STASH_WL = C::RB * 64 * stash_lane_bytes<PREC>();
};

// Offset of the cosines of (layer j, block rb) in a wavefront's stash.
template <int PREC, int WP>
__device__ __forceinline__ int stash_at(int j, int rb) {
  return ((j - 1) * Cfg<PREC, WP>::RB + rb) * 64 * stash_lane_bytes<PREC>();
}

// One forward hidden layer j: in -> out, cosines stashed, or (last: the
// tile's exit layer) packed into out; returns the tail partial sums.
template <int PREC, int WP, int ACT>
__device__ __forceinline__ void adj_fwd_layer(float kf, __amdgpu_buffer_rsrc_t hidden, char* ring,
                                              int wave,
                                              int lane, int g, int& c, int nc, int j, bool last,
                                              const typename Tr<PREC>::V (&in)[Cfg<PREC, WP>::KS],
                                              typename Tr<PREC>::V (&out)[Cfg<PREC, WP>::KS],
                                              const Stash& stash, float& s0, float& s1) {
  using C = Cfg<PREC, WP>;
  using A = AdjCfg<PREC, WP>;
  using T = Tr<PREC>;
  using V = typename T::V;
  s0 = s1 = 0.0f;
  // lane-derived values (addresses, the constant bias operand) are rebuilt
  // per layer from opaque copies rather than kept live across the tile loop
  asm volatile("" : "+v"(lane), "+v"(g));
  const V bb = T::bias_b(g);
#pragma unroll
  for (int rb = 0; rb < C::RB; ++rb) {
    const bool pre = c + 1 < nc;
    if (pre)
      load_chunk_buf<C::CH, C::NW, kFreshCopy<PREC, ACT>>(
          hidden, (c + 1) * C::CH, ring + ((c + 1) & 1) * A::SLOT, wave, lane);
    const char* slot = ring + (c & 1) * A::SLOT;
    // bias step first, then the K steps: the forward kernel's order, so the
    // recomputed values are bit-identical to a plain query (the bias tile
    // follows the KS weight tiles in the chunk)
    const typename T::Acc acc = mma_chain<PREC, C::KS + 1, kAdjPF>(
        slot, lane, [](int s) { return s == 0 ? C::KS : s - 1; },
        [&](int s) -> V { return s == 0 ? bb : in[s - 1]; });
    // The next chunk's copy must have landed before the barrier below. The
    // wait comes before this block's epilogue, so that it covers the previous
    // block's stash stores (long done) rather than this one's. A count that
    // left stores outstanding is not safe: vector-memory loads and stores are
    // not counted down in issue order with respect to each other, so it can
    // pass with a chunk piece still in flight (seen as rare wrong gradients
    // of the FINER FP32 form at width 352).
    if (pre) wait_chunk();
    if (last)
      fwd_epilogue<PREC, C::KS, FE_REGS, ACT>(kf, slot + C::TAIL_OFF, g, rb, acc, out, s0, s1,
                                              stash, 0);
    else
      fwd_epilogue<PREC, C::KS, FE_STASH, ACT>(kf, slot + C::TAIL_OFF, g, rb, acc, out, s0, s1,
                                               stash, stash_at<PREC, WP>(j, rb));
    barrier_no_fence();
    ++c;
  }
}

// One backward layer j (j >= 2): in = delta'_j -> out = delta'_{j-1} with
// the stashed cosines of layer j - 1, or (FIRST: j == 2) the input gradient,
// with layer 1's cosines recomputed from the point (l1: the layer-1 chunks
// in LDS; its product is four inputs deep) and `out` untouched. The two
// forms are separate copies so that neither holds the other's registers.
template <int PREC, int WP, int ACT, bool FIRST>
__device__ __forceinline__ void adj_bwd_layer(float kf1, __amdgpu_buffer_rsrc_t bwd, char* ring,
                                              int wave,
                                              int lane, int g, int& c, int nc, int d, int j,
                                              const char* l1, float px, float py, float pz,
                                              const typename Tr<PREC>::V (&in)[Cfg<PREC, WP>::KS],
                                              typename Tr<PREC>::V (&out)[Cfg<PREC, WP>::KS],
                                              const Stash& stash, char* sst, float v0, float v1,
                                              const char* w1t,
                                              float (&gx)[3]) {
  using C = Cfg<PREC, WP>;
  using A = AdjCfg<PREC, WP>;
  using T = Tr<PREC>;
  using V = typename T::V;
  asm volatile("" : "+v"(lane), "+v"(g));   // see adj_fwd_layer
#pragma unroll
  for (int rb = 0; rb < C::RB; ++rb) {
    const bool pre = c + 1 < nc;
    if (pre) {
      // chunks run layer d, d-1, ..., 2 and blocks 0..RB-1 within a layer
      const int c1 = c + 1;
      const int jn = d - c1 / C::RB, rn = c1 % C::RB;
      load_chunk_buf<C::CH_B, C::NW, kFreshCopy<PREC, ACT>>(
          bwd, ((jn - 2) * C::RB + rn) * C::CH_B, ring + (c1 & 1) * A::SLOT, wave, lane);
      // and that block's cosines of layer jn - 1 (none for layer 2, whose
      // layer-1 cosines are recomputed)
      if (A::LSTASH && jn >= 3)
        stash_fetch<PREC>(stash, stash_at<PREC, WP>(jn - 1, rn), sst + (c1 & 1) * C::NW * A::SB,
                          lane);
    }
    const char* slot = ring + (c & 1) * A::SLOT;
    const typename T::Acc acc = mma_chain<PREC, C::KS, kAdjPF>(
        slot, lane, [](int s) { return s; }, [&](int s) -> V { return in[s]; });
    float cs[T::NR];
    if constexpr (FIRST) {
      typename T::Acc z = {};
#pragma unroll
      for (int st = 0; st < T::L1S; ++st)
        z = T::mma1(T::l1_a(l1 + rb * C::L1C, st, lane), T::l1_b(st, g, px, py, pz), z);
#pragma unroll
      for (int e = 0; e < T::NR; ++e) cs[e] = act_slope<ACT>(z[e], act_arg<ACT>(z[e], kf1), kf1);
    } else {
      if constexpr (A::LSTASH)
        stash_lds<PREC>(sst + (c & 1) * C::NW * A::SB, lane, cs);
      else
        stash_get<PREC>(stash, stash_at<PREC, WP>(j - 1, rb), cs);
    }
    bwd_epilogue<PREC, C::KS>((const float*)(slot + C::TAIL_OFF_B), T::BM, g, rb, acc, v0, v1, cs,
                              out, FIRST, w1t, gx);
    if (pre) wait_chunk();
    __syncthreads();
    ++c;
  }
}

template <int PREC, int WP, int ACT>
__global__ __launch_bounds__((Cfg<PREC, WP>::NT)) void k_adjoint(AdjointArgs a) {
  using C = Cfg<PREC, WP>;
  using A = AdjCfg<PREC, WP>;
  using T = Tr<PREC>;
  using V = typename T::V;
  constexpr int Q = C::Q;
  constexpr int NQ = T::NQ;
  __shared__ __attribute__((aligned(16))) char lds[A::LDS];
  char* ring = lds;
  char* l1 = lds + 2 * A::SLOT;
  char* w1t = l1 + C::L1B;
  float* ust = (float*)(w1t + A::W1T);
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const QueryArgs& q = a.q;

  __shared__ Plan splan;   // the plan's bucket bounds, read per tile
  // Each lane's point (x, y, z, dy) and index for the current tile, parked in
  // LDS between layer 1 and their next use (layer 1 again, at the end of the
  // backward pass; the stores at the end of the tile), so that they hold no
  // registers through the hidden layers.
  __shared__ f32x4 spt[C::NT];
  __shared__ int32_t sgi[C::NT];
  for (int i = tid; i < C::L1B / 16; i += C::NT) ((uint4*)l1)[i] = ((const uint4*)q.m.chunks)[i];
  for (int i = tid; i < A::W1T / 16; i += C::NT) ((uint4*)w1t)[i] = ((const uint4*)a.w1t)[i];
  if (q.plan)
    for (int i = tid; i < (int)(sizeof(Plan) / 8); i += C::NT)
      ((int64_t*)&splan)[i] = ((const int64_t*)q.plan)[i];
  __syncthreads();
  const int L = q.m.L;
  // the weight streams as buffers (uniform bases, 32-bit lane offsets)
  const __amdgpu_buffer_rsrc_t hidden = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char*>(q.m.chunks + C::L1B), 0, (L - 1) * C::RB * C::CH, kBufferWord3);
  const __amdgpu_buffer_rsrc_t bwd = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char*>(a.bwd), 0, (L - 1) * C::RB * C::CH_B, kBufferWord3);
  const int64_t total = uniform64(q.plan ? splan.total_tiles : (q.n + Q - 1) / Q);
  const __amdgpu_buffer_rsrc_t stash_rs = __builtin_amdgcn_make_buffer_rsrc(
      a.stash + (size_t)blockIdx.x * a.stash_wg + (size_t)wave * L * A::STASH_WL, 0,
      L * A::STASH_WL, kBufferWord3);
  float* uw = ust + wave * kMaxLayers * NQ * 2;   // [layer][point][2]
  char* sst = (char*)ust + A::UST + wave * A::SB;   // this wavefront's stash ring

  // Tiles (deepest first) are drawn one at a time from a counter, so a
  // workgroup that drew deep tiles draws fewer and none ends a whole deep
  // tile after the others (a static round robin gave some workgroups one
  // depth-L tile more).
  __shared__ uint32_t drawn;
  for (;;) {
    if (wave == 0 && lane_now() == 0) drawn = atomicAdd(a.next_tile, 1u);
    __syncthreads();
    const int64_t tile = drawn;
    __syncthreads();
    if (tile >= total) break;
    // Lane-derived values are rebuilt per tile from lane_now(): kept live
    // across the tile loop they would not fit the register budget beside the
    // two activation buffers.
    int lane = lane_now();
    const int g = T::grp(lane), col = T::col(lane);
    const Stash stash{stash_rs, lane * stash_lane_bytes<PREC>()};
    int d;
    int64_t start, cnt;
    if (q.plan) {
      d = 1;
      for (int dd = L; dd >= 1; --dd)
        if (tile < splan.tile_end[dd]) {
          d = dd;
          break;
        }
      const int64_t local = tile - splan.tile_end[d + 1];
      start = splan.start[d] + local * Q;
      cnt = splan.count[d] - local * Q;
    } else {
      d = q.full_depth;
      start = tile * Q;
      cnt = q.n - start;
    }
    if (cnt > Q) cnt = Q;

    const int qi = wave * NQ + col;
    const bool ok = qi < cnt;
    int64_t gi = 0;
    float px = 0.0f, py = 0.0f, pz = 0.0f, dy = 0.0f;
    if (ok) {
      gi = q.perm ? (int64_t)q.perm[start + qi] : start + qi;
      const float* p = q.xyz + 3 * gi;
      px = p[0];
      py = p[1];
      pz = p[2];
      dy = a.dy ? a.dy[gi] : 1.0f;
    }
    {
      const int t = wave * 64 + lane_now();
      spt[t] = f32x4{px, py, pz, dy};
      sgi[t] = ok ? (int32_t)gi : -1;
    }

    // ---------------- forward recompute with stash ----------------
    V actA[C::KS], actB[C::KS];
    float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb) {
      const char* ch = l1 + rb * C::L1C;
      typename T::Acc acc = {};
#pragma unroll
      for (int st = 0; st < T::L1S; ++st)
        acc = T::mma1(T::l1_a(ch, st, lane), T::l1_b(st, g, px, py, pz), acc);
      if (T::VB == 16 && d == 1) {
        if constexpr (T::VB == 16) {
          // FP32 cosines of block rb: four vectors at 4 rb.. of the pair
          // (actA, actB), which no hidden layer needs in a depth-1 tile
          float cf[T::NR];
          fwd_epilogue<PREC, C::KS, FE_F32, ACT>(q.m.kf[0], ch + T::L1S * T::L1AB, g, rb, acc,
                                                 actA, s0, s1, stash, 0, cf);
#pragma unroll
          for (int i = 0; i < T::NR / 4; ++i) {
            const V v = __builtin_bit_cast(V, f32x4{cf[4 * i], cf[4 * i + 1], cf[4 * i + 2],
                                                    cf[4 * i + 3]});
            const int qv = (T::NR / 4) * rb + i;
            if (qv < C::KS) actA[qv] = v; else actB[qv - C::KS] = v;
          }
        }
      } else if (d == 1) {
        fwd_epilogue<PREC, C::KS, FE_REGS, ACT>(q.m.kf[0], ch + T::L1S * T::L1AB, g, rb, acc, actA,
                                                s0, s1, stash, 0);
      } else
        fwd_epilogue<PREC, C::KS, FE_NONE, ACT>(q.m.kf[0], ch + T::L1S * T::L1AB, g, rb, acc, actA,
                                                s0, s1, stash, 0);
    }
    float u0 = adj_lane_sum<PREC>(s0) + q.m.c0[0], u1 = adj_lane_sum<PREC>(s1) + q.m.c1[0];
    float y = fmaf(u0, u1, 0.0f);
    if (g == 0) {
      uw[col * 2] = u0;
      uw[col * 2 + 1] = u1;
    }
    const int nc = (d - 1) * C::RB;
    int c = 0;
    if (nc > 0) {
      load_chunk_buf<C::CH, C::NW, kFreshCopy<PREC, ACT>>(hidden, 0, ring, wave, lane);
      wait_chunk();
      __syncthreads();
    }
    for (int j = 2; j <= d; ++j) {
      if (j & 1)
        adj_fwd_layer<PREC, WP, ACT>(q.m.kf[1], hidden, ring, wave, lane, g, c, nc, j, j == d, actB,
                                     actA, stash, s0, s1);
      else
        adj_fwd_layer<PREC, WP, ACT>(q.m.kf[1], hidden, ring, wave, lane, g, c, nc, j, j == d, actA,
                                     actB, stash, s0, s1);
      u0 = adj_lane_sum<PREC>(s0) + q.m.c0[j - 1];
      u1 = adj_lane_sum<PREC>(s1) + q.m.c1[j - 1];
      y = fmaf(u0, u1, y);
      if (g == 0) {
        uw[((j - 1) * NQ + col) * 2] = u0;
        uw[((j - 1) * NQ + col) * 2 + 1] = u1;
      }
    }
    if (q.sdf && g == 0 && ok) q.sdf[sgi[wave * 64 + lane_now()]] = y;

    // ---------------- backward ----------------
    // exit tail of layer d: delta'_d = cos_d * (u1 a0 + u0 a1), into actA;
    // cos_d is in layer d's output registers (actA for odd d, actB for even)
    float gx[3] = {0.0f, 0.0f, 0.0f};
    {
      const float* tl = a.tails + (size_t)(d - 1) * 2 * WP;
      auto exit_tail = [&](const V (&cosv)[C::KS]) {
#pragma unroll
        for (int rb = 0; rb < C::RB; ++rb) {
          const typename T::Acc zero = {};
          float cs[T::NR];
          bool f32 = false;
          if constexpr (T::VB == 16) {
            if (d == 1) {
#pragma unroll
              for (int i = 0; i < T::NR / 4; ++i) {
                const int qv = (T::NR / 4) * rb + i;
                const f32x4 v =
                    __builtin_bit_cast(f32x4, qv < C::KS ? actA[qv] : actB[qv - C::KS]);
#pragma unroll
                for (int k = 0; k < 4; ++k) cs[4 * i + k] = v[k];
              }
              f32 = true;
            }
          }
          if (!f32) {
            cos_from_regs<PREC, C::KS>(cosv, rb, cs);
          }
          bwd_epilogue<PREC, C::KS>(tl + T::BM * rb, WP, g, rb, zero, u0, u1, cs, actA, d == 1,
                                    w1t, gx);
        }
      };
      if (d & 1)
        exit_tail(actA);
      else
        exit_tail(actB);
    }
    const int ncb = (d - 1) * C::RB;
    c = 0;
    if (ncb > 0) {
      // the forward's stash stores have completed before the stash is read
      wait_chunk();
      load_chunk_buf<C::CH_B, C::NW, kFreshCopy<PREC, ACT>>(bwd, (d - 2) * C::RB * C::CH_B, ring,
                                                            wave, lane);
      if (A::LSTASH && d >= 3) stash_fetch<PREC>(stash, stash_at<PREC, WP>(d - 1, 0), sst, lane);
      wait_chunk();
      __syncthreads();
    }
    // layers d..3 pass delta' on (actA -> actB -> actA ...); layer 2 then
    // ends in the input gradient from whichever buffer holds delta'_2
    for (int j = d; j >= 3; j -= 2) {
      adj_bwd_layer<PREC, WP, ACT, false>(q.m.kf[0], bwd, ring, wave, lane, g, c, ncb, d, j, l1, px,
                                          py, pz, actA, actB, stash, sst,
                                          uw[((j - 2) * NQ + col) * 2],
                                          uw[((j - 2) * NQ + col) * 2 + 1], w1t, gx);
      if (j - 1 < 3) break;
      adj_bwd_layer<PREC, WP, ACT, false>(q.m.kf[0], bwd, ring, wave, lane, g, c, ncb, d, j - 1, l1,
                                          px, py, pz, actB, actA, stash, sst,
                                          uw[((j - 3) * NQ + col) * 2],
                                          uw[((j - 3) * NQ + col) * 2 + 1], w1t, gx);
    }
    if (d >= 2) {
      const float v0 = uw[col * 2], v1 = uw[col * 2 + 1];
      const f32x4 pt = spt[wave * 64 + lane_now()];
      if (((d - 2) & 1) == 0)
        adj_bwd_layer<PREC, WP, ACT, true>(q.m.kf[0], bwd, ring, wave, lane, g, c, ncb, d, 2, l1,
                                           pt[0], pt[1], pt[2], actA, actB, stash, sst, v0, v1, w1t,
                                           gx);
      else
        adj_bwd_layer<PREC, WP, ACT, true>(q.m.kf[0], bwd, ring, wave, lane, g, c, ncb, d, 2, l1,
                                           pt[0], pt[1], pt[2], actB, actA, stash, sst, v0, v1, w1t,
                                           gx);
    }
    const float gxs = adj_lane_sum<PREC>(gx[0]), gys = adj_lane_sum<PREC>(gx[1]),
                gzs = adj_lane_sum<PREC>(gx[2]);
    const int tl = wave * 64 + lane_now();
    const int32_t go = sgi[tl];
    if (g == 0 && go >= 0) {
      const float dyo = spt[tl][3];
      float* o = a.grad + 3 * (int64_t)go;
      o[0] = dyo * gxs;
      o[1] = dyo * gys;
      o[2] = dyo * gzs;
    }
  }
}

template <int PREC, int WP, int ACT>
hipError_t launch_adj_one(const AdjointArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_adjoint<PREC, WP, ACT>), dim3((unsigned)grid), dim3(Cfg<PREC, WP>::NT), 0,
                     s, a);
  return hipGetLastError();
}

template <int PREC, int ACT>
hipError_t launch_adj_prec(const AdjointArgs& a, int grid, hipStream_t s) {
  switch (a.q.m.WP) {
    case 64: return launch_adj_one<PREC, 64, ACT>(a, grid, s);
    case 128: return launch_adj_one<PREC, 128, ACT>(a, grid, s);
    case 256: return launch_adj_one<PREC, 256, ACT>(a, grid, s);
    case 352: return launch_adj_one<PREC, 352, ACT>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

template <int ACT>
hipError_t launch_adjoint_act(int prec, const AdjointArgs& a, int grid, hipStream_t s) {
  if (prec == PREC_FP32) return launch_adj_prec<PREC_FP32, ACT>(a, grid, s);
  if (prec == PREC_BF16) return launch_adj_prec<PREC_BF16, ACT>(a, grid, s);
  return launch_adj_prec<PREC_FP16, ACT>(a, grid, s);
}

}  // namespace sand
