// gfx950 kernels of the localized style-transfer loss and gradient.
//
// Layout: activations are NHWC per tile window (channels fastest), one workspace slot
// per tile of a batch.  Every kernel takes a Batch (per-tile geometry by value) and maps
// blockIdx.x to (tile, work block) through the Batch prefix sums, so one launch covers
// all tiles of a batch, ragged or not.
//
// Numerics: FP32 accumulation everywhere (MFMA f32 accumulators); FP64 for Gram
// partial reductions across chunks/tiles and for all energy sums.  All reductions run
// in a fixed order, so results are bitwise reproducible and independent of the batch
// size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <stdint.h>
#include <stdio.h>

#include "kernels.h"

namespace nst {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// CK: input channels staged per LDS chunk (64 bytes per pixel for both precisions).
template <typename T> struct Tr;
template <> struct Tr<float> { static constexpr int CK = 16; };
template <> struct Tr<bf16> { static constexpr int CK = 32; };

__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(bf16 v) { return (float)v; }
template <typename T> __device__ __forceinline__ T from_f(float v);
template <> __device__ __forceinline__ float from_f<float>(float v) { return v; }
template <> __device__ __forceinline__ bf16 from_f<bf16>(float v) { return (bf16)v; }

// One lane's operand fragment: the CK/2 consecutive channels of its k-half.
// The 32x32 MFMAs pair A-lane (row m, k-half g, element j) with B-lane (col n, g, j),
// so any assignment of channels to (g, j) that A and B share gives the same sum.
template <typename T> struct Mma;
template <> struct Mma<float> {
  struct Frag { f32x4 v[2]; };
  static __device__ __forceinline__ Frag load(const float *p) {
    Frag f;
    f.v[0] = *(const f32x4 *)p;
    f.v[1] = *(const f32x4 *)(p + 4);
    return f;
  }
  static __device__ __forceinline__ void mma(f32x16 &acc, const Frag &a, const Frag &b) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[h][j], b.v[h][j], acc, 0, 0, 0);
  }
};
template <> struct Mma<bf16> {
  struct Frag { bf16x8 v[2]; };
  static __device__ __forceinline__ Frag load(const bf16 *p) {
    Frag f;
    f.v[0] = *(const bf16x8 *)p;
    f.v[1] = *(const bf16x8 *)(p + 8);
    return f;
  }
  static __device__ __forceinline__ void mma(f32x16 &acc, const Frag &a, const Frag &b) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v[0], b.v[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v[1], b.v[1], acc, 0, 0, 0);
  }
};

__device__ __forceinline__ int find_tile(const Batch &g, int bid) {
  int t = 0;
  while (t + 1 < g.n && bid >= g.pfx[t + 1]) ++t;
  return t;
}

// Width of the k_conv3 patches (see below); conv1_1 (k_conv_img) keeps 8 x 32.
constexpr int kConvPW = 16;

// Pixel (within its 32-pixel MFMA operand block) of operand column l32.  The measured LDS
// bank conflicts fit a ds_read_b128 that serves 8 lanes per cycle, lanes {0-3, 20-23},
// {4-7, 16-19}, {8-11, 28-31}, {12-15, 24-27} (and the same + 32), over 64 four-byte
// banks.  With 80-byte halo rows, halo row P starts on bank group 5 P mod 16, so 32
// consecutive rows are conflict-free in every cycle.  A block of two 16-pixel patch rows
// puts its second run at P + 18 instead of P + 16; its columns are rotated by two so that
// every lane reads a halo row congruent to l32 mod 16, the bank groups of one consecutive
// run.  Any pixel order is valid as long as the operand reads and the epilogues use the
// same one.
template <int PW> __device__ __forceinline__ int blk_pixel(int l32) {
  if constexpr (PW == 16) return l32 < 16 ? l32 : 16 + ((l32 - 2) & 15);
  else return l32;
}

// ---------------------------------------------------------------------------------------
// Pipelined implicit-GEMM 3x3 convolution (NHWC input) on MFMA.
//   Work block: a PH x PW output patch (PW = kConvPW = 16, M = PH PW pixels) x BN output
//   channels, WM x WN waves.  The K loop runs over stages (channel chunk c, filter row
//   ky): each stage holds the 3 taps of one filter row for BN channels in LDS, and the
//   first stage of a chunk also the (PH + 2) x (PW + 2) halo patch of that chunk.  Stages are double-buffered and
//   filled by LDS DMA (global_load_lds_dwordx4: each lane's 16 bytes go straight to LDS
//   at the wave's base + 16 x lane, no registers or LDS store instructions involved): the
//   next stage's loads are issued between the current stage's first MFMAs and are in
//   flight during the rest of it; halfway through its last k-step a stage waits for the
//   wave's own loads and passes one barrier.  With one halo buffer (SA) the next chunk's
//   halo is loaded between chunks instead.
//   A 32-row MFMA operand block is two patch rows of 16 pixels, i.e. two runs of 16
//   consecutive LDS rows with a gap between them, read in the column order of blk_pixel
//   (bank-conflict free like one run of 32 rows).  32-wide patches would need no such
//   order, but the regions a pass computes are ragged (e.g. 132-138 px wide at stride 8 for 1024 px tiles): 16 x 16 patches pad the
//   deep layers' MFMA work by 8.0% instead of 9.9% at 6048 x 8064 and measured 3% faster
//   over the whole evaluation.  Halo-patch rows are
//   padded to 80 bytes (unit p of a chunk is row p / 5, 16-byte chunk p % 5; chunk 4 is
//   padding), so every tap and filter-row shift of an operand block is a constant byte
//   offset; weight rows are 64 bytes with the 16-byte chunk XOR-swizzled by (row / 4)
//   mod 4 (applied on the global side of the DMA), which tap shifts (multiples of BN
//   rows) leave unchanged.  Halo positions outside the window and padding units read a
//   zero row.
//   Segment 1 (optional) adds the centre tap over in2 (the style residual V D~).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int swz64(int row, int chunk, int ck, int vec) {
  return row * ck + ((chunk ^ ((row >> 2) & 3)) * vec);
}

// One k-step of a stage: filter tap ti, channel half kh of the 64-byte LDS rows (16 BF16
// or 4 FP32 channels per lane).  Operand fragments are one 16-byte LDS read per 32-row A
// block and per 32-column B block.  Tap by tap, first half then second, each
// accumulator sees the same sequence of MFMAs as a whole-row loop would give it.
template <int TM, int TN> struct KFrag { u32x4 a[TM], b[TN]; };

template <typename T, int TM, int TN, int BN, int CK, int VEC>
__device__ __forceinline__ void load_kstep(KFrag<TM, TN> &f, const T *A, const T *B,
                                           const int (&pidx)[TM], int toff, int ti, int kh, int bcol,
                                           int half) {
  const int chunk = 2 * half + kh;
#pragma unroll
  for (int tm = 0; tm < TM; ++tm) f.a[tm] = *(const u32x4 *)(&A[(pidx[tm] + toff) * (CK + VEC) + chunk * VEC]);
#pragma unroll
  for (int tn = 0; tn < TN; ++tn)
    f.b[tn] = *(const u32x4 *)(&B[swz64(ti * BN + bcol + tn * 32, chunk, CK, VEC)]);
}

// The weights fragment is the MFMA's first operand: block (tm, tn) accumulates the
// transposed 32 x 32 tile, channels by pixels, so that lane (l32, half) holds column l32 of
// the block and channels 8 (r / 4) + 4 half + (r mod 4) in element r: four consecutive
// channels per group of four elements.
template <typename T, int TM, int TN>
__device__ __forceinline__ void mma_kstep(f32x16 (&acc)[TM][TN], const KFrag<TM, TN> &f) {
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
      if constexpr (sizeof(T) == 2) {
        acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, f.b[tn]),
                                                               __builtin_bit_cast(bf16x8, f.a[tm]),
                                                               acc[tm][tn], 0, 0, 0);
      } else {
        const f32x4 av = __builtin_bit_cast(f32x4, f.a[tm]), bv = __builtin_bit_cast(f32x4, f.b[tn]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x2f32(bv[j], av[j], acc[tm][tn], 0, 0, 0);
      }
    }
}

// Passes of the LDS epilogue: the fewest that divide TN and fit the FP32 tile
// (BM x (WN x TN / passes x 32 + 4) floats) into the stage buffers.  A row pitch of 4
// mod 64 words keeps the 16-byte writes of 16 consecutive pixels on distinct banks.
constexpr int epi_passes(int bm, int wn, int tn, int smem_bytes) {
  for (int p = 1; p <= tn; ++p)
    if (tn % p == 0 && bm * (wn * (tn / p) * 32 + 4) * 4 <= smem_bytes) return p;
  return 0;
}

// Workgroup barrier for the conv kernels: waits for this wave's LDS reads and writes
// (lgkmcnt 0), not for its global loads.  __syncthreads() (and an LDS-only fence, which
// counts LDS DMA as pending LDS writes) would wait for every outstanding load, vmcnt 0;
// the stage code waits explicitly for the DMA that the next stage reads and leaves later
// DMA (the next chunk's halo) in flight, and the epilogue does not wait for its global
// stores between passes.  The asm is a compiler memory barrier.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Single-pass BF16 epilogue (BF16 layers without the FP32 content residual): phase 1
// applies bias + ReLU (forward) to the accumulators in registers, rounds to BF16 and
// writes 8-byte rows of four channels to LDS (the whole BM x BN tile fits); phase 2 copies
// 16-byte rows of eight channels to the output and, forward, takes the 2 x 2 pooling
// maximum, backward, applies the ReLU mask.  Forward outputs have their sign bit cleared
// (a ReLU output of -0 becomes +0), so all values are non-negative and the integer order of
// their bits is their order as numbers: the integer maximum is the first maximum in
// window order that a separate pooling pass would keep.  The mask is a selection, so
// rounding before it gives the same bits as rounding after it.
template <int BN, int WM, int WN, int PH, int PW, int EPI, int SMEM_BYTES>
__device__ __forceinline__ void epi_bf16(f32x16 (&acc)[PH * PW / (WM * 32)][BN / (WN * 32)], bf16 *sm,
                                         const ConvArgs &a, long long slot, int y0, int x0, int h, int w, int n0,
                                         int tid, int wm, int wn, int lpx, int half) {
  constexpr int BM = PH * PW, NT = WM * WN * 64;
  constexpr int TM = BM / (WM * 32), TN = BN / (WN * 32);
  constexpr int RS = BN + 8;   // row pitch in BF16: 4 mod 64 words for even BN / 32
  static_assert(BM * RS * 2 <= SMEM_BYTES, "BF16 epilogue tile");
  typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
  typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
  const int cout = a.cout;
  // backward: an optional per-channel constant joins the adjoint before the mask
  const bool bwd_bias = EPI != EPI_FWD && a.bias != nullptr;
  // phase 1: block (tm, tn), lane: pixel lpx, channels 8 jj + 4 half + (0..3) (mma_kstep)
#pragma unroll
  for (int tn = 0; tn < TN; ++tn)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int cl = wn * TN * 32 + tn * 32 + 8 * jj + 4 * half;
      f32x4 b = {0.f, 0.f, 0.f, 0.f};
      if (EPI == EPI_FWD || bwd_bias) b = *(const f32x4 *)(a.bias + (n0 + cl < cout ? n0 + cl : 0));
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        const int m = wm * TM * 32 + tm * 32 + lpx;
        u16x4 o;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float v = acc[tm][tn][4 * jj + e];
          if constexpr (EPI == EPI_FWD) v = fmaxf(v + b[e], 0.f);
          else if (bwd_bias) v += b[e];
          o[e] = __builtin_bit_cast(unsigned short, (bf16)v);
          if constexpr (EPI == EPI_FWD) o[e] &= (unsigned short)0x7fff;
        }
        *(u16x4 *)(&sm[m * RS + cl]) = o;
      }
      // one (tn, jj) group at a time: hoisting every accumulator read would need 256 VGPRs
      __builtin_amdgcn_sched_barrier(0);
    }
  lds_barrier();
  // phase 2: thread chunk of eight channels lc (the same for all its items)
  constexpr int CPR = BN / 8, ISTEP = NT / CPR;
  static_assert(NT % CPR == 0, "epilogue items");
  const int lc = (tid % CPR) * 8, ib = tid / CPR;
  const int n = n0 + lc;
  const bool nok = n < cout;
  if constexpr (EPI == EPI_FWD) {
    // 2 x 2 windows q = ib + k ISTEP (k < NW)
    constexpr int PWO = PW / 2, PO = (PH / 2) * PWO, NW = PO * CPR / NT;
    static_assert((PO * CPR) % NT == 0, "epilogue windows");
    bf16 *outb = a.out ? (bf16 *)a.out + slot * a.out_ss + n : nullptr;
    bf16 *poolb = a.pool ? (bf16 *)a.pool + slot * a.pool_ss + n : nullptr;
    const bool pavg = a.pool_avg != 0;
    const int ho = h >> 1, wo = w >> 1;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int q = ib + k * ISTEP;
      const int qy = q / PWO, qx = q % PWO;
      u16x8 best;
      float sum[8];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int ly = 2 * qy + (kk >> 1), lx = 2 * qx + (kk & 1);
        const int py = y0 + ly, px = x0 + lx;
        const u16x8 u = *(const u16x8 *)(&sm[(ly * PW + lx) * RS + lc]);
        best = kk == 0 ? u : __builtin_elementwise_max(best, u);
        if (pavg) {
          // average pool: the mean of the four stored values, rounded once
#pragma unroll
          for (int e = 0; e < 8; ++e) sum[e] = (kk == 0 ? 0.f : sum[e]) + __builtin_bit_cast(float, (unsigned)u[e] << 16);
        }
        if (outb && nok && py < h && px < w) *(u16x8 *)(outb + (long long)(py * w + px) * cout) = u;
      }
      if (pavg) {
#pragma unroll
        for (int e = 0; e < 8; ++e) best[e] = __builtin_bit_cast(unsigned short, (bf16)(0.25f * sum[e]));
      }
      const int oy = (y0 >> 1) + qy, ox = (x0 >> 1) + qx;   // patch origins are even
      if (poolb && nok && oy < ho && ox < wo) *(u16x8 *)(poolb + (long long)(oy * wo + ox) * cout) = best;
    }
  } else {
    // pixels m = ib + i ISTEP (i < NIT), masks loaded in groups of G
    constexpr int NIT = BM * CPR / NT, G = NIT < 8 ? NIT : 8;
    static_assert((BM * CPR) % NT == 0 && NIT % G == 0, "epilogue items");
    static_assert(ISTEP % PW == 0 || PW % ISTEP == 0, "epilogue pixel stride");
    auto item = [&](int i, int &ly, int &lx) __attribute__((always_inline)) {
      if constexpr (ISTEP % PW == 0) {
        ly = ib / PW + i * (ISTEP / PW);
        lx = ib % PW;
      } else {
        ly = i / (PW / ISTEP);
        lx = ib + (i % (PW / ISTEP)) * ISTEP;   // ib < ISTEP
      }
    };
    bf16 *outb = (bf16 *)a.out + slot * a.out_ss + n;
    const bf16 *mskb = a.mask ? (const bf16 *)a.mask + slot * a.mask_ss + (nok ? n : 0) : nullptr;
#pragma unroll
    for (int g0 = 0; g0 < NIT; g0 += G) {
      u16x8 mk[G];
      if (mskb) {
#pragma unroll
        for (int j = 0; j < G; ++j) {
          int ly, lx;
          item(g0 + j, ly, lx);
          const int py = min(y0 + ly, h - 1), px = min(x0 + lx, w - 1);
          mk[j] = *(const u16x8 *)(mskb + (long long)(py * w + px) * cout);
        }
      }
#pragma unroll
      for (int j = 0; j < G; ++j) {
        int ly, lx;
        item(g0 + j, ly, lx);
        const int py = y0 + ly, px = x0 + lx;
        if (py >= h || px >= w || !nok) continue;
        u16x8 u = *(const u16x8 *)(&sm[(ly * PW + lx) * RS + lc]);
        if (mskb) {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (!(__builtin_bit_cast(float, (unsigned)mk[j][e] << 16) > 0.f)) u[e] = 0;
        }
        *(u16x8 *)(outb + (long long)(py * w + px) * cout) = u;
      }
    }
  }
}

// Conv epilogue through LDS (the caller's last barrier has released its stage buffers,
// SMEM_BYTES of them at sm), in NPASS passes over the wave's TN column blocks: phase 1
// writes the raw FP32 accumulators of the pass, phase 2 reads VEC consecutive channels of
// one pixel with 16-byte LDS reads and applies bias + ReLU (+ content difference), or
// content residual + ReLU mask, with 16-byte global loads and stores.  The arithmetic per
// element is the same as applying it to the accumulator directly.
//   A thread keeps the same VEC channels for the whole pass (NT is a multiple of the
// CPR channel chunks of a pixel row).  The forward epilogue walks 2 x 2 pooling windows:
// it rounds each of the window's four outputs once, stores them and, for a pooled layer,
// the first maximum of the rounded values in row-major window order, as a separate
// pooling pass would.  The backward epilogue walks pixels in groups of G whose loads
// (residual, mask) are issued together, the first group before phase 1.  Addresses are a
// per-pass base plus a 64-bit element offset (pixel index times cout: a whole-image
// window can hold more than 2^31 elements).
template <typename T, int BN, int WM, int WN, int PH, int PW, int EPI, int SMEM_BYTES, bool F32E>
__device__ __forceinline__ void conv_epilogue(f32x16 (&acc)[PH * PW / (WM * 32)][BN / (WN * 32)], T *sm,
                                              const ConvArgs &a, const Batch &g, int t, long long slot,
                                              int y0, int x0, int h, int w, int n0, int tid, int wm, int wn,
                                              int lpx, int half) {
  constexpr int BM = PH * PW, NT = WM * WN * 64;
  constexpr int TM = BM / (WM * 32), TN = BN / (WN * 32);
  constexpr int VEC = 16 / sizeof(T), NQ = VEC / 4;
  constexpr int NPASS = epi_passes(BM, WN, TN, SMEM_BYTES);
  constexpr int TNP = TN / NPASS, CW = TNP * 32, RSW = WN * CW + 4;
  constexpr int CPR = WN * CW / VEC;
  static_assert(NT % CPR == 0 && PH % 2 == 0, "epilogue tiling");
  typedef T TV __attribute__((ext_vector_type(VEC)));
  // BF16 without the content residual: single pass (the choice is a template argument,
  // F32E, so that each kernel holds one epilogue: with both behind a run-time test the
  // compiler copies every accumulator to VGPRs ahead of it and spills)
  if constexpr (sizeof(T) == 2 && !F32E) {
    epi_bf16<BN, WM, WN, PH, PW, EPI, SMEM_BYTES>(acc, (bf16 *)sm, a, slot, y0, x0, h, w, n0, tid, wm, wn, lpx, half);
    return;
  }
  float *so = (float *)sm;
  const int cout = a.cout;
  const int lc = (tid % CPR) * VEC, ib = tid / CPR;
  // forward: windows q = ib + k QSTEP (k < NW); backward: pixels m = ib + i MSTEP (i < NIT)
  constexpr int PWO = PW / 2, PO = (PH / 2) * PWO, QSTEP = NT / CPR, NW = PO * CPR / NT;
  constexpr int MSTEP = NT / CPR, NIT = BM * CPR / NT;
  static_assert((PO * CPR) % NT == 0 && (BM * CPR) % NT == 0, "epilogue items");
  static_assert(MSTEP % PW == 0 || PW % MSTEP == 0, "epilogue pixel stride");
  constexpr int GW = NW < 2 ? NW : 2;            // forward: windows per load group
  constexpr int G = EPI == EPI_FWD ? 4 * GW : (NIT < 8 ? NIT : 8);
  static_assert(NW % GW == 0 && NIT % G == 0, "epilogue groups");
  const bool fwd_rc = EPI == EPI_FWD && a.rc != nullptr, bwd_rc = EPI != EPI_FWD && a.rc != nullptr;
  const bool bwd_mask = EPI != EPI_FWD && a.mask != nullptr;
  const bool bwd_bias = EPI != EPI_FWD && a.bias != nullptr;
  // local (row, column) of item j of group g0
  auto item_fwd = [&](int k, int kk, int &ly, int &lx) __attribute__((always_inline)) {
    const int q = ib + k * QSTEP;
    ly = 2 * (q / PWO) + (kk >> 1);
    lx = 2 * (q % PWO) + (kk & 1);
  };
  auto item_bwd = [&](int i, int &ly, int &lx) __attribute__((always_inline)) {
    if constexpr (MSTEP % PW == 0) {
      ly = ib / PW + i * (MSTEP / PW);
      lx = ib % PW;
    } else {
      ly = i / (PW / MSTEP);
      lx = ib + (i % (PW / MSTEP)) * MSTEP;   // ib < MSTEP
    }
  };
  TV mk[G];
  f32x4 dq[G][NQ];
  // loads of group g0 at clamped addresses (every lane loads; items outside the window
  // or past cout are not stored)
  auto load_group = [&](int g0, int nc) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < G; ++j) {
      int ly, lx;
      if constexpr (EPI == EPI_FWD)
        item_fwd(g0 / 4 + j / 4, j % 4, ly, lx);
      else
        item_bwd(g0 + j, ly, lx);
      const int py = min(y0 + ly, h - 1), px = min(x0 + lx, w - 1);
      if (fwd_rc) {
        const float *f = a.fc + ((long long)(g.gy[t] + py) * a.fc_w + (g.gx[t] + px)) * cout + nc;
#pragma unroll
        for (int q = 0; q < NQ; ++q) dq[j][q] = *(const f32x4 *)(f + 4 * q);
      }
      const long long po = (long long)(py * w + px) * cout;
      if (bwd_rc) {
        const float *rc = a.rc + slot * a.rc_ss + nc + po;
#pragma unroll
        for (int q = 0; q < NQ; ++q) dq[j][q] = *(const f32x4 *)(rc + 4 * q);
      }
      if (bwd_mask) mk[j] = *(const TV *)((const T *)a.mask + slot * a.mask_ss + nc + po);
    }
  };
#pragma unroll
  for (int p = 0; p < NPASS; ++p) {
    const int n = n0 + (lc / CW) * TN * 32 + p * CW + lc % CW;   // this thread's channels
    const bool nok = n < cout;
    const int nc = nok ? n : 0;
    float bv[VEC];
    if (EPI == EPI_FWD || bwd_bias) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const f32x4 b = *(const f32x4 *)(a.bias + nc + 4 * q);
#pragma unroll
        for (int e = 0; e < 4; ++e) bv[4 * q + e] = b[e];
      }
    }
    T *outb = a.out ? (T *)a.out + slot * a.out_ss + n : nullptr;
    // the first group's loads are in flight while the accumulators go to LDS
    if (fwd_rc || bwd_rc || bwd_mask) load_group(0, nc);
    if (p > 0) lds_barrier();
    // accumulator block (tm, tq): pixel lpx, channels 8 jj + 4 half + (0..3) (see mma_kstep)
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
      for (int tq = 0; tq < TNP; ++tq)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int m = wm * TM * 32 + tm * 32 + lpx;
          const f32x16 &av = acc[tm][p * TNP + tq];
          const f32x4 v = {av[4 * jj], av[4 * jj + 1], av[4 * jj + 2], av[4 * jj + 3]};
          *(f32x4 *)(&so[m * RSW + wn * CW + tq * 32 + 8 * jj + 4 * half]) = v;
        }
    lds_barrier();
    if constexpr (EPI == EPI_FWD) {
      T *poolb = a.pool ? (T *)a.pool + slot * a.pool_ss + n : nullptr;
      const bool pavg = a.pool_avg != 0;
      const int ho = h >> 1, wo = w >> 1;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        if (k > 0 && k % GW == 0 && fwd_rc) load_group(4 * k, nc);
        TV best;
        float bf[VEC];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          int ly, lx;
          item_fwd(k, kk, ly, lx);
          const int m = ly * PW + lx;
          const int py = y0 + ly, px = x0 + lx;
          float v[VEC];
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const f32x4 u = *(const f32x4 *)(&so[m * RSW + lc + 4 * q]);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[4 * q + e] = fmaxf(u[e] + bv[4 * q + e], 0.f);
          }
          TV o;
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            o[e] = from_f<T>(v[e]);
            const float f = to_f(o[e]);
            if (pavg) {
              bf[e] = (kk == 0 ? 0.f : bf[e]) + f;   // average pool: sum of the stored values
            } else if (kk == 0 || f > bf[e]) {
              bf[e] = f;
              best[e] = o[e];
            }
          }
          if (py < h && px < w && nok) {
            const long long po = (long long)(py * w + px) * cout;
            if (fwd_rc) {
              const int j = (k % GW) * 4 + kk;
              float *rc = a.rc + slot * a.rc_ss + n + po;
#pragma unroll
              for (int q = 0; q < NQ; ++q) {
                f32x4 d;
#pragma unroll
                for (int e = 0; e < 4; ++e) d[e] = v[4 * q + e] - dq[j][q][e];
                *(f32x4 *)(rc + 4 * q) = d;
              }
            }
            if (outb) *(TV *)(outb + po) = o;
          }
        }
        if (poolb && pavg) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) best[e] = from_f<T>(0.25f * bf[e]);
        }
        if (poolb) {
          const int q = ib + k * QSTEP;
          const int oy = (y0 >> 1) + q / PWO, ox = (x0 >> 1) + q % PWO;   // patch origins are even
          if (oy < ho && ox < wo && nok) *(TV *)(poolb + (long long)(oy * wo + ox) * cout) = best;
        }
      }
    } else {
#pragma unroll
      for (int g0 = 0; g0 < NIT; g0 += G) {
        if (g0 > 0 && (bwd_rc || bwd_mask)) load_group(g0, nc);
#pragma unroll
        for (int j = 0; j < G; ++j) {
          int ly, lx;
          item_bwd(g0 + j, ly, lx);
          const int m = ly * PW + lx;
          const int py = y0 + ly, px = x0 + lx;
          if (py >= h || px >= w || !nok) continue;
          float v[VEC];
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const f32x4 u = *(const f32x4 *)(&so[m * RSW + lc + 4 * q]);
            v[4 * q] = u[0]; v[4 * q + 1] = u[1]; v[4 * q + 2] = u[2]; v[4 * q + 3] = u[3];
          }
          if (bwd_bias) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] += bv[e];
          }
          if (bwd_rc) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
              for (int e = 0; e < 4; ++e) v[4 * q + e] += a.two_alpha * dq[j][q][e];
          }
          if (bwd_mask) {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
              if (!(to_f(mk[j][e]) > 0.f)) v[e] = 0.f;
          }
          TV o;
#pragma unroll
          for (int e = 0; e < VEC; ++e) o[e] = from_f<T>(v[e]);
          *(TV *)(outb + (long long)(py * w + px) * cout) = o;
        }
      }
    }
  }
}

__device__ __attribute__((aligned(16))) unsigned kZeroRow[4] = {0u, 0u, 0u, 0u};

typedef __attribute__((address_space(3))) void lds_void;

// One 16-byte LDS DMA unit per lane: unit i of the wave writes LDS at dst + (i NT + 64 wv)
// units + 16 bytes x lane.  A unit that is off (no next stage, halo position outside the
// window or in the padding) reads the zero row, so every wave issues every unit and the
// issue has no branches; an off unit only ever writes a buffer that is not read again
// (the last stage's free buffers) or the padding of the halo buffer.
template <typename T, int NT, int VEC>
__device__ __forceinline__ void dma_unit_b(T *__restrict__ dst, const T *wbase, unsigned boff, bool on, int i,
                                           int wv) {
  const void *gp = on ? (const void *)((const char *)wbase + boff) : (const void *)kZeroRow;
  __builtin_amdgcn_global_load_lds(gp, (lds_void *)(dst + (i * NT + wv * 64) * VEC), 16, 0, 0);
}

template <typename T, int NT, int VEC>
__device__ __forceinline__ void dma_unit_a(T *__restrict__ dst, const T *base, unsigned arel, bool on, int cin,
                                           int i, int wv, int tid) {
  const unsigned unit = (unsigned)((i * NT + tid) % 5);
  const unsigned off = (arel * (unsigned)cin + unit * VEC) * (unsigned)sizeof(T);
  const void *gp = on ? (const void *)((const char *)base + off) : (const void *)kZeroRow;
  __builtin_amdgcn_global_load_lds(gp, (lds_void *)(dst + (i * NT + wv * 64) * VEC), 16, 0, 0);
}

template <typename T, int NT, int ANVD, int VEC>
__device__ __forceinline__ void dma_a(T *__restrict__ dst, const T *base, const unsigned (&arel)[ANVD],
                                      unsigned okbits, int cin, int wv, int tid) {
#pragma unroll
  for (int i = 0; i < ANVD; ++i)
    dma_unit_a<T, NT, VEC>(dst, base, arel[i], (okbits >> i) & 1u, cin, i, wv, tid);
}

template <typename T, int NT, int BNV, int VEC>
__device__ __forceinline__ void dma_b(T *__restrict__ dst, const T *wbase, const unsigned (&boff)[BNV],
                                      int wv) {
#pragma unroll
  for (int i = 0; i < BNV; ++i) dma_unit_b<T, NT, VEC>(dst, wbase, boff[i], true, i, wv);
}

// Weight-row offsets with the LDS swizzle on the global side: unit p = i NT + tid of a
// stage is weight row p / 4 (tap row ti < NROWS, channel n), physical chunk p % 4, which
// holds logical chunk (p % 4) ^ ((row / 4) mod 4).  Rows past the stage's taps repeat tap 0.
template <typename T, int NT, int BNV, int BN, int CK, int VEC>
__device__ __forceinline__ void dma_boff(unsigned (&boff)[BNV], int nrows, int cout_pad, int n0, int tid) {
#pragma unroll
  for (int i = 0; i < BNV; ++i) {
    const int row = (i * NT + tid) >> 2;
    int ti = row / BN;
    const int n = row - ti * BN;
    ti = ti < nrows ? ti : 0;
    const int lchunk = (tid & 3) ^ ((row >> 2) & 3);
    boff[i] = (unsigned)(((ti * cout_pad + n0 + n) * CK + lchunk * VEC) * (int)sizeof(T));
  }
}

// One stage: the k-step pipeline over this stage's buffers, with the DMA of the next
// stage's weights (then optionally the next halo chunk) spread over its first KD k-steps
// (at most four, never the last).  Spreading the DMA keeps the CU's address and L1 path
// (about 64 bytes per clock) below saturation; issued all at once after a barrier, the
// DMA of the four waves would stall them for most of a thousand cycles before the first
// MFMA.
//   f[0] holds the stage's first k-step fragments on entry.  The last k-step's fragments
// are in registers before it starts, so halfway through its MFMAs the stage is done with
// its buffers: it waits for this wave's DMA except the last VMW loads (a halo chunk left
// in flight), passes the workgroup barrier, reads the next stage's first fragments
// (buffers An, Bn, offset toffn) into f[0], and then runs the second half of the MFMAs,
// which cover the latency of those reads.
template <typename T, int TM, int TN, int BN, int CK, int VEC, int NTAP, int NT, int ANVD, int BNV, bool DA,
          int VMW, bool MIDA = false>
__device__ __forceinline__ void stage_dma(f32x16 (&acc)[TM][TN], KFrag<TM, TN> (&f)[2], const T *__restrict__ A,
                                          const T *__restrict__ B, const int (&pidx)[TM], int toff0, int bcol,
                                          int half, T *__restrict__ adst, const T *abase,
                                          const unsigned (&arel)[ANVD], unsigned okbits, int cin,
                                          T *__restrict__ bdst, const T *wbase, const unsigned (&boff)[BNV],
                                          bool issue_b, bool issue_a, const T *__restrict__ An,
                                          const T *__restrict__ Bn, int toffn, bool has_next, int wv, int tid) {
  constexpr int NK = 2 * NTAP;
  constexpr int ND = BNV + (DA ? ANVD : 0);   // DMA units per lane: weights first, then halo
  constexpr int KD = NK - 1 < 4 ? NK - 1 : 4;  // k-steps that issue DMA (never the last)
  constexpr int DPK = (ND + KD - 1) / KD;
  const bool aon = DA && issue_a;
  // all of the first k-step's reads (lgkmcnt 0): the compiler counts pending LDS DMA as
  // LDS traffic and would otherwise wait again inside the k-step, after the next
  // fragment reads have started
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_sched_barrier(0);
  // the next k-step's NLD fragment reads are interleaved with the first MFMAs of this
  // k-step (one MFMA, then one read), so they are in flight during the rest of it, the
  // LDS counter (4 bits) never tracks two k-steps of reads, and the only LDS wait of a
  // k-step, before its first MFMA, covers reads issued during the previous one.  With
  // fewer than two MFMAs per read the reads all go first.  The k-step's DMA units follow
  // its MFMAs one by one.
  constexpr int NLD = TM + TN, NMF = TM * TN * (sizeof(T) == 2 ? 1 : 4);
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    if (j + 1 < NK)
      load_kstep<T, TM, TN, BN, CK, VEC>(f[(j + 1) & 1], A, B, pidx, toff0 + (j + 1) / 2, (j + 1) / 2,
                                         (j + 1) & 1, bcol, half);
    if (j == NK - 1) {
      // last k-step: the first half of its MFMAs (same operand order as mma_kstep), the
      // stage's waits and barrier, the next stage's first reads, the second half
      const KFrag<TM, TN> &fl = f[j & 1];
#pragma unroll
      for (int tm = 0; tm < TM / 2; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
          if constexpr (sizeof(T) == 2) {
            acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fl.b[tn]),
                                                                   __builtin_bit_cast(bf16x8, fl.a[tm]),
                                                                   acc[tm][tn], 0, 0, 0);
          } else {
            const f32x4 av = __builtin_bit_cast(f32x4, fl.a[tm]), bv = __builtin_bit_cast(f32x4, fl.b[tn]);
#pragma unroll
            for (int q = 0; q < 4; ++q)
              acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x2f32(bv[q], av[q], acc[tm][tn], 0, 0, 0);
          }
        }
      __builtin_amdgcn_sched_barrier(0);
      // a halo chunk issued in this stage (the last VMW loads, as loads complete in issue
      // order) may stay in flight; lgkmcnt 0 visible to the compiler, so that it does not
      // wait for the next stage's reads before the second half
      if (aon)
        __builtin_amdgcn_s_waitcnt(0xf70 | VMW);
      else
        __builtin_amdgcn_s_waitcnt(0xf70);
      __builtin_amdgcn_s_waitcnt(0xc07f);
      lds_barrier();
      KFrag<TM, TN> keep = fl;   // f[0] is overwritten by the next stage's reads
      if constexpr (MIDA) {
        // single halo buffer: no wave reads it any more, so the next chunk's halo (adst,
        // abase, cin, issue_a) goes out now; the caller waits for it
        if (issue_a) dma_a<T, NT, ANVD, VEC>(adst, abase, arel, okbits, cin, wv, tid);
      } else {
        if (has_next) load_kstep<T, TM, TN, BN, CK, VEC>(f[0], An, Bn, pidx, toffn, 0, 0, bcol, half);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int tm = TM / 2; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
          if constexpr (sizeof(T) == 2) {
            acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, keep.b[tn]),
                                                                   __builtin_bit_cast(bf16x8, keep.a[tm]),
                                                                   acc[tm][tn], 0, 0, 0);
          } else {
            const f32x4 av = __builtin_bit_cast(f32x4, keep.a[tm]), bv = __builtin_bit_cast(f32x4, keep.b[tn]);
#pragma unroll
            for (int q = 0; q < 4; ++q)
              acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x2f32(bv[q], av[q], acc[tm][tn], 0, 0, 0);
          }
        }
      __builtin_amdgcn_sched_barrier(0);
      continue;
    }
    mma_kstep<T, TM, TN>(acc, f[j & 1]);
    const int u0 = j * DPK, u1 = (j + 1) * DPK < ND ? (j + 1) * DPK : ND;
#pragma unroll
    for (int u = u0; u < u1; ++u) {
      if (u < BNV)
        dma_unit_b<T, NT, VEC>(bdst, wbase, boff[u], issue_b, u, wv);
      else
        dma_unit_a<T, NT, VEC>(adst, abase, arel[u - BNV], aon && ((okbits >> (u - BNV)) & 1u), cin, u - BNV, wv,
                               tid);
    }
    const int nld = j + 1 < NK ? NLD : 0, ndma = u1 > u0 ? u1 - u0 : 0;
    if constexpr (NMF >= 2 * NLD) {
#pragma unroll
      for (int q = 0; q < NMF; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if (q < nld) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        if (q < ndma) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
      }
    } else {
#pragma unroll
      for (int q = 0; q < NLD; ++q)
        if (q < nld) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
#pragma unroll
      for (int q = 0; q < NMF; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if (q < ndma) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
      }
    }
#pragma unroll
    for (int q = NMF; q < DPK; ++q)
      if (q < ndma) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// SA (single halo buffer) kernels are made to fit several resident blocks per CU: three
// for 64-channel tiles, two for 128-channel ones
template <typename T, int BN, int WM, int WN, int PH, int EPI, bool SEG2, bool F32E, bool SA>
__global__ __launch_bounds__(WM * WN * 64, SA ? (BN <= 64 ? 3 : 2) : 1) void k_conv3(ConvArgs a, Batch g) {
  constexpr int PW = kConvPW, BM = PH * PW;
  constexpr int NT = WM * WN * 64;
  constexpr int TM = BM / (WM * 32), TN = BN / (WN * 32);
  static_assert(TM >= 1 && TN >= 1 && TM * WM * 32 == BM && TN * WN * 32 == BN, "bad wave tiling");
  constexpr int CK = Tr<T>::CK;
  constexpr int VEC = 16 / sizeof(T);
  constexpr int HP = PH + 2, WP = PW + 2;
  constexpr int AROWS = HP * WP;
  constexpr int ANVD = (AROWS * 5 + NT - 1) / NT;   // 16-byte units per thread per halo chunk
  constexpr int AUNITS = ANVD * NT;                   // units written (every wave, padding included)
  constexpr int BNV = (3 * BN * 4 + NT - 1) / NT;
  constexpr int ASZ = AUNITS * VEC, BSZ = BNV * NT * VEC;
  // SA: one halo buffer (more resident blocks per CU; the next chunk's halo is loaded
  // between chunks, while the other blocks compute)
  constexpr int NA = SA ? 1 : 2, SMEM = (NA * ASZ + 2 * BSZ) * (int)sizeof(T);
  static_assert(ANVD <= 32, "halo mask bits");
  static_assert(epi_passes(BM, WN, TN, SMEM) > 0, "epilogue does not fit");
  constexpr bool WIDE = TM * TN >= 16;
  __shared__ __attribute__((aligned(16))) T sm[NA * ASZ + 2 * BSZ];
  if constexpr (WIDE) asm volatile("" ::: "a0");

  // XCD-aware block order: workgroup L runs on XCD L mod 8, which takes the contiguous
  // patch range [xcd PPX, (xcd + 1) PPX) with the NB column blocks of a patch back to
  // back, so those re-read the patch's halo input (and neighbours their shared halo
  // rows) from that XCD's L2
  const int npatch = g.pfx[g.n], nbn = (a.cout + BN - 1) / BN;
  const int ppx = (npatch + 7) / 8;
  const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
  const int patch = xcd * ppx + seq / nbn;
  if (patch >= npatch) return;   // whole block: before any barrier
  const int t = find_tile(g, patch);
  const int lb = patch - g.pfx[t];
  const int h = g.h[t], w = g.w[t];
  // output region a0..a3 of the window (the image-gradient stitch: the tile's owned pixels;
  // the other convolutions: what the pass needs; a pooled layer's region starts on even
  // rows and columns)
  const int oy = g.a0[t], ox = g.a2[t];
  const int ey = g.a1[t], ex = g.a3[t];
  const int nbx = (ex - ox + PW - 1) / PW;
  const int y0 = oy + (lb / nbx) * PH, x0 = ox + (lb % nbx) * PW;
  const int n0 = (seq % nbn) * BN;
  const long long slot = g.slot[t];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wv / WN, wn = wv % WN;
  const int l32 = lane & 31, half = lane >> 5;
  const int lpx = blk_pixel<PW>(l32);   // this lane's pixel in each operand block

  int pidx[TM];
#pragma unroll
  for (int tm = 0; tm < TM; ++tm) {
    const int m = wm * TM * 32 + tm * 32 + lpx;
    pidx[tm] = (m / PW) * WP + (m % PW);
  }
  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const T *in0 = (const T *)a.in + slot * a.in_ss;
  const T *in1 = SEG2 ? (const T *)a.in2 + slot * a.in2_ss : nullptr;
  const T *wp0 = (const T *)a.wp;
  const T *wp1 = (const T *)a.wp2;
  const int nck = a.cin / CK;
  const int nck2 = SEG2 ? a.cin2 / CK : 0;

  // per-lane DMA sources, computed once: halo pixel relative to the block's clamped origin
  // (by, bx) with a valid bit (inside the window, a data unit, inside the patch)
  const int by = max(y0 - 1, 0), bx = max(x0 - 1, 0);
  unsigned arel[ANVD], okbits = 0u, boff[BNV];
#pragma unroll
  for (int i = 0; i < ANVD; ++i) {
    const int p = i * NT + tid;
    const int row = p / 5, unit = p - row * 5;
    const int py = row / WP, px = row - py * WP;
    const int yy = y0 - 1 + py, xx = x0 - 1 + px;
    const int cy = min(max(yy, 0), h - 1), cx = min(max(xx, 0), w - 1);
    arel[i] = (unsigned)((cy - by) * w + (cx - bx));
    const bool ok = row < AROWS && unit < 4 && yy >= 0 && yy < h && xx >= 0 && xx < w;
    okbits |= (ok ? 1u : 0u) << i;
  }
  // no 3x3 segment (nck = 0: the top layer's seeds): the first stage is segment 1's
  const bool seg1_first = nck == 0;
  dma_boff<T, NT, BNV, BN, CK, VEC>(boff, seg1_first ? 1 : 3, a.cout_pad, n0, tid);
  const T *abase0 = seg1_first ? nullptr : in0 + ((long long)by * w + bx) * a.cin;
  const long long wrow = (long long)a.cout_pad * CK;

  T *const A0 = sm, *const A1 = sm + (NA - 1) * ASZ, *const B0 = sm + NA * ASZ, *const B1 = sm + NA * ASZ + BSZ;
  if (!seg1_first) {
    dma_a<T, NT, ANVD, VEC>(A0, abase0, arel, okbits, a.cin, wv, tid);
    dma_b<T, NT, BNV, VEC>(B0, wp0, boff, wv);
  } else if (nck2 > 0) {
    dma_a<T, NT, ANVD, VEC>(A0, in1 + ((long long)by * w + bx) * a.cin2, arel, okbits, a.cin2, wv, tid);
    dma_b<T, NT, BNV, VEC>(B0, wp1, boff, wv);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const int bcol = wn * TN * 32 + l32;
  // halo loads per chunk and wave (a stage may leave them in flight)
  static_assert(ANVD >= 1 && ANVD <= 15, "vmcnt range");
  // each stage passes the workgroup barrier itself and leaves the next stage's first
  // fragments in fr[0]
  KFrag<TM, TN> fr[2];
  if (!seg1_first || nck2 > 0)
    load_kstep<T, TM, TN, BN, CK, VEC>(fr[0], A0, B0, pidx, seg1_first ? WP + 1 : 0, 0, 0, bcol, half);
  if constexpr (SA) {
    // one halo buffer A0: each chunk's last stage issues the next halo chunk (or segment
    // 1's first) halfway through its last k-step; the wait and barrier follow the stage
#pragma unroll 1
    for (int c = 0; c < nck; ++c) {
      const bool odd = c & 1;
      T *const Bx = odd ? B1 : B0, *const By = odd ? B0 : B1;
      const bool more = c + 1 < nck;
      const bool seg = !more && SEG2 && nck2 > 0;
      stage_dma<T, TM, TN, BN, CK, VEC, 3, NT, ANVD, BNV, false, 0>(
          acc, fr, A0, Bx, pidx, 0, bcol, half, nullptr, nullptr, arel, okbits, 0, By, wp0 + (c * 9 + 3) * wrow,
          boff, true, false, A0, By, WP, true, wv, tid);
      stage_dma<T, TM, TN, BN, CK, VEC, 3, NT, ANVD, BNV, false, 0>(
          acc, fr, A0, By, pidx, WP, bcol, half, nullptr, nullptr, arel, okbits, 0, Bx, wp0 + (c * 9 + 6) * wrow,
          boff, true, false, A0, Bx, 2 * WP, true, wv, tid);
      if (seg) dma_boff<T, NT, BNV, BN, CK, VEC>(boff, 1, a.cout_pad, n0, tid);
      const T *wnext = more ? wp0 + (c + 1) * 9 * wrow : wp1;
      const T *anext = more ? abase0 + (c + 1) * CK : (SEG2 ? in1 + ((long long)by * w + bx) * a.cin2 : abase0);
      stage_dma<T, TM, TN, BN, CK, VEC, 3, NT, ANVD, BNV, false, 0, true>(
          acc, fr, A0, Bx, pidx, 2 * WP, bcol, half, A0, anext, arel, okbits, more ? a.cin : a.cin2, By, wnext, boff,
          more || seg, more || seg, A0, By, 0, false, wv, tid);
      __builtin_amdgcn_s_waitcnt(0);
      lds_barrier();
      if (more || seg) load_kstep<T, TM, TN, BN, CK, VEC>(fr[0], A0, By, pidx, more ? 0 : WP + 1, 0, 0, bcol, half);
    }
    if constexpr (SEG2) {
      const T *abase1 = in1 + ((long long)by * w + bx) * a.cin2;
#pragma unroll 1
      for (int c2 = 0; c2 < nck2; ++c2) {
        const int st = 3 * nck + c2;
        const bool more = c2 + 1 < nck2;
        stage_dma<T, TM, TN, BN, CK, VEC, 1, NT, ANVD, BNV, false, 0, true>(
            acc, fr, A0, (st & 1) ? B1 : B0, pidx, WP + 1, bcol, half, A0, abase1 + (c2 + 1) * CK, arel, okbits,
            a.cin2, (st & 1) ? B0 : B1, wp1 + (long long)(c2 + 1) * wrow, boff, more, more, A0, B0, 0, false, wv,
            tid);
        __builtin_amdgcn_s_waitcnt(0);
        lds_barrier();
        if (more) load_kstep<T, TM, TN, BN, CK, VEC>(fr[0], A0, (st & 1) ? B0 : B1, pidx, WP + 1, 0, 0, bcol, half);
      }
    }
  } else {
#pragma unroll 1
  for (int c = 0; c < nck; ++c) {
    const bool odd = c & 1;
    T *const Ac = odd ? A1 : A0, *const An = odd ? A0 : A1;
    T *const Bx = odd ? B1 : B0, *const By = odd ? B0 : B1;
    const bool more = c + 1 < nck;
    const bool seg = !more && SEG2 && nck2 > 0;
    // filter row 0 (B buffer x): prefetch row 1 into y, then the next chunk's halo patch
    // (or segment 1's) into the other A buffer, which has two stages to arrive
    const T *anext = more ? abase0 + (c + 1) * CK : (SEG2 ? in1 + ((long long)by * w + bx) * a.cin2 : abase0);
    stage_dma<T, TM, TN, BN, CK, VEC, 3, NT, ANVD, BNV, true, ANVD>(
        acc, fr, Ac, Bx, pidx, 0, bcol, half, An, anext, arel, okbits, more ? a.cin : a.cin2, By,
        wp0 + (c * 9 + 3) * wrow, boff, true, more || seg, Ac, By, WP, true, wv, tid);
    // filter row 1 (y); prefetch row 2 into x (the halo patch lands with it)
    stage_dma<T, TM, TN, BN, CK, VEC, 3, NT, ANVD, BNV, false, 0>(
        acc, fr, Ac, By, pidx, WP, bcol, half, nullptr, nullptr, arel, okbits, 0, Bx, wp0 + (c * 9 + 6) * wrow,
        boff, true, false, Ac, Bx, 2 * WP, true, wv, tid);
    // filter row 2 (x); prefetch the next chunk's row 0 (or segment 1's weights) into y;
    // the next stage is the next chunk's row 0 or segment 1's first stage
    if (seg) dma_boff<T, NT, BNV, BN, CK, VEC>(boff, 1, a.cout_pad, n0, tid);
    const T *wnext = more ? wp0 + (c + 1) * 9 * wrow : wp1;
    stage_dma<T, TM, TN, BN, CK, VEC, 3, NT, ANVD, BNV, false, 0>(
        acc, fr, Ac, Bx, pidx, 2 * WP, bcol, half, nullptr, nullptr, arel, okbits, 0, By, wnext, boff,
        more || seg, false, An, By, more ? 0 : WP + 1, more || seg, wv, tid);
  }
  if constexpr (SEG2) {
    const T *abase1 = in1 + ((long long)by * w + bx) * a.cin2;
#pragma unroll 1
    for (int c2 = 0; c2 < nck2; ++c2) {
      const int st = 3 * nck + c2, ac = nck + c2;
      const bool more = c2 + 1 < nck2;
      stage_dma<T, TM, TN, BN, CK, VEC, 1, NT, ANVD, BNV, true, 0>(
          acc, fr, (ac & 1) ? A1 : A0, (st & 1) ? B1 : B0, pidx, WP + 1, bcol, half, (ac & 1) ? A0 : A1,
          abase1 + (c2 + 1) * CK, arel, okbits, a.cin2, (st & 1) ? B0 : B1, wp1 + (long long)(c2 + 1) * wrow,
          boff, more, more, (ac & 1) ? A0 : A1, (st & 1) ? B0 : B1, WP + 1, more, wv, tid);
    }
  }
  }
  if constexpr (EPI == EPI_STITCH) {
    // image gradient (FP32 CHW) at the owned pixels: channels 0..2 of the padded 32
    // accumulator element r of lanes 0..31 is channel r of pixel lpx (see mma_kstep)
#pragma unroll
    for (int tm = 0; tm < TM; ++tm) {
      const int m = wm * TM * 32 + tm * 32 + lpx;
      const int py = y0 + m / PW, px = x0 + m % PW;
      if (half == 0 && py < ey && px < ex) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
          a.grad[((long long)r * a.img_h + (g.gy[t] + py)) * a.img_w + (g.gx[t] + px)] = acc[tm][0][r];
      }
    }
  } else {
    conv_epilogue<T, BN, WM, WN, PH, PW, EPI, SMEM, F32E>(acc, sm, a, g, t, slot, y0, x0, h, w, n0, tid, wm, wn, lpx,
                                                      half);
  }
}

template <typename T, int BN, int WM, int WN, int PH, int EPI, bool SEG2, bool F32E = false, bool SA = false>
static hipError_t run_conv3(const ConvArgs &a, const Batch &g, hipStream_t s) {
  const int nblk = g.pfx[g.n];
  if (nblk == 0) return hipSuccess;
  // one-dimensional grid in XCD-aware order (see k_conv3)
  dim3 grid(8 * ((nblk + 7) / 8) * ((a.cout + BN - 1) / BN));
  hipLaunchKernelGGL((k_conv3<T, BN, WM, WN, PH, EPI, SEG2, F32E, SA>), grid, dim3(WM * WN * 64), 0, s, a, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// conv1_1 forward straight from the whole FP32 CHW image (fuses the halo crop).
//   Work item: an 8 x 32 output patch x all 64 output channels, 4 waves (64 px x 64 ch
//   each).  Persistent blocks: a block loads the 64 x 32 weight operand once, then loops
//   over patches.  For each it stages the 3 x 10 x 34 FP32 image patch in LDS (the values
//   were loaded into registers during the previous patch), thread t writes pixel t's
//   im2col row of the 27 (filter tap, colour) values, zero-padded to 32, K = 32 runs on
//   MFMA, and the LDS epilogue applies bias + ReLU and writes 16-byte rows of channels.
// ---------------------------------------------------------------------------------------
// resident blocks per CU: BF16 three (LDS 3 x 50 KB, registers for 3 waves per SIMD),
// FP32 two (its operands need more registers)
template <typename T> constexpr int kImgBlocksPerCU = sizeof(T) == 2 ? 3 : 2;

template <typename T>
__device__ __forceinline__ void img_patch_load(float (&v)[4], const ConvArgs &a, const Batch &g, int patch,
                                               int tid) {
  constexpr int PH = 8, PW = 32, HP = PH + 2, WP = PW + 2;
  const int t = find_tile(g, patch);
  const int lb = patch - g.pfx[t];
  const int h = g.h[t], w = g.w[t];
  const int nbx = (g.a3[t] - g.a2[t] + PW - 1) / PW;   // output region a0..a3
  const int y0 = g.a0[t] + (lb / nbx) * PH, x0 = g.a2[t] + (lb % nbx) * PW;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = tid + i * 256;
    const int c = e / (HP * WP), r = (e / WP) % HP, q = e % WP;
    const int yy = y0 - 1 + r, xx = x0 - 1 + q;
    v[i] = 0.f;
    if (e < 3 * HP * WP && yy >= 0 && yy < h && xx >= 0 && xx < w)
      v[i] = a.img[((long long)c * a.img_h + (g.gy[t] + yy)) * a.img_w + (g.gx[t] + xx)];
  }
}

template <typename T>
__global__ __launch_bounds__(256, kImgBlocksPerCU<T>) void k_conv_img(ConvArgs a, Batch g) {
  constexpr int PH = 8, PW = 32, BM = 256, BN = 64, TM = 2, TN = 2, KP = 32;
  constexpr int HP = PH + 2, WP = PW + 2;               // image patch with its 1-pixel halo
  constexpr int RS = KP + 16 / (int)sizeof(T);         // LDS row stride (elements), 16 B pad
  // im2col rows, then (reused) the two-pass FP32 epilogue tile; weights and the image
  // patch live apart so they survive the epilogue
  constexpr int SMEM = BM * RS * (int)sizeof(T) > BM * (32 + 8) * 4 ? BM * RS * (int)sizeof(T)
                                                                   : BM * (32 + 8) * 4;
  static_assert(3 * HP * WP <= 4 * 256, "image patch exceeds four values per thread");
  __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];
  __shared__ __attribute__((aligned(16))) T Bs[BN * RS];
  __shared__ __attribute__((aligned(16))) float ip[3 * HP * WP];
  T *const As = (T *)smem;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int npatch = g.pfx[g.n];
  {
    // weight operand: packed [KP / CK][1][64][CK]; row n of B = the 32 k-values of n
    const T *wp = (const T *)a.wp;
    constexpr int CK = Tr<T>::CK;
    for (int e = tid; e < BN * KP; e += 256) {
      const int n = e / KP, k = e - n * KP;
      Bs[n * RS + k] = wp[((long long)(k / CK) * a.cout_pad + n) * CK + (k % CK)];
    }
  }
  float iv[4];
  if (blockIdx.x < npatch) img_patch_load<T>(iv, a, g, blockIdx.x, tid);
#pragma unroll 1
  for (int patch = blockIdx.x; patch < npatch; patch += gridDim.x) {
    const int t = find_tile(g, patch);
    const int lb = patch - g.pfx[t];
    const int h = g.h[t], w = g.w[t];
    const int nbx = (g.a3[t] - g.a2[t] + PW - 1) / PW;   // output region a0..a3
    const int y0 = g.a0[t] + (lb / nbx) * PH, x0 = g.a2[t] + (lb % nbx) * PW;
    const long long slot = g.slot[t];
    __syncthreads();   // the previous patch's epilogue is done with smem and ip
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (tid + i * 256 < 3 * HP * WP) ip[tid + i * 256] = iv[i];
    __syncthreads();
    if (patch + (int)gridDim.x < npatch) img_patch_load<T>(iv, a, g, patch + gridDim.x, tid);
    {
      const int ty = tid / PW, tx = tid % PW;
      T row[KP];
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        float v = 0.f;
        if (k < 27) {
          const int tap = k / 3, c = k - 3 * (k / 3);
          v = ip[(c * HP + ty + tap / 3) * WP + tx + tap % 3];
        }
        row[k] = from_f<T>(v);
      }
#pragma unroll
      for (int k = 0; k < KP; ++k) As[tid * RS + k] = row[k];
    }
    __syncthreads();
    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    // lane half g covers k in [16 g, 16 g + 16)
    typename Mma<T>::Frag af[TM], bfr[TN];
    if constexpr (sizeof(T) == 2) {
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        const T *p = &As[(wave * 64 + tm * 32 + l32) * RS + half * 16];
        af[tm].v[0] = *(const bf16x8 *)p;
        af[tm].v[1] = *(const bf16x8 *)(p + 8);
      }
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) {
        const T *p = &Bs[(tn * 32 + l32) * RS + half * 16];
        bfr[tn].v[0] = *(const bf16x8 *)p;
        bfr[tn].v[1] = *(const bf16x8 *)(p + 8);
      }
#pragma unroll
      for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) Mma<T>::mma(acc[tm][tn], bfr[tn], af[tm]);   // channels x pixels
    } else {
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
          const T *p = &As[(wave * 64 + tm * 32 + l32) * RS + half * 16 + hh * 8];
          af[tm].v[0] = *(const f32x4 *)p;
          af[tm].v[1] = *(const f32x4 *)(p + 4);
        }
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
          const T *p = &Bs[(tn * 32 + l32) * RS + half * 16 + hh * 8];
          bfr[tn].v[0] = *(const f32x4 *)p;
          bfr[tn].v[1] = *(const f32x4 *)(p + 4);
        }
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
          for (int tn = 0; tn < TN; ++tn) Mma<T>::mma(acc[tm][tn], bfr[tn], af[tm]);
      }
    }
    __syncthreads();   // the epilogue reuses the im2col buffer
    conv_epilogue<T, BN, 4, 1, PH, PW, EPI_FWD, SMEM, false>(acc, (T *)smem, a, g, t, slot, y0, x0, h, w, 0, tid, wave,
                                                         0, l32, half);
  }
}

// k_conv3 tile configurations: BN output channels, WM x WN waves, PH x 16 pixel patches,
// sa = one halo buffer.  BF16 layers with 256 or 512 output channels and long K loops
// (K = 9 C_in + C_in2 >= 2304) use 4 waves with 128 x 128 wave tiles (AGPR accumulators,
// one block and one wave per SIMD).  Shorter K loops (K = 576 or 1152: every 64- and
// 128-channel layer and conv3_1 with its 128 input channels; K = 512: the top layer's
// residual segment alone), where each block's set-up (about 2 us before its first MFMA) and
// epilogue weigh most, use one halo buffer and several resident blocks per CU, whose
// phases overlap: 64-channel tiles with three (52 KB of LDS), BF16 128-channel tiles (4
// waves of 128 px x 64 ch) with two (76 KB).  FP32 keeps two waves per SIMD throughout.
struct Conv2Cfg { int bn, wm, wn, ph; bool sa; };
constexpr int kLongK = 9 * 256;
static Conv2Cfg conv2_cfg(int precision, int cout, int k = kLongK) {
  if (precision == 1) {
    if (cout <= 64) return {64, 4, 1, 16, true};
    if (cout % 256 == 0 && k >= kLongK) return {256, 2, 2, 16, false};
    return {128, 2, 2, 16, true};
  }
  if (cout <= 64) return {64, 4, 1, 16, true};
  if (cout % 256 == 0) return {256, 2, 4, 16, false};
  return {128, 4, 2, 16, false};
}

int conv_block_rows(int precision, int in_mode, int epi, int cout) {
  if (in_mode == IN_IMAGE) return 8;                       // k_conv_img
  if (epi == EPI_STITCH) return 256 / kConvPW;              // k_conv3 stitch
  return conv2_cfg(precision, cout).ph;                      // k_conv3
}
int conv_block_cols(int precision, int in_mode, int epi, int cout) {
  (void)precision; (void)epi; (void)cout;
  return in_mode == IN_IMAGE ? 32 : kConvPW;
}
int conv_block_px(int precision, int in_mode, int epi, int cout) {
  return conv_block_cols(precision, in_mode, epi, cout) * conv_block_rows(precision, in_mode, epi, cout);
}
int ck_of(int precision) { return precision == 1 ? Tr<bf16>::CK : Tr<float>::CK; }
size_t elem_size(int precision) { return precision == 1 ? 2 : 4; }

template <typename T>
static hipError_t conv_dispatch(int in_mode, int epi, const ConvArgs &a, const Batch &g,
                                hipStream_t s) {
  const bool seg2 = a.in2 != nullptr && a.cin2 > 0;
  if (epi == EPI_STITCH) {
    if (in_mode != IN_NHWC || seg2 || a.cout > 3 || a.cout_pad != 32) return hipErrorInvalidValue;
    return run_conv3<T, 32, 4, 1, 256 / kConvPW, EPI_STITCH, false, false, true>(a, g, s);   // one halo buffer
  }
  const bool small = a.cout <= 64;
  // BF16: the 256-channel tile for long K loops only (see conv2_cfg)
  const bool long256 = a.cout % 256 == 0 && 9 * a.cin + (seg2 ? a.cin2 : 0) >= kLongK;
  if (epi == EPI_FWD) {
    if (seg2) return hipErrorInvalidValue;
    if (in_mode == IN_IMAGE) {
      if (a.cout != 64 || a.rc) return hipErrorInvalidValue;
      const int nblk = g.pfx[g.n];
      if (nblk == 0) return hipSuccess;
      int dev = 0, ncu = 0;
      hipError_t e = hipGetDevice(&dev);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      const int grid = std::min(nblk, kImgBlocksPerCU<T> * ncu);
      hipLaunchKernelGGL(k_conv_img<T>, dim3(grid), dim3(256), 0, s, a, g);
      return hipGetLastError();
    }
    if (in_mode != IN_NHWC) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 2) {
      // F32E: the content layer's FP32 residual needs the FP32 epilogue
#define NST_CONV3_FWD(BN_, WM_, WN_, PH_, SA_)                                             \
  return a.rc ? run_conv3<T, BN_, WM_, WN_, PH_, EPI_FWD, false, true, SA_>(a, g, s)     \
              : run_conv3<T, BN_, WM_, WN_, PH_, EPI_FWD, false, false, SA_>(a, g, s)
      if (small) NST_CONV3_FWD(64, 4, 1, 16, true);
      if (long256) NST_CONV3_FWD(256, 2, 2, 16, false);
      NST_CONV3_FWD(128, 2, 2, 16, true);
#undef NST_CONV3_FWD
    } else {
      if (small) return run_conv3<T, 64, 4, 1, 16, EPI_FWD, false, false, true>(a, g, s);
      if (a.cout % 256 == 0) return run_conv3<T, 256, 2, 4, 16, EPI_FWD, false>(a, g, s);
      return run_conv3<T, 128, 4, 2, 16, EPI_FWD, false>(a, g, s);
    }
  }
  // EPI_BWD; IN_NONE: no 3x3 segment (the top layer's seeds: segment 1 and the epilogue)
  if (in_mode == IN_NONE && (a.cin != 0 || a.in != nullptr)) return hipErrorInvalidValue;
  if (in_mode == IN_NHWC || in_mode == IN_NONE) {
#define NST_CONV3_BWD(BN_, WM_, WN_, PH_, RC_, SA_)                                        \
  return seg2 ? run_conv3<T, BN_, WM_, WN_, PH_, EPI_BWD, true, RC_, SA_>(a, g, s)        \
              : run_conv3<T, BN_, WM_, WN_, PH_, EPI_BWD, false, RC_, SA_>(a, g, s)
    if constexpr (sizeof(T) == 2) {
      if (a.rc) {   // the content residual enters in FP32 (F32E)
        if (small) NST_CONV3_BWD(64, 4, 1, 16, true, true);
        if (long256) NST_CONV3_BWD(256, 2, 2, 16, true, false);
        NST_CONV3_BWD(128, 2, 2, 16, true, true);
      }
      if (small) NST_CONV3_BWD(64, 4, 1, 16, false, true);
      if (long256) NST_CONV3_BWD(256, 2, 2, 16, false, false);
      NST_CONV3_BWD(128, 2, 2, 16, false, true);
    } else {
      if (small) NST_CONV3_BWD(64, 4, 1, 16, false, true);
      if (a.cout % 256 == 0) NST_CONV3_BWD(256, 2, 4, 16, false, false);
      NST_CONV3_BWD(128, 4, 2, 16, false, false);
    }
#undef NST_CONV3_BWD
  }
  return hipErrorInvalidValue;
}

const char *conv_kernel_name(int precision, int in_mode, int epi, const ConvArgs &a) {
  static char buf[8][160];
  static int k = 0;
  char *o = buf[k++ & 7];
  const bool seg2 = a.in2 != nullptr && a.cin2 > 0;
  const char *ty = precision == 1 ? "__bf16" : "float";
  if (in_mode == IN_IMAGE) {
    snprintf(o, 160, "void nst::k_conv_img<%s>(nst::ConvArgs, nst::Batch)", ty);
  } else if (epi == EPI_STITCH) {
    snprintf(o, 160, "void nst::k_conv3<%s, 32, 4, 1, %d, %d, false, false, true>(nst::ConvArgs, nst::Batch)", ty,
             256 / kConvPW, EPI_STITCH);
  } else {
    const Conv2Cfg k = conv2_cfg(precision, a.cout, 9 * a.cin + (seg2 ? a.cin2 : 0));
    const bool f32e = precision == 1 && a.rc != nullptr;
    snprintf(o, 160, "void nst::k_conv3<%s, %d, %d, %d, %d, %d, %s, %s, %s>(nst::ConvArgs, nst::Batch)", ty, k.bn,
             k.wm, k.wn, k.ph, epi, seg2 ? "true" : "false", f32e ? "true" : "false", k.sa ? "true" : "false");
  }
  return o;
}

hipError_t launch_conv(int precision, int in_mode, int epi, const ConvArgs &a, const Batch &g,
                       hipStream_t s) {
  return precision == 1 ? conv_dispatch<bf16>(in_mode, epi, a, g, s)
                        : conv_dispatch<float>(in_mode, epi, a, g, s);
}

// ---------------------------------------------------------------------------------------
// 16-byte vector helpers (VEC = 16 / sizeof(T) channels)
// ---------------------------------------------------------------------------------------
template <typename T> struct Vec {
  static constexpr int N = 16 / sizeof(T);
  union {
    uint4 u;
    T e[N];
  };
};

// Max-pool backward fused with the content seed and the ReLU mask of the pre-pool layer:
//   dZ = ([p is the first maximum of its window] dP + 2 alpha rc) * [A > 0]
// Work item = (pooling window, channel vector); windows cut by floor mode get dP = 0.
template <typename T>
__global__ __launch_bounds__(256) void k_pool_bwd(const T *dp, long long dp_ss, const T *act,
                                                  long long act_ss, const float *rc,
                                                  long long rc_ss, float two_alpha, T *dz,
                                                  long long dz_ss, int C, bool avg, Batch g) {
  const int t = find_tile(g, blockIdx.x);
  const int item = (blockIdx.x - g.pfx[t]) * 256 + threadIdx.x;
  const int h = g.h[t], w = g.w[t];
  // pooling windows of the region a0..a1 x a2..a3 (pooled coordinates; a window past the
  // floor-mode size covers the dropped last row / column, which gets 0)
  const int rw2 = g.a3[t] - g.a2[t];
  constexpr int N = Vec<T>::N;
  const int nv = C / N;
  if (item >= (g.a1[t] - g.a0[t]) * rw2 * nv) return;
  const int v = item % nv, p = item / nv, wy = g.a0[t] + p / rw2, wx = g.a2[t] + p % rw2;
  const long long slot = g.slot[t];
  const bool full = (2 * wy + 1 < h) && (2 * wx + 1 < w);
  Vec<T> av[4], dv;
  bool valid[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int yy = 2 * wy + (k >> 1), xx = 2 * wx + (k & 1);
    valid[k] = yy < h && xx < w;
    av[k].u = make_uint4(0u, 0u, 0u, 0u);
    if (valid[k]) av[k].u = *(const uint4 *)(act + slot * act_ss + ((long long)yy * w + xx) * C + v * N);
  }
  dv.u = make_uint4(0u, 0u, 0u, 0u);
  if (full) dv.u = *(const uint4 *)(dp + slot * dp_ss + ((long long)wy * (w / 2) + wx) * C + v * N);
  // max pool: dP goes to the first maximum in window order; average pool: a quarter to
  // each input (exact in BF16 and FP32)
  int arg[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    float m = to_f(av[0].e[j]);
    int best = 0;
#pragma unroll
    for (int k = 1; k < 4; ++k)
      if (to_f(av[k].e[j]) > m) {
        m = to_f(av[k].e[j]);
        best = k;
      }
    arg[j] = full ? best : -1;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!valid[k]) continue;
    const int yy = 2 * wy + (k >> 1), xx = 2 * wx + (k & 1);
    const long long pix = (long long)yy * w + xx;
    Vec<T> o;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      float val = avg ? (full ? 0.25f * to_f(dv.e[j]) : 0.f) : ((arg[j] == k) ? to_f(dv.e[j]) : 0.f);
      if (rc) val += two_alpha * rc[slot * rc_ss + pix * C + v * N + j];
      if (!(to_f(av[k].e[j]) > 0.f)) val = 0.f;
      o.e[j] = from_f<T>(val);
    }
    *(uint4 *)(dz + slot * dz_ss + pix * C + v * N) = o.u;
  }
}

hipError_t launch_pool_bwd(int precision, const void *dp, long long dp_ss, const void *act,
                           long long act_ss, const float *rc, long long rc_ss, float two_alpha,
                           void *dz, long long dz_ss, int C, bool avg, const Batch &g, hipStream_t s) {
  const int nblk = g.pfx[g.n];
  if (nblk == 0) return hipSuccess;
  if (precision == 1)
    hipLaunchKernelGGL(k_pool_bwd<bf16>, dim3(nblk), dim3(256), 0, s, (const bf16 *)dp, dp_ss,
                       (const bf16 *)act, act_ss, rc, rc_ss, two_alpha, (bf16 *)dz, dz_ss, C, avg, g);
  else
    hipLaunchKernelGGL(k_pool_bwd<float>, dim3(nblk), dim3(256), 0, s, (const float *)dp, dp_ss,
                       (const float *)act, act_ss, rc, rc_ss, two_alpha, (float *)dz, dz_ss, C,
                       avg, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Per-tile Gram partials over owned features (Step 1 of Algorithm 1):
//   part[slot][chunk] = V_chunk^T V_chunk, chunk = kGramChunk owned pixels in row-major
//   order over the owned rectangle.  One workgroup = one 64x64 upper-triangle block of
//   one chunk; wave (wi, wj) computes a 32x32 quadrant with fp32 MFMA 32x32x2, where
//   lane l supplies channel (i0 or j0) + l mod 32 of pixel q + l / 32: both operands are
//   plain coalesced NHWC reads.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gram(const T *act, long long act_ss, int C, Batch g,
                                              float *part, long long part_ss) {
  const int t = find_tile(g, blockIdx.x);
  const int k = blockIdx.x - g.pfx[t];
  const int nb = C / 64;
  int pair = blockIdx.y, bi = 0;
  while (pair >= nb - bi) {
    pair -= nb - bi;
    ++bi;
  }
  const int bj = bi + pair;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int i0 = bi * 64 + (wave >> 1) * 32, j0 = bj * 64 + (wave & 1) * 32;
  const int w = g.w[t];
  const int r0 = g.a0[t], r1 = g.a1[t], c0 = g.a2[t], c1 = g.a3[t];
  const int ow = c1 - c0;
  const int npx = (r1 - r0) * ow;
  const int q0 = k * kGramChunk;
  const int q1 = min(npx, q0 + kGramChunk);
  const T *b = act + g.slot[t] * act_ss;
  int qq = q0 + half;
  int y = r0 + qq / ow, x = c0 + qq % ow;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int q = q0; q < q1; q += 2) {
    float av = 0.f, bv = 0.f;
    if (qq < q1) {
      const long long p = ((long long)y * w + x) * C;
      av = to_f(b[p + i0 + l32]);
      bv = to_f(b[p + j0 + l32]);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    qq += 2;
    x += 2;
    while (x >= c1) {
      x -= ow;
      ++y;
    }
  }
  float *o = part + g.slot[t] * part_ss + (long long)k * C * C;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = i0 + 8 * (r >> 2) + 4 * half + (r & 3);
    o[(long long)i * C + j0 + l32] = acc[r];
  }
}

// BF16 Gram partials: same chunks and output layout as k_gram, on bf16 MFMA.  A stage of
// 64 owned pixels is written channel-major into LDS (row = channel, 64 pixels + pad), so
// that each lane's operand is 8 consecutive pixels of one channel; products are exact in
// FP32 and accumulate in FP32 within the chunk.  One LDS stage buffer (the next stage's
// loads are in registers during the MFMAs; a second barrier per stage guards the buffer),
// so that three workgroups fit on a CU and keep more loads in flight.  Block CB x CB of
// the Gram per workgroup, 4 waves in 2 x 2.
template <int CB>
__global__ __launch_bounds__(256, 3) void k_gram_bf16(const bf16 *act, long long act_ss, int C,
                                                   Batch g, float *part, long long part_ss) {
  constexpr int SP = 64, RS = SP + 8;                  // pixels per stage, LDS row stride
  constexpr int TB = CB / 64;                           // 32x32 blocks per wave per dim
  // stage loads: item u of an operand = (pixel pair u % 32, channel group u / 32), two
  // 16-byte loads; lanes 0-31 of a wave cover one group's 64 pixels, lanes 32-63 the next
  // group, so the packed 32-bit channel-major writes hit 64 distinct banks
  constexpr int NI = (SP / 2) * (CB / 8);               // items per operand per stage
  constexpr int PT = 2 * NI / 256;                      // items per thread (both operands)
  static_assert((2 * NI) % 256 == 0 && SP == 64, "stage items per thread");
  // channel-major stage: the next stage's loads are in registers while the MFMAs of the
  // current one run
  __shared__ __attribute__((aligned(16))) bf16 At[1][CB * RS];
  __shared__ __attribute__((aligned(16))) bf16 Bt[1][CB * RS];
  const int t = find_tile(g, blockIdx.x);
  const int k = blockIdx.x - g.pfx[t];
  const int nb = C / CB;
  int pair = blockIdx.y, bi = 0;
  while (pair >= nb - bi) {
    pair -= nb - bi;
    ++bi;
  }
  const int bj = bi + pair;
  const bool diag = bi == bj;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int wi = wave >> 1, wj = wave & 1;
  const int w = g.w[t];
  const int r0 = g.a0[t], c0 = g.a2[t], c1 = g.a3[t];
  const int ow = c1 - c0;
  const int npx = (g.a1[t] - r0) * ow;
  const int q0 = k * kGramChunk;
  const int q1 = min(npx, q0 + kGramChunk);
  const bf16 *b = act + g.slot[t] * act_ss;
  f32x16 acc[TB][TB];
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  Vec<bf16> pre[PT][2];
  auto load_stage = [&](int qs) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int v = tid + i * 256;
      const int op = v >= NI, u = v - op * NI;
      const int pp = u & 31, cg = u >> 5;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int q = qs + 2 * pp + e;
        pre[i][e].u = make_uint4(0u, 0u, 0u, 0u);
        if (q < q1 && (!op || !diag)) {
          const int y = r0 + q / ow, x = c0 + q % ow;
          pre[i][e].u = *(const uint4 *)(b + ((long long)y * w + x) * C + (op ? bj : bi) * CB + cg * 8);
        }
      }
    }
  };
  load_stage(q0);
  const int buf = 0;
  for (int qs = q0; qs < q1; qs += SP) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int v = tid + i * 256;
      const int op = v >= NI, u = v - op * NI;
      const int pp = u & 31, cg = u >> 5;
      if (op && diag) continue;
      unsigned *dst = (unsigned *)(op ? Bt[buf] : At[buf]);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const unsigned lo = __builtin_bit_cast(unsigned short, pre[i][0].e[j]);
        const unsigned hi = __builtin_bit_cast(unsigned short, pre[i][1].e[j]);
        dst[((cg * 8 + j) * RS + 2 * pp) >> 1] = lo | (hi << 16);
      }
    }
    __syncthreads();
    if (qs + SP < q1) load_stage(qs + SP);
    const bf16 *Asrc = At[buf];
    const bf16 *Bsrc = diag ? At[buf] : Bt[buf];
#pragma unroll
    for (int ks = 0; ks < SP / 16; ++ks) {
      bf16x8 fa[TB], fb[TB];
#pragma unroll
      for (int i = 0; i < TB; ++i)
        fa[i] = *(const bf16x8 *)(&Asrc[(wi * 32 * TB + i * 32 + l32) * RS + ks * 16 + half * 8]);
#pragma unroll
      for (int j = 0; j < TB; ++j)
        fb[j] = *(const bf16x8 *)(&Bsrc[(wj * 32 * TB + j * 32 + l32) * RS + ks * 16 + half * 8]);
#pragma unroll
      for (int i = 0; i < TB; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  float *o = part + g.slot[t] * part_ss + (long long)k * C * C;
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ii = bi * CB + wi * 32 * TB + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        const int jj = bj * CB + wj * 32 * TB + j * 32 + l32;
        o[(long long)ii * C + jj] = acc[i][j][r];
      }
}

// tilesum[t][i][j] = sum over the tile's chunks (in order) of part[.][k][min(i,j)][max(i,j)]
__global__ __launch_bounds__(256) void k_gram_tile_reduce(const float *part, long long part_ss,
                                                          int C, Batch g, double *tilesum) {
  const int t = blockIdx.y;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= C * C) return;
  const int i = e / C, j = e - i * C;
  const int ii = min(i, j), jj = max(i, j);
  const int nch = g.pfx[t + 1] - g.pfx[t];
  const float *p = part + g.slot[t] * part_ss + (long long)ii * C + jj;
  double s = 0.0;
  for (int k = 0; k < nch; ++k) s += (double)p[(long long)k * C * C];
  tilesum[(long long)t * C * C + e] = s;
}

// The same sums over 32 x 32 output tiles with coalesced loads: thread (ty, tx) of an
// output tile sums, in chunk order, the partial at row ty, column tx of the upper-triangle
// tile that holds the tile or its mirror image; through LDS the lower-triangle outputs
// take the transposed sums.  Every output element gets the same sequence of additions as
// above; for C not a multiple of 32 the kernel above is used.
__global__ __launch_bounds__(1024) void k_gram_tile_reduce32(const float *part, long long part_ss, int C,
                                                             Batch g, double *tilesum) {
  __shared__ double sm[32][33];
  const int t = blockIdx.y;
  const int nb = C / 32;
  const int bi = blockIdx.x / nb, bj = blockIdx.x - (blockIdx.x / nb) * nb;
  const int si = min(bi, bj), sj = max(bi, bj);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int nch = g.pfx[t + 1] - g.pfx[t];
  const long long cc = (long long)C * C;
  const float *q = part + g.slot[t] * part_ss + (long long)(si * 32 + ty) * C + sj * 32 + tx;
  // in chunk order; the loads of 16 chunks go out together
  double s = 0.0;
  int k = 0;
  for (; k + 16 <= nch; k += 16) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = q[(k + u) * cc];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += (double)v[u];
  }
  for (; k < nch; ++k) s += (double)q[k * cc];
  sm[ty][tx] = s;   // sum of part[.][si 32 + ty][sj 32 + tx]
  __syncthreads();
  // output (i, j) = (bi 32 + ty, bj 32 + tx) needs part[min(i, j)][max(i, j)]
  const double v = bi < bj ? sm[ty][tx] : bi > bj ? sm[tx][ty] : (ty <= tx ? sm[ty][tx] : sm[tx][ty]);
  tilesum[(long long)t * cc + (long long)(bi * 32 + ty) * C + bj * 32 + tx] = v;
}

__global__ __launch_bounds__(256) void k_gram_accum(const double *tilesum, int n_tiles, int CC,
                                                    double *gacc) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= CC) return;
  double s = gacc[e];
  for (int t = 0; t < n_tiles; ++t) s += tilesum[(long long)t * CC + e];
  gacc[e] = s;
}

hipError_t launch_gram(int precision, const void *act, long long act_ss, int C, const Batch &g,
                       float *part, long long part_ss, hipStream_t s) {
  const int nblk = g.pfx[g.n];
  if (nblk == 0) return hipSuccess;
  if (precision == 1) {
    const int cb = C >= 128 ? 128 : 64;
    const int nb = C / cb;
    dim3 grid(nblk, nb * (nb + 1) / 2);
    if (cb == 128)
      hipLaunchKernelGGL(k_gram_bf16<128>, grid, dim3(256), 0, s, (const bf16 *)act, act_ss, C, g,
                         part, part_ss);
    else
      hipLaunchKernelGGL(k_gram_bf16<64>, grid, dim3(256), 0, s, (const bf16 *)act, act_ss, C, g,
                         part, part_ss);
    return hipGetLastError();
  }
  const int nb = C / 64;
  dim3 grid(nblk, nb * (nb + 1) / 2);
  hipLaunchKernelGGL(k_gram<float>, grid, dim3(256), 0, s, (const float *)act, act_ss, C, g, part,
                     part_ss);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Channel sums of the owned style features (the mean of Sec. 3.2, Algorithm 1 Step 1):
// per 2048-pixel chunk of a tile's owned region (the Gram's chunks) an FP32 sum per channel,
// then per tile an FP64 sum over its chunks in chunk order, added to the global sums in
// tile order.  In a chunk, thread (pixel group pg, channel vector cg) adds pixels
// pg, pg + PG, ... with 16-byte loads; the PG group sums are then added in group order.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_chan_partial(const T *act, long long act_ss, int C, Batch g,
                                                      float *part, long long part_ss) {
  constexpr int VEC = 16 / sizeof(T);
  __shared__ float red[256 * VEC];
  const int t = find_tile(g, blockIdx.x);
  const int j = blockIdx.x - g.pfx[t];
  const int w = g.w[t];
  const int r0 = g.a0[t], c0 = g.a2[t], ow = g.a3[t] - g.a2[t];
  const int npx = (g.a1[t] - r0) * ow;
  const int p0 = j * kGramChunk, p1 = min(npx, p0 + kGramChunk);
  const int cpv = C / VEC, pgs = 256 / cpv;          // threads per pixel, pixel groups
  const int cg = threadIdx.x % cpv, pg = threadIdx.x / cpv;
  const T *b = act + g.slot[t] * act_ss + cg * VEC;
  float acc[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
  if (pg < pgs) {
    for (int p = p0 + pg; p < p1; p += pgs) {
      const int y = r0 + p / ow, x = c0 + p % ow;
      typedef T TV __attribute__((ext_vector_type(VEC)));
      const TV v = *(const TV *)(b + ((long long)y * w + x) * C);
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] += to_f(v[e]);
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) red[pg * C + cg * VEC + e] = acc[e];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += 256) {
    float s = 0.f;
    for (int q = 0; q < pgs; ++q) s += red[q * C + c];
    part[g.slot[t] * part_ss + (long long)j * C + c] = s;
  }
}

__global__ __launch_bounds__(256) void k_chan_accum(const float *part, long long part_ss, int C, Batch g,
                                                    double *csum) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= C) return;
  double s = csum[c];
  for (int t = 0; t < g.n; ++t) {
    const float *q = part + g.slot[t] * part_ss + c;
    double st = 0.0;
    for (int j = 0; j < g.pfx[t + 1] - g.pfx[t]; ++j) st += (double)q[(long long)j * C];
    s += st;
  }
  csum[c] = s;
}

hipError_t launch_chan_sums(int precision, const void *act, long long act_ss, int C, const Batch &g,
                            float *part, long long part_ss, double *csum, hipStream_t s) {
  const int nblk = g.pfx[g.n];
  if (nblk == 0) return hipSuccess;
  if (precision == 1)
    hipLaunchKernelGGL(k_chan_partial<bf16>, dim3(nblk), dim3(256), 0, s, (const bf16 *)act, act_ss, C, g, part,
                       part_ss);
  else
    hipLaunchKernelGGL(k_chan_partial<float>, dim3(nblk), dim3(256), 0, s, (const float *)act, act_ss, C, g,
                       part, part_ss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chan_accum, dim3((C + 255) / 256), dim3(256), 0, s, part, part_ss, C, g, csum);
  return hipGetLastError();
}

hipError_t launch_gram_tile_reduce(const float *part, long long part_ss, int C, const Batch &g,
                                   double *tilesum, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  if (C % 32 == 0) {
    dim3 grid((C / 32) * (C / 32), g.n);
    hipLaunchKernelGGL(k_gram_tile_reduce32, grid, dim3(1024), 0, s, part, part_ss, C, g, tilesum);
  } else {
    dim3 grid((C * C + 255) / 256, g.n);
    hipLaunchKernelGGL(k_gram_tile_reduce, grid, dim3(256), 0, s, part, part_ss, C, g, tilesum);
  }
  return hipGetLastError();
}

hipError_t launch_gram_accum(const double *tilesum, int n_tiles, int C, double *gacc,
                             hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram_accum, dim3((C * C + 255) / 256), dim3(256), 0, s, tilesum, n_tiles,
                     C * C, gacc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Content energy partials over owned content features: sum of rc^2 (rc = V - F_c), FP64,
// fixed-order block reduction; then a single-thread accumulation in (tile, block) order.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_content_partial(const float *rc, long long rc_ss, int C,
                                                         Batch g, double *part,
                                                         long long part_ss) {
  __shared__ double red[256];
  const int t = find_tile(g, blockIdx.x);
  const int blk = blockIdx.x - g.pfx[t];
  const int w = g.w[t];
  const int r0 = g.a0[t], r1 = g.a1[t], c0 = g.a2[t], c1 = g.a3[t];
  const int ow = c1 - c0, npx = (r1 - r0) * ow;
  const float *b = rc + g.slot[t] * rc_ss;
  double s = 0.0;
  // element e = pl C + c, e = tid + 256 m in order of m; pixel pl and channel c advance
  // incrementally and the pixel's address is recomputed only when pl changes
  int pl = threadIdx.x / C, c = threadIdx.x - pl * C;
  int cur = -1;
  const float *row = b;
  for (int e = threadIdx.x; e < kContentBlockPx * C; e += 256) {
    const int q = blk * kContentBlockPx + pl;
    if (q < npx) {
      if (pl != cur) {
        cur = pl;
        row = b + ((long long)(r0 + q / ow) * w + (c0 + q % ow)) * C;
      }
      const double d = row[c];
      s += d * d;
    }
    c += 256;
    while (c >= C) {
      c -= C;
      ++pl;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[g.slot[t] * part_ss + blk] = red[0];
}

// acc += the block partials of the batch, tile by tile in tile order: a tile's partials
// are added by a fixed tree (thread j sums the partials j, j + 256, ... in order, then
// the 256 sums pairwise), and each tile sum is added to acc in turn.  The order depends
// only on the tile, not on how tiles are grouped into launches, so any tile batching
// gives the same bits.
__global__ __launch_bounds__(256) void k_content_accum(const double *part, long long part_ss, Batch g,
                                                       double *acc) {
  __shared__ double red[256];
  double total = threadIdx.x == 0 ? acc[0] : 0.0;
  for (int t = 0; t < g.n; ++t) {
    const int nb = g.pfx[t + 1] - g.pfx[t];
    const double *p = part + g.slot[t] * part_ss;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += p[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) total += red[0];
    __syncthreads();   // red is rewritten by the next tile
  }
  if (threadIdx.x == 0) acc[0] = total;
}

hipError_t launch_content_partial(const float *rc, long long rc_ss, int C, const Batch &g,
                                  double *part, long long part_ss, hipStream_t s) {
  const int nblk = g.pfx[g.n];
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_content_partial, dim3(nblk), dim3(256), 0, s, rc, rc_ss, C, g, part,
                     part_ss);
  return hipGetLastError();
}

hipError_t launch_content_accum(const double *part, long long part_ss, const Batch &g,
                                double *acc, hipStream_t s) {
  hipLaunchKernelGGL(k_content_accum, dim3(1), dim3(256), 0, s, part, part_ss, g, acc);
  return hipGetLastError();
}

// Owned features of a layer -> whole-image fp32 map (h x w x C).
template <typename T>
__global__ __launch_bounds__(256) void k_stitch_feats(const T *act, long long act_ss, int C,
                                                      Batch g, float *feats, int fw) {
  const int t = find_tile(g, blockIdx.x);
  const int item = (blockIdx.x - g.pfx[t]) * 256 + threadIdx.x;
  constexpr int N = Vec<T>::N;
  const int nv = C / N;
  const int r0 = g.a0[t], r1 = g.a1[t], c0 = g.a2[t], c1 = g.a3[t];
  const int ow = c1 - c0;
  if (item >= (r1 - r0) * ow * nv) return;
  const int v = item % nv, p = item / nv;
  const int y = r0 + p / ow, x = c0 + p % ow;
  Vec<T> q;
  q.u = *(const uint4 *)(act + g.slot[t] * act_ss + ((long long)y * g.w[t] + x) * C + v * N);
  float *o = feats + ((long long)(g.gy[t] + y) * fw + (g.gx[t] + x)) * C + v * N;
#pragma unroll
  for (int j = 0; j < N; ++j) o[j] = to_f(q.e[j]);
}

hipError_t launch_stitch_feats(int precision, const void *act, long long act_ss, int C,
                               const Batch &g, float *feats, int feats_w, hipStream_t s) {
  const int nblk = g.pfx[g.n];
  if (nblk == 0) return hipSuccess;
  if (precision == 1)
    hipLaunchKernelGGL(k_stitch_feats<bf16>, dim3(nblk), dim3(256), 0, s, (const bf16 *)act,
                       act_ss, C, g, feats, feats_w);
  else
    hipLaunchKernelGGL(k_stitch_feats<float>, dim3(nblk), dim3(256), 0, s, (const float *)act,
                       act_ss, C, g, feats, feats_w);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Small utility kernels
// ---------------------------------------------------------------------------------------
__global__ void k_fill_f64(double *p, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f32(float *p, size_t n, float v) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float *p, size_t n, float v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ void k_fill_u32(unsigned *p, size_t n, unsigned v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Grid-stride count of non-finite elements: a per-thread count, one atomic per wave.
template <typename T>
__global__ __launch_bounds__(256) void k_count_nonfinite(const T *p, size_t n, unsigned *count) {
  unsigned c = 0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    c += isfinite(p[i]) ? 0u : 1u;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

template <typename T>
static hipError_t count_nonfinite(const T *p, size_t n, unsigned *count, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_count_nonfinite<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, count);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite_f32(const float *p, size_t n, unsigned *count, hipStream_t s) {
  return count_nonfinite(p, n, count, s);
}

hipError_t launch_count_nonfinite_f64(const double *p, size_t n, unsigned *count, hipStream_t s) {
  return count_nonfinite(p, n, count, s);
}

__global__ void k_div_f64(const double *in, double *out, size_t n, double d) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = in[i] / d;
}
hipError_t launch_gram_normalize(const double *gacc, double *g, size_t n, double n_p,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_div_f64, dim3((n + 255) / 256), dim3(256), 0, s, gacc, g, n, n_p);
  return hipGetLastError();
}

// Style energy terms, one workgroup per style layer, and the packed residual operand,
// one thread per element:
//   e_style[l] = w_l sum_ij (G - Ghat)_ij^2                      (Eq. 3)
//   B[k = i][n = j] = (2 w_l / n_p) (D_ij + D_ji), D = G - Ghat   (Table 1, Gram row)
// packed as [i / CK][j][i mod CK] in compute precision.  Each energy sum runs over the
// elements in a fixed order (thread stride, then a tree over the workgroup).
__global__ __launch_bounds__(256) void k_style_energy(const double *g, const double *gt, StyleTermsArgs a,
                                                      double *e_style) {
  __shared__ double red[256];
  const int l = blockIdx.x;
  const int C = a.C[l];
  const double *G = g + a.off[l], *H = gt + a.off[l];
  double s = 0.0;
  // elements e = tid + 256 m in order of m; the loads of 8 consecutive m go out together
  // (a few workgroups only: the latency of one load per step would not be hidden)
  const int CC = C * C;
  int e = threadIdx.x;
  for (; e + 7 * 256 < CC; e += 8 * 256) {
    double gv[8], hv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      gv[q] = G[e + q * 256];
      hv[q] = H[e + q * 256];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double dij = gv[q] - hv[q];
      s += dij * dij;
    }
  }
  for (; e < CC; e += 256) {
    const double dij = G[e] - H[e];
    s += dij * dij;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  double el = a.w[l] * red[0];
  if (a.mx) {
    // Eq. 5: w' ||mean_x - mean_t||^2 + w'' ||std_x - std_t||^2, std = (diag G - mean^2)^(1/2)
    __syncthreads();
    const double *mx = a.mx + a.moff[l], *mt = a.mt + a.moff[l];
    double sm = 0.0, ss = 0.0;
    for (int c = threadIdx.x; c < C; c += 256) {
      const double dm = mx[c] - mt[c];
      const double sx = sqrt(fmax(G[(long long)c * C + c] - mx[c] * mx[c], 0.0));
      const double st = sqrt(fmax(H[(long long)c * C + c] - mt[c] * mt[c], 0.0));
      sm += dm * dm;
      ss += (sx - st) * (sx - st);
    }
    red[threadIdx.x] = a.w1[l] * sm + a.w2[l] * ss;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    el += red[0];
  }
  if (threadIdx.x == 0) e_style[l] = el;
}

template <typename T>
__global__ __launch_bounds__(256) void k_style_pack(const double *g, const double *gt, StyleTermsArgs a, T *dt) {
  constexpr int CK = Tr<T>::CK;
  const int l = blockIdx.y;
  const int C = a.C[l];
  const long long u = (long long)blockIdx.x * 256 + threadIdx.x;   // packed index
  if (u >= (long long)((C + CK - 1) / CK) * C * CK) return;
  const int i_lo = (int)(u % CK);
  const long long r = u / CK;
  const int j = (int)(r % C), i = (int)(r / C) * CK + i_lo;
  if (i >= C) return;
  const double *G = g + a.off[l], *H = gt + a.off[l];
  const double coef = 2.0 * a.w[l] * a.inv_np[l];
  const double dij = G[(long long)i * C + j] - H[(long long)i * C + j];
  const double dji = G[(long long)j * C + i] - H[(long long)j * C + i];
  double v = coef * (dij + dji);
  if (a.mx && i == j) {
    // Table 1 rows 3-4: the std seed (2 w'' / n_p)(V - mean)(std - std_t) / std is
    // V diag(r) - mean r with r = (2 w'' / n_p)(std - std_t) / std (0 where std = 0); diag(r)
    // joins the residual operand, and the per-channel rest, with the mean seed
    // (2 w' / n_p)(mean - mean_t), is the constant ms added to every pixel's adjoint
    const double mx = a.mx[a.moff[l] + i], mt = a.mt[a.moff[l] + i];
    const double sx = sqrt(fmax(G[(long long)i * C + i] - mx * mx, 0.0));
    const double st = sqrt(fmax(H[(long long)i * C + i] - mt * mt, 0.0));
    const double r = sx > 0.0 ? 2.0 * a.w2[l] * a.inv_np[l] * (sx - st) / sx : 0.0;
    v += r;
    a.msb[a.moff[l] + i] = (float)(2.0 * a.w1[l] * a.inv_np[l] * (mx - mt) - r * mx);
  }
  dt[a.dt_off[l] + u] = from_f<T>((float)v);
}

hipError_t launch_style_terms(int precision, const double *g, const double *gt,
                              const StyleTermsArgs &a, void *dt, double *e_style, hipStream_t s) {
  if (a.n_style == 0) return hipSuccess;
  hipLaunchKernelGGL(k_style_energy, dim3(a.n_style), dim3(256), 0, s, g, gt, a, e_style);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int ck = precision == 1 ? Tr<bf16>::CK : Tr<float>::CK;
  long long most = 0;
  for (int l = 0; l < a.n_style; ++l)
    most = std::max(most, (long long)((a.C[l] + ck - 1) / ck) * a.C[l] * ck);
  const dim3 grid((unsigned)((most + 255) / 256), a.n_style);
  if (precision == 1)
    hipLaunchKernelGGL(k_style_pack<bf16>, grid, dim3(256), 0, s, g, gt, a, (bf16 *)dt);
  else
    hipLaunchKernelGGL(k_style_pack<float>, grid, dim3(256), 0, s, g, gt, a, (float *)dt);
  return hipGetLastError();
}

__global__ void k_energy_total(const double *ec, const double *e_style, int n_style,
                               double alpha, double *energy) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double c = alpha * ec[0];
  double e = c;
  for (int l = 0; l < n_style; ++l) {
    energy[2 + l] = e_style[l];
    e += e_style[l];
  }
  energy[0] = e;
  energy[1] = c;
}

hipError_t launch_energy_total(const double *ec, const double *e_style, int n_style,
                               double alpha, double *energy, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_total, dim3(1), dim3(64), 0, s, ec, e_style, n_style, alpha,
                     energy);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Device scratch for the allocation-free entry point: one static array per GPU the library
// runs on, held until the process ends.  Host code never uses the array's name as an
// address; scratch_init looks up each device's copy once, with that device current, and
// later calls take the stored address.
// ---------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void *scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace nst
