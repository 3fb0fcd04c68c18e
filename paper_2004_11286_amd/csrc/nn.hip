// nn.hip -- the learned surrogate of libmclbm (include/mclbm_nn.h): 3-D
// convolutions with 3x3x3 kernels as implicit GEMMs on gfx950's BF16 matrix
// cores (v_mfma_f32_32x32x16_bf16), their two backward passes, the loss, Adam
// and the mole-content residual.
//
// Activations are BF16, 16 channels of a node contiguous, so one lane's 16-byte
// load is 8 consecutive channels of one node. A convolution computes
// out^T[co][node] = sum_tap W_tap[co][ci] in[node + d_tap][ci]: the weights of a
// tap (row co, ci contiguous) are the MFMA's A operand, staged in LDS and shared
// by the four waves of a workgroup; the neighbour activations are the B operand,
// staged in LDS per group of three taps; the accumulator holds 4 consecutive
// output channels of one node per lane group, so results leave as 8- or 16-byte
// vector stores. A workgroup computes 256 nodes of one tube (64 per wave, two
// 32-node column blocks) for all output channels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mclbm_nn.h"
#include "nn_internal.hpp"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TILE = 256;      // nodes per workgroup
constexpr int WIDTH = 64;      // hidden channels
constexpr int CIN0 = 32;       // input channels of layer 0 (fields, second terms, conditioning, zeros)
constexpr int COUTL = 32;      // output channels of the last layer (padded)
constexpr int NTAP = 27;
constexpr int MAXC = 16;
constexpr size_t ALIGN = 256;

inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct NTube {
  int64_t base;
  int32_t nx, ny, nz;
  int32_t first_tile, ntiles;
  int32_t pad;
  int64_t ntot;   // nodes of all tubes (the stride of the activation layout)
};

// Activations and activation gradients (BF16) are chunk-major: [C / 16][n][16]
// over the n nodes of all tubes, so the 16 channels one MFMA step takes from a
// node are 32 contiguous bytes and a wavefront's gather of consecutive nodes
// covers whole cache lines (node-major rows of 64 channels would use 32 bytes of
// each 128-byte line per load). Channel counts are multiples of 16.
__device__ __forceinline__ size_t aidx(const NTube& tb, int64_t gnode, int c)
{
  return (size_t)(c >> 4) * (size_t)tb.ntot * 16 + (size_t)gnode * 16 + (size_t)(c & 15);
}

// Workgroup b of a launch runs on XCD b mod 8, each with its own L2. The
// convolution of a tile reads the rows one y or z step away, tiles nx / TILE and
// nx ny / TILE further on; renumbering so that XCD k takes the tiles
// [k q, (k + 1) q) (q = nb / 8, the last nb mod 8 unchanged) keeps those rows in
// the L2 of the XCD that staged them.
__device__ inline int xcd_tile(int b, int nb)
{
  constexpr int NXCD = 8;
  const int q = nb / NXCD;
  if (b >= q * NXCD) return b;
  return (b % NXCD) * q + b / NXCD;
}

// The last layer's raw FP32 output is channel-major, [COUTL][n] over the n nodes
// of all tubes: the kernels that read it take one channel of consecutive nodes
// per load (node-major rows would put each lane on a cache line of its own).
__device__ __forceinline__ size_t yidx(const NTube& tb, int64_t gnode, int c)
{
  return (size_t)c * (size_t)tb.ntot + (size_t)gnode;
}

// The tube and tube-local node of lane-independent tile `tile`.
__device__ inline NTube tube_of(const NTube* tubes, const int32_t* tile_tube, int ntubes, int tile)
{
  return tubes[ntubes > 1 ? tile_tube[tile] : 0];
}

__device__ inline int64_t wrap_index(const NTube& tb, int x, int y, int z)
{
  y += (y < 0) ? tb.ny : 0;
  y -= (y >= tb.ny) ? tb.ny : 0;
  z += (z < 0) ? tb.nz : 0;
  z -= (z >= tb.nz) ? tb.nz : 0;
  return tb.base + x + (int64_t)tb.nx * (y + (int64_t)tb.ny * z);
}

// ---------------------------------------------------------------------------
// Convolution (forward, and backward with respect to the input)
// ---------------------------------------------------------------------------
// EPI 0: + bias, ReLU, BF16 out; EPI 1: + bias, FP32 out (channel-major, yidx); EPI 2: times the
// ReLU mask (mask > 0), BF16 out. EPI 0 and 1 gather forward, in(x + d) with x
// clamped to the tube (replicate padding at the walls) and y, z wrapped; EPI 2
// is the adjoint, in(x - d) with nothing from outside the tube, plus, at a wall
// node, the ghost's share.
//
// The 27 taps run as 9 groups (dy, dz) of three dx taps. For a group, the
// activations the tile's nodes need are the nodes t0 - 1 .. t0 + TILE of the
// tile's range shifted by (dy, dz), with y and z wrapped: TILE + 2 rows of CIN
// channels, staged in LDS once and read by the group's three taps (gathering
// every tap from the caches instead moves three times the data through them).
// Node p of the tile reads row p + 1 + dx while x + dx stays in the tube (the node
// p + dx of the same x row); beyond a wall the forward reads row p + 1 (replicate
// padding) and the adjoint zero, plus row p + 1 as the ghost's share at a wall
// node. The next group's rows are loaded into registers while the
// current group's products run.
template <int CIN, int COUT, int EPI>
__global__ __launch_bounds__(256) void k_conv(const NTube* __restrict__ tubes, const int32_t* __restrict__ tile_tube,
                                                int ntubes, const bf16* __restrict__ W, const float* __restrict__ bias,
                                                const bf16* __restrict__ in, const bf16* __restrict__ mask,
                                                void* __restrict__ out)
{
  static_assert(CIN % 16 == 0 && COUT % 32 == 0, "channel counts must fit the 32x32x16 MFMA");
  constexpr int SIGN = EPI == 2 ? -1 : 1;
  constexpr int LS = CIN + 8;              // LDS row stride (bf16) of weights and staged rows
  constexpr int MB = COUT / 32;
  constexpr int KC = CIN / 16;
  constexpr int CHUNKS = COUT * CIN / 8;   // 16-byte pieces of one tap's weights
  constexpr int PT = (CHUNKS + 255) / 256;
  constexpr int RCH = CIN / 8;             // 16-byte pieces of one staged row
  static_assert(2 * RCH <= 256, "the two extra rows are spread over the first threads");
  __shared__ __attribute__((aligned(16))) bf16 wl[2][COUT * LS];
  __shared__ __attribute__((aligned(16))) bf16 sl[(TILE + 2) * LS];

  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const NTube tb = tube_of(tubes, tile_tube, ntubes, tile);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n_t = tb.nx * tb.ny * tb.nz;
  const int t0 = (tile - tb.first_tile) * TILE;
  int pos[2], xs[2];
  bool valid[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    pos[b] = wave * 64 + b * 32 + (lane & 31);
    valid[b] = t0 + pos[b] < n_t;
    xs[b] = valid[b] ? (t0 + pos[b]) % tb.nx : 0;
  }
  // staged rows of this thread: row threadIdx.x (all its pieces), and one piece
  // of the rows TILE and TILE + 1 on the first 2 RCH threads
  const int r1 = TILE + (int)threadIdx.x / RCH, c1 = (int)threadIdx.x % RCH;
  const bool extra = threadIdx.x < 2 * RCH;
  int jx[2], jy[2], jz[2];
  bool jin[2];
  {
    const int rows[2] = {(int)threadIdx.x, r1};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int j = t0 + rows[k] - 1;
      jin[k] = j >= 0 && j < n_t && (k == 0 || extra);
      const int i = jin[k] ? j : 0;
      jx[k] = i % tb.nx;
      const int r = i / tb.nx;
      jy[k] = r % tb.ny;
      jz[k] = r / tb.ny;
    }
  }
  bf16x8 sreg[RCH], sx1;
  auto sload = [&](int g) {
    const int dy = SIGN * (g % 3 - 1), dz = SIGN * (g / 3 - 1);
    const int64_t nb0 = wrap_index(tb, jx[0], jy[0] + dy, jz[0] + dz);
#pragma unroll
    for (int c = 0; c < RCH; ++c) {
      if (jin[0]) {
        sreg[c] = *(const bf16x8*)(in + aidx(tb, nb0, c * 8));
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) sreg[c][e] = (bf16)0.f;
      }
    }
    if (jin[1]) {
      const int64_t nb1 = wrap_index(tb, jx[1], jy[1] + dy, jz[1] + dz);
      sx1 = *(const bf16x8*)(in + aidx(tb, nb1, c1 * 8));
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) sx1[e] = (bf16)0.f;
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int c = 0; c < RCH; ++c) *(bf16x8*)(&sl[threadIdx.x * LS + c * 8]) = sreg[c];
    if (extra) *(bf16x8*)(&sl[r1 * LS + c1 * 8]) = sx1;
  };
  f32x16 acc[MB][2];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[mb][b][v] = 0.f;

  bf16x8 wreg[PT];
  auto load_w = [&](int tap) {
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      const int ch = threadIdx.x + p * 256;
      if (ch < CHUNKS) wreg[p] = *(const bf16x8*)(W + (size_t)tap * COUT * CIN + (size_t)ch * 8);
    }
  };
  auto store_w = [&](int buf) {
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      const int ch = threadIdx.x + p * 256;
      if (ch < CHUNKS) {
        const int row = ch / (CIN / 8), col = (ch % (CIN / 8)) * 8;
        *(bf16x8*)(&wl[buf][row * LS + col]) = wreg[p];
      }
    }
  };
  const int khalf = 8 * (lane >> 5);
  // a tube one node wide in y and z wraps every (dy, dz) onto the node itself:
  // the nine groups stage the same rows, so they are staged once
  const bool restage = tb.ny > 1 || tb.nz > 1;
  sload(0);
  sstore();
  load_w(0);
  store_w(0);
  __syncthreads();
  for (int g = 0; g < 9; ++g) {
    if (g + 1 < 9 && restage) sload(g + 1);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int tap = 3 * g + d;
      const int buf = tap & 1;
      if (tap + 1 < NTAP) load_w(tap + 1);
      const int dx = SIGN * (d - 1);
      bf16x8 bop[2][KC];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int x = xs[b] + dx;
        const bool inside = x >= 0 && x < tb.nx;
        const int row = pos[b] + 1 + (inside ? dx : 0);
        const bool use = valid[b] && (SIGN > 0 || inside);
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
          if (use) {
            bop[b][kc] = *(const bf16x8*)(&sl[row * LS + kc * 16 + khalf]);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) bop[b][kc][e] = (bf16)0.f;
          }
        }
        if constexpr (SIGN < 0) {
          // the ghost's share: at a wall node the forward took the ghost of tap
          // dx = -1 at x = 0 (dx = +1 at x = nx - 1) from the wall node itself, so
          // the wall node also collects in(wall node) under that tap; the two
          // operands are added in FP32 and rounded once
          const bool wall = valid[b] && ((xs[b] == 0 && dx == 1) || (xs[b] == tb.nx - 1 && dx == -1));
          if (wall) {
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
              const bf16x8 e8 = *(const bf16x8*)(&sl[(pos[b] + 1) * LS + kc * 16 + khalf]);
#pragma unroll
              for (int e = 0; e < 8; ++e) bop[b][kc][e] = (bf16)((float)bop[b][kc][e] + (float)e8[e]);
            }
          }
        }
      }
#pragma unroll
      for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const bf16x8 a = *(const bf16x8*)(&wl[buf][(mb * 32 + (lane & 31)) * LS + kc * 16 + khalf]);
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[mb][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bop[b][kc], acc[mb][b], 0, 0, 0);
        }
      if (tap + 1 < NTAP) store_w(buf ^ 1);
      __syncthreads();
    }
    if (g + 1 < 9 && restage) {
      sstore();
      __syncthreads();
    }
  }
  // epilogue: lane holds channels co0 .. co0+3 of its node for each group g
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    if (!valid[b]) continue;
    const int64_t gn = tb.base + t0 + pos[b];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int co0 = mb * 32 + 8 * g + 4 * (lane >> 5);
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = acc[mb][b][4 * g + j];
        if (EPI == 0 || EPI == 1) {
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] += bias[co0 + j];
        }
        if (EPI == 0) {
          bf16x4 o;
#pragma unroll
          for (int j = 0; j < 4; ++j) o[j] = (bf16)fmaxf(v[j], 0.f);
          *(bf16x4*)((bf16*)out + aidx(tb, gn, co0)) = o;
        } else if (EPI == 1) {
#pragma unroll
          for (int j = 0; j < 4; ++j) ((float*)out)[yidx(tb, gn, co0 + j)] = v[j];
        } else {
          const bf16x4 mk = *(const bf16x4*)(mask + aidx(tb, gn, co0));
          bf16x4 o;
#pragma unroll
          for (int j = 0; j < 4; ++j) o[j] = (bf16)((float)mk[j] > 0.f ? v[j] : 0.f);
          *(bf16x4*)((bf16*)out + aidx(tb, gn, co0)) = o;
        }
      }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[tap][co][ci] = sum_nodes dY[node][co] X[node + d_tap][ci]
// (the forward's gather: x clamped to the tube, y and z wrapped)
// ---------------------------------------------------------------------------
// The reduction runs over nodes, so both operands are staged transposed in LDS
// (channel rows, node columns) for 128-node chunks; workgroup (g, (dy, dz)) sums
// the chunks g, g + G, ... for the taps dx = -1, 0, +1 and writes its partials
// [g][tap][COUT][CINP]. With yz_fixed >= 0 the grid has one (dy, dz) column, that
// one: when every tube is one node wide in y and z, the y and z shifts wrap onto
// the node itself and the nine (dy, dz) columns would sum the same products in
// the same order, so k_wgrad_reduce reads the one for all of them. The partials
// are then [g][dx][COUT][CINP], and nine times as many workgroups share the
// chunks (the same buffer).
constexpr int WCH = 128;   // nodes per staged chunk

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad(const NTube* __restrict__ tubes, const int32_t* __restrict__ tile_tube,
                                               int ntubes, int nchunks, const bf16* __restrict__ dY,
                                               const bf16* __restrict__ X, float* __restrict__ partial,
                                               int yz_fixed)
{
  constexpr int CINP = CIN < 32 ? 32 : CIN;
  constexpr int S = WCH + 8;
  constexpr int NB = (COUT / 32) * (CINP / 32);
  constexpr int PW = (NB + 3) / 4;
  // one workgroup takes the three taps dx = -1, 0, +1 of one (dy, dz): the output
  // gradient chunk is staged once for all three, and the three shifted input
  // windows overlap (two of them come from the cache)
  __shared__ __attribute__((aligned(16))) bf16 dyt[COUT * S];
  __shared__ __attribute__((aligned(16))) bf16 xt[3][CINP * S];
  const int yz = yz_fixed >= 0 ? yz_fixed : (int)blockIdx.y, g = blockIdx.x, G = gridDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int dy = yz % 3 - 1, dz = yz / 3 - 1;
  const int tap0 = 9 * (dz + 1) + 3 * (dy + 1);   // taps tap0 + k, dx = k - 1
  f32x16 acc[3][PW];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int q = 0; q < PW; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[k][q][v] = 0.f;
  if (CIN < CINP) {
    for (int e = threadIdx.x; e < 3 * (CINP - CIN) * S; e += 256) {
      const int k = e / ((CINP - CIN) * S);
      xt[k][CIN * S + e % ((CINP - CIN) * S)] = (bf16)0.f;
    }
  }
  const int khalf = 8 * (lane >> 5);
  // 4 * WCH staging items over 256 threads, two each: item < WCH stages dY of node
  // item, item WCH + k WCH + i stages X of node i shifted by dx = k - 1. A chunk's
  // items are loaded into registers while the previous chunk's MFMAs run.
  constexpr int C8 = (COUT > CIN ? COUT : CIN) / 8;
  bf16x8 st[2][C8];
  auto load_items = [&](int ch) {
    const int tile = ch >> 1;
    const NTube tb = tube_of(tubes, tile_tube, ntubes, tile);
    const int n_t = tb.nx * tb.ny * tb.nz;
    const int node0 = (tile - tb.first_tile) * TILE + (ch & 1) * WCH;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int item = threadIdx.x + 256 * r;
      const int node = node0 + (item & (WCH - 1));
      const bool valid = node < n_t;
      if (item < WCH) {
#pragma unroll
        for (int c8 = 0; c8 < COUT / 8; ++c8) {
          if (valid) {
            st[r][c8] = *(const bf16x8*)(dY + aidx(tb, tb.base + node, c8 * 8));
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) st[r][c8][j] = (bf16)0.f;
          }
        }
      } else {
        const int dx = item / WCH - 2;
        int x = 0, y = 0, z = 0;
        if (valid) {
          x = node % tb.nx;
          const int rr = node / tb.nx;
          y = rr % tb.ny;
          z = rr / tb.ny;
        }
        // replicate padding: x clamped to the tube; y, z wrapped
        const int xx = x + dx < 0 ? 0 : (x + dx >= tb.nx ? tb.nx - 1 : x + dx);
        const int64_t nb = wrap_index(tb, xx, y + dy, z + dz);
#pragma unroll
        for (int c8 = 0; c8 < CIN / 8; ++c8) {
          if (valid) {
            st[r][c8] = *(const bf16x8*)(X + aidx(tb, nb, c8 * 8));
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) st[r][c8][j] = (bf16)0.f;
          }
        }
      }
    }
  };
  auto store_items = [&]() {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int item = threadIdx.x + 256 * r;
      const int i = item & (WCH - 1);
      if (item < WCH) {
#pragma unroll
        for (int c8 = 0; c8 < COUT / 8; ++c8)
#pragma unroll
          for (int j = 0; j < 8; ++j) dyt[(c8 * 8 + j) * S + i] = st[r][c8][j];
      } else {
        const int k = item / WCH - 1;
#pragma unroll
        for (int c8 = 0; c8 < CIN / 8; ++c8)
#pragma unroll
          for (int j = 0; j < 8; ++j) xt[k][(c8 * 8 + j) * S + i] = st[r][c8][j];
      }
    }
  };
  if (g < nchunks) load_items(g);
  for (int ch = g; ch < nchunks; ch += G) {
    store_items();
    __syncthreads();
    if (ch + G < nchunks) load_items(ch + G);
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      const int blk = wave + 4 * q;
      if (blk < NB) {
        const int mb = blk / (CINP / 32), cb = blk % (CINP / 32);
#pragma unroll 2
        for (int k0 = 0; k0 < WCH; k0 += 16) {
          const bf16x8 a = *(const bf16x8*)(&dyt[(mb * 32 + (lane & 31)) * S + k0 + khalf]);
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const bf16x8 b = *(const bf16x8*)(&xt[k][(cb * 32 + (lane & 31)) * S + k0 + khalf]);
            acc[k][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[k][q], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      const int blk = wave + 4 * q;
      if (blk >= NB) continue;
      const int mb = blk / (CINP / 32), cb = blk % (CINP / 32);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = mb * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
        const int col = cb * 32 + (lane & 31);
        const size_t pt = yz_fixed >= 0 ? (size_t)g * 3 + k : (size_t)g * NTAP + tap0 + k;
        partial[(pt * COUT + row) * CINP + col] = acc[k][q][v];
      }
    }
}

// grad[tap][co][j] += sum_g partial[g][tap][co][col] over the parameters of a
// layer (co < co_r, j < ci_r) from the padded partials [G][tap][COUTP][CINP],
// fixed order. With second terms (P > 0, layer 0) parameter column j < C also
// collects column C + j (j < P) divided by 256, and the conditioning
// parameters j >= C sit at column j + P. With flat != 0 (tubes one node wide in
// y and z) the partials are [G][dx][COUTP][CINP]: each sum is formed once per dx
// and added to the gradient of its nine taps.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ partial, int G, int COUTP,
                                                      int CINP, int co_r, int ci_r, int C, int P,
                                                      float* __restrict__ grad, int flat)
{
  // 32 outputs per workgroup, each summed by 8 threads over a slice of g; the
  // slices are then added in order (flat: one output per dx, whose nine taps
  // share the sum; else one per tap)
  constexpr int NSL = 8;
  __shared__ float red[NSL][32][2];
  const int jj = threadIdx.x & 31, sl = threadIdx.x >> 5;
  const int k = blockIdx.x * 32 + jj;
  const int nout = (flat ? 3 : NTAP) * co_r * ci_r;
  const int npt = flat ? 3 : NTAP;
  float s = 0.f, s2 = 0.f;
  int j = 0, co = 0, tap = 0;
  if (k < nout) {
    j = k % ci_r;
    co = (k / ci_r) % co_r;
    tap = k / (ci_r * co_r);                   // flat: tap = dx + 1
    const int col = (P > 0 && j >= C) ? j + P : j;
    const int g0 = (int)((int64_t)G * sl / NSL), g1 = (int)((int64_t)G * (sl + 1) / NSL);
    for (int g = g0; g < g1; ++g) {
      const size_t row = (((size_t)g * npt + tap) * COUTP + co) * CINP;
      s += partial[row + col];
      if (P > 0 && j < P) s2 += partial[row + C + j];
    }
  }
  red[sl][jj][0] = s;
  red[sl][jj][1] = s2;
  __syncthreads();
  if (sl != 0 || k >= nout) return;
  float t = 0.f, t2 = 0.f;
#pragma unroll
  for (int q = 0; q < NSL; ++q) {
    t += red[q][jj][0];
    t2 += red[q][jj][1];
  }
  const float v = t + t2 * (1.f / 256.f);
  if (!flat) {
    grad[k] += v;
    return;
  }
  for (int yz = 0; yz < 9; ++yz)               // tap 9 (dz + 1) + 3 (dy + 1) + (dx + 1)
    grad[((size_t)(3 * yz + tap) * co_r + co) * ci_r + j] += v;
}

// Bias gradient partials: partial[tile][c] = sum over the tile's nodes of dY[node][c]
// (C = 16, 32 or 64). Wave w takes the 16-channel chunk w % (C / 16) of every
// (4 / (C / 16))-th group of 64 nodes starting at group w / (C / 16): each lane
// reads the chunk's 32 contiguous bytes of its nodes (a wave covers whole
// lines), sums them per channel, the lanes are added by a butterfly and the
// waves of a chunk in order.
__global__ __launch_bounds__(256) void k_bgrad(const NTube* __restrict__ tubes, const int32_t* __restrict__ tile_tube,
                                               int ntubes, int C, const bf16* __restrict__ dY,
                                               float* __restrict__ partial)
{
  __shared__ float red[4][16];
  const int tile = blockIdx.x;
  const NTube tb = tube_of(tubes, tile_tube, ntubes, tile);
  const int n_t = tb.nx * tb.ny * tb.nz;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nch = C / 16, nparts = 4 / nch;
  const int ch = wave % nch, part = wave / nch;
  const int t0 = (tile - tb.first_tile) * TILE;
  float s[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) s[k] = 0.f;
  for (int i = part * 64 + lane; i < TILE; i += 64 * nparts) {
    if (t0 + i < n_t) {
      const bf16x8* src = (const bf16x8*)(dY + aidx(tb, tb.base + t0 + i, ch * 16));
      const bf16x8 a = src[0], b = src[1];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        s[e] += (float)a[e];
        s[8 + e] += (float)b[e];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s[k] += __shfl_xor(s[k], off, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 16; ++k) red[wave][k] = s[k];
  }
  __syncthreads();
  if ((int)threadIdx.x < C) {
    const int c = threadIdx.x;
    float t = 0.f;
    for (int p = 0; p < nparts; ++p) t += red[p * nch + c / 16][c % 16];
    partial[(size_t)tile * C + c] = t;
  }
}

// grad[c] += sum_t partial[t][c] for the real channels c < count (row stride C):
// block c, thread i sums tiles i, i + 256, ..., then a tree in LDS; a fixed order,
// so the result is deterministic.
__global__ __launch_bounds__(256) void k_bgrad_reduce(const float* __restrict__ partial, int ntiles, int C,
                                                      int count, float* __restrict__ grad)
{
  __shared__ float red[256];
  const int c = blockIdx.x;
  if (c >= count) return;
  float s = 0.f;
  for (int t = threadIdx.x; t < ntiles; t += 256) s += partial[(size_t)t * C + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[c] += red[0];
}

// ---------------------------------------------------------------------------
// Input packing, output unpacking, loss
// ---------------------------------------------------------------------------
struct Norm {
  float in_shift[MAXC], in_scale[MAXC], out_scale[COUTL], weight[COUTL];
};

// act0[node][c]: for c < C the normalised field v_c = (f_c - shift_c) scale_c
// in BF16 (hi_c); for C <= c < C + P the second term lo = bf16((v - hi) 256)
// of field c - C; for C + P <= c < C + P + S the tube's conditioning values;
// zero above.
__global__ __launch_bounds__(256) void k_pack_in(const NTube* __restrict__ tubes, const int32_t* __restrict__ tile_tube,
                                                 int ntubes, int C, int P, int S, Norm nm, const float* __restrict__ f,
                                                 const float* __restrict__ cond, bf16* __restrict__ act0)
{
  const int tile = blockIdx.x;
  const int t = ntubes > 1 ? tile_tube[tile] : 0;
  const NTube tb = tubes[t];
  const int n_t = tb.nx * tb.ny * tb.nz;
  const int node = (tile - tb.first_tile) * TILE + threadIdx.x;
  if (node >= n_t) return;
  const float* ft = f + (size_t)C * tb.base;
  auto value = [&](int c) -> float {
    if (c < C) return (ft[(size_t)c * n_t + node] - nm.in_shift[c]) * nm.in_scale[c];
    if (c < C + P) {
      const int k = c - C;
      const float v = (ft[(size_t)k * n_t + node] - nm.in_shift[k]) * nm.in_scale[k];
      return (v - (float)(bf16)v) * 256.f;
    }
    if (c < C + P + S) return cond[(size_t)t * S + (c - C - P)];
    return 0.f;
  };
#pragma unroll
  for (int c8 = 0; c8 < CIN0 / 8; ++c8) {
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (bf16)value(c8 * 8 + j);
    *(bf16x8*)(act0 + aidx(tb, tb.base + node, c8 * 8)) = v;
  }
}

// fields_out[c][node] = f[c][node] + y[c][node] out_scale_c.
__global__ __launch_bounds__(256) void k_unpack_out(const NTube* __restrict__ tubes, const int32_t* __restrict__ tile_tube,
                                                    int ntubes, int C, Norm nm, const float* __restrict__ f,
                                                    const float* __restrict__ y, float* __restrict__ fo)
{
  const int tile = blockIdx.x;
  const NTube tb = tube_of(tubes, tile_tube, ntubes, tile);
  const int n_t = tb.nx * tb.ny * tb.nz;
  const int node = (tile - tb.first_tile) * TILE + threadIdx.x;
  if (node >= n_t) return;
  const size_t o = (size_t)C * tb.base;
  for (int c = 0; c < C; ++c)
    fo[o + (size_t)c * n_t + node] = f[o + (size_t)c * n_t + node] + y[yidx(tb, tb.base + node, c)] * nm.out_scale[c];
}

// Loss and its gradient with respect to the raw output y: with the target
// change r_c = (target_c - f_c) / out_scale_c, loss = (1/N) sum w_c (y_c - r_c)^2.
__global__ __launch_bounds__(256) void k_loss(const NTube* __restrict__ tubes, const int32_t* __restrict__ tile_tube,
                                              int ntubes, int C, Norm nm, double inv_n, const float* __restrict__ f,
                                              const float* __restrict__ target, const float* __restrict__ y,
                                              bf16* __restrict__ dY, double* __restrict__ partial)
{
  __shared__ double red[256];
  const int tile = blockIdx.x;
  const NTube tb = tube_of(tubes, tile_tube, ntubes, tile);
  const int n_t = tb.nx * tb.ny * tb.nz;
  const int node = (tile - tb.first_tile) * TILE + threadIdx.x;
  double l = 0.0;
  if (node < n_t) {
    const size_t o = (size_t)C * tb.base;
    const int64_t gn = tb.base + node;
    bf16 d[COUTL];
#pragma unroll
    for (int c = 0; c < COUTL; ++c) d[c] = (bf16)0.f;
    for (int c = 0; c < C; ++c) {
      const size_t k = o + (size_t)c * n_t + node;
      const double r = ((double)target[k] - (double)f[k]) / nm.out_scale[c];
      const double e = (double)y[yidx(tb, gn, c)] - r;
      l += nm.weight[c] * e * e;
      d[c] = (bf16)(float)(2.0 * nm.weight[c] * e * inv_n);
    }
#pragma unroll
    for (int c8 = 0; c8 < COUTL / 8; ++c8) {
      bf16x8 v;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = d[c8 * 8 + j];
      *(bf16x8*)(dY + aidx(tb, gn, c8 * 8)) = v;
    }
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[tile] = red[0];
}

// ---------------------------------------------------------------------------
// Conservative output: the network predicts, for each species s, the fluxes of
// its molar density n_s = p X_s / T through the faces between a node x and
// x + e_a (a = x, y, z), and the changes of T and u. The new densities are
// n_s - sum_a (F_a(x) - F_a(x - e_a)): a discrete divergence, so every tube
// keeps its moles of each species exactly. The faces at the walls carry no
// flux; y and z are periodic. Then p = T sum_s n_s and X_s = n_s / sum n.
// Output channels: F for species s and direction a at 3 s + a, then T, u.
// ---------------------------------------------------------------------------
struct Geo {
  int x, y, z;
};

__device__ inline Geo geo_of(const NTube& tb, int node)
{
  const int r = node / tb.nx;
  return {node % tb.nx, r % tb.ny, r / tb.ny};
}

// Face from node g towards +e_a exists (a wall face at x = nx - 1 does not).
__device__ inline bool face_open(const NTube& tb, const Geo& g, int a) { return a != 0 || g.x + 1 < tb.nx; }

__device__ inline int64_t shifted(const NTube& tb, Geo g, int a, int d)
{
  if (a == 0) g.x += d;
  if (a == 1) g.y += d;
  if (a == 2) g.z += d;
  return wrap_index(tb, g.x, g.y, g.z);
}

__device__ inline Geo shifted_geo(const NTube& tb, Geo g, int a, int d)
{
  if (a == 0) g.x += d;
  if (a == 1) g.y = (g.y + d + tb.ny) % tb.ny;
  if (a == 2) g.z = (g.z + d + tb.nz) % tb.nz;
  return g;
}

__global__ __launch_bounds__(256) void k_unpack_cons(const NTube* __restrict__ tubes,
                                                     const int32_t* __restrict__ tile_tube, int ntubes, int M,
                                                     Norm nm, const float* __restrict__ f,
                                                     const float* __restrict__ y, float* __restrict__ fo)
{
  const int tile = blockIdx.x;
  const NTube tb = tube_of(tubes, tile_tube, ntubes, tile);
  const int n_t = tb.nx * tb.ny * tb.nz;
  const int node = (tile - tb.first_tile) * TILE + threadIdx.x;
  if (node >= n_t) return;
  const int C = M + 5;
  const size_t o = (size_t)C * tb.base;
  auto fld = [&](int c) -> double { return (double)f[o + (size_t)c * n_t + node]; };
  const Geo g = geo_of(tb, node);
  const int64_t gn = tb.base + node;
  const double T = fld(M), p = fld(M + 4);
  double nn[MAXC], sum = 0.0;
  for (int s = 0; s < M; ++s) {
    double div = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double sc = nm.out_scale[3 * s + a];
      if (face_open(tb, g, a)) div += (double)y[yidx(tb, gn, 3 * s + a)] * sc;
      const bool lower = a != 0 || g.x > 0;
      if (lower) div -= (double)y[yidx(tb, shifted(tb, g, a, -1), 3 * s + a)] * sc;
    }
    nn[s] = p * fld(s) / T - div;
    sum += nn[s];
  }
  const double T1 = T + (double)y[yidx(tb, gn, 3 * M)] * nm.out_scale[3 * M];
  for (int s = 0; s < M; ++s) fo[o + (size_t)s * n_t + node] = (float)(nn[s] / sum);
  fo[o + (size_t)M * n_t + node] = (float)T1;
  for (int k = 0; k < 3; ++k)
    fo[o + (size_t)(M + 1 + k) * n_t + node] =
        (float)(fld(M + 1 + k) + (double)y[yidx(tb, gn, 3 * M + 1 + k)] * nm.out_scale[3 * M + 1 + k]);
  fo[o + (size_t)(M + 4) * n_t + node] = (float)(T1 * sum);
}

// Target fluxes through the x faces: along each x row of a tube, F*_s(x) =
// -sum_{x' <= x} (n*_s - n_s)(x'), with n = p X / T of the input fields f and of
// the target. On a tube with walls and fields uniform in y and z this is the one
// flux field whose divergence gives the target change (zero through the left
// wall); it pins the uniform flux offset that the divergence alone cannot see.
// Two passes: k_flux_change writes each node's n*_s - n_s (formed in FP64) into
// fs [n][M], one thread per node; k_flux_target then scans every (row, species)
// in FP64, one thread each, in place.
__global__ __launch_bounds__(256) void k_flux_change(const NTube* __restrict__ tubes,
                                                     const int32_t* __restrict__ tile_tube, int ntubes, int M,
                                                     const float* __restrict__ f, const float* __restrict__ target,
                                                     float* __restrict__ fs)
{
  const int tile = blockIdx.x;
  const NTube tb = tube_of(tubes, tile_tube, ntubes, tile);
  const int n_t = tb.nx * tb.ny * tb.nz;
  const int node = (tile - tb.first_tile) * TILE + threadIdx.x;
  if (node >= n_t) return;
  const size_t o = (size_t)(M + 5) * tb.base;
  auto at = [&](const float* a, int c) -> double { return (double)a[o + (size_t)c * n_t + node]; };
  for (int s = 0; s < M; ++s)
    fs[(tb.base + node) * M + s] =
        (float)(at(target, M + 4) * at(target, s) / at(target, M) - at(f, M + 4) * at(f, s) / at(f, M));
}

// Row r of tube t (ny nz rows of nx nodes), species s: wave ((t's first row + r)
// M + s) of a launch over every row of every tube (row_first[t]: rows of the
// tubes before t) turns the row's flux-change values into the x fluxes they
// imply, F(x) = -sum_{x' <= x} d(x'), an inclusive prefix sum in FP64 over 64
// nodes at a time with the running total carried between them.
__global__ __launch_bounds__(256) void k_flux_target(const NTube* __restrict__ tubes, const int32_t* __restrict__ row_first,
                                                     int ntubes, int64_t nrows, int M, float* __restrict__ fs)
{
  const int64_t id = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (id >= nrows * M) return;                 // uniform over the wave
  const int64_t row = id / M;
  const int s = (int)(id % M);
  int lo = 0, hi = ntubes - 1;                 // the tube: last t with row_first[t] <= row
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (row_first[mid] <= row) lo = mid;
    else hi = mid - 1;
  }
  const NTube tb = tubes[lo];
  float* p = fs + (tb.base + (row - row_first[lo]) * tb.nx) * M + s;
  double carry = 0.0;
  for (int x0 = 0; x0 < tb.nx; x0 += 64) {
    const int x = x0 + lane;
    double v = x < tb.nx ? -(double)p[(size_t)x * M] : 0.0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double t = __shfl_up(v, off, 64);
      if (lane >= off) v += t;
    }
    v += carry;
    if (x < tb.nx) p[(size_t)x * M] = (float)v;
    carry = __shfl(v, 63, 64);
  }
}

// Loss of the conservative output on the conserved and transported variables,
// in physical units: (1/N) sum [ sum_s w_s (n_s - n*_s)^2 + w_T (T - T*)^2 +
// sum_k w_u,k (u_k - u*_k)^2 + w_F sum_s (F_s,x - F*_s,x)^2 (open x faces) ],
// weights w = nm.weight[0..M+4] (w_F in the p slot, which this form does not
// fit), F* from k_flux_target. Writes the loss partials, dL/dn_s per node into
// gn_out [n][M], and the T and u part of the output gradient (the flux part
// follows in k_loss_cons_flux).
__global__ __launch_bounds__(256) void k_loss_cons(const NTube* __restrict__ tubes,
                                                   const int32_t* __restrict__ tile_tube, int ntubes, int M,
                                                   Norm nm, double inv_n, const float* __restrict__ fo,
                                                   const float* __restrict__ target, const float* __restrict__ y,
                                                   const float* __restrict__ fs, float* __restrict__ gn_out,
                                                   bf16* __restrict__ dY, double* __restrict__ partial)
{
  __shared__ double red[256];
  const int tile = blockIdx.x;
  const NTube tb = tube_of(tubes, tile_tube, ntubes, tile);
  const int n_t = tb.nx * tb.ny * tb.nz;
  const int node = (tile - tb.first_tile) * TILE + threadIdx.x;
  double l = 0.0;
  if (node < n_t) {
    const int C = M + 5;
    const size_t o = (size_t)C * tb.base;
    const int64_t gn = tb.base + node;
    auto at = [&](const float* a, int c) -> double { return (double)a[o + (size_t)c * n_t + node]; };
    for (int s = 0; s < M; ++s) {
      const double e = at(fo, M + 4) * at(fo, s) / at(fo, M) - at(target, M + 4) * at(target, s) / at(target, M);
      l += nm.weight[s] * e * e;
      gn_out[gn * M + s] = (float)(2.0 * nm.weight[s] * e * inv_n);
    }
    const double wf = nm.weight[M + 4];
    if (wf != 0.0 && node % tb.nx + 1 < tb.nx) {
      for (int s = 0; s < M; ++s) {
        const double e = (double)y[yidx(tb, gn, 3 * s)] * nm.out_scale[3 * s] - (double)fs[gn * M + s];
        l += wf * e * e;
      }
    }
    bf16 d[COUTL];
#pragma unroll
    for (int c = 0; c < COUTL; ++c) d[c] = (bf16)0.f;
    for (int k = 0; k < 4; ++k) {
      const double e = at(fo, M + k) - at(target, M + k);
      l += nm.weight[M + k] * e * e;
      d[3 * M + k] = (bf16)(float)(2.0 * nm.weight[M + k] * e * nm.out_scale[3 * M + k] * inv_n);
    }
#pragma unroll
    for (int c8 = 0; c8 < COUTL / 8; ++c8) {
      bf16x8 v;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = d[c8 * 8 + j];
      *(bf16x8*)(dY + aidx(tb, gn, c8 * 8)) = v;
    }
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[tile] = red[0];
}

// Flux part of the output gradient: F_a(x) lowers n at x and raises it at
// x + e_a, so dL/dF_a(x) = dL/dn(x + e_a) - dL/dn(x) on an open face, 0 on a wall;
// on an open x face the flux term adds 2 w_F (F_x - F*_x) / N.
__global__ __launch_bounds__(256) void k_loss_cons_flux(const NTube* __restrict__ tubes,
                                                        const int32_t* __restrict__ tile_tube, int ntubes, int M,
                                                        Norm nm, double inv_n, const float* __restrict__ gn_in,
                                                        const float* __restrict__ y, const float* __restrict__ fs,
                                                        bf16* __restrict__ dY)
{
  const int tile = blockIdx.x;
  const NTube tb = tube_of(tubes, tile_tube, ntubes, tile);
  const int n_t = tb.nx * tb.ny * tb.nz;
  const int node = (tile - tb.first_tile) * TILE + threadIdx.x;
  if (node >= n_t) return;
  const Geo g = geo_of(tb, node);
  const int64_t gn = tb.base + node;
  for (int a = 0; a < 3; ++a) {
    const bool open = face_open(tb, g, a);
    const int64_t up = open ? shifted(tb, g, a, +1) : gn;
    for (int s = 0; s < M; ++s) {
      double v = open ? (double)(gn_in[up * M + s] - gn_in[gn * M + s]) : 0.0;
      if (a == 0 && open && nm.weight[M + 4] != 0.f)
        v += 2.0 * nm.weight[M + 4] * ((double)y[yidx(tb, gn, 3 * s)] * nm.out_scale[3 * s] - (double)fs[gn * M + s]) *
             inv_n;
      dY[aidx(tb, gn, 3 * s + a)] = (bf16)(float)(v * nm.out_scale[3 * s + a]);
    }
  }
}

// Per-tile moles S_s = sum p X_s / T (species s < M, T at component M, p at
// component M + 4), FP64.
__global__ __launch_bounds__(256) void k_mole_sums(const NTube* __restrict__ tubes, const int32_t* __restrict__ tile_tube,
                                                   int ntubes, int C, int M, const float* __restrict__ f,
                                                   double* __restrict__ partial)
{
  __shared__ double red[256];
  const int tile = blockIdx.x;
  const NTube tb = tube_of(tubes, tile_tube, ntubes, tile);
  const int n_t = tb.nx * tb.ny * tb.nz;
  const int node = (tile - tb.first_tile) * TILE + threadIdx.x;
  const size_t o = (size_t)C * tb.base;
  for (int s = 0; s < M; ++s) {
    double v = 0.0;
    if (node < n_t)
      v = (double)f[o + (size_t)(M + 4) * n_t + node] * (double)f[o + (size_t)s * n_t + node] /
          (double)f[o + (size_t)M * n_t + node];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)tile * M + s] = red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Optimiser and weight packing
// ---------------------------------------------------------------------------
// Adam (Kingma and Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// w -= lr (m / bc1) / (sqrt(v / bc2) + eps); then g = 0.
__global__ void k_adam(int64_t n, float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       float* __restrict__ g, float lr, float b1, float b2, float eps, float bc1, float bc2)
{
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  w[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
  g[k] = 0.f;
}

// Input column i of layer 0 -> parameter column, and its weight factor: the
// field columns c < C are parameters c, the second terms C <= i < C + P reuse
// the weights of fields i - C divided by 256 (hi + lo / 256 is the field), the
// conditioning columns follow. Other layers (P = 0) map i to i.
__device__ inline int tied_column(int i, int IN, int C, int P, float& factor)
{
  factor = 1.f;
  if (P == 0) return i < IN ? i : -1;
  if (i < C) return i;
  if (i < C + P) {
    factor = 1.f / 256.f;
    return i - C;
  }
  return i - P < IN ? i - P : -1;
}

// BF16 copies of a layer's weights: forward layout [tap][OUTP][INP] (padding
// zero) and backward-input layout [tap][INP][OUTP].
__global__ void k_pack_w(const float* __restrict__ w, int OUT, int IN, int OUTP, int INP, int C, int P,
                         bf16* __restrict__ wf, bf16* __restrict__ wb)
{
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NTAP * OUTP * INP) return;
  const int i = k % INP, o = (k / INP) % OUTP, tap = k / (INP * OUTP);
  float factor;
  const int src = tied_column(i, IN, C, P, factor);
  const float v = (o < OUT && src >= 0) ? w[((size_t)tap * OUT + o) * IN + src] * factor : 0.f;
  wf[k] = (bf16)v;
  if (wb) wb[((size_t)tap * INP + i) * OUTP + o] = (bf16)v;
}

__global__ void k_pack_b(const float* __restrict__ b, int OUT, int OUTP, float* __restrict__ bp)
{
  const int k = threadIdx.x;
  if (k < OUTP) bp[k] = k < OUT ? b[k] : 0.f;
}

// Sum of squares of g[0..n) in FP64, one partial per block (grid-stride, fixed order).
__global__ __launch_bounds__(256) void k_sumsq(const float* __restrict__ g, int64_t n, double* __restrict__ partial)
{
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = g[i];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_scale(float* __restrict__ g, int64_t n, float f)
{
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] *= f;
}

__global__ void k_zero(float* __restrict__ p, int64_t n)
{
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0.f;
}

thread_local std::string g_nn_error;

}  // namespace

// ---------------------------------------------------------------------------
// Network object
// ---------------------------------------------------------------------------
struct mclbm_nn {
  int C = 0, P = 0, S = 0, depth = 0, ntubes = 0;
  int Ms = 0;                           // species of the conservative output (0: direct output)
  int Cout = 0;                         // output channels: C, or 3 Ms + 4
  int64_t n = 0, ntiles = 0;
  bool flat_yz = false;                 // every tube is one node wide in y and z
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<NTube> hTubes;
  std::vector<int32_t> hTileTube;
  std::vector<int32_t> hRowFirst;
  Norm norm{};
  // per layer: real and padded sizes, offsets into the parameter arrays
  std::vector<int> in_r, out_r, in_p, out_p;
  std::vector<int64_t> w_off, b_off;    // offsets (floats) of W and b in master/m/v/grad
  int64_t nparam = 0;
  int64_t step = 0;
  // device regions
  NTube* dTubes = nullptr;
  int32_t* dTileTube = nullptr;
  int32_t* dRowFirst = nullptr;         // x rows of the tubes before each tube
  int64_t nrows = 0;                    // x rows of all tubes
  float *master = nullptr, *mom1 = nullptr, *mom2 = nullptr, *grad = nullptr;
  std::vector<bf16*> wf, wb;            // packed BF16 weights per layer
  std::vector<float*> bp;               // padded biases per layer
  std::vector<bf16*> act;               // act[0] packed input, act[l+1] output of layer l (hidden)
  float* yout = nullptr;                // raw output of the last layer [COUTL][n]
  bf16* dy[2] = {nullptr, nullptr};     // activation gradients (ping-pong), [n][WIDTH]
  bf16* dyl = nullptr;                  // gradient of the last layer's output [n][COUTL]
  float* wpart = nullptr;               // weight-gradient partials
  int wG = 0;                           // workgroups along the chunks (nine (dy, dz) columns each)
  int wGf = 0;                          // the same with one column (flat_yz): up to nine times wG
  float* bpart = nullptr;               // bias-gradient partials [ntiles][WIDTH]
  double* dpart = nullptr;              // loss / residual partials
  float* cond = nullptr;                // [ntubes][S] conditioning values
  float* fin = nullptr;                 // [C][n] input fields
  float* fout = nullptr;                // [C][n] predicted fields
};

namespace {

int nn_fail(mclbm_nn* net, int code, const std::string& msg)
{
  if (net) net->err = msg; else g_nn_error = msg;
  return code;
}

#define NN_TRY(net, call)                                                                          \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return nn_fail((net), MCLBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int nn_check(mclbm_nn* net, const char* what)
{
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return nn_fail(net, MCLBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return MCLBM_OK;
}

struct NNLayout {
  size_t tubes, tile_tube, row_first, master, mom1, mom2, grad, wf, wb, bp, act, yout, dy, dyl, wpart, bpart, dpart, cond, fin, fout,
      total;
  int64_t n, ntiles, nparam, nparam_p;
  int wG;
};

void layer_sizes(int C, int Cout, int P, int S, int depth, std::vector<int>& in_r, std::vector<int>& out_r, std::vector<int>& in_p,
                 std::vector<int>& out_p)
{
  in_r.assign(depth, WIDTH);
  out_r.assign(depth, WIDTH);
  in_p.assign(depth, WIDTH);
  out_p.assign(depth, WIDTH);
  in_r[0] = C + S;            // parameters; the second terms reuse the field weights
  in_p[0] = CIN0;
  out_r[depth - 1] = Cout;
  out_p[depth - 1] = COUTL;
}

int out_channels(int C, int Ms) { return Ms > 0 ? 3 * Ms + 4 : C; }

int validate_nn(int C, int P, int S, int Ms, int depth, const int32_t* dims, int ntubes, std::string& err)
{
  if (Ms < 0 || (Ms > 0 && (C != Ms + 5 || 3 * Ms + 4 > COUTL))) {
    err = "a conservative output needs channels = species + 5 (X, T, u, p) and 3 species + 4 <= 32";
    return MCLBM_EARG;
  }
  if (C < 1 || C > MAXC || P < 0 || P > C || S < 0 || C + P + S > CIN0) {
    err = "need 1 <= channels <= 16, 0 <= two_term <= channels, conditioning >= 0, "
          "channels + two_term + conditioning <= 32";
    return MCLBM_EARG;
  }
  if (depth < 2 || depth > 16) { err = "depth must be in 2..16"; return MCLBM_EARG; }
  if (!dims || ntubes < 1) { err = "tube dimensions must be given"; return MCLBM_EARG; }
  int64_t tiles = 0;
  for (int t = 0; t < ntubes; ++t) {
    const int64_t nx = dims[3 * t], ny = dims[3 * t + 1], nz = dims[3 * t + 2];
    if (nx < 1 || ny < 1 || nz < 1) { err = "tube sizes must be positive"; return MCLBM_EARG; }
    if (nx * ny * nz >= ((int64_t)1 << 30)) { err = "tube too large"; return MCLBM_EARG; }
    tiles += (nx * ny * nz + TILE - 1) / TILE;
  }
  if (tiles >= ((int64_t)1 << 30)) { err = "too many nodes"; return MCLBM_EARG; }
  return MCLBM_OK;
}

NNLayout nn_layout(int C, int P, int S, int Ms, int depth, const int32_t* dims, int ntubes)
{
  NNLayout l{};
  l.n = 0;
  l.ntiles = 0;
  for (int t = 0; t < ntubes; ++t) {
    const int64_t n = (int64_t)dims[3 * t] * dims[3 * t + 1] * dims[3 * t + 2];
    l.n += n;
    l.ntiles += (n + TILE - 1) / TILE;
  }
  std::vector<int> in_r, out_r, in_p, out_p;
  layer_sizes(C, out_channels(C, Ms), P, S, depth, in_r, out_r, in_p, out_p);
  l.nparam = 0;
  l.nparam_p = 0;
  size_t wfb = 0, bpb = 0;
  for (int k = 0; k < depth; ++k) {
    l.nparam += (int64_t)NTAP * out_r[k] * in_r[k] + out_r[k];
    wfb += align_up(sizeof(bf16) * NTAP * out_p[k] * in_p[k]);
    bpb += align_up(sizeof(float) * out_p[k]);
  }
  // weight-gradient groups: 56 x 9 (dy, dz) workgroups fill the 256 compute units
  // two deep (the 64 -> 64 kernel stages 68 KB of LDS: two workgroups per unit)
  l.wG = (int)std::min<int64_t>(2 * l.ntiles, 56);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
  l.tubes = take(sizeof(NTube) * ntubes);
  l.tile_tube = take(sizeof(int32_t) * l.ntiles);
  l.row_first = take(sizeof(int32_t) * ntubes);
  l.master = take(sizeof(float) * l.nparam);
  l.mom1 = take(sizeof(float) * l.nparam);
  l.mom2 = take(sizeof(float) * l.nparam);
  l.grad = take(sizeof(float) * l.nparam);
  l.wf = take(wfb);
  l.wb = take(wfb);
  l.bp = take(bpb);
  const size_t npad = (size_t)l.ntiles * TILE;   // room for whole tiles is not needed: nodes index by tube
  (void)npad;
  l.act = take(sizeof(bf16) * (size_t)l.n * CIN0) ;
  for (int k = 0; k + 1 < depth; ++k) off += align_up(sizeof(bf16) * (size_t)l.n * WIDTH);
  l.yout = take(sizeof(float) * (size_t)l.n * COUTL);
  l.dy = take(sizeof(bf16) * (size_t)l.n * WIDTH);
  off += align_up(sizeof(bf16) * (size_t)l.n * WIDTH);      // second ping-pong buffer
  l.dyl = take(sizeof(bf16) * (size_t)l.n * COUTL);
  l.wpart = take(sizeof(float) * (size_t)l.wG * NTAP * WIDTH * WIDTH);
  l.bpart = take(sizeof(float) * (size_t)l.ntiles * WIDTH);
  l.dpart = take(sizeof(double) * (size_t)l.ntiles * MAXC);
  l.cond = take(sizeof(float) * (size_t)ntubes * (S > 0 ? S : 1));
  l.fin = take(sizeof(float) * (size_t)l.n * C);
  l.fout = take(sizeof(float) * (size_t)l.n * C);
  l.total = off;
  return l;
}

unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Reduce per-tile double partials [ntiles][nv] to per-tube sums on the host.
int tube_sums(mclbm_nn* net, int nv, std::vector<double>& out)
{
  std::vector<double> part((size_t)net->ntiles * nv);
  NN_TRY(net, hipMemcpyAsync(part.data(), net->dpart, sizeof(double) * part.size(), hipMemcpyDeviceToHost,
                             net->stream));
  NN_TRY(net, hipStreamSynchronize(net->stream));
  out.assign((size_t)net->ntubes * nv, 0.0);
  for (int t = 0; t < net->ntubes; ++t)
    for (int k = 0; k < net->hTubes[t].ntiles; ++k)
      for (int v = 0; v < nv; ++v) out[(size_t)t * nv + v] += part[(size_t)(net->hTubes[t].first_tile + k) * nv + v];
  return MCLBM_OK;
}

int repack(mclbm_nn* net)
{
  for (int k = 0; k < net->depth; ++k) {
    const int total = NTAP * net->out_p[k] * net->in_p[k];
    hipLaunchKernelGGL(k_pack_w, dim3(blocks_for(total, 256)), dim3(256), 0, net->stream, net->master + net->w_off[k],
                       net->out_r[k], net->in_r[k], net->out_p[k], net->in_p[k], k == 0 ? net->C : net->in_r[k],
                       k == 0 ? net->P : 0, net->wf[k], k > 0 ? net->wb[k] : nullptr);
    hipLaunchKernelGGL(k_pack_b, dim3(1), dim3(64), 0, net->stream, net->master + net->b_off[k], net->out_r[k],
                       net->out_p[k], net->bp[k]);
  }
  return nn_check(net, "k_pack_w");
}

template <int CIN, int COUT, int EPI>
void conv(mclbm_nn* net, const bf16* W, const float* b, const bf16* in, const bf16* mask, void* out)
{
  hipLaunchKernelGGL((k_conv<CIN, COUT, EPI>), dim3((unsigned)net->ntiles), dim3(256), 0, net->stream, net->dTubes,
                     net->dTileTube, net->ntubes, W, b, in, mask, out);
}

template <int CIN, int COUT>
void wgrad(mclbm_nn* net, const bf16* dY, const bf16* X, int layer)
{
  constexpr int CINP = CIN < 32 ? 32 : CIN;
  const int nchunks = (int)(2 * net->ntiles);
  const int G = net->flat_yz ? net->wGf : net->wG;
  hipLaunchKernelGGL((k_wgrad<CIN, COUT>), dim3(G, net->flat_yz ? 1 : NTAP / 3), dim3(256), 0, net->stream,
                     net->dTubes, net->dTileTube, net->ntubes, nchunks, dY, X, net->wpart, net->flat_yz ? 4 : -1);
  // only the real channels have parameters (the padded ones stay zero)
  const int co_r = net->out_r[layer], ci_r = net->in_r[layer];
  const int n = (net->flat_yz ? 3 : NTAP) * co_r * ci_r;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks_for(n, 32)), dim3(256), 0, net->stream, net->wpart, G,
                     COUT, CINP, co_r, ci_r, layer == 0 ? net->C : ci_r, layer == 0 ? net->P : 0,
                     net->grad + net->w_off[layer], net->flat_yz ? 1 : 0);
}

void bgrad(mclbm_nn* net, const bf16* dY, int C, int layer)
{
  hipLaunchKernelGGL(k_bgrad, dim3((unsigned)net->ntiles), dim3(256), 0, net->stream, net->dTubes, net->dTileTube,
                     net->ntubes, C, dY, net->bpart);
  hipLaunchKernelGGL(k_bgrad_reduce, dim3((unsigned)net->out_r[layer]), dim3(256), 0, net->stream, net->bpart,
                     (int)net->ntiles, C, net->out_r[layer], net->grad + net->b_off[layer]);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" size_t mclbm_nn_workspace_bytes(int32_t channels, int32_t two_term, int32_t conditioning,
                                           int32_t species, int32_t depth, const int32_t* dims, int32_t ntubes)
{
  std::string err;
  if (validate_nn(channels, two_term, conditioning, species, depth, dims, ntubes, err) != MCLBM_OK) {
    g_nn_error = err;
    return 0;
  }
  return nn_layout(channels, two_term, conditioning, species, depth, dims, ntubes).total;
}

extern "C" int mclbm_nn_create(int32_t channels, int32_t two_term, int32_t conditioning, int32_t species,
                               int32_t depth, const int32_t* dims, int32_t ntubes, void* dev_workspace,
                               size_t bytes, void* hip_stream, mclbm_nn** out)
{
  if (!out) return nn_fail(nullptr, MCLBM_EARG, "out is NULL");
  *out = nullptr;
  std::string err;
  int rc = validate_nn(channels, two_term, conditioning, species, depth, dims, ntubes, err);
  if (rc) return nn_fail(nullptr, rc, err);
  const NNLayout lay = nn_layout(channels, two_term, conditioning, species, depth, dims, ntubes);
  if (!dev_workspace) return nn_fail(nullptr, MCLBM_EARG, "workspace is NULL");
  if (((uintptr_t)dev_workspace) % ALIGN) return nn_fail(nullptr, MCLBM_EARG, "workspace must be 256-byte aligned");
  if (bytes < lay.total) return nn_fail(nullptr, MCLBM_EARG, "workspace too small");
  mclbm_nn* net = new (std::nothrow) mclbm_nn();
  if (!net) return nn_fail(nullptr, MCLBM_EARG, "out of host memory");
  net->C = channels;
  net->P = two_term;
  net->S = conditioning;
  net->Ms = species;
  net->Cout = out_channels(channels, species);
  net->depth = depth;
  net->ntubes = ntubes;
  net->n = lay.n;
  net->ntiles = lay.ntiles;
  net->stream = (hipStream_t)hip_stream;
  net->wG = lay.wG;
  net->wGf = (int)std::min<int64_t>(2 * lay.ntiles, 9 * (int64_t)lay.wG);
  layer_sizes(channels, net->Cout, two_term, conditioning, depth, net->in_r, net->out_r, net->in_p, net->out_p);
  int64_t off = 0;
  for (int k = 0; k < depth; ++k) {
    net->w_off.push_back(off);
    off += (int64_t)NTAP * net->out_r[k] * net->in_r[k];
    net->b_off.push_back(off);
    off += net->out_r[k];
  }
  net->nparam = off;
  char* ws = (char*)dev_workspace;
  net->dTubes = (NTube*)(ws + lay.tubes);
  net->dTileTube = (int32_t*)(ws + lay.tile_tube);
  net->dRowFirst = (int32_t*)(ws + lay.row_first);
  net->master = (float*)(ws + lay.master);
  net->mom1 = (float*)(ws + lay.mom1);
  net->mom2 = (float*)(ws + lay.mom2);
  net->grad = (float*)(ws + lay.grad);
  size_t wo = lay.wf, bo = lay.bp, wbo = lay.wb;
  for (int k = 0; k < depth; ++k) {
    net->wf.push_back((bf16*)(ws + wo));
    net->wb.push_back((bf16*)(ws + wbo));
    const size_t wbytes = align_up(sizeof(bf16) * NTAP * net->out_p[k] * net->in_p[k]);
    wo += wbytes;
    wbo += wbytes;
    net->bp.push_back((float*)(ws + bo));
    bo += align_up(sizeof(float) * net->out_p[k]);
  }
  size_t ao = lay.act;
  net->act.push_back((bf16*)(ws + ao));
  ao += align_up(sizeof(bf16) * (size_t)lay.n * CIN0);
  for (int k = 0; k + 1 < depth; ++k) {
    net->act.push_back((bf16*)(ws + ao));
    ao += align_up(sizeof(bf16) * (size_t)lay.n * WIDTH);
  }
  net->yout = (float*)(ws + lay.yout);
  net->dy[0] = (bf16*)(ws + lay.dy);
  net->dy[1] = (bf16*)(ws + lay.dy + align_up(sizeof(bf16) * (size_t)lay.n * WIDTH));
  net->dyl = (bf16*)(ws + lay.dyl);
  net->wpart = (float*)(ws + lay.wpart);
  net->bpart = (float*)(ws + lay.bpart);
  net->dpart = (double*)(ws + lay.dpart);
  net->cond = (float*)(ws + lay.cond);
  net->fin = (float*)(ws + lay.fin);
  net->fout = (float*)(ws + lay.fout);
  // tubes and the tile -> tube map
  net->hTubes.resize(ntubes);
  net->hTileTube.resize(lay.ntiles);
  int64_t base = 0;
  int32_t tile = 0;
  for (int t = 0; t < ntubes; ++t) {
    NTube& tb = net->hTubes[t];
    tb.base = base;
    tb.nx = dims[3 * t];
    tb.ny = dims[3 * t + 1];
    tb.nz = dims[3 * t + 2];
    const int64_t n = (int64_t)tb.nx * tb.ny * tb.nz;
    tb.first_tile = tile;
    tb.ntiles = (int32_t)((n + TILE - 1) / TILE);
    tb.pad = 0;
    tb.ntot = lay.n;
    for (int k = 0; k < tb.ntiles; ++k) net->hTileTube[tile + k] = t;
    tile += tb.ntiles;
    base += n;
  }
  net->flat_yz = true;
  for (const NTube& tb : net->hTubes) net->flat_yz = net->flat_yz && tb.ny == 1 && tb.nz == 1;
  net->hRowFirst.resize(ntubes);
  net->nrows = 0;
  for (int t = 0; t < ntubes; ++t) {
    net->hRowFirst[t] = (int32_t)net->nrows;
    net->nrows += (int64_t)net->hTubes[t].ny * net->hTubes[t].nz;
  }
  for (int c = 0; c < MAXC; ++c) {
    net->norm.in_shift[c] = 0.f;
    net->norm.in_scale[c] = 1.f;
  }
  for (int c = 0; c < COUTL; ++c) {
    net->norm.out_scale[c] = 1.f;
    net->norm.weight[c] = 1.f;
  }
  hipError_t e = hipMemcpyAsync(net->dTubes, net->hTubes.data(), sizeof(NTube) * ntubes, hipMemcpyHostToDevice,
                                net->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(net->dTileTube, net->hTileTube.data(), sizeof(int32_t) * lay.ntiles, hipMemcpyHostToDevice,
                       net->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(net->dRowFirst, net->hRowFirst.data(), sizeof(int32_t) * ntubes, hipMemcpyHostToDevice,
                       net->stream);
  if (e == hipSuccess) {
    // parameters, moments and gradients start at zero (set_params gives the weights)
    for (float* p : {net->master, net->mom1, net->mom2, net->grad})
      hipLaunchKernelGGL(k_zero, dim3(blocks_for(net->nparam, 256)), dim3(256), 0, net->stream, p, net->nparam);
    const int64_t nc = (int64_t)ntubes * (conditioning > 0 ? conditioning : 1);
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(nc, 256)), dim3(256), 0, net->stream, net->cond, nc);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) {
    g_nn_error = std::string("device setup: ") + hipGetErrorString(e);
    delete net;
    return MCLBM_EDEVICE;
  }
  rc = repack(net);
  if (rc) {
    g_nn_error = net->err;
    delete net;
    return rc;
  }
  *out = net;
  return MCLBM_OK;
}

extern "C" void mclbm_nn_destroy(mclbm_nn* net)
{
  if (!net) return;
  (void)hipStreamSynchronize(net->stream);
  delete net;
}

extern "C" const char* mclbm_nn_last_error(const mclbm_nn* net) { return net ? net->err.c_str() : g_nn_error.c_str(); }

extern "C" int64_t mclbm_nn_param_count(const mclbm_nn* net) { return net ? net->nparam : -1; }

extern "C" int mclbm_nn_set_params(mclbm_nn* net, const float* host)
{
  if (!net) return MCLBM_EARG;
  if (!host) return nn_fail(net, MCLBM_EARG, "params is NULL");
  NN_TRY(net, hipMemcpyAsync(net->master, host, sizeof(float) * net->nparam, hipMemcpyHostToDevice, net->stream));
  for (float* p : {net->mom1, net->mom2, net->grad})
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(net->nparam, 256)), dim3(256), 0, net->stream, p, net->nparam);
  net->step = 0;
  int rc = repack(net);
  if (rc) return rc;
  NN_TRY(net, hipStreamSynchronize(net->stream));
  return MCLBM_OK;
}

extern "C" int mclbm_nn_get_params(mclbm_nn* net, float* host)
{
  if (!net) return MCLBM_EARG;
  if (!host) return nn_fail(net, MCLBM_EARG, "buffer is NULL");
  NN_TRY(net, hipMemcpyAsync(host, net->master, sizeof(float) * net->nparam, hipMemcpyDeviceToHost, net->stream));
  NN_TRY(net, hipStreamSynchronize(net->stream));
  return MCLBM_OK;
}

extern "C" int mclbm_nn_get_grads(mclbm_nn* net, float* host)
{
  if (!net) return MCLBM_EARG;
  if (!host) return nn_fail(net, MCLBM_EARG, "buffer is NULL");
  NN_TRY(net, hipMemcpyAsync(host, net->grad, sizeof(float) * net->nparam, hipMemcpyDeviceToHost, net->stream));
  NN_TRY(net, hipStreamSynchronize(net->stream));
  return MCLBM_OK;
}

extern "C" int mclbm_nn_set_norm(mclbm_nn* net, const float* in_shift, const float* in_scale, const float* out_scale)
{
  if (!net) return MCLBM_EARG;
  if (!in_shift || !in_scale || !out_scale) return nn_fail(net, MCLBM_EARG, "normalisation arrays must be given");
  for (int c = 0; c < net->C; ++c) {
    if (!(std::isfinite(in_shift[c]) && in_scale[c] > 0.f))
      return nn_fail(net, MCLBM_EARG, "scales must be positive and shifts finite");
    net->norm.in_shift[c] = in_shift[c];
    net->norm.in_scale[c] = in_scale[c];
  }
  for (int c = 0; c < net->Cout; ++c) {
    if (!(out_scale[c] > 0.f)) return nn_fail(net, MCLBM_EARG, "output scales must be positive");
    net->norm.out_scale[c] = out_scale[c];
  }
  return MCLBM_OK;
}

extern "C" int mclbm_nn_set_conditioning(mclbm_nn* net, const float* host)
{
  if (!net) return MCLBM_EARG;
  if (!host) return nn_fail(net, MCLBM_EARG, "conditioning is NULL");
  if (net->S == 0) return MCLBM_OK;
  NN_TRY(net, hipMemcpyAsync(net->cond, host, sizeof(float) * net->ntubes * net->S, hipMemcpyHostToDevice,
                             net->stream));
  NN_TRY(net, hipStreamSynchronize(net->stream));
  return MCLBM_OK;
}

extern "C" int mclbm_nn_io(mclbm_nn* net, float** fields_in, float** fields_out)
{
  if (!net) return MCLBM_EARG;
  if (fields_in) *fields_in = net->fin;
  if (fields_out) *fields_out = net->fout;
  return MCLBM_OK;
}

extern "C" int mclbm_nn_forward(mclbm_nn* net)
{
  if (!net) return MCLBM_EARG;
  const unsigned grid = (unsigned)net->ntiles;
  hipLaunchKernelGGL(k_pack_in, dim3(grid), dim3(256), 0, net->stream, net->dTubes, net->dTileTube, net->ntubes,
                     net->C, net->P, net->S, net->norm, net->fin, net->cond, net->act[0]);
  const int D = net->depth;
  conv<CIN0, WIDTH, 0>(net, net->wf[0], net->bp[0], net->act[0], nullptr, net->act[1]);
  for (int k = 1; k + 1 < D; ++k) conv<WIDTH, WIDTH, 0>(net, net->wf[k], net->bp[k], net->act[k], nullptr, net->act[k + 1]);
  conv<WIDTH, COUTL, 1>(net, net->wf[D - 1], net->bp[D - 1], net->act[D - 1], nullptr, net->yout);
  if (net->Ms > 0)
    hipLaunchKernelGGL(k_unpack_cons, dim3(grid), dim3(256), 0, net->stream, net->dTubes, net->dTileTube,
                       net->ntubes, net->Ms, net->norm, net->fin, net->yout, net->fout);
  else
    hipLaunchKernelGGL(k_unpack_out, dim3(grid), dim3(256), 0, net->stream, net->dTubes, net->dTileTube,
                       net->ntubes, net->C, net->norm, net->fin, net->yout, net->fout);
  return nn_check(net, "mclbm_nn_forward");
}

extern "C" int mclbm_nn_loss(mclbm_nn* net, const float* target, const float* channel_weight, double* loss)
{
  if (!net) return MCLBM_EARG;
  if (!target) return nn_fail(net, MCLBM_EARG, "target is NULL");
  Norm nm = net->norm;
  for (int c = 0; c < net->C; ++c) nm.weight[c] = channel_weight ? channel_weight[c] : 1.f;
  const unsigned grid = (unsigned)net->ntiles;
  if (net->Ms > 0) {
    // dL/dn and the target x fluxes per node, [n][M] each, in the first
    // activation-gradient buffer (free until backward; WIDTH BF16 = 128 bytes per node)
    float* gnode = (float*)net->dy[0];
    float* fstar = gnode + (size_t)net->n * net->Ms;
    hipLaunchKernelGGL(k_flux_change, dim3(grid), dim3(256), 0, net->stream, net->dTubes, net->dTileTube,
                       net->ntubes, net->Ms, net->fin, target, fstar);
    hipLaunchKernelGGL(k_flux_target, dim3(blocks_for(net->nrows * net->Ms, 4)), dim3(256), 0, net->stream,
                       net->dTubes, net->dRowFirst, net->ntubes, net->nrows, net->Ms, fstar);
    hipLaunchKernelGGL(k_loss_cons, dim3(grid), dim3(256), 0, net->stream, net->dTubes, net->dTileTube,
                       net->ntubes, net->Ms, nm, 1.0 / (double)net->n, net->fout, target, net->yout, fstar, gnode,
                       net->dyl, net->dpart);
    hipLaunchKernelGGL(k_loss_cons_flux, dim3(grid), dim3(256), 0, net->stream, net->dTubes, net->dTileTube,
                       net->ntubes, net->Ms, nm, 1.0 / (double)net->n, gnode, net->yout, fstar, net->dyl);
  } else {
    hipLaunchKernelGGL(k_loss, dim3(grid), dim3(256), 0, net->stream, net->dTubes, net->dTileTube, net->ntubes,
                       net->C, nm, 1.0 / (double)net->n, net->fin, target, net->yout, net->dyl, net->dpart);
  }
  int rc = nn_check(net, "k_loss");
  if (rc) return rc;
  std::vector<double> part(net->ntiles);
  NN_TRY(net, hipMemcpyAsync(part.data(), net->dpart, sizeof(double) * net->ntiles, hipMemcpyDeviceToHost,
                             net->stream));
  NN_TRY(net, hipStreamSynchronize(net->stream));
  double s = 0.0;
  for (double v : part) s += v;
  if (loss) *loss = s / (double)net->n;
  return MCLBM_OK;
}

extern "C" int mclbm_nn_backward(mclbm_nn* net)
{
  if (!net) return MCLBM_EARG;
  const int D = net->depth;
  // last layer: dW from dyl and act[D-1]; then the gradient of act[D-1]
  wgrad<WIDTH, COUTL>(net, net->dyl, net->act[D - 1], D - 1);
  bgrad(net, net->dyl, COUTL, D - 1);
  conv<COUTL, WIDTH, 2>(net, net->wb[D - 1], nullptr, net->dyl, net->act[D - 1], net->dy[0]);
  int cur = 0;
  for (int k = D - 2; k >= 1; --k) {
    wgrad<WIDTH, WIDTH>(net, net->dy[cur], net->act[k], k);
    bgrad(net, net->dy[cur], WIDTH, k);
    conv<WIDTH, WIDTH, 2>(net, net->wb[k], nullptr, net->dy[cur], net->act[k], net->dy[cur ^ 1]);
    cur ^= 1;
  }
  wgrad<CIN0, WIDTH>(net, net->dy[cur], net->act[0], 0);
  bgrad(net, net->dy[cur], WIDTH, 0);
  return nn_check(net, "mclbm_nn_backward");
}

extern "C" int mclbm_nn_clip_grad_norm(mclbm_nn* net, double max_norm, double* norm)
{
  if (!net) return MCLBM_EARG;
  if (!(max_norm >= 0.0)) return nn_fail(net, MCLBM_EARG, "max_norm must be >= 0");
  // partials in the loss buffer (ntiles * MAXC doubles, at least 16)
  const unsigned nb = (unsigned)std::min<int64_t>(256, (int64_t)net->ntiles * MAXC);
  hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(256), 0, net->stream, net->grad, net->nparam, net->dpart);
  int rc = nn_check(net, "k_sumsq");
  if (rc) return rc;
  std::vector<double> part(nb);
  NN_TRY(net, hipMemcpyAsync(part.data(), net->dpart, sizeof(double) * nb, hipMemcpyDeviceToHost, net->stream));
  NN_TRY(net, hipStreamSynchronize(net->stream));
  double s = 0.0;
  for (double v : part) s += v;
  const double nrm = std::sqrt(s);
  if (norm) *norm = nrm;
  if (max_norm > 0.0 && std::isfinite(nrm) && nrm > max_norm) {
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(net->nparam, 256)), dim3(256), 0, net->stream, net->grad, net->nparam,
                       (float)(max_norm / nrm));
    return nn_check(net, "k_scale");
  }
  return MCLBM_OK;
}

extern "C" int mclbm_nn_zero_grad(mclbm_nn* net)
{
  if (!net) return MCLBM_EARG;
  hipLaunchKernelGGL(k_zero, dim3(blocks_for(net->nparam, 256)), dim3(256), 0, net->stream, net->grad, net->nparam);
  return nn_check(net, "k_zero");
}

extern "C" int mclbm_nn_adam_step(mclbm_nn* net, float lr, float beta1, float beta2, float eps)
{
  if (!net) return MCLBM_EARG;
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return nn_fail(net, MCLBM_EARG, "need lr > 0, 0 <= beta < 1, eps > 0");
  net->step += 1;
  const float bc1 = 1.f - (float)std::pow((double)beta1, (double)net->step);
  const float bc2 = 1.f - (float)std::pow((double)beta2, (double)net->step);
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(net->nparam, 256)), dim3(256), 0, net->stream, net->nparam, net->master,
                     net->mom1, net->mom2, net->grad, lr, beta1, beta2, eps, bc1, bc2);
  int rc = nn_check(net, "k_adam");
  if (rc) return rc;
  return repack(net);
}

extern "C" int mclbm_nn_mole_residual(mclbm_nn* net, int32_t species, const float* a, const float* b, double* out)
{
  if (!net) return MCLBM_EARG;
  if (!a || !b || !out) return nn_fail(net, MCLBM_EARG, "pointers must be given");
  if (species < 1 || species + 5 > net->C) return nn_fail(net, MCLBM_EARG, "need 1 <= species <= channels - 5");
  std::vector<double> sa, sb;
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_mole_sums, dim3((unsigned)net->ntiles), dim3(256), 0, net->stream, net->dTubes,
                       net->dTileTube, net->ntubes, net->C, species, pass ? b : a, net->dpart);
    int rc = nn_check(net, "k_mole_sums");
    if (rc) return rc;
    rc = tube_sums(net, species, pass ? sb : sa);
    if (rc) return rc;
  }
  for (int t = 0; t < net->ntubes; ++t) {
    double r = 0.0;
    for (int s = 0; s < species; ++s) {
      const double x = sa[(size_t)t * species + s], y = sb[(size_t)t * species + s];
      const double d = std::fabs(y - x) / std::fabs(x);
      r = std::max(r, std::isfinite(d) ? d : HUGE_VAL);
    }
    out[t] = r;
  }
  return MCLBM_OK;
}

void mclbm::nn::geometry(const mclbm_nn* net, int* channels, int* species, std::vector<int>* dims)
{
  *channels = net->C;
  *species = net->Ms;
  dims->clear();
  for (const NTube& tb : net->hTubes) {
    dims->push_back(tb.nx);
    dims->push_back(tb.ny);
    dims->push_back(tb.nz);
  }
}
