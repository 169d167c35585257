// Convolutional neural operator for the magnetic-field subcycle
// (libhvpic.so, gfx950).
//
// A stand-in for the subcycled Faraday/Ohm advance of arXiv 2305.05600,
// Sec. II.A, on 2D periodic grids: four periodic 3x3 convolutions
// 7 -> 32 -> 32 -> 32 -> 3 channels with tanh between them map the
// normalised (B^n, n^{n+1/2}, J_i^{n+1/2}) to the normalised increment
// B^{n+1} - B^n.  Inference and training run here: BF16 operands on the
// matrix cores (v_mfma_f32_16x16x16_bf16) with FP32 accumulation, FP32 master
// weights and Adam.
//
// Layout: activations are pixel-major with the channels contiguous ([pixel]
// [channel], BF16), so that one lane's 4 consecutive channels are one 8-byte
// load; a layer is an implicit GEMM (out channels) x (pixels) with K = 9 taps
// x in channels, the taps wrapping around each image.  Channel counts are
// padded to 16 (7 inputs, 3 outputs) with zero weights.  The weight gradient
// stages 64-pixel segments in LDS channel-major, so its operands are also
// 8-byte reads; blocks leave partial sums that one pass adds in a fixed order.
#include <string.h>

#include <algorithm>

#include "hvpic_internal.hpp"

namespace hvpic {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kNL = 4;
constexpr int kCin[kNL] = {7, 32, 32, 32}, kCout[kNL] = {32, 32, 32, 3};
constexpr int kCinP[kNL] = {16, 32, 32, 32}, kCoutP[kNL] = {32, 32, 32, 16};
constexpr int wsize(int l) { return kCoutP[l] * 9 * kCinP[l]; }
constexpr int woff(int l) { return l == 0 ? 0 : woff(l - 1) + wsize(l - 1); }
constexpr int boff(int l) { return l == 0 ? 0 : boff(l - 1) + kCoutP[l - 1]; }
constexpr int kW = woff(kNL), kB = boff(kNL);  // 27648 weights, 112 biases (padded)
constexpr int bwoff(int l) { return l <= 1 ? 0 : bwoff(l - 1) + wsize(l - 1); }  // layers 1..3
constexpr int kWb = bwoff(kNL);

// The parameter block (device, caller-owned), byte offsets.
struct PB {
  static constexpr size_t w = 0;                         // f32 [kW] master weights
  static constexpr size_t b = w + 4 * kW;                // f32 [kB]
  static constexpr size_t mw = b + 4 * kB;               // Adam moments
  static constexpr size_t vw = mw + 4 * kW;
  static constexpr size_t mb = vw + 4 * kW;
  static constexpr size_t vb = mb + 4 * kB;
  static constexpr size_t gw = vb + 4 * kB;              // gradient accumulators
  static constexpr size_t gb = gw + 4 * kW;
  static constexpr size_t norm = gb + 4 * kB;            // f32 mean[8], std[8], out_std[16]
  static constexpr size_t step = norm + 4 * 32;          // int32 Adam step count
  static constexpr size_t wf = step + 256;               // bf16 [kW] forward weights
  static constexpr size_t wb = wf + 2 * kW;              // bf16 [kWb] backward-data weights
  static constexpr size_t total = (wb + 2 * kWb + 255) & ~(size_t)255;
};

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even of the upper 16 bits (finite inputs)
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// pixel q of the same image as p, shifted by (dy, dx) with periodic wrap
__device__ __forceinline__ int64_t shifted(int64_t img0, int y, int x, int dy, int dx, int nx,
                                          int ny) {
  int yy = y + dy, xx = x + dx;
  yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
  xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
  return img0 + (int64_t)yy * nx + xx;
}

// One periodic 3x3 layer over N = nimg*ny*nx pixels.  W: bf16
// [COUTP][9][CINP].  MODE 0: out bf16 = tanh(acc + bias); 1: out f32 = acc +
// bias; 2: out bf16 = acc * (1 - h^2) with h from H [N][COUTP] (the
// backward-data product of a tanh layer, no bias).  A wavefront takes 16
// consecutive pixels; lane (ln, lq) = (lane % 16, lane / 16) holds the
// channels 4lq..4lq+3 of pixel ln for the B operand and of output row ln for
// the A operand, and receives out channels 4lq..4lq+3 of pixel ln.
template <int CINP, int COUTP, int MODE>
__global__ __launch_bounds__(256) void k_conv3x3(const uint16_t* __restrict__ X,
                                                 const uint16_t* __restrict__ W,
                                                 const float* __restrict__ bias,
                                                 const uint16_t* __restrict__ Hact,
                                                 void* __restrict__ out, int64_t N, int nx,
                                                 int ny) {
  constexpr int MT = COUTP / 16, KB = CINP / 16, NW = COUTP * 9 * CINP;
  __shared__ uint16_t sw[NW];
  for (int i = threadIdx.x; i < NW / 4; i += 256)
    reinterpret_cast<uint2*>(sw)[i] = reinterpret_cast<const uint2*>(W)[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int ln = lane & 15, lq = lane >> 4;
  const int64_t P = (int64_t)nx * ny;
  const int64_t ntiles = (N + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wid; tile < ntiles;
       tile += (int64_t)gridDim.x * 4) {
    const int64_t p = tile * 16 + ln;
    const bool live = p < N;
    const int64_t img = live ? p / P : 0;
    const int r = live ? (int)(p - img * P) : 0;
    const int y = r / nx, x = r - (r / nx) * nx;
    v4f acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int64_t q = shifted(img * P, y, x, t / 3 - 1, t % 3 - 1, nx, ny);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        v4s b = v4s{0, 0, 0, 0};
        if (live) b = *reinterpret_cast<const v4s*>(X + q * CINP + kb * 16 + lq * 4);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const v4s a =
              *reinterpret_cast<const v4s*>(sw + ((mt * 16 + ln) * 9 + t) * CINP + kb * 16 + lq * 4);
          acc[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[mt], 0, 0, 0);
        }
      }
    }
    if (!live) continue;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int co = mt * 16 + lq * 4;
      if (MODE == 1) {
        float4 v;
        v.x = acc[mt][0] + bias[co];
        v.y = acc[mt][1] + bias[co + 1];
        v.z = acc[mt][2] + bias[co + 2];
        v.w = acc[mt][3] + bias[co + 3];
        *reinterpret_cast<float4*>(static_cast<float*>(out) + p * COUTP + co) = v;
      } else {
        uint16_t o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v;
          if (MODE == 0) {
            v = tanhf(acc[mt][i] + bias[co + i]);
          } else {
            const float h = bf2f(Hact[p * COUTP + co + i]);
            v = acc[mt][i] * (1.0f - h * h);
          }
          o[i] = f2bf(v);
        }
        uint2 pk;
        pk.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
        pk.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
        *reinterpret_cast<uint2*>(static_cast<uint16_t*>(out) + p * COUTP + co) = pk;
      }
    }
  }
}

// Weight gradient of a periodic 3x3 layer: dW[co][t][ci] = sum_p dZ[p][co]
// X[p + off(t)][ci], db[co] = sum_p dZ[p][co], as per-block partials
// part[block][COUTP*9*CINP + COUTP].  A block takes 64-pixel segments: dZ and
// the 9 shifted copies of X go to LDS channel-major, then each wavefront
// accumulates its share of the 9 * (COUTP/16) * (CINP/16) output tiles over
// the segment's four 16-pixel steps.
constexpr int kSeg = 64;
template <int CINP, int COUTP>
__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const uint16_t* __restrict__ X,
                                                       const uint16_t* __restrict__ dZ,
                                                       float* __restrict__ part, int64_t N, int nx,
                                                       int ny) {
  constexpr int MT = COUTP / 16, NT = CINP / 16, TILES = 9 * MT * NT, TPW = (TILES + 3) / 4;
  constexpr int NWT = COUTP * 9 * CINP;
  __shared__ uint16_t sz[COUTP * kSeg];
  __shared__ uint16_t sx[9 * CINP * kSeg];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int ln = lane & 15, lq = lane >> 4;
  const int64_t P = (int64_t)nx * ny;
  v4f acc[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
  float dbacc = 0.f;
  const int64_t nseg = (N + kSeg - 1) / kSeg;
  for (int64_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
    const int64_t p0 = sg * kSeg;
    for (int e = threadIdx.x; e < kSeg * COUTP / 4; e += 256) {
      const int px = e / (COUTP / 4), cq = (e % (COUTP / 4)) * 4;
      const int64_t p = p0 + px;
      uint2 v = make_uint2(0u, 0u);
      if (p < N) v = *reinterpret_cast<const uint2*>(dZ + p * COUTP + cq);
      sz[(cq + 0) * kSeg + px] = (uint16_t)(v.x & 0xFFFFu);
      sz[(cq + 1) * kSeg + px] = (uint16_t)(v.x >> 16);
      sz[(cq + 2) * kSeg + px] = (uint16_t)(v.y & 0xFFFFu);
      sz[(cq + 3) * kSeg + px] = (uint16_t)(v.y >> 16);
    }
    for (int e = threadIdx.x; e < 9 * kSeg * CINP / 4; e += 256) {
      const int t = e / (kSeg * CINP / 4), rem = e % (kSeg * CINP / 4);
      const int px = rem / (CINP / 4), cq = (rem % (CINP / 4)) * 4;
      const int64_t p = p0 + px;
      uint2 v = make_uint2(0u, 0u);
      if (p < N) {
        const int64_t img = p / P;
        const int r = (int)(p - img * P), y = r / nx, x = r - (r / nx) * nx;
        const int64_t q = shifted(img * P, y, x, t / 3 - 1, t % 3 - 1, nx, ny);
        v = *reinterpret_cast<const uint2*>(X + q * CINP + cq);
      }
      uint16_t* d = sx + ((size_t)t * CINP + cq) * kSeg + px;
      d[0] = (uint16_t)(v.x & 0xFFFFu);
      d[kSeg] = (uint16_t)(v.x >> 16);
      d[2 * kSeg] = (uint16_t)(v.y & 0xFFFFu);
      d[3 * kSeg] = (uint16_t)(v.y >> 16);
    }
    __syncthreads();
    if (threadIdx.x < COUTP)
      for (int k = 0; k < kSeg; ++k) dbacc += bf2f(sz[threadIdx.x * kSeg + k]);
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const int q = wid + 4 * j;
      if (q < TILES) {
        const int t = q / (MT * NT), mt = (q / NT) % MT, nt = q % NT;
#pragma unroll
        for (int k0 = 0; k0 < kSeg; k0 += 16) {
          const v4s a = *reinterpret_cast<const v4s*>(sz + (mt * 16 + ln) * kSeg + k0 + lq * 4);
          const v4s b = *reinterpret_cast<const v4s*>(
              sx + ((size_t)t * CINP + nt * 16 + ln) * kSeg + k0 + lq * 4);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  float* mine = part + (size_t)blockIdx.x * (NWT + COUTP);
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int q = wid + 4 * j;
    if (q < TILES) {
      const int t = q / (MT * NT), mt = (q / NT) % MT, nt = q % NT;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        mine[((mt * 16 + lq * 4 + i) * 9 + t) * CINP + nt * 16 + ln] = acc[j][i];
    }
  }
  if (threadIdx.x < COUTP) mine[NWT + threadIdx.x] = dbacc;
}

// gw[i] += sum over nb blocks of part[b][i] (fixed order); i < n weights
// followed by nbias biases of the layer
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nb, int nwt, int nbias,
                               float* __restrict__ gw, float* __restrict__ gb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = nwt + nbias;
  if (i >= n) return;
  float s = 0.f;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * n + i];
  if (i < nwt)
    gw[i] += s;
  else
    gb[i - nwt] += s;
}

// The 7 normalised input channels (padded to 16) of sample idx[s] (s if idx
// is null) at every pixel: X0[s*P + r][c].
__global__ void k_no_pack(const float* __restrict__ B, const float* __restrict__ n,
                          const float* __restrict__ J, const int32_t* __restrict__ idx, int S,
                          int64_t P, const float* __restrict__ norm, uint16_t* __restrict__ X0) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)S * P) return;
  const int s = (int)(p / P);
  const int64_t r = p - (int64_t)s * P;
  const int64_t smp = idx ? idx[s] : s;
  const float v[7] = {B[smp * 3 * P + r], B[smp * 3 * P + P + r], B[smp * 3 * P + 2 * P + r],
                      n[smp * P + r],   J[smp * 3 * P + r], J[smp * 3 * P + P + r],
                      J[smp * 3 * P + 2 * P + r]};
  uint16_t o[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) o[c] = c < 7 ? f2bf((v[c] - norm[c]) / norm[8 + c]) : (uint16_t)0;
  uint4* dst = reinterpret_cast<uint4*>(X0 + p * 16);
  uint4 a, b;
  a.x = o[0] | ((uint32_t)o[1] << 16);
  a.y = o[2] | ((uint32_t)o[3] << 16);
  a.z = o[4] | ((uint32_t)o[5] << 16);
  a.w = o[6] | ((uint32_t)o[7] << 16);
  b.x = o[8] | ((uint32_t)o[9] << 16);
  b.y = o[10] | ((uint32_t)o[11] << 16);
  b.z = o[12] | ((uint32_t)o[13] << 16);
  b.w = o[14] | ((uint32_t)o[15] << 16);
  dst[0] = a;
  dst[1] = b;
}

// Loss of the normalised increment and its gradient: d = D[p][c] - (Bt - B)
// / out_std for c < 3; dZ4 = bf16(2 d / (3 S P)); per-block FP64 partials of
// sum d^2.
__global__ __launch_bounds__(256) void k_no_loss(const float* __restrict__ D,
                                                 const float* __restrict__ B,
                                                 const float* __restrict__ Bt,
                                                 const int32_t* __restrict__ idx, int S, int64_t P,
                                                 const float* __restrict__ norm,
                                                 uint16_t* __restrict__ dZ, double* part) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[1] = {0.0};
  if (p < (int64_t)S * P) {
    const int s = (int)(p / P);
    const int64_t r = p - (int64_t)s * P;
    const int64_t smp = idx ? idx[s] : s;
    const float scale = 2.0f / (float)(3.0 * (double)S * (double)P);
    uint16_t o[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) o[c] = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float tgt = (Bt[smp * 3 * P + c * P + r] - B[smp * 3 * P + c * P + r]) / norm[16 + c];
      const float d = D[p * 16 + c] - tgt;
      v[0] += (double)d * (double)d;
      o[c] = f2bf(scale * d);
    }
    uint4* dst = reinterpret_cast<uint4*>(dZ + p * 16);
    uint4 a, b;
    a.x = o[0] | ((uint32_t)o[1] << 16);
    a.y = o[2] | ((uint32_t)o[3] << 16);
    a.z = a.w = 0u;
    b.x = b.y = b.z = b.w = 0u;
    dst[0] = a;
    dst[1] = b;
  }
  block_partial<1, 1>(v, part);
}

__global__ void k_no_loss_final(const double* part, int nb, int64_t count, double* out) {
  double r[1];
  sum_partials<1, 1>(part, nb, r);
  if (threadIdx.x == 0) out[0] = r[0] / (double)count;
}

// mask of the real (unpadded) entries of weight i of the concatenated
// padded array (layer l, out co, in ci)
__device__ __forceinline__ bool weight_live(int i, int& l, int& co, int& t, int& ci) {
  l = 0;
  while (l < kNL - 1 && i >= woff(l + 1)) ++l;
  const int j = i - woff(l);
  co = j / (9 * kCinP[l]);
  t = (j / kCinP[l]) % 9;
  ci = j % kCinP[l];
  return co < kCout[l] && ci < kCin[l];
}

// One Adam step (bias-corrected) over the padded weights and biases, the
// gradient accumulators cleared, the BF16 forward copies and the flipped,
// transposed backward-data copies (layers 1..3) rewritten.  With lr = 0 only
// the copies are refreshed (after loading weights).
__global__ void k_no_adam(char* pb, float lr, float b1, float b2, float eps, int do_update) {
  float* w = reinterpret_cast<float*>(pb + PB::w);
  float* b = reinterpret_cast<float*>(pb + PB::b);
  float* mw = reinterpret_cast<float*>(pb + PB::mw);
  float* vw = reinterpret_cast<float*>(pb + PB::vw);
  float* mb = reinterpret_cast<float*>(pb + PB::mb);
  float* vb = reinterpret_cast<float*>(pb + PB::vb);
  float* gw = reinterpret_cast<float*>(pb + PB::gw);
  float* gb = reinterpret_cast<float*>(pb + PB::gb);
  uint16_t* wf = reinterpret_cast<uint16_t*>(pb + PB::wf);
  uint16_t* wbk = reinterpret_cast<uint16_t*>(pb + PB::wb);
  const int step = *reinterpret_cast<const int*>(pb + PB::step) + (do_update ? 1 : 0);
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  auto upd = [&](float& p, float& m, float& v, float& g) {
    m = b1 * m + (1.0f - b1) * g;
    v = b2 * v + (1.0f - b2) * g * g;
    p -= lr * (m / c1) / (sqrtf(v / c2) + eps);
    g = 0.0f;
  };
  if (i < kW) {
    int l, co, t, ci;
    const bool live = weight_live(i, l, co, t, ci);
    if (!live) {
      w[i] = 0.0f;
      gw[i] = 0.0f;
    } else if (do_update) {
      upd(w[i], mw[i], vw[i], gw[i]);
    }
    const uint16_t h = f2bf(w[i]);
    wf[i] = h;
    if (l >= 1) {
      // backward data of layer l: [CINP_l][9][COUTP_l], tap flipped
      wbk[bwoff(l) + (ci * 9 + (8 - t)) * kCoutP[l] + co] = h;
    }
  } else if (i < kW + kB) {
    const int j = i - kW;
    int l = 0;
    while (l < kNL - 1 && j >= boff(l + 1)) ++l;
    const bool live = j - boff(l) < kCout[l];
    if (!live) {
      b[j] = 0.0f;
      gb[j] = 0.0f;
    } else if (do_update) {
      upd(b[j], mb[j], vb[j], gb[j]);
    }
  }
  if (i == 0 && do_update) *reinterpret_cast<int*>(pb + PB::step) = step;
}

// Loads logical weights w_l [Cout][9][Cin] (concatenated), biases and the
// normalisation (mean[7], std[7], out_std[3]) into the padded block; clears
// Adam's state and the gradients.
__global__ void k_no_load(char* pb, const float* __restrict__ wl, const float* __restrict__ bl,
                          const float* __restrict__ norm) {
  float* w = reinterpret_cast<float*>(pb + PB::w);
  float* b = reinterpret_cast<float*>(pb + PB::b);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kW) {
    int l, co, t, ci;
    const bool live = weight_live(i, l, co, t, ci);
    int lo = 0;
    for (int k = 0; k < l; ++k) lo += kCout[k] * 9 * kCin[k];
    w[i] = live ? wl[lo + (co * 9 + t) * kCin[l] + ci] : 0.0f;
    reinterpret_cast<float*>(pb + PB::mw)[i] = 0.0f;
    reinterpret_cast<float*>(pb + PB::vw)[i] = 0.0f;
    reinterpret_cast<float*>(pb + PB::gw)[i] = 0.0f;
  } else if (i < kW + kB) {
    const int j = i - kW;
    int l = 0;
    while (l < kNL - 1 && j >= boff(l + 1)) ++l;
    int lo = 0;
    for (int k = 0; k < l; ++k) lo += kCout[k];
    const int co = j - boff(l);
    b[j] = co < kCout[l] ? bl[lo + co] : 0.0f;
    reinterpret_cast<float*>(pb + PB::mb)[j] = 0.0f;
    reinterpret_cast<float*>(pb + PB::vb)[j] = 0.0f;
    reinterpret_cast<float*>(pb + PB::gb)[j] = 0.0f;
  } else if (i < kW + kB + 32) {
    const int k = i - kW - kB;
    float v = 0.0f;
    if (k < 7) v = norm[k];
    else if (k >= 8 && k < 15) v = norm[7 + k - 8];
    else if (k >= 16 && k < 19) v = norm[14 + k - 16];
    else if (k >= 8) v = 1.0f;  // scale slots of padding channels
    reinterpret_cast<float*>(pb + PB::norm)[k] = v;
  }
  if (i == 0) *reinterpret_cast<int*>(pb + PB::step) = 0;
}

__global__ void k_no_store(const char* pb, float* __restrict__ wl, float* __restrict__ bl) {
  const float* w = reinterpret_cast<const float*>(pb + PB::w);
  const float* b = reinterpret_cast<const float*>(pb + PB::b);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kW) {
    int l, co, t, ci;
    if (weight_live(i, l, co, t, ci)) {
      int lo = 0;
      for (int k = 0; k < l; ++k) lo += kCout[k] * 9 * kCin[k];
      wl[lo + (co * 9 + t) * kCin[l] + ci] = w[i];
    }
  } else if (i < kW + kB) {
    const int j = i - kW;
    int l = 0;
    while (l < kNL - 1 && j >= boff(l + 1)) ++l;
    int lo = 0;
    for (int k = 0; k < l; ++k) lo += kCout[k];
    const int co = j - boff(l);
    if (co < kCout[l]) bl[lo + co] = b[j];
  }
}

// B_out[c][r] = B[c][r] + out_std[c] * D[r][c] (one sample)
__global__ void k_no_out(const float* __restrict__ B, const float* __restrict__ D, int64_t P,
                         const float* __restrict__ norm, float* __restrict__ Bo) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= P) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) Bo[c * P + r] = B[c * P + r] + norm[16 + c] * D[r * 16 + c];
}

// activation buffers of a workspace for S samples of P pixels
struct Acts {
  uint16_t *x0, *h1, *h2, *h3, *dz4, *dza, *dzb;
  float* d4;
  float* part;    // weight-gradient partials
  double* lpart;  // loss partials
};
constexpr int kWgradBlocks = 256;
int64_t lpart_slots(int64_t N) { return ceil_div(N, 256); }

size_t acts_bytes(int64_t N) {
  size_t off = 0;
  auto take = [&](size_t b) { off += (b + 255) & ~(size_t)255; };
  take(2 * 16 * N);                                    // x0
  for (int k = 0; k < 3; ++k) take(2 * 32 * N);        // h1..h3
  take(2 * 16 * N);                                    // dz4
  take(2 * 32 * N);                                    // dza
  take(2 * 32 * N);                                    // dzb
  take(4 * 16 * N);                                    // d4
  take(4 * (size_t)kWgradBlocks * (32 * 9 * 32 + 32)); // partials
  take(8 * lpart_slots(N));
  return off;
}

Acts acts_of(void* ws, int64_t N) {
  char* base = static_cast<char*>(ws);
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = base + off;
    off += (b + 255) & ~(size_t)255;
    return p;
  };
  Acts a;
  a.x0 = (uint16_t*)take(2 * 16 * N);
  a.h1 = (uint16_t*)take(2 * 32 * N);
  a.h2 = (uint16_t*)take(2 * 32 * N);
  a.h3 = (uint16_t*)take(2 * 32 * N);
  a.dz4 = (uint16_t*)take(2 * 16 * N);
  a.dza = (uint16_t*)take(2 * 32 * N);
  a.dzb = (uint16_t*)take(2 * 32 * N);
  a.d4 = (float*)take(4 * 16 * N);
  a.part = (float*)take(4 * (size_t)kWgradBlocks * (32 * 9 * 32 + 32));
  a.lpart = (double*)take(8 * lpart_slots(N));
  return a;
}

int conv_grid(int64_t N) { return (int)std::min<int64_t>(ceil_div(ceil_div(N, 16), 4), 4096); }

template <int CINP, int COUTP, int MODE>
void conv(hipStream_t s, const uint16_t* X, const uint16_t* W, const float* bias,
          const uint16_t* H, void* out, int64_t N, int nx, int ny) {
  hipLaunchKernelGGL((k_conv3x3<CINP, COUTP, MODE>), dim3(conv_grid(N)), dim3(256), 0, s, X, W,
                     bias, H, out, N, nx, ny);
}

template <int CINP, int COUTP>
void wgrad(hipStream_t s, const uint16_t* X, const uint16_t* dZ, float* part, float* gw,
           float* gb, int64_t N, int nx, int ny) {
  const int nb = (int)std::min<int64_t>(ceil_div(N, kSeg), kWgradBlocks);
  hipLaunchKernelGGL((k_conv3x3_wgrad<CINP, COUTP>), dim3(nb), dim3(256), 0, s, X, dZ, part, N,
                     nx, ny);
  const int n = COUTP * 9 * CINP + COUTP;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s,
                     (const float*)part, nb, COUTP * 9 * CINP, COUTP, gw, gb);
}

// the forward pass of S samples: X0 -> d4 (normalised increment)
void forward(hipStream_t s, const char* pb, const Acts& a, int64_t N, int nx, int ny) {
  const uint16_t* wf = reinterpret_cast<const uint16_t*>(pb + PB::wf);
  const float* b = reinterpret_cast<const float*>(pb + PB::b);
  conv<16, 32, 0>(s, a.x0, wf + woff(0), b + boff(0), nullptr, a.h1, N, nx, ny);
  conv<32, 32, 0>(s, a.h1, wf + woff(1), b + boff(1), nullptr, a.h2, N, nx, ny);
  conv<32, 32, 0>(s, a.h2, wf + woff(2), b + boff(2), nullptr, a.h3, N, nx, ny);
  conv<32, 16, 1>(s, a.h3, wf + woff(3), b + boff(3), nullptr, a.d4, N, nx, ny);
}

bool grid_ok(int nx, int ny) { return nx >= 1 && ny >= 1 && (int64_t)nx * ny < (1ll << 28); }

}  // namespace

size_t no_params_bytes() { return PB::total; }

// The proposal B_out of the operator for one sample (B, n, J on an nx x ny
// grid), enqueued on s.
int no_predict(hipStream_t s, const void* params, void* ws, int nx, int ny, const float* B,
               const float* n, const float* J, float* B_out) {
  const int64_t P = (int64_t)nx * ny;
  const Acts a = acts_of(ws, P);
  const char* pb = static_cast<const char*>(params);
  const float* norm = reinterpret_cast<const float*>(pb + PB::norm);
  hipLaunchKernelGGL(k_no_pack, dim3((unsigned)ceil_div(P, 256)), dim3(256), 0, s, B, n, J,
                     (const int32_t*)nullptr, 1, P, norm, a.x0);
  forward(s, pb, a, P, nx, ny);
  hipLaunchKernelGGL(k_no_out, dim3((unsigned)ceil_div(P, 256)), dim3(256), 0, s, B,
                     (const float*)a.d4, P, norm, B_out);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace hvpic

using namespace hvpic;

extern "C" {

int hvpic_no_params_bytes(size_t* bytes) {
  if (!bytes) return HVPIC_EINVAL;
  *bytes = PB::total;
  return HVPIC_OK;
}

int hvpic_no_workspace_bytes(int nx, int ny, int batch, size_t* bytes) {
  if (!bytes || !grid_ok(nx, ny) || batch < 1 || batch > 4096) return HVPIC_EINVAL;
  *bytes = acts_bytes((int64_t)nx * ny * batch);
  return HVPIC_OK;
}

int hvpic_no_load(void* params, const float* w, const float* b, const float* norm,
                  void* hip_stream) {
  if (!params || !w || !b || !norm) return HVPIC_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int n = kW + kB + 32;
  hipLaunchKernelGGL(k_no_load, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s,
                     static_cast<char*>(params), w, b, norm);
  hipLaunchKernelGGL(k_no_adam, dim3((unsigned)ceil_div(kW + kB, 256)), dim3(256), 0, s,
                     static_cast<char*>(params), 0.0f, 0.9f, 0.999f, 1e-8f, 0);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int hvpic_no_store(const void* params, float* w, float* b, void* hip_stream) {
  if (!params || !w || !b) return HVPIC_EINVAL;
  hipLaunchKernelGGL(k_no_store, dim3((unsigned)ceil_div(kW + kB, 256)), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), static_cast<const char*>(params), w, b);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int hvpic_no_predict(const void* params, void* workspace, int nx, int ny, const float* B,
                     const float* n, const float* J, float* B_out, void* hip_stream) {
  if (!params || !workspace || !grid_ok(nx, ny) || !B || !n || !J || !B_out) return HVPIC_EINVAL;
  return no_predict(static_cast<hipStream_t>(hip_stream), params, workspace, nx, ny, B, n, J,
                    B_out);
}

int hvpic_no_train_step(void* params, void* workspace, int nx, int ny, const float* B,
                        const float* n, const float* J, const float* B_target, const int32_t* idx,
                        int batch, float lr, double* loss_out, void* hip_stream) {
  if (!params || !workspace || !grid_ok(nx, ny) || !B || !n || !J || !B_target || batch < 1 ||
      batch > 4096 || !(lr >= 0.0f))
    return HVPIC_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t P = (int64_t)nx * ny, N = P * batch;
  const Acts a = acts_of(workspace, N);
  char* pb = static_cast<char*>(params);
  const float* norm = reinterpret_cast<const float*>(pb + PB::norm);
  const uint16_t* wbk = reinterpret_cast<const uint16_t*>(pb + PB::wb);
  float* gw = reinterpret_cast<float*>(pb + PB::gw);
  float* gb = reinterpret_cast<float*>(pb + PB::gb);
  const unsigned pix = (unsigned)ceil_div(N, 256);
  hipLaunchKernelGGL(k_no_pack, dim3(pix), dim3(256), 0, s, B, n, J, idx, batch, P, norm, a.x0);
  forward(s, pb, a, N, nx, ny);
  hipLaunchKernelGGL(k_no_loss, dim3(pix), dim3(256), 0, s, (const float*)a.d4, B, B_target, idx,
                     batch, P, norm, a.dz4, a.lpart);
  // layer 3 (32 -> 16): weights, then the gradient at its input through tanh
  wgrad<32, 16>(s, a.h3, a.dz4, a.part, gw + woff(3), gb + boff(3), N, nx, ny);
  conv<16, 32, 2>(s, a.dz4, wbk + bwoff(3), nullptr, a.h3, a.dza, N, nx, ny);
  wgrad<32, 32>(s, a.h2, a.dza, a.part, gw + woff(2), gb + boff(2), N, nx, ny);
  conv<32, 32, 2>(s, a.dza, wbk + bwoff(2), nullptr, a.h2, a.dzb, N, nx, ny);
  wgrad<32, 32>(s, a.h1, a.dzb, a.part, gw + woff(1), gb + boff(1), N, nx, ny);
  conv<32, 32, 2>(s, a.dzb, wbk + bwoff(1), nullptr, a.h1, a.dza, N, nx, ny);
  wgrad<16, 32>(s, a.x0, a.dza, a.part, gw + woff(0), gb + boff(0), N, nx, ny);
  if (loss_out)
    hipLaunchKernelGGL(k_no_loss_final, dim3(1), dim3(1024), 0, s, (const double*)a.lpart,
                       (int)pix, (int64_t)(3 * N), loss_out);
  hipLaunchKernelGGL(k_no_adam, dim3((unsigned)ceil_div(kW + kB, 256)), dim3(256), 0, s, pb, lr,
                     0.9f, 0.999f, 1e-8f, 1);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int hvpic_field_advance_no(hvpic_ctx* ctx, const void* params, void* workspace, float* B,
                           const float* n_half, const float* J_half, const float* n_prev,
                           const float* J_prev, float* E_out, double* diag_out, float tol,
                           double* stats) {
  if (!ctx || ctx->magic != kMagic) return HVPIC_ESTATE;
  const hvpic_params& p = ctx->p;
  if (p.ndim != 2 || p.energy_eq || p.open_x || p.eta_h != 0.0 || p.nsub < 1) return HVPIC_EINVAL;
  if (!params || !workspace || !B || !n_half || !J_half || !n_prev || !J_prev || !E_out ||
      !(tol >= 0.0f))
    return HVPIC_EINVAL;
  float* Bno = ctx->fscratch + 22ll * ctx->ncell;  // the proposal [3][ncell]
  int rc = no_predict(ctx->stream, params, workspace, p.nx, p.ny, B, n_half, J_half, Bno);
  if (rc != HVPIC_OK) return rc;
  return launch_field_advance_no(ctx, B, n_half, J_half, n_prev, J_prev, E_out, diag_out, Bno,
                                 tol, stats);
}

// Single layers, for checking the kernels: a periodic 3x3 layer over nimg
// images (x bf16 [N][cinp], w bf16 [coutp][9][cinp]) and its weight gradient
// (added to dw [coutp][9][cinp] and db [coutp]).
int hvpic_no_conv3x3(int nimg, int nx, int ny, int cinp, int coutp, int mode, const void* x,
                     const void* w, const float* bias, const void* h, void* out,
                     void* hip_stream) {
  if (nimg < 1 || !grid_ok(nx, ny) || !x || !w || !out) return HVPIC_EINVAL;
  if (mode < 0 || mode > 2 || (mode != 2 && !bias) || (mode == 2 && !h)) return HVPIC_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t N = (int64_t)nx * ny * nimg;
  const uint16_t* X = static_cast<const uint16_t*>(x);
  const uint16_t* W = static_cast<const uint16_t*>(w);
  const uint16_t* H = static_cast<const uint16_t*>(h);
  const int key = cinp * 1000 + coutp * 10 + mode;
  switch (key) {
    case 16320: conv<16, 32, 0>(s, X, W, bias, H, out, N, nx, ny); break;
    case 32320: conv<32, 32, 0>(s, X, W, bias, H, out, N, nx, ny); break;
    case 32161: conv<32, 16, 1>(s, X, W, bias, H, out, N, nx, ny); break;
    case 16322: conv<16, 32, 2>(s, X, W, bias, H, out, N, nx, ny); break;
    case 32322: conv<32, 32, 2>(s, X, W, bias, H, out, N, nx, ny); break;
    default: return HVPIC_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int hvpic_no_conv3x3_wgrad(int nimg, int nx, int ny, int cinp, int coutp, const void* x,
                           const void* dz, float* dw, float* db, void* workspace,
                           void* hip_stream) {
  if (nimg < 1 || !grid_ok(nx, ny) || !x || !dz || !dw || !db || !workspace) return HVPIC_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t N = (int64_t)nx * ny * nimg;
  const Acts a = acts_of(workspace, N);
  const uint16_t* X = static_cast<const uint16_t*>(x);
  const uint16_t* Z = static_cast<const uint16_t*>(dz);
  if (cinp == 32 && coutp == 16)
    wgrad<32, 16>(s, X, Z, a.part, dw, db, N, nx, ny);
  else if (cinp == 32 && coutp == 32)
    wgrad<32, 32>(s, X, Z, a.part, dw, db, N, nx, ny);
  else if (cinp == 16 && coutp == 32)
    wgrad<16, 32>(s, X, Z, a.part, dw, db, N, nx, ny);
  else
    return HVPIC_EINVAL;
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // extern "C"
