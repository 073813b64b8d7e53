// Fingerprint extraction (section 5.1; section 5.2 statistics from a
// sample): one channel's continuous samples -> binary fingerprints, the
// sorted index lists the search takes.
//
//   spectrogram  power of the short-time Fourier transform (periodic Hann
//                window) in the kept frequency band, frames every `hop`
//                samples (k_stft);
//   image        per fingerprint, fp_frames consecutive frames averaged
//                time_ds at a time into a rows x cols spectral image;
//   wavelet      2-D orthonormal Haar transform (every row, then every
//                column; per axis: final average, then details from the
//                coarsest level to the finest);
//   normalize    z = (w - median) / MAD per coefficient (0 where MAD = 0),
//                median and MAD (lower middle values) over the fingerprints
//                whose ids the caller samples;
//   top-K        the K coefficients of largest |z| (ties: smaller index),
//                z != 0 only;
//   binarize     coefficient c with z > 0 -> bit 2c, z < 0 -> bit 2c + 1.
//
// GPU form.  The spectrogram is a product of the frames' samples (frames x
// window, rows overlapping by window - hop) with the band's Hann-weighted
// cosine and sine rows (window x 2 bins).  k_stft_mfma: a workgroup takes
// 256 consecutive frames and 32 bins, stages their samples and the basis
// rows in LDS, and forms the product with fp32 16 x 16 x 4 MFMA steps.
// k_stft, the vector form for windows and hops whose staging would not fit
// 64 KB: each lane accumulates 4 frames (64 apart) x 8 bins (real and
// imaginary parts) over the window with fp32 FMA.
// k_fp: one wavefront per fingerprint: the image is assembled in LDS, the
// Haar levels run in place (every lane reads its pairs, then writes), the
// normalized |z| of the lane's 32 consecutive coefficients are kept in
// registers as ordered integers, the K-th largest is found by a four-digit
// radix select with LDS histograms, and the selected bits are written in
// coefficient order at offsets from a wavefront scan.  Median and MAD come
// from segmented radix sorts (one segment per coefficient) of the sample's
// coefficients and of their absolute deviations.
#include <string.h>

#include <algorithm>

#include "host.hpp"

using namespace fl;

namespace {

constexpr int kFT = 256;             // threads per workgroup
constexpr int kFramesPerBlock = 256; // k_stft frames per workgroup
constexpr int kMaxWindow = 256;
constexpr int kMaxCoef = 2048;       // rows * cols
constexpr int kPitchPad = 1;         // LDS row padding of the image

struct FpArgs {
  const float* x;
  uint64_t n;          // samples
  uint32_t window, hop, band_lo, rows, fp_frames, time_ds, cols, fp_lag, top_k;
  uint32_t lrows, lcols;  // log2 of rows and cols (both powers of two)
  uint64_t n_frames, n_fp;
};

// LDS reads of one wavefront see its own earlier LDS writes and atomics.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Floats as unsigned integers in the same order.
__device__ __forceinline__ uint32_t f2o(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float o2f(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

// Power spectrogram of the kept band, frame-major: spec[frame * rows + bin].
__global__ __launch_bounds__(kFT) void k_stft(FpArgs a, float* spec) {
  extern __shared__ float lds[];
  const uint32_t W = a.window;
  float* xs = lds;                                                    // kFramesPerBlock * hop + W samples
  float* basis = xs + (((size_t)kFramesPerBlock * a.hop + W + 3) & ~(size_t)3);  // [4 waves][W][16], 16-byte aligned
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t f0 = (uint64_t)blockIdx.x * kFramesPerBlock;
  const uint64_t s0 = f0 * a.hop;
  const uint32_t span = kFramesPerBlock * a.hop + W;
  for (uint32_t e = tid; e < span; e += kFT) xs[e] = s0 + e < a.n ? a.x[s0 + e] : 0.0f;
  // this wavefront's bins: kb0 .. kb0 + 7 of the kept band
  const uint32_t kb0 = blockIdx.y * 32 + wave * 8;
  float* B = basis + (size_t)wave * W * 16;
  for (uint32_t e = lane; e < W * 8; e += 64) {
    const uint32_t nn = e >> 3, j = e & 7;
    const uint32_t k = a.band_lo + kb0 + j;
    float sn, cs;
    sincospif(2.0f * (float)((k * nn) % W) / (float)W, &sn, &cs);
    const float h = 0.5f * (1.0f - cospif(2.0f * (float)nn / (float)W));
    B[nn * 16 + 2 * j] = cs * h;
    B[nn * 16 + 2 * j + 1] = -sn * h;
  }
  __syncthreads();
  float acc[4][16];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[q][j] = 0.0f;
  // lane l takes frames l, l + 64, l + 128, l + 192 of the block, so that in
  // every sample step the wave reads samples hop apart (a few banks each)
  const float* xl = xs + (size_t)lane * a.hop;
  const uint32_t qs = 64 * a.hop;
  for (uint32_t nn = 0; nn < W; ++nn) {
    float b[16];
    const float4* bp = reinterpret_cast<const float4*>(B + nn * 16);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float4 t = bp[v];
      b[4 * v] = t.x;
      b[4 * v + 1] = t.y;
      b[4 * v + 2] = t.z;
      b[4 * v + 3] = t.w;
    }
    float xv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) xv[q] = xl[q * qs + nn];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[q][j] = fmaf(xv[q], b[j], acc[q][j]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint64_t f = f0 + lane + 64 * q;
    if (f >= a.n_frames) continue;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t kb = kb0 + j;
      if (kb < a.rows) spec[f * a.rows + kb] = acc[q][2 * j] * acc[q][2 * j] + acc[q][2 * j + 1] * acc[q][2 * j + 1];
    }
  }
}

// In-place Haar levels along one axis of the image v (pitch P): `lines`
// lines of length `len`, element (line, i) at v[line * ls + i * es].  All
// waves of the workgroup run the same levels (barriers).
__device__ __forceinline__ void haar_axis(float* v, uint32_t lines, uint32_t llen, uint32_t ls, uint32_t es,
                                          uint32_t lane) {
  const float s = 0.70710678118654752f;
  for (uint32_t lh = llen; lh > 0; --lh) {  // level with 2^lh elements per line
    const uint32_t half = 1u << (lh - 1), items = lines * half;
    float av[kMaxCoef / 2 / 64], dv[kMaxCoef / 2 / 64];
    uint32_t k = 0;
    for (uint32_t e = lane; e < items; e += 64, ++k) {
      const uint32_t line = e >> (lh - 1), j = e & (half - 1);
      const float x0 = v[line * ls + (2 * j) * es], x1 = v[line * ls + (2 * j + 1) * es];
      av[k] = (x0 + x1) * s;
      dv[k] = (x0 - x1) * s;
    }
    __syncthreads();
    k = 0;
    for (uint32_t e = lane; e < items; e += 64, ++k) {
      const uint32_t line = e >> (lh - 1), j = e & (half - 1);
      v[line * ls + j * es] = av[k];
      v[line * ls + (half + j) * es] = dv[k];
    }
    __syncthreads();
  }
}

// Hann-weighted cosine and sine rows of the kept band for the matrix-core
// form of the spectrogram: basis[yb][t][n][16], column c = 16 t + j of bin
// group yb (32 bins) = bin 32 yb + c / 2, cos for even c, -sin for odd c, at
// sample n of the window; zero past the window (n < wpad, the window rounded
// up to 4) and past the band.
__global__ __launch_bounds__(kFT) void k_stft_basis(FpArgs a, uint32_t wpad, uint32_t nyb, float* basis) {
  const uint32_t W = a.window;
  const uint64_t total = (uint64_t)nyb * 4 * wpad * 16;
  for (uint64_t e = (uint64_t)blockIdx.x * kFT + threadIdx.x; e < total; e += (uint64_t)gridDim.x * kFT) {
    const uint32_t j = (uint32_t)(e & 15), nn = (uint32_t)((e >> 4) % wpad);
    const uint32_t t = (uint32_t)((e >> 4) / wpad % 4), yb = (uint32_t)((e >> 4) / wpad / 4);
    const uint32_t c = 16 * t + j, kb = 32 * yb + c / 2;
    float v = 0.0f;
    if (nn < W && kb < a.rows) {
      const uint32_t k = a.band_lo + kb;
      float sn, cs;
      sincospif(2.0f * (float)((k * nn) % W) / (float)W, &sn, &cs);
      const float h = 0.5f * (1.0f - cospif(2.0f * (float)nn / (float)W));
      v = (c & 1) ? -sn * h : cs * h;
    }
    basis[e] = v;
  }
}

// The spectrogram on the matrix cores: per workgroup 256 consecutive frames
// and one bin group (32 bins, 64 basis columns).  The frames' samples and
// the group's basis rows are staged in LDS; wavefront w takes frames
// 64 w .. 64 w + 63 as four 16-frame tiles against the four 16-column basis
// tiles, accumulating frames x window x basis with 16 x 16 x 4 fp32 MFMA
// steps (A: frame row i, samples n0 + k in lane i + 16 k; B: basis rows
// n0 + k, column j in lane j + 16 k; D: row 4 (lane / 16) + r, column
// lane % 16 in element r).  The power of a bin is re^2 + im^2 of two
// neighbouring columns, which sit in neighbouring lanes.
__global__ __launch_bounds__(kFT) void k_stft_mfma(FpArgs a, const float* basis, uint32_t wpad, float* spec) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  extern __shared__ float lds[];
  const uint32_t hop = a.hop;
  float* xs = lds;  // 255 * hop + wpad samples
  const uint32_t span = (kFramesPerBlock - 1) * hop + wpad;
  float* bl = xs + ((span + 3) & ~3u);  // [4][wpad][16]
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t f0 = (uint64_t)blockIdx.x * kFramesPerBlock;
  const uint64_t s0 = f0 * hop;
  for (uint32_t e = tid; e < span; e += kFT) xs[e] = s0 + e < a.n ? a.x[s0 + e] : 0.0f;
  {
    const float4* src = reinterpret_cast<const float4*>(basis + (uint64_t)blockIdx.y * 4 * wpad * 16);
    float4* dst = reinterpret_cast<float4*>(bl);
    for (uint32_t e = tid; e < wpad * 16; e += kFT) dst[e] = src[e];  // 4 * wpad * 16 floats
  }
  __syncthreads();
  const uint32_t li = lane & 15, lk = lane >> 4;
  const float* xw = xs + (wave * 64 + li) * hop + lk;
  const float* bw = bl + lk * 16 + li;
  f4 acc[4][4];
#pragma unroll
  for (int ft = 0; ft < 4; ++ft)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[ft][t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  for (uint32_t n0 = 0; n0 < wpad; n0 += 4) {
    float av[4], bv[4];
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) av[ft] = xw[ft * 16 * hop + n0];
#pragma unroll
    for (int t = 0; t < 4; ++t) bv[t] = bw[(t * wpad + n0) * 16];
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[ft][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ft], bv[t], acc[ft][t], 0, 0, 0);
  }
#pragma unroll
  for (int ft = 0; ft < 4; ++ft)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float v = acc[ft][t][r];
        const float w = __shfl_xor(v, 1, 64);
        const uint64_t f = f0 + wave * 64 + 16 * ft + 4 * lk + r;
        const uint32_t kb = 32 * blockIdx.y + (16 * t + li) / 2;
        if (!(li & 1) && f < a.n_frames && kb < a.rows) spec[f * a.rows + kb] = v * v + w * w;
      }
}


// One wavefront per fingerprint.  mode 0 (sample): fingerprint sample_ids[s]
// writes its coefficients as ordered keys into keys_t[c * n_sample + s];
// mode 1 (main): fingerprint i writes its top-K bits to out[i * K ..] and
// its count to cnt[i] (when cnt is given); unused slots hold 0xFFFF.
__global__ __launch_bounds__(kFT) void k_fp(FpArgs a, const float* spec, int mode, const uint64_t* sample_ids,
                                            uint64_t n_items, uint64_t* keys_t, const float* med, const float* mad,
                                            uint16_t* out, uint32_t* cnt) {
  extern __shared__ float lds2[];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t R = a.rows, C = a.cols, NC = R * C, P = C + kPitchPad;
  float* v = lds2 + (size_t)wave * (R * P + 256);  // image, then 256 histogram words
  uint32_t* hist = reinterpret_cast<uint32_t*>(v + R * P);
  // consecutive fingerprints share most of their frames: keep them on one
  // XCD's L2
  const uint64_t item = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * 4 + wave;
  const bool live = item < n_items;
  const uint64_t fi = !live ? 0 : (mode == 0 ? sample_ids[item] : item);
  // 1. spectral image: column c averages frames c*ds .. c*ds+ds-1 of the
  // fingerprint's window
  const uint64_t F0 = fi * a.fp_lag;
  const float inv = 1.0f / (float)a.time_ds;
  for (uint32_t e = lane; e < NC; e += 64) {
    const uint32_t c = e >> a.lrows, r = e & (R - 1);  // consecutive lanes: consecutive bins of one frame
    float sum = 0.0f;
    if (live)
      for (uint32_t d = 0; d < a.time_ds; ++d) sum += spec[(F0 + (uint64_t)c * a.time_ds + d) * R + r];
    v[r * P + c] = sum * inv;
  }
  __syncthreads();
  // 2. Haar: rows (length C), then columns (length R)
  haar_axis(v, R, a.lcols, P, 1, lane);
  haar_axis(v, C, a.lrows, 1, P, lane);
  if (mode == 0) {
    if (live)
      for (uint32_t e = lane; e < NC; e += 64) {
        const uint32_t r = e >> a.lcols, c = e & (C - 1);
        keys_t[(uint64_t)e * n_items + item] = f2o(v[r * P + c]);
      }
    return;
  }
  // 3. normalize: lane holds coefficients [lane * per, lane * per + per)
  const uint32_t per = NC / 64;  // NC is a multiple of 64
  uint32_t key[kMaxCoef / 64];
  uint32_t neg = 0;  // bit q: z < 0
  uint32_t nz = 0;
  for (uint32_t q = 0; q < per; ++q) {
    const uint32_t e = lane * per + q;
    const uint32_t r = e >> a.lcols, c = e & (C - 1);
    const float w = v[r * P + c];
    const float m = mad[e];
    const float z = m > 0.0f ? (w - med[e]) / m : 0.0f;
    key[q] = __float_as_uint(fabsf(z));
    if (z < 0.0f) neg |= 1u << q;
    nz += key[q] != 0u;
  }
  for (int o = 32; o > 0; o >>= 1) nz += __shfl_xor(nz, o, 64);
  // 4. the K-th largest key T (radix select over four 8-bit digits: the top
  // one by wavefront counts, the others by LDS histograms), and how many
  // keys equal to T are taken (the smallest indices first); each wavefront
  // works on its own histogram, so only wavefront-level syncs
  uint32_t T = 0, take_eq = 0;
  const bool all_nonzero = nz <= a.top_k;
  if (!all_nonzero) {
    uint32_t remaining = a.top_k;
    // top digit: the keys' top bytes (sign and exponent) take few values, so
    // instead of a histogram (whose atomics would all meet in those few
    // bins) the occupied values are visited from the largest down with
    // wavefront counts until the K-th key's value is reached
    uint32_t d = 0;
    for (uint32_t q = 0; q < per; ++q) d = max(d, key[q] >> 24);
    for (int o = 32; o > 0; o >>= 1) d = max(d, (uint32_t)__shfl_xor(d, o, 64));
    for (;;) {
      uint32_t c = 0, below = 0;
      for (uint32_t q = 0; q < per; ++q) {
        const uint32_t t = key[q] >> 24;
        c += key[q] != 0u && t == d;
        if (key[q] != 0u && t < d) below = max(below, t);
      }
      for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        below = max(below, (uint32_t)__shfl_xor(below, o, 64));
      }
      if (c >= remaining) break;  // more than top_k keys are non-zero, so this ends
      remaining -= c;
      d = below;
    }
    uint32_t prefix = d << 24, mask = 0xFF000000u;
    for (int shift = 16; shift >= 0; shift -= 8) {
      for (uint32_t b = lane; b < 256; b += 64) hist[b] = 0;
      wave_lds_sync();
      for (uint32_t q = 0; q < per; ++q)
        if (key[q] != 0u && (key[q] & mask) == prefix) atomicAdd(&hist[(key[q] >> shift) & 255u], 1u);
      wave_lds_sync();
      // lane l holds digits 255 - 4l .. 252 - 4l (descending); suffix counts
      uint32_t h4[4], s4 = 0;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        h4[d] = hist[255 - 4 * lane - d];
        s4 += h4[d];
      }
      uint32_t incl = s4;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o) incl += y;
      }
      uint32_t before = incl - s4;  // keys with a larger digit (lanes before)
      uint32_t digit = 0, above = 0;
      bool found = false;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        if (!found && before < remaining && before + h4[d] >= remaining) {
          found = true;
          digit = 255 - 4 * lane - d;
          above = before;
        }
        before += h4[d];
      }
      const uint64_t fm = __ballot(found);
      const int src = __ffsll((long long)fm) - 1;
      digit = __shfl(digit, src, 64);
      above = __shfl(above, src, 64);
      remaining -= above;
      prefix |= digit << shift;
      mask |= 255u << shift;
      wave_lds_sync();  // every lane has read the histogram before the next clear
    }
    T = prefix;
    take_eq = remaining;
  }
  // 5. selection and emission in coefficient order
  uint32_t eq_here = 0;
  if (!all_nonzero)
    for (uint32_t q = 0; q < per; ++q) eq_here += key[q] == T;
  uint32_t eq_incl = eq_here;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(eq_incl, o, 64);
    if (lane >= (uint32_t)o) eq_incl += y;
  }
  uint32_t eq_rank = eq_incl - eq_here;  // equal keys at smaller indices
  uint32_t selm = 0, nsel = 0;
  for (uint32_t q = 0; q < per; ++q) {
    bool sel;
    if (all_nonzero) {
      sel = key[q] != 0u;
    } else {
      sel = key[q] > T || (key[q] == T && eq_rank < take_eq);
      eq_rank += key[q] == T;
    }
    if (sel) {
      selm |= 1u << q;
      ++nsel;
    }
  }
  uint32_t pos_incl = nsel;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(pos_incl, o, 64);
    if (lane >= (uint32_t)o) pos_incl += y;
  }
  const uint32_t total = __shfl(pos_incl, 63, 64);
  if (!live) return;
  uint16_t* o = out + fi * a.top_k;
  uint32_t p = pos_incl - nsel;
  for (uint32_t q = 0; q < per; ++q)
    if (selm >> q & 1u) o[p++] = (uint16_t)(2u * (lane * per + q) + ((neg >> q) & 1u));
  for (uint32_t e = total + lane; e < a.top_k; e += 64) o[e] = 0xFFFFu;
  if (cnt && lane == 0) cnt[fi] = total;
}

// The lower middle value of each coefficient's sorted segment:
// out[c] = o2f(sorted[c * m + (m - 1) / 2]).
__global__ __launch_bounds__(kFT) void k_seg_median(const uint64_t* sorted, uint64_t m, uint32_t nc, float* out) {
  const uint32_t c = blockIdx.x * kFT + threadIdx.x;
  if (c < nc) out[c] = o2f((uint32_t)sorted[(uint64_t)c * m + (m - 1) / 2]);
}

// Absolute deviations from each coefficient's median, as ordered keys.
__global__ __launch_bounds__(kFT) void k_seg_dev(const uint64_t* sorted, uint64_t m, uint32_t nc, const float* med,
                                                 uint64_t* dev) {
  const uint64_t total = m * nc;
  for (uint64_t e = (uint64_t)blockIdx.x * kFT + threadIdx.x; e < total; e += (uint64_t)gridDim.x * kFT) {
    const uint32_t c = (uint32_t)(e / m);
    dev[e] = f2o(fabsf(o2f((uint32_t)sorted[e]) - med[c]));
  }
}

unsigned grid_f(uint64_t n) {
  const uint64_t b = (n + kFT - 1) / kFT;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 8u * device_cus()));
}

bool pow2(uint32_t v) { return v && !(v & (v - 1)); }

size_t stft_lds_bytes(uint32_t window, uint32_t hop) {
  return ((((size_t)kFramesPerBlock * hop + window + 3) & ~(size_t)3) + 4ull * window * 16) * sizeof(float);
}

size_t stft_mfma_lds_bytes(uint32_t window, uint32_t hop) {
  const size_t wpad = (window + 3) & ~3u;
  return (((((size_t)kFramesPerBlock - 1) * hop + wpad + 3) & ~(size_t)3) + 4 * wpad * 16) * sizeof(float);
}

}  // namespace

extern "C" int fast_lsh_fingerprints(fast_lsh_ctx* c, const float* samples, uint64_t n_samples,
                                     const fast_lsh_fp_params* prm, const uint64_t* sample_ids, uint64_t n_sample,
                                     uint16_t* out, uint32_t* out_count, uint64_t capacity, uint64_t* n_fp,
                                     float* med_mad) {
  if (!c) return fl_fail(FAST_LSH_E_INVALID, "ctx is NULL");
  if (!prm || !n_fp) return fl_fail(FAST_LSH_E_INVALID, "params or n_fp is NULL");
  *n_fp = 0;
  const uint32_t W = prm->window, rows = prm->band_hi - prm->band_lo;
  if (W < 2 || W > (uint32_t)kMaxWindow || prm->hop < 1 || prm->hop > 64)
    return fl_fail(FAST_LSH_E_INVALID, "window %u must be in [2, %d] and hop %u in [1, 64]", W, kMaxWindow, prm->hop);
  if (prm->band_hi <= prm->band_lo || prm->band_hi > W / 2 + 1 || !pow2(rows) || rows < 8 || rows > 64)
    return fl_fail(FAST_LSH_E_INVALID, "band [%u, %u) must hold 8, 16, 32 or 64 bins of the %u-sample window",
                   prm->band_lo, prm->band_hi, W);
  if (prm->time_ds < 1 || prm->fp_frames % prm->time_ds || !pow2(prm->fp_frames / prm->time_ds))
    return fl_fail(FAST_LSH_E_INVALID, "fp_frames / time_ds must be a power of two");
  const uint32_t cols = prm->fp_frames / prm->time_ds, nc = rows * cols;
  if (nc < 64 || nc > (uint32_t)kMaxCoef)
    return fl_fail(FAST_LSH_E_INVALID, "image of %u x %u coefficients outside [64, %d]", rows, cols, kMaxCoef);
  if (prm->fp_lag < 1 || prm->top_k < 1 || prm->top_k > nc)
    return fl_fail(FAST_LSH_E_INVALID, "fp_lag must be >= 1 and top_k in [1, %u]", nc);
  if (n_sample < 1 || !sample_ids) return fl_fail(FAST_LSH_E_INVALID, "the normalization sample is empty");
  if (stft_lds_bytes(W, prm->hop) > 65536)
    return fl_fail(FAST_LSH_E_INVALID, "window %u and hop %u need more than 64 KB of LDS (window * 65 + 256 * hop "
                   "must be at most 16384)", W, prm->hop);
  FpArgs a;
  memset(&a, 0, sizeof a);
  a.x = samples;
  a.n = n_samples;
  a.window = W;
  a.hop = prm->hop;
  a.band_lo = prm->band_lo;
  a.rows = rows;
  a.fp_frames = prm->fp_frames;
  a.time_ds = prm->time_ds;
  a.cols = cols;
  a.lrows = (uint32_t)__builtin_ctz(rows);
  a.lcols = (uint32_t)__builtin_ctz(cols);
  a.fp_lag = prm->fp_lag;
  a.top_k = prm->top_k;
  a.n_frames = n_samples < W ? 0 : (n_samples - W) / prm->hop + 1;
  a.n_fp = a.n_frames < prm->fp_frames ? 0 : (a.n_frames - prm->fp_frames) / prm->fp_lag + 1;
  *n_fp = a.n_fp;
  if (a.n_fp == 0) return FAST_LSH_OK;
  if (a.n_fp > capacity)
    return fl_fail(FAST_LSH_E_CAPACITY, "%llu fingerprints do not fit capacity %llu", (unsigned long long)a.n_fp,
                   (unsigned long long)capacity);
  if (!samples || !out) return fl_fail(FAST_LSH_E_INVALID, "samples or out is NULL");
  HIPCK(hipSetDevice(c->device));
  hipStream_t s = c->stream;
  // the sample's ids must name fingerprints (checked on the host copy)
  {
    std::vector<uint64_t> ids(n_sample);
    HIPCK(hipMemcpyAsync(ids.data(), sample_ids, n_sample * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    for (uint64_t k = 0; k < n_sample; ++k)
      if (ids[k] >= a.n_fp)
        return fl_fail(FAST_LSH_E_INVALID, "sample id %llu >= %llu fingerprints", (unsigned long long)ids[k],
                       (unsigned long long)a.n_fp);
  }
  float* spec;
  RC(ws<float>(c, "fp_spec", a.n_frames * rows, &spec));
  // 1. spectrogram (on the matrix cores when the staged rows fit 64 KB)
  {
    const dim3 grid((unsigned)((a.n_frames + kFramesPerBlock - 1) / kFramesPerBlock), (rows + 31) / 32);
    const uint32_t wpad = (W + 3) & ~3u;
    if (stft_mfma_lds_bytes(W, a.hop) <= 65536) {
      float* basis;
      RC(ws<float>(c, "fp_basis", (uint64_t)grid.y * 4 * wpad * 16, &basis));
      prof_begin(c, FAST_LSH_STAGE_SPECTROGRAM);
      hipLaunchKernelGGL(k_stft_basis, dim3(grid.y * wpad / 4), dim3(kFT), 0, s, a, wpad, grid.y, basis);
      hipLaunchKernelGGL(k_stft_mfma, grid, dim3(kFT), stft_mfma_lds_bytes(W, a.hop), s, a, basis, wpad, spec);
      prof_end(c);
    } else {
      prof_begin(c, FAST_LSH_STAGE_SPECTROGRAM);
      hipLaunchKernelGGL(k_stft, grid, dim3(kFT), stft_lds_bytes(W, a.hop), s, a, spec);
      prof_end(c);
    }
  }
  LAUNCHCK();
  const size_t fp_lds = 4ull * (rows * (cols + kPitchPad) + 256) * sizeof(float);
  // 2. the sample's coefficients, then median and MAD per coefficient
  uint64_t *k0, *k1;
  uint32_t *v0, *v1, *hist, *sums;
  float *med, *mad;
  const uint64_t tot = (uint64_t)nc * n_sample;
  RC(ws<uint64_t>(c, "fp_k0", tot, &k0));
  RC(ws<uint64_t>(c, "fp_k1", tot, &k1));
  RC(ws<uint32_t>(c, "fp_v0", tot, &v0));
  RC(ws<uint32_t>(c, "fp_v1", tot, &v1));
  const uint32_t nt = radix_tiles(n_sample, 0);
  RC(ws<uint32_t>(c, "fp_hist", (uint64_t)256 * nt * nc, &hist));
  RC(ws<uint32_t>(c, "fp_sums", scan_sums_elems((uint64_t)256 * nt, nc), &sums));
  RC(ws<float>(c, "fp_stats", 2ull * nc, &med));
  mad = med + nc;
  prof_begin(c, FAST_LSH_STAGE_FINGERPRINTS);
  hipLaunchKernelGGL(k_fp, dim3((unsigned)((n_sample + 3) / 4)), dim3(kFT), fp_lds, s, a, spec, 0, sample_ids,
                     n_sample, k0, nullptr, nullptr, nullptr, nullptr);
  for (int pass = 0; pass < 2; ++pass) {
    bool first = true;
    for (uint32_t sh = 0; sh < 32; sh += 8) {
      radix_pass(k0, first ? nullptr : v0, k1, v1, n_sample, nc, sh, hist, sums, 0, s);
      first = false;
      std::swap(k0, k1);
      std::swap(v0, v1);
    }
    if (pass == 0) {
      hipLaunchKernelGGL(k_seg_median, dim3((nc + kFT - 1) / kFT), dim3(kFT), 0, s, k0, n_sample, nc, med);
      hipLaunchKernelGGL(k_seg_dev, dim3(grid_f(tot)), dim3(kFT), 0, s, k0, n_sample, nc, med, k1);
      std::swap(k0, k1);
    } else {
      hipLaunchKernelGGL(k_seg_median, dim3((nc + kFT - 1) / kFT), dim3(kFT), 0, s, k0, n_sample, nc, mad);
    }
  }
  // 3. every fingerprint: normalize, top-K, binarize
  hipLaunchKernelGGL(k_fp, dim3((unsigned)((a.n_fp + 3) / 4)), dim3(kFT), fp_lds, s, a, spec, 1, nullptr, a.n_fp,
                     nullptr, med, mad, out, out_count);
  prof_end(c);
  LAUNCHCK();
  if (med_mad) HIPCK(hipMemcpyAsync(med_mad, med, 2ull * nc * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIPCK(hipStreamSynchronize(s));
  prof_collect(c);
  return FAST_LSH_OK;
}
