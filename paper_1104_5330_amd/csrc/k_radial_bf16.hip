// Mixed-precision radial pass: cos(Theta) * (D_r Y) with D_r and Y each split
// into three bf16 terms (D = D1 + D2 + D3, Y = Y1 + Y2 + Y3) and the six leading
// cross products D1Y1, D1Y2, D2Y1, D1Y3, D2Y2, D3Y1 accumulated in FP32 on
// v_mfma_f32_16x16x32_bf16 (the "bf16x3" scheme of Henry, Tang and Heinecke,
// ARITH 2019).  Together they carry about 24 significant bits, the precision of
// the FP32 stage copies they act on.
//
// Operand layouts of v_mfma_f32_16x16x32_bf16 (lane l, element e = 0..7):
//   A (16 x 32): A[l % 16][8 (l / 16) + e];  B (32 x 16): B[8 (l / 16) + e][l % 16];
//   C (16 x 16): register v holds C[4 (l / 16) + v][l % 16].
#include <cstring>

#include "k_common.h"

namespace {

constexpr int CB = 256;
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

SP6_DEV void split3(float x, __bf16& a, __bf16& b, __bf16& c) {
  a = (__bf16)x;
  const float r1 = x - float(a);
  b = (__bf16)r1;
  c = (__bf16)(r1 - float(b));
}

// NRT row tiles of 16, KS k-steps of 32 (n_r <= 32 KS, 16 NRT)
template <int NRT, bool ACCUM, typename TI>
__global__ __launch_bounds__(CB) void k_radial_bf16x3(KDims d, KTab t, const TI* __restrict__ Y,
                                                      float* __restrict__ T) {
  constexpr int KS = (NRT + 1) / 2;
  constexpr int NWV = CB / 64;
  const int lane = threadIdx.x & 63, wave = wave_uniform(threadIdx.x >> 6);
  const int lr = lane & 15, lg = lane >> 4;
  // A operands: three bf16 planes of the padded matrix, 8 consecutive k per lane
  v8bf A[3][NRT][KS];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const uint16_t* src = t.Dsplit + (size_t(p) * t.NRP + 16 * rt + lr) * t.KP3 + 32 * s + 8 * lg;
        const uint4 raw = *reinterpret_cast<const uint4*>(src);
        __builtin_memcpy(&A[p][rt][s], &raw, 16);
      }
  const int gpe = int(d.M / 16);
  const int ngroups = gpe * d.n_eps;
  // the resident workgroups advance through the groups together, in the
  // direction d.rev
  const int gstride = int(gridDim.x) * NWV;
  const int64_t M = d.M;
  const int n_r = d.n_r;
  // wave-uniform row pointers plus 32-bit per-lane byte offsets (B rows 8 lg + q,
  // C rows 4 lg + v).  Only the last k-step and the last row tile can reach past
  // n_r; every other load and store is unconditional.
  const uint32_t offB = (uint32_t(8 * lg) * uint32_t(M) + uint32_t(lr)) * uint32_t(sizeof(TI));
  const uint32_t offC = (uint32_t(4 * lg) * uint32_t(M) + uint32_t(lr)) * 4u;
  auto ldY = [&](const TI* row) { return *reinterpret_cast<const TI*>(reinterpret_cast<const char*>(row) + offB); };
  auto atT = [&](float* row) { return reinterpret_cast<float*>(reinterpret_cast<char*>(row) + offC); };
  // every extent is a power of two: divisions become shifts
  const int sh_g = __builtin_ctz(gpe), sh_P = __builtin_ctz(d.n_Ph);
  // a wavefront takes the two column groups of a 128-byte FP32 row segment one
  // after the other, so that the second half of each line is read while the
  // first half's fetch is still in L2; with few row tiles (registers to spare)
  // both groups' loads are issued before either group's products
  constexpr int TVN = ACCUM ? NRT * 4 : 1;
  constexpr bool PAIRLOAD = NRT <= 3;
  struct Group {
    float y[KS][8];
    float tv[TVN];
    float cT;
    int64_t gb;
  };
  auto load = [&](int k, Group& G) {
    const int g = d.rev ? ngroups - 1 - k : k;
    const int e = g >> sh_g;
    const int c0 = (g & (gpe - 1)) * 16;
    G.cT = float(t.cos_Th[((c0 + lr) >> sh_P) & (d.n_Th - 1)]);
    G.gb = int64_t(e) * n_r * M + c0;
    const TI* __restrict__ Yg = Y + G.gb;
    float* __restrict__ Tg = T + G.gb;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const TI* row = Yg + int64_t(32 * s + q) * M;
        if (s < KS - 1)
          G.y[s][q] = float(ldY(row));
        else
          G.y[s][q] = 32 * s + 8 * lg + q < n_r ? float(ldY(row)) : 0.0f;
      }
    if constexpr (ACCUM) {
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float* row = Tg + int64_t(16 * rt + v) * M;
          if (rt < NRT - 1)
            G.tv[rt * 4 + v] = *atT(row);
          else
            G.tv[rt * 4 + v] = 16 * rt + 4 * lg + v < n_r ? *atT(row) : 0.0f;
        }
    }
  };
  auto compute = [&](const Group& G) {
    float* __restrict__ Tg = T + G.gb;
    v8bf B[3][KS];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        __bf16 b1, b2, b3;
        split3(G.y[s][q], b1, b2, b3);
        B[0][s][q] = b1;
        B[1][s][q] = b2;
        B[2][s][q] = b3;
      }
    v4f acc[NRT];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) {
      acc[rt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        // smallest products first
        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2][rt][s], B[0][s], acc[rt], 0, 0, 0);
        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1][rt][s], B[1][s], acc[rt], 0, 0, 0);
        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0][rt][s], B[2][s], acc[rt], 0, 0, 0);
        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1][rt][s], B[0][s], acc[rt], 0, 0, 0);
        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0][rt][s], B[1][s], acc[rt], 0, 0, 0);
        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0][rt][s], B[0][s], acc[rt], 0, 0, 0);
      }
    }
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (rt < NRT - 1 || 16 * rt + 4 * lg + v < n_r) {
          const float val = G.cT * acc[rt][v];
          float* dst = atT(Tg + int64_t(16 * rt + v) * M);
          if constexpr (ACCUM)
            *dst = G.tv[rt * 4 + v] + val;
          else
            *dst = val;
        }
      }
  };
  for (int k2 = int(blockIdx.x) * NWV + wave; 2 * k2 < ngroups; k2 += gstride) {
    const bool two = 2 * k2 + 1 < ngroups;
    if constexpr (PAIRLOAD) {
      Group G0, G1;
      load(2 * k2, G0);
      if (two) load(2 * k2 + 1, G1);
      compute(G0);
      if (two) compute(G1);
    } else {
      Group G0;
      load(2 * k2, G0);
      compute(G0);
      if (two) {
        load(2 * k2 + 1, G0);
        compute(G0);
      }
    }
  }
}

template <int NRT, typename TI>
void launch_t(const KDims& d, const KTab& t, const void* Y, float* T, bool accum, hipStream_t s) {
  const int64_t ngroups = (d.M / 16) * d.n_eps;
  // one resident round of workgroups, advancing through the column groups together
  auto blocks_for = [&](auto kernel) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, CB, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    const int64_t blocks = (ngroups + 3) / 4, cap = int64_t(d.ncu) * per_cu;
    return unsigned(blocks < cap ? blocks : cap);
  };
  const TI* y = static_cast<const TI*>(Y);
  if (accum)
    k_radial_bf16x3<NRT, true, TI><<<blocks_for(k_radial_bf16x3<NRT, true, TI>), CB, 0, s>>>(d, t, y, T);
  else
    k_radial_bf16x3<NRT, false, TI><<<blocks_for(k_radial_bf16x3<NRT, false, TI>), CB, 0, s>>>(d, t, y, T);
}

template <typename TI>
hipError_t launch_ti(const KDims& d, const KTab& t, const void* Y, float* T, bool accum, hipStream_t s) {
  switch (t.NRP / 16) {
    case 1: launch_t<1, TI>(d, t, Y, T, accum, s); break;
    case 2: launch_t<2, TI>(d, t, Y, T, accum, s); break;
    case 3: launch_t<3, TI>(d, t, Y, T, accum, s); break;
    case 4: launch_t<4, TI>(d, t, Y, T, accum, s); break;
    case 5: launch_t<5, TI>(d, t, Y, T, accum, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// round a double to bf16 (round to nearest even through FP32)
uint16_t to_bf16(double x) {
  float f = float(x);
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

double from_bf16(uint16_t b) {
  uint32_t u = uint32_t(b) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return double(f);
}

}  // namespace

hipError_t launch_radial_bf16x3(const KDims& d, const KTab& t, const void* Y, bool y_f32, float* T, bool accum,
                                hipStream_t s) {
  return y_f32 ? launch_ti<float>(d, t, Y, T, accum, s) : launch_ti<double>(d, t, Y, T, accum, s);
}

void build_radial_split(const HostTables& h, int n_r, std::vector<uint16_t>& out, int* KP3) {
  const int NRP = h.NRP;
  const int kp3 = ((n_r + 31) / 32) * 32;
  *KP3 = kp3;
  out.assign(size_t(3) * NRP * kp3, 0);
  for (int i = 0; i < n_r; ++i)
    for (int j = 0; j < n_r; ++j) {
      double x = h.Dr[size_t(i) * n_r + j];
      for (int p = 0; p < 3; ++p) {
        const uint16_t b = to_bf16(x);
        out[(size_t(p) * NRP + i) * kp3 + j] = b;
        x -= from_bf16(b);
      }
    }
}
