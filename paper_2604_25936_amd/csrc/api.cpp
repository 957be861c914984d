// C ABI of the SAND query library: model loading and packing, depth maps,
// and the query entry points (argument checks, scratch, launch sequence).

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sand.h"
#include "sand_internal.h"
#include "sand_host.h"

using namespace sand;

// ---------------------------------------------------------------- errors --

namespace sand {

static thread_local std::string g_last_error;

sand_status fail(sand_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

sand_status device_fail(hipError_t e, const char* what) {
  return fail(SAND_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

DeviceGuard::DeviceGuard(int dev) {
  ok = hipGetDevice(&prev) == hipSuccess;
  if (ok && prev != dev) ok = hipSetDevice(dev) == hipSuccess;
}
DeviceGuard::~DeviceGuard() {
  int cur = -1;
  if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
}

}  // namespace sand

extern "C" const char* sand_status_str(sand_status s) {
  // a C caller may pass any int: read the value as one, not as the enum
  int32_t v;
  static_assert(sizeof(v) == sizeof(s), "sand_status is an int");
  std::memcpy(&v, &s, sizeof(v));
  switch (v) {
    case SAND_OK: return "ok";
    case SAND_ERR_INVALID: return "invalid argument";
    case SAND_ERR_FORMAT: return "malformed model or map";
    case SAND_ERR_NOMEM: return "out of memory";
    case SAND_ERR_DEVICE: return "device error";
    case SAND_ERR_BUDGET: return "request exceeds the memory budget";
    case SAND_ERR_UNSUPPORTED: return "unsupported";
    case SAND_ERR_TIMEOUT: return "timed out";
  }
  return "unknown status";
}

extern "C" const char* sand_last_error(void) { return g_last_error.c_str(); }

extern "C" void sand_query_opts_init(sand_query_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = SAND_FP32;
  o->mode = SAND_ADAPTIVE;
}

// ---------------------------------------------------------------- models --

namespace {

struct Blob {
  int L = 0, W = 0;
  float om[2] = {0, 0};
  uint8_t kind[kMaxLayers] = {};
  int act = ACT_SINE;
  std::vector<const float*> Wm, b;      // per layer
  std::vector<const float*> a0, a1;     // per tail (a1 null for linear)
  std::vector<float> c0, c1;            // per tail (c1 = 1 for linear)
};

uint32_t rd32(const unsigned char* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

sand_status parse_blob(const void* data, size_t nbytes, Blob& B, std::vector<float>& store) {
  const unsigned char* p = (const unsigned char*)data;
  if (nbytes < 64 || std::memcmp(p, "SANDTMLP", 8) != 0)
    return fail(SAND_ERR_FORMAT, "model blob: bad magic or shorter than the 64-byte header");
  const uint32_t version = rd32(p + 8), L = rd32(p + 12), W = rd32(p + 16), din = rd32(p + 20);
  if (version != 1) return fail(SAND_ERR_FORMAT, "model blob: version %u, expected 1", version);
  if (din != 3) return fail(SAND_ERR_FORMAT, "model blob: input dimension %u, expected 3", din);
  if (L < 1 || L > (uint32_t)kMaxLayers)
    return fail(SAND_ERR_FORMAT, "model blob: %u layers, expected 1..%d", L, kMaxLayers);
  if (W < 1) return fail(SAND_ERR_FORMAT, "model blob: width 0");
  if (W > (uint32_t)kMaxWidth)
    return fail(SAND_ERR_UNSUPPORTED, "model blob: width %u exceeds %d", W, kMaxWidth);
  for (int i = 0; i < 16; ++i) {
    const uint8_t k = p[32 + i];
    if ((uint32_t)i < L ? (k > 1) : (k != 0))
      return fail(SAND_ERR_FORMAT, "model blob: bad tail kind %u at layer %d", k, i + 1);
  }
  if (p[48] > ACT_FINER)
    return fail(SAND_ERR_FORMAT, "model blob: unknown activation %u (0 sine, 1 FINER)", p[48]);
  for (int i = 49; i < 64; ++i)
    if (p[i] != 0) return fail(SAND_ERR_FORMAT, "model blob: reserved header bytes not zero");
  size_t nf = (size_t)W * 3 + W + (size_t)(L - 1) * ((size_t)W * W + W);
  for (uint32_t i = 0; i < L; ++i) nf += (size_t)(W + 1) * (p[32 + i] ? 2 : 1);
  if (nbytes != 64 + 4 * nf)
    return fail(SAND_ERR_FORMAT, "model blob: %zu bytes, expected %zu for L=%u W=%u", nbytes,
                64 + 4 * nf, L, W);
  store.resize(nf + 2);
  std::memcpy(store.data(), p + 64, 4 * nf);   // little-endian host
  std::memcpy(&store[nf], p + 24, 8);          // the two omegas
  for (size_t i = 0; i < nf + 2; ++i)
    if (!std::isfinite(store[i])) return fail(SAND_ERR_FORMAT, "model blob: non-finite value");
  if (p[48] == ACT_FINER && (store[nf] == 0.0f || store[nf + 1] == 0.0f))
    return fail(SAND_ERR_FORMAT, "model blob: a FINER model needs nonzero omegas");
  B.L = (int)L;
  B.W = (int)W;
  B.act = p[48];
  B.om[0] = store[nf];
  B.om[1] = store[nf + 1];
  const float* q = store.data();
  B.Wm.push_back(q); q += (size_t)W * 3;
  B.b.push_back(q); q += W;
  for (uint32_t j = 1; j < L; ++j) {
    B.Wm.push_back(q); q += (size_t)W * W;
    B.b.push_back(q); q += W;
  }
  for (uint32_t i = 0; i < L; ++i) {
    B.kind[i] = p[32 + i];
    if (B.kind[i] == 0) {
      B.a0.push_back(q); q += W;
      B.c0.push_back(*q++);
      B.a1.push_back(nullptr);
      B.c1.push_back(1.0f);
    } else {
      B.a0.push_back(q); q += W;
      B.c0.push_back(*q++);
      B.a1.push_back(q); q += W;
      B.c1.push_back(*q++);
    }
  }
  return SAND_OK;
}

uint16_t to_bf16(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  const uint32_t lsb = (x >> 16) & 1u;
  return (uint16_t)((x + 0x7fffu + lsb) >> 16);   // round to nearest even (finite inputs)
}

uint16_t to_f16(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  const uint32_t sign = (x >> 16) & 0x8000u;
  const int32_t e = (int32_t)((x >> 23) & 0xff) - 127 + 15;
  uint32_t m = x & 0x7fffffu;
  if (e >= 31) return (uint16_t)(sign | 0x7c00u);
  if (e <= 0) {
    if (e < -10) return (uint16_t)sign;
    m |= 0x800000u;
    const int shift = 14 - e;
    uint32_t h = m >> shift;
    const uint32_t rem = m & ((1u << shift) - 1), half = 1u << (shift - 1);
    if (rem > half || (rem == half && (h & 1))) ++h;
    return (uint16_t)(sign | h);
  }
  uint32_t h = sign | ((uint32_t)e << 10) | (m >> 13);
  const uint32_t rem = m & 0x1fffu;
  if (rem > 0x1000u || (rem == 0x1000u && (h & 1))) ++h;
  return (uint16_t)h;
}

float from_16(uint16_t v, int prec) {
  if (prec == PREC_BF16) {
    const uint32_t x = (uint32_t)v << 16;
    float f;
    std::memcpy(&f, &x, 4);
    return f;
  }
  const uint32_t sign = (uint32_t)(v & 0x8000u) << 16;
  const int e = (v >> 10) & 0x1f;
  const uint32_t m = v & 0x3ffu;
  float f;
  if (e == 0) {
    f = std::ldexp((float)m, -24);
  } else {
    const uint32_t x = ((uint32_t)(e - 15 + 127) << 23) | (m << 13);
    std::memcpy(&f, &x, 4);
  }
  return sign ? -f : f;
}

// Host-side geometry of the packed layout (mirrors the kernel's Tr/Cfg).
struct Geo {
  int BM, L1S, VB, KPS, TAILB;
  int RB, KS, CH, L1C;
  Geo(int prec, int WP) {
    if (prec == PREC_FP32) {
      BM = 16; L1S = 1; VB = 4; KPS = 4; TAILB = BM * 8;
    } else {
      BM = 32; L1S = 2; VB = 16; KPS = 16; TAILB = 2 * 64 * 4;
    }
    RB = WP / BM;
    KS = WP / KPS;
    CH = (KS + 1) * 64 * VB + TAILB;
    L1C = L1S * (prec == PREC_FP32 ? 256 : 64 * 16) + TAILB;
  }
};

// Pack one precision's chunks (layout in sand_internal.h).
std::vector<char> pack(const Blob& B, int prec, int WP) {
  const Geo G(prec, WP);
  const int W = B.W;
  const size_t total = (size_t)G.RB * G.L1C + (size_t)(B.L - 1) * G.RB * G.CH;
  std::vector<char> buf(total, 0);
  const double s1 = (double)B.om[0] / kTwoPi, sh = (double)B.om[1] / kTwoPi;
  auto tail_w = [&](int f, int layer, int u) {
    const float* a = f == 0 ? B.a0[layer] : B.a1[layer];
    return (u < W && a) ? a[u] : 0.0f;
  };
  auto tails = [&](float* dst, int layer, int rb) {
    if (prec == PREC_FP32) {
      // a0[BM], a1[BM] in unit order
      for (int i = 0; i < G.BM; ++i)
        for (int f = 0; f < 2; ++f) dst[f * G.BM + i] = tail_w(f, layer, G.BM * rb + i);
    } else {
      // lane-indexed: lane l holds the unit of its register e = l & 15 in
      // row group l >> 5 (accumulator row 8 (e / 4) + 4 (l / 32) + e % 4)
      for (int l = 0; l < 64; ++l) {
        const int e = l & 15, row = 8 * (e >> 2) + 4 * (l >> 5) + (e & 3);
        for (int f = 0; f < 2; ++f) dst[f * 64 + l] = tail_w(f, layer, G.BM * rb + row);
      }
    }
  };
  // layer 1
  // v = h + m + l, each part a BF16 (the kernels' 16-bit paths evaluate
  // layer 1 on BF16 MFMAs over three-way splits of weights and coordinates)
  auto split3 = [](double v, uint16_t (&p)[3]) {
    for (int i = 0; i < 3; ++i) {
      p[i] = to_bf16((float)v);
      v -= (double)from_16(p[i], PREC_BF16);
    }
  };
  for (int rb = 0; rb < G.RB; ++rb) {
    char* ch = buf.data() + (size_t)rb * G.L1C;
    for (int st = 0; st < G.L1S; ++st)
      for (int l = 0; l < 64; ++l) {
        if (prec == PREC_FP32) {
          // K = (x, y, z, 1) across the four 16-lane groups
          const int m = l & 15, k = l >> 4, u = G.BM * rb + m;
          double v = 0.0;
          if (u < W) v = s1 * (k < 3 ? (double)B.Wm[0][u * 3 + k] : (double)B.b[0][u]);
          ((float*)ch)[st * 64 + l] = (float)v;
        } else {
          // lane half hh of step st holds coordinate c = 2 st + hh: the
          // weight parts of the products (wh, wh, wm, wh, wm, wl) whose
          // coordinate parts are (ch, cm, ch, cl, cm, ch), then bias parts
          // against constant 1s: bh, bm (step 0, half 0), bl (step 0, half 1)
          const int m = l & 31, hh = l >> 5, u = G.BM * rb + m, c = 2 * st + hh;
          uint16_t* A = (uint16_t*)(ch + ((size_t)st * 64 + l) * 16);
          for (int p = 0; p < 8; ++p) A[p] = 0;
          if (u >= W) continue;
          uint16_t w[3];
          if (c < 3) {
            split3(s1 * (double)B.Wm[0][u * 3 + c], w);
            const int part[6] = {0, 0, 1, 0, 1, 2};
            for (int i = 0; i < 6; ++i) A[i] = w[part[i]];
          }
          if (st == 0) {
            split3(s1 * (double)B.b[0][u], w);
            if (hh == 0) {
              A[6] = w[0];
              A[7] = w[1];
            } else {
              A[6] = w[2];
            }
          }
        }
      }
    tails((float*)(ch + (size_t)G.L1C - G.TAILB), 0, rb);
  }
  // hidden layers
  for (int j = 1; j < B.L; ++j) {
    const float* Wj = B.Wm[j];
    const float* bj = B.b[j];
    for (int rb = 0; rb < G.RB; ++rb) {
      char* ch = buf.data() + (size_t)G.RB * G.L1C + ((size_t)(j - 1) * G.RB + rb) * G.CH;
      for (int s = 0; s <= G.KS; ++s)
        for (int l = 0; l < 64; ++l) {
          if (prec == PREC_FP32) {
            const int m = l & 15, g = l >> 4, uo = 16 * rb + m;
            double v = 0.0;
            if (s < G.KS) {
              const int ui = 16 * (s >> 2) + 4 * g + (s & 3);
              if (uo < W && ui < W) v = sh * (double)Wj[(size_t)uo * W + ui];
            } else if (g == 0 && uo < W) {
              v = sh * (double)bj[uo];
            }
            ((float*)ch)[s * 64 + l] = (float)v;
          } else {
            const int m = l & 31, h = l >> 5, uo = 32 * rb + m;
            uint16_t* A = (uint16_t*)(ch + ((size_t)s * 64 + l) * 16);
            auto r16 = [&](double v) { return prec == PREC_BF16 ? to_bf16((float)v) : to_f16((float)v); };
            for (int p = 0; p < 8; ++p) {
              double v = 0.0;
              if (s < G.KS) {
                const int ui = 16 * s + 8 * (p >> 2) + 4 * h + (p & 3);
                if (uo < W && ui < W) v = sh * (double)Wj[(size_t)uo * W + ui];
                A[p] = r16(v);
              } else {
                A[p] = 0;
              }
            }
            if (s == G.KS && h == 0 && uo < W) {
              const double bv = sh * (double)bj[uo];
              const uint16_t hi = r16(bv);
              A[0] = hi;
              A[1] = r16(bv - (double)from_16(hi, prec));
            }
          }
        }
      tails((float*)(ch + (size_t)(G.KS + 1) * 64 * G.VB), j, rb);
    }
  }
  return buf;
}

// Adjoint data of one precision: transposed chunks of layers 2..L (rows =
// units of layer j-1, K = units of layer j in the permuted order, values
// omega_j W_j[k][row]) followed by the tails of layer j-1 (layout in
// sand_internal.h, without the bias step).
std::vector<char> pack_bwd(const Blob& B, int prec, int WP) {
  const Geo G(prec, WP);
  const int W = B.W;
  const size_t chb = (size_t)G.KS * 64 * G.VB + G.BM * 8;
  std::vector<char> buf((size_t)(B.L - 1) * G.RB * chb, 0);
  const double om = B.om[1];
  for (int jl = 2; jl <= B.L; ++jl) {
    const float* Wj = B.Wm[jl - 1];
    for (int rb = 0; rb < G.RB; ++rb) {
      char* ch = buf.data() + ((size_t)(jl - 2) * G.RB + rb) * chb;
      for (int s = 0; s < G.KS; ++s)
        for (int l = 0; l < 64; ++l) {
          if (prec == PREC_FP32) {
            const int m = l & 15, g = l >> 4;
            const int ui = 16 * rb + m, uo = 16 * (s >> 2) + 4 * g + (s & 3);
            const double v = (ui < W && uo < W) ? om * (double)Wj[(size_t)uo * W + ui] : 0.0;
            ((float*)ch)[s * 64 + l] = (float)v;
          } else {
            const int m = l & 31, h = l >> 5, ui = 32 * rb + m;
            uint16_t* A = (uint16_t*)(ch + ((size_t)s * 64 + l) * 16);
            for (int p = 0; p < 8; ++p) {
              const int uo = 16 * s + 8 * (p >> 2) + 4 * h + (p & 3);
              const double v = (ui < W && uo < W) ? om * (double)Wj[(size_t)uo * W + ui] : 0.0;
              A[p] = prec == PREC_BF16 ? to_bf16((float)v) : to_f16((float)v);
            }
          }
        }
      float* t = (float*)(ch + (size_t)G.KS * 64 * G.VB);
      for (int i = 0; i < G.BM; ++i) {
        const int u = G.BM * rb + i;
        t[i] = u < W ? B.a0[jl - 2][u] : 0.0f;
        t[G.BM + i] = (u < W && B.a1[jl - 2]) ? B.a1[jl - 2][u] : 0.0f;
      }
    }
  }
  return buf;
}

// omega_1 W_1 rows ([WP][4], last entry 0) and the tail table [L][2][WP].
std::vector<char> pack_grad_tables(const Blob& B, int WP) {
  std::vector<char> buf((size_t)WP * 16 + (size_t)B.L * 2 * WP * 4, 0);
  float* w1 = (float*)buf.data();
  for (int u = 0; u < B.W; ++u)
    for (int k = 0; k < 3; ++k) w1[u * 4 + k] = (float)((double)B.om[0] * B.Wm[0][u * 3 + k]);
  float* t = (float*)(buf.data() + (size_t)WP * 16);
  for (int l = 0; l < B.L; ++l)
    for (int u = 0; u < B.W; ++u) {
      t[(size_t)l * 2 * WP + u] = B.a0[l][u];
      t[(size_t)l * 2 * WP + WP + u] = B.a1[l] ? B.a1[l][u] : 0.0f;
    }
  return buf;
}

}  // namespace

extern "C" sand_status sand_load_model(const void* blob, size_t nbytes, int device,
                                       sand_model* out) {
  if (!blob || !out) return fail(SAND_ERR_INVALID, "sand_load_model: null blob or out");
  *out = nullptr;
  Blob B;
  std::vector<float> store;
  sand_status st = parse_blob(blob, nbytes, B, store);
  if (st != SAND_OK) return st;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(SAND_ERR_INVALID, "sand_load_model: device %d not available (%d devices)", device,
                ndev);
  const int WP = padded_width(B.W);
  // forward packs (3 precisions), adjoint packs (3), then the FP32 tables
  std::vector<char> packs[7];
  size_t offs[7], total = 0;
  for (int p = 0; p < 3; ++p) {
    packs[p] = pack(B, p, WP);
    packs[3 + p] = pack_bwd(B, p, WP);
  }
  packs[6] = pack_grad_tables(B, WP);
  for (int p = 0; p < 7; ++p) {
    offs[p] = total;
    total += (packs[p].size() + 255) & ~(size_t)255;
  }
  const size_t args_off = total;
  total += 3 * ((sizeof(ModelArgs) + 255) & ~(size_t)255);
  DeviceGuard guard(device);
  if (!guard.ok) return fail(SAND_ERR_DEVICE, "sand_load_model: cannot select device %d", device);
  int num_cu = 0;
  hipError_t e = hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return device_fail(e, "sand_load_model: device query");
  char* dev = nullptr;
  e = hipMalloc((void**)&dev, total);
  if (e != hipSuccess) return fail(SAND_ERR_NOMEM, "sand_load_model: %zu device bytes", total);
  for (int p = 0; p < 7; ++p) {
    if (packs[p].empty()) continue;
    e = hipMemcpy(dev + offs[p], packs[p].data(), packs[p].size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(dev);
      return device_fail(e, "sand_load_model: upload");
    }
  }
  sand_model m = new sand_model_s();
  m->device = device;
  m->L = B.L;
  m->W = B.W;
  m->WP = WP;
  m->act = B.act;
  m->num_cu = num_cu;
  m->dev = dev;
  m->bytes = total;
  for (int p = 0; p < 3; ++p) m->bwd[p] = dev + offs[3 + p];
  m->w1t = (const float*)(dev + offs[6]);
  m->tails = (const float*)(dev + offs[6] + (size_t)WP * 16);
  for (int p = 0; p < 3; ++p) {
    ModelArgs& a = m->args[p];
    std::memset(&a, 0, sizeof(a));
    a.chunks = dev + offs[p];
    a.L = B.L;
    a.WP = WP;
    a.chunk_bytes = Geo(p, WP).CH;
    a.act = B.act;
    a.kf[0] = (float)(kTwoPi / std::fabs((double)B.om[0]));
    a.kf[1] = (float)(kTwoPi / std::fabs((double)B.om[1]));
    for (int i = 0; i < B.L; ++i) {
      a.c0[i] = B.c0[i];
      a.c1[i] = B.c1[i];
      if (B.kind[i] == 0) a.lin_mask |= 1u << i;
    }
  }
  for (int p = 0; p < 3; ++p) {
    char* dst = dev + args_off + p * ((sizeof(ModelArgs) + 255) & ~(size_t)255);
    e = hipMemcpy(dst, &m->args[p], sizeof(ModelArgs), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(dev);
      delete m;
      return device_fail(e, "sand_load_model: upload");
    }
    m->args_dev[p] = (const ModelArgs*)dst;
  }
  *out = m;
  return SAND_OK;
}

extern "C" void sand_free_model(sand_model m) {
  if (!m) return;
  DeviceGuard guard(m->device);
  (void)hipFree(m->dev);
  delete m;
}

extern "C" sand_status sand_model_info(sand_model m, int32_t* L, int32_t* W) {
  if (!m) return fail(SAND_ERR_INVALID, "sand_model_info: null model");
  if (L) *L = m->L;
  if (W) *W = m->W;
  return SAND_OK;
}

// ------------------------------------------------------------ depth maps --

extern "C" sand_status sand_build_depthmap(sand_model m, const uint8_t* depth_host, int32_t R,
                                           const float* far_host, sand_depthmap* out) {
  if (!m || !depth_host || !out)
    return fail(SAND_ERR_INVALID, "sand_build_depthmap: null model, map or out");
  *out = nullptr;
  if (R < 2 || R > 1024 || (R & (R - 1)) != 0)
    return fail(SAND_ERR_INVALID, "sand_build_depthmap: R=%d is not a power of two in 2..1024", R);
  const size_t cells = (size_t)R * R * R;
  bool has_zero = false;
  for (size_t i = 0; i < cells; ++i) {
    if (depth_host[i] > m->L)
      return fail(SAND_ERR_FORMAT, "sand_build_depthmap: depth %u at cell %zu exceeds L=%d",
                  depth_host[i], i, m->L);
    has_zero |= depth_host[i] == 0;
  }
  if (has_zero && !far_host)
    return fail(SAND_ERR_FORMAT, "sand_build_depthmap: depth-0 cells need far-field values");
  DeviceGuard guard(m->device);
  if (!guard.ok) return fail(SAND_ERR_DEVICE, "sand_build_depthmap: cannot select device");
  uint8_t* d = nullptr;
  float* f = nullptr;
  hipError_t e = hipMalloc((void**)&d, cells);
  if (e != hipSuccess) return fail(SAND_ERR_NOMEM, "sand_build_depthmap: %zu bytes", cells);
  e = hipMemcpy(d, depth_host, cells, hipMemcpyHostToDevice);
  if (e == hipSuccess && far_host) {
    e = hipMalloc((void**)&f, cells * 4);
    if (e == hipSuccess) e = hipMemcpy(f, far_host, cells * 4, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    (void)hipFree(d);
    if (f) (void)hipFree(f);
    return device_fail(e, "sand_build_depthmap: upload");
  }
  sand_depthmap dm = new sand_depthmap_s();
  dm->model = m;
  dm->device = m->device;
  dm->R = R;
  dm->depth = d;
  dm->far = f;
  *out = dm;
  return SAND_OK;
}

extern "C" void sand_free_depthmap(sand_depthmap dm) {
  if (!dm) return;
  DeviceGuard guard(dm->device);
  if (dm->depth) (void)hipFree(dm->depth);
  if (dm->far) (void)hipFree(dm->far);
  if (dm->oct) (void)hipFree(dm->oct);
  for (void* p : dm->owned) (void)hipFree(p);
  delete dm;
}

// ---------------------------------------------------- map construction --

namespace {

// Device buffers of one construction, freed together.
struct DevBufs {
  std::vector<void*> p;
  template <class T>
  hipError_t get(T** out, size_t bytes) {
    *out = nullptr;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes > 0 ? bytes : 1);
    if (e == hipSuccess) {
      p.push_back(q);
      *out = (T*)q;
    }
    return e;
  }
  void release() {
    for (void* q : p) (void)hipFree(q);
    p.clear();
  }
  ~DevBufs() { release(); }
};

constexpr int64_t kMapChunk = 1 << 24;   // samples per full-depth pass

}  // namespace

extern "C" sand_status sand_construct_depthmap(sand_model m, const uint8_t* near_host,
                                               const float* center_sdf_host, int32_t R,
                                               int32_t sps, float r, int32_t precision,
                                               void* stream, sand_depthmap* out,
                                               uint8_t* depth_host, sand_map_info* info) {
  const char* who = "sand_construct_depthmap";
  if (!m || !near_host || !center_sdf_host || !out)
    return fail(SAND_ERR_INVALID, "%s: null model, mask, centre values or out", who);
  *out = nullptr;
  if (R < 2 || R > 1024 || (R & (R - 1)) != 0)
    return fail(SAND_ERR_INVALID, "%s: R=%d is not a power of two in 2..1024", who, R);
  if (sps != 1 && sps != 2 && sps != 4 && sps != 8)
    return fail(SAND_ERR_INVALID, "%s: s=%d is not 1, 2, 4 or 8", who, sps);
  if (!(r > 0.0f) || !std::isfinite(r))
    return fail(SAND_ERR_INVALID, "%s: threshold r must be finite and > 0", who);
  if (precision < 0 || precision > 2)
    return fail(SAND_ERR_INVALID, "%s: precision %d", who, precision);
  const int64_t cells = (int64_t)R * R * R;
  int64_t nnear = 0;
  for (int64_t v = 0; v < cells; ++v) nnear += near_host[v] != 0;
  const int64_t s3 = (int64_t)sps * sps * sps, nsamp = nnear * s3;
  if (nnear > 2147483647LL)
    return fail(SAND_ERR_INVALID, "%s: %lld near voxels", who, (long long)nnear);
  DeviceGuard guard(m->device);
  if (!guard.ok) return fail(SAND_ERR_DEVICE, "%s: cannot select device", who);
  hipStream_t st = (hipStream_t)stream;
  const int64_t chunk = nsamp < kMapChunk ? nsamp : kMapChunk;
  const int L = m->L;
  DevBufs tmp;
  uint8_t *near_d = nullptr, *depth_d = nullptr;
  float *csdf_d = nullptr, *far_d = nullptr, *xyz = nullptr, *yall = nullptr, *ylast = nullptr;
  int32_t* list = nullptr;
  uint32_t *count = nullptr, *depth32 = nullptr;
  hipError_t e = tmp.get(&near_d, cells);
  if (e == hipSuccess) e = tmp.get(&csdf_d, cells * 4);
  if (e == hipSuccess) e = tmp.get(&list, nnear * 4);
  if (e == hipSuccess) e = tmp.get(&count, 4);
  if (e == hipSuccess) e = tmp.get(&depth32, cells * 4);
  if (e == hipSuccess) e = tmp.get(&xyz, chunk * 12);
  if (e == hipSuccess) e = tmp.get(&yall, chunk * L * 4);
  if (e == hipSuccess) e = tmp.get(&ylast, chunk * 4);
  if (e != hipSuccess) return fail(SAND_ERR_NOMEM, "%s: scratch for %lld samples", who,
                                   (long long)nsamp);
  // the map's own arrays, handed to the map object on success
  e = hipMalloc((void**)&depth_d, cells);
  if (e == hipSuccess) e = hipMalloc((void**)&far_d, cells * 4);
  auto drop_map = [&]() {
    if (depth_d) (void)hipFree(depth_d);
    if (far_d) (void)hipFree(far_d);
  };
  if (e != hipSuccess) {
    drop_map();
    return fail(SAND_ERR_NOMEM, "%s: map of R=%d", who, R);
  }
  e = hipMemcpyAsync(near_d, near_host, cells, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(csdf_d, center_sdf_host, cells * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(count, 0, 4, st);
  if (e == hipSuccess) e = hipMemsetAsync(depth32, 0, cells * 4, st);
  if (e == hipSuccess) e = launch_map_list(near_d, cells, list, count, st);
  QueryArgs qa{};
  qa.m = m->args[precision];
  qa.xyz = xyz;
  qa.sdf = ylast;           // y_L again (also the last column of y_all)
  qa.full_depth = L;
  qa.y_all = yall;
  for (int64_t first = 0; e == hipSuccess && first < nsamp; first += chunk) {
    const int64_t k = nsamp - first < chunk ? nsamp - first : chunk;
    e = launch_map_samples(list, first, k, R, sps, xyz, st);
    qa.n = k;
    if (e == hipSuccess) e = launch_tmlp(precision, qa, m->num_cu, st);
    if (e == hipSuccess) e = launch_map_pool(yall, L, list, first, k, sps, r, depth32, st);
  }
  if (e == hipSuccess) e = launch_map_finish(near_d, csdf_d, depth32, cells, depth_d, far_d, st);
  if (e == hipSuccess && depth_host)
    e = hipMemcpyAsync(depth_host, depth_d, cells, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(st);
    drop_map();
    return device_fail(e, "sand_construct_depthmap");
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->near_voxels = nnear;
    info->samples = nsamp;
    std::vector<uint8_t> h;
    const uint8_t* dh = depth_host;
    if (!dh) {
      h.resize(cells);
      e = hipMemcpy(h.data(), depth_d, cells, hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        drop_map();
        return device_fail(e, "sand_construct_depthmap: read back");
      }
      dh = h.data();
    }
    for (int64_t v = 0; v < cells; ++v) info->depth_counts[dh[v] <= 16 ? dh[v] : 16]++;
  }
  sand_depthmap dm = new sand_depthmap_s();
  dm->model = m;
  dm->device = m->device;
  dm->R = R;
  dm->depth = depth_d;
  dm->far = far_d;
  *out = dm;
  return SAND_OK;
}

// ---------------------------------------------------------------- octree --

namespace {

// Device arrays owned by an octree under construction; handed to the map
// object on success, freed otherwise.
struct Owned {
  std::vector<void*> p;
  size_t bytes = 0;
  template <class T>
  hipError_t get(T** out, size_t n_bytes, hipStream_t s, bool zero = false) {
    *out = nullptr;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, n_bytes > 0 ? n_bytes : 1);
    if (e != hipSuccess) return e;
    p.push_back(q);
    bytes += n_bytes;
    if (zero) e = hipMemsetAsync(q, 0, n_bytes > 0 ? n_bytes : 1, s);
    *out = (T*)q;
    return e;
  }
  void release() {
    for (void* q : p) (void)hipFree(q);
    p.clear();
  }
};

}  // namespace

extern "C" sand_status sand_construct_octree(sand_model m, int32_t D, int32_t sps, float r,
                                             int32_t precision, void* stream, sand_depthmap* out,
                                             sand_octree_info* info) {
  const char* who = "sand_construct_octree";
  if (!m || !out) return fail(SAND_ERR_INVALID, "%s: null model or out", who);
  *out = nullptr;
  if (D < 1 || D > kMaxOctDepth)
    return fail(SAND_ERR_INVALID, "%s: D=%d is not in 1..%d", who, D, kMaxOctDepth);
  if (sps != 1 && sps != 2 && sps != 4 && sps != 8)
    return fail(SAND_ERR_INVALID, "%s: s=%d is not 1, 2, 4 or 8", who, sps);
  if (!(r > 0.0f) || !std::isfinite(r))
    return fail(SAND_ERR_INVALID, "%s: threshold r must be finite and > 0", who);
  if (precision < 0 || precision > 2) return fail(SAND_ERR_INVALID, "%s: precision %d", who, precision);
  DeviceGuard guard(m->device);
  if (!guard.ok) return fail(SAND_ERR_DEVICE, "%s: cannot select device", who);
  hipStream_t st = (hipStream_t)stream;
  const int L = m->L;
  const int64_t chunk_max = kMapChunk;
  Owned own;       // the octree's arrays
  DevBufs tmp;     // scratch of the build
  OctreeArgs oa{};
  oa.D = D;
  sand_octree_info inf{};
  inf.D = D;
  auto bail = [&](hipError_t e) {
    (void)hipStreamSynchronize(st);
    own.release();
    return device_fail(e, who);
  };

  // scratch for the full-depth passes: points, final values, all outputs
  float *xyz = nullptr, *ylast = nullptr, *yall = nullptr;
  hipError_t e = tmp.get(&xyz, chunk_max * 12);
  if (e == hipSuccess) e = tmp.get(&ylast, chunk_max * 4);
  if (e == hipSuccess) e = tmp.get(&yall, chunk_max * L * 4);
  int64_t* total_d = nullptr;
  uint32_t* near_count_d = nullptr;
  if (e == hipSuccess) e = tmp.get(&total_d, 8);
  if (e == hipSuccess) e = tmp.get(&near_count_d, 4);
  if (e != hipSuccess) return fail(SAND_ERR_NOMEM, "%s: build scratch", who);

  QueryArgs qa{};
  qa.m = m->args[precision];
  qa.full_depth = L;
  auto y_at = [&](const float* pts, float* yout, int64_t n) {
    qa.xyz = pts;
    qa.sdf = yout;
    qa.n = n;
    return launch_tmlp(precision, qa, m->num_cu, st);
  };

  // level 0: the root
  const float root_c[3] = {0.0f, 0.0f, 0.0f};
  float y0 = 0.0f;
  e = hipMemcpyAsync(xyz, root_c, 12, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = y_at(xyz, ylast, 1);
  if (e == hipSuccess) e = hipMemcpyAsync(&y0, ylast, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return bail(e);
  const float h0 = (float)std::sqrt(3.0);
  uint64_t* parents = nullptr;   // internal codes of the previous level, Morton order
  int64_t np = 0;
  if (std::fabs(y0) <= h0) {
    uint64_t one = 1ull, zero64 = 0ull;
    uint32_t rank0 = 0;
    uint64_t* b0 = nullptr;
    uint32_t* r0 = nullptr;
    e = own.get(&b0, 8, st);
    if (e == hipSuccess) e = own.get(&r0, 4, st);
    if (e == hipSuccess) e = tmp.get(&parents, 8);
    if (e == hipSuccess) e = hipMemcpyAsync(b0, &one, 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(r0, &rank0, 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(parents, &zero64, 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // host sources are on the stack
    if (e != hipSuccess) return bail(e);
    oa.bits[0] = b0;
    oa.rank[0] = r0;
    np = 1;
    inf.internal_nodes[0] = 1;
  } else {
    oa.root_leaf = 1;
    oa.root_value = y0;
    inf.leaves[0] = 1;
  }

  int32_t* near_slots = nullptr;
  int64_t nnear = 0, nslots_D = 0;
  uint64_t* parents_D = nullptr;
  uint8_t* depth_D = nullptr;
  for (int l = 1; l <= D && np > 0; ++l) {
    const int64_t nslots = 8 * np;
    uint8_t* dep = nullptr;
    float* val = nullptr;
    uint64_t* bits = nullptr;
    uint32_t* rank = nullptr;
    const int64_t words = l < D ? (((int64_t)1 << (3 * l)) + 63) / 64 : 0;
    e = own.get(&dep, nslots, st);
    if (e == hipSuccess) e = own.get(&val, nslots * 4, st);
    if (e == hipSuccess && l < D) e = own.get(&bits, words * 8, st, true);
    if (e == hipSuccess && l < D) e = own.get(&rank, words * 4, st);
    if (e == hipSuccess && l == D) e = tmp.get(&near_slots, nslots * 4);
    if (e == hipSuccess) e = hipMemsetAsync(near_count_d, 0, 4, st);
    if (e != hipSuccess) return bail(e);
    oa.depth[l] = dep;
    oa.value[l] = val;
    const float h = (float)(std::sqrt(3.0) * std::ldexp(1.0, -l));
    for (int64_t first = 0; e == hipSuccess && first < nslots; first += chunk_max) {
      const int64_t k = nslots - first < chunk_max ? nslots - first : chunk_max;
      e = launch_oct_centres(parents, first, k, l, xyz, st);
      if (e == hipSuccess) e = y_at(xyz, ylast, k);
      if (e == hipSuccess)
        e = launch_oct_classify(parents, ylast, first, k, l, D, h, bits, dep, val, near_slots,
                                near_count_d, st);
    }
    if (e != hipSuccess) return bail(e);
    if (l < D) {
      int64_t total = 0;
      e = launch_oct_rank(bits, words, rank, total_d, st);
      if (e == hipSuccess) e = hipMemcpyAsync(&total, total_d, 8, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return bail(e);
      oa.bits[l] = bits;
      oa.rank[l] = rank;
      inf.internal_nodes[l] = total;
      inf.leaves[l] = nslots - total;
      uint64_t* next = nullptr;
      if (total > 0) {
        e = tmp.get(&next, total * 8);
        if (e == hipSuccess) e = launch_oct_list(bits, rank, words, next, st);
        if (e != hipSuccess) return bail(e);
      }
      parents = next;
      np = total;
    } else {
      uint32_t nn = 0;
      e = hipMemcpyAsync(&nn, near_count_d, 4, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return bail(e);
      nnear = nn;
      nslots_D = nslots;
      parents_D = parents;
      depth_D = dep;
      inf.leaves[l] = nslots;
    }
  }

  // near leaves at level D: Eq. 5 over s^3 sub-cell samples, max-pooled (Eq. 6)
  const int64_t s3 = (int64_t)sps * sps * sps, nsamp = nnear * s3;
  if (nnear > 0) {
    uint32_t* depth32 = nullptr;
    e = tmp.get(&depth32, nslots_D * 4);
    if (e == hipSuccess) e = hipMemsetAsync(depth32, 0, nslots_D * 4, st);
    qa.y_all = yall;
    for (int64_t first = 0; e == hipSuccess && first < nsamp; first += chunk_max) {
      const int64_t k = nsamp - first < chunk_max ? nsamp - first : chunk_max;
      e = launch_oct_samples(near_slots, parents_D, first, k, D, sps, xyz, st);
      if (e == hipSuccess) e = y_at(xyz, ylast, k);
      if (e == hipSuccess) e = launch_map_pool(yall, L, near_slots, first, k, sps, r, depth32, st);
    }
    qa.y_all = nullptr;
    if (e == hipSuccess) e = launch_oct_finish(near_slots, nnear, depth32, depth_D, st);
    if (e != hipSuccess) return bail(e);
  }
  inf.near_leaves = nnear;
  inf.samples = nsamp;

  // dense index of level K = min(D - 1, 6): most points end in a leaf at or
  // above it and need one load
  if (!oa.root_leaf && D >= 2) {
    const int K = D - 1 < 6 ? D - 1 : 6;
    uint2* top = nullptr;
    e = own.get(&top, ((size_t)1 << (3 * K)) * sizeof(uint2), st);
    if (e == hipSuccess) e = launch_oct_top(oa, K, top, st);
    if (e != hipSuccess) return bail(e);
    oa.top = top;
    oa.top_level = K;
  }

  // the descriptor
  OctreeArgs* oa_d = nullptr;
  e = hipMalloc((void**)&oa_d, sizeof(OctreeArgs));
  if (e == hipSuccess) e = hipMemcpyAsync(oa_d, &oa, sizeof(OctreeArgs), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    if (oa_d) (void)hipFree(oa_d);
    return bail(e);
  }
  inf.bytes = own.bytes + sizeof(OctreeArgs);
  if (info) {
    // leaves per stored depth: far leaves at every level, near leaves by depth
    inf.depth_counts[0] = 0;
    for (int l = 0; l <= D; ++l) inf.depth_counts[0] += (int32_t)inf.leaves[l];
    inf.depth_counts[0] -= (int32_t)nnear;
    if (nnear > 0) {
      std::vector<uint8_t> dh((size_t)nslots_D);
      e = hipMemcpy(dh.data(), depth_D, (size_t)nslots_D, hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        (void)hipFree(oa_d);
        return bail(e);
      }
      for (uint8_t v : dh)
        if (v >= 1 && v <= 16) inf.depth_counts[v]++;
    }
    *info = inf;
  }
  sand_depthmap dm = new sand_depthmap_s();
  dm->model = m;
  dm->device = m->device;
  dm->R = 1 << D;
  dm->oct = oa_d;
  dm->owned = own.p;
  own.p.clear();
  *out = dm;
  return SAND_OK;
}

// --------------------------------------------------------------- queries --

namespace sand {

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

WorkspaceLayout workspace_layout(int64_t n) {
  WorkspaceLayout w{};
  if (n <= 0) return w;
  const size_t nblk = (size_t)((n + kLookupChunk - 1) / kLookupChunk);
  w.depth = 0;
  w.perm = al((size_t)n);
  w.counts = w.perm + al(4 * (size_t)n);
  w.plan = w.counts + al(nblk * kBuckets * 4);
  w.groups = w.plan + al(sizeof(Plan));
  w.qcount = w.groups + al((nblk + kScanGroup - 1) / kScanGroup * kBuckets * 4);
  w.total = w.qcount + al(nblk * 4);
  w.nblk = (int64_t)nblk;
  return w;
}

sand_status check_query(const char* who, sand_model m, sand_depthmap dm, const float* xyz,
                        int64_t n, const void* out, const sand_query_opts& o) {
  if (!m) return fail(SAND_ERR_INVALID, "%s: null model", who);
  if (n < 0 || n > 2147483647LL) return fail(SAND_ERR_INVALID, "%s: n=%lld out of range", who,
                                             (long long)n);
  if (n > 0 && (!xyz || !out)) return fail(SAND_ERR_INVALID, "%s: null point or output buffer", who);
  if (((uintptr_t)xyz & 3u) != 0) return fail(SAND_ERR_INVALID, "%s: points not 4-byte aligned", who);
  if (o.precision < 0 || o.precision > 2)
    return fail(SAND_ERR_INVALID, "%s: precision %d", who, o.precision);
  if (o.mode < 0 || o.mode > 3) return fail(SAND_ERR_INVALID, "%s: mode %d", who, o.mode);
  if (o.max_depth < 0) return fail(SAND_ERR_INVALID, "%s: max_depth %d", who, o.max_depth);
  if (o.mode == SAND_DYNAMIC) {
    if (!(o.dynamic_r > 0.0f) || !std::isfinite(o.dynamic_r))
      return fail(SAND_ERR_INVALID, "%s: dynamic mode needs a finite dynamic_r > 0", who);
    if (o.dynamic_checkpoint < -1 || o.dynamic_checkpoint == 1)
      return fail(SAND_ERR_INVALID, "%s: dynamic_checkpoint %d (need -1, 0 or >= 2)", who,
                  o.dynamic_checkpoint);
  } else if (o.dynamic_r != 0.0f || o.dynamic_checkpoint != 0) {
    return fail(SAND_ERR_INVALID, "%s: dynamic_r and dynamic_checkpoint are only for dynamic mode",
                who);
  }
  if (dm && dm->model != m) return fail(SAND_ERR_INVALID, "%s: map belongs to another model", who);
  if (o.mode == SAND_ADAPTIVE && !dm) return fail(SAND_ERR_INVALID, "%s: adaptive mode needs a map", who);
  if (o.mode == SAND_FORCED && n > 0 && !o.forced_depth)
    return fail(SAND_ERR_INVALID, "%s: forced mode needs forced_depth", who);
  if (o.workspace && o.workspace_bytes < workspace_layout(n).total)
    return fail(SAND_ERR_INVALID, "%s: workspace of %zu bytes, need %zu", who, o.workspace_bytes,
                workspace_layout(n).total);
  return SAND_OK;
}

size_t grad_stash_bytes(sand_model m, int prec) {
  return (size_t)m->num_cu * adjoint_stash_bytes_per_wg(prec, m->WP, m->L);
}

sand_status run_bucketing(sand_model m, sand_depthmap dm, const float* xyz, int64_t n, float* sdf,
                          float* grad, const sand_query_opts& o, char* ws, hipStream_t s,
                          int tile_q, hipEvent_t* ev, const int32_t** perm_out,
                          const Plan** plan_out) {
  auto mark = [&](int i) {
    if (ev && ev[i]) (void)hipEventRecord(ev[i], s);
  };
  const WorkspaceLayout w = workspace_layout(n);
  uint8_t* depth = o.depth_out ? o.depth_out : (uint8_t*)(ws + w.depth);
  int32_t* perm = (int32_t*)(ws + w.perm);
  int32_t* counts = (int32_t*)(ws + w.counts);
  Plan* plan = (Plan*)(ws + w.plan);
  const uint8_t* map = dm ? dm->depth : nullptr;
  const float* far = dm ? dm->far : nullptr;
  const OctreeArgs* oct = dm ? dm->oct : nullptr;
  const int R = dm ? dm->R : 2;
  hipError_t e;
  mark(0);
  // the octree's deferred points queue in the permutation buffer, which the
  // scatter fills only after they are resolved
  if ((e = launch_lookup_count(xyz, n, map, R, far, oct, o.forced_depth, o.mode, m->L, o.max_depth, depth,
                               sdf, grad, counts, perm, (int32_t*)(ws + w.qcount), s)) !=
      hipSuccess)
    return device_fail(e, "lookup launch");
  mark(1);
  if ((e = launch_scan(counts, w.nblk, m->L, tile_q, plan, (int32_t*)(ws + w.groups), s)) !=
      hipSuccess)
    return device_fail(e, "scan launch");
  mark(2);
  if ((e = launch_scatter(depth, n, counts, perm, s)) != hipSuccess)
    return device_fail(e, "scatter launch");
  mark(3);
  *perm_out = perm;
  *plan_out = plan;
  return SAND_OK;
}

// Lookup + bucketing + T-MLP for n points. `ws` must hold workspace_layout(n).
namespace {

constexpr int64_t kDynSampleMin = int64_t(1) << 22;   // queries that pick their own checkpoint
constexpr int64_t kDynSample = 65536;                 // points in the sample
constexpr size_t kDynArenaBytes = size_t(1) << 31;    // compaction arena limit

// Checkpoint layer for compacted dynamic exit, from the exit depths of a
// strided sample of the query: with s_c the fraction of points still
// running after layer c, compaction at c costs about (c - 1) + s_c (a + d -
// c) hidden-layer evaluations per point against d - 1 without (a tile runs
// as deep as its deepest point); a is the cost of writing and reading back
// a record, in hidden-layer evaluations. Returns -1 when compaction does not
// pay.
int choose_checkpoint(sand_model m, int prec, const float* xyz, int64_t n, int d, float r,
                      hipStream_t s, sand_status& st) {
  st = SAND_OK;
  if (n < kDynSampleMin || d < 4) return -1;
  const int64_t ns = kDynSample, stride = n / ns;
  char* tmp = nullptr;
  if (hipMallocAsync((void**)&tmp, (size_t)ns * 17, s) != hipSuccess) return -1;
  float* sx = (float*)tmp;
  float* sy = sx + 3 * ns;
  uint8_t* sd = (uint8_t*)(sy + ns);
  QueryArgs qa{};
  qa.m = m->args[prec];
  qa.xyz = sx;
  qa.sdf = sy;
  qa.n = ns;
  qa.full_depth = d;
  qa.dyn_r = r;
  qa.depth_out = sd;
  std::vector<uint8_t> h((size_t)ns);
  hipError_t e = launch_gather_points(xyz, stride, ns, sx, s);
  if (e == hipSuccess) e = launch_tmlp(prec, qa, m->num_cu, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), sd, (size_t)ns, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFreeAsync(tmp, s);
  if (e != hipSuccess) {
    st = device_fail(e, "dynamic checkpoint sample");
    return -1;
  }
  std::vector<int64_t> hist(kBuckets, 0);
  for (uint8_t v : h) ++hist[v < kBuckets ? v : kBuckets - 1];
  const double a = prec == PREC_FP32 ? 0.4 : 1.7;
  double best = (double)(d - 1);
  int bc = -1;
  int64_t running = ns;
  for (int c = 1; c < d; ++c) {
    running -= hist[c];
    if (c < 2) continue;
    const double cost = (c - 1) + (double)running / ns * (a + d - c);
    if (cost < 0.95 * best) {
      best = cost;
      bc = c;
    }
  }
  return bc;
}

// Dynamic exit with compaction after layer cp: per slab of at most `cap`
// points (the records the arena holds), the spilling launch, then the
// resumed tiles of its records.
sand_status run_dynamic_compacted(sand_model m, int prec, const QueryArgs& base, int cp,
                                  hipStream_t s) {
  const int64_t rec = dyn_record_bytes(prec, m->WP);
  int64_t cap = (int64_t)(kDynArenaBytes / (size_t)rec);
  if (cap > base.n) cap = base.n;
  char* arena = nullptr;
  if (hipMallocAsync((void**)&arena, 256 + (size_t)cap * rec, s) != hipSuccess)
    return fail(SAND_ERR_NOMEM, "sand_query: compaction arena of %lld bytes",
                (long long)(256 + cap * rec));
  hipError_t e = hipSuccess;
  for (int64_t s0 = 0; s0 < base.n && e == hipSuccess; s0 += cap) {
    QueryArgs qa = base;
    qa.xyz = base.xyz + 3 * s0;
    qa.sdf = base.sdf + s0;
    qa.n = base.n - s0 < cap ? base.n - s0 : cap;
    if (base.depth_out) qa.depth_out = base.depth_out + s0;
    qa.spill.arena = arena + 256;
    qa.spill.count = (int*)arena;
    qa.spill.cap = cap;
    qa.spill.layer = cp;
    e = launch_fill_u8((uint8_t*)arena, 4, 0, s);
    if (e == hipSuccess) e = launch_tmlp(prec, qa, m->num_cu, s);
    if (e == hipSuccess) e = launch_tmlp_resume(prec, qa, m->num_cu, s);
  }
  (void)hipFreeAsync(arena, s);
  return e == hipSuccess ? SAND_OK : device_fail(e, "compacted dynamic launch");
}

}  // namespace

sand_status run_forward(sand_model m, sand_depthmap dm, const float* xyz, int64_t n, float* sdf,
                        const sand_query_opts& o, char* ws, hipStream_t s, hipEvent_t* ev) {
  auto mark = [&](int i) {
    if (ev && ev[i]) (void)hipEventRecord(ev[i], s);
  };
  const int prec = o.precision;
  QueryArgs qa{};
  qa.m = m->args[prec];
  qa.xyz = xyz;
  qa.sdf = sdf;
  qa.n = n;
  hipError_t e;
  if (o.mode == SAND_FULL || o.mode == SAND_DYNAMIC) {
    const int d = (o.max_depth > 0 && o.max_depth < m->L) ? o.max_depth : m->L;
    qa.full_depth = d;
    if (o.mode == SAND_DYNAMIC) {
      qa.dyn_r = o.dynamic_r;
      qa.depth_out = o.depth_out;
      for (int i = 0; i < 4; ++i) mark(i);   // the checkpoint sample counts as t-mlp time
      int cp = o.dynamic_checkpoint;
      if (cp == 0) {
        sand_status st = SAND_OK;
        cp = choose_checkpoint(m, prec, xyz, n, d, o.dynamic_r, s, st);
        if (st != SAND_OK) return st;
      }
      if (cp >= 2 && cp < d) {
        const sand_status st = run_dynamic_compacted(m, prec, qa, cp, s);
        mark(4);
        return st;
      }
    } else {
      for (int i = 0; i < 4; ++i) mark(i);
    }
    if ((e = launch_tmlp(prec, qa, m->num_cu, s)) != hipSuccess) return device_fail(e, "t-mlp launch");
    mark(4);
    if (o.mode == SAND_FULL && o.depth_out &&
        (e = launch_fill_u8(o.depth_out, n, (uint8_t)d, s)) != hipSuccess)
      return device_fail(e, "depth fill launch");
    return SAND_OK;
  }
  sand_status st = run_bucketing(m, dm, xyz, n, sdf, nullptr, o, ws, s, tmlp_tile_points(prec, m->WP), ev,
                                 &qa.perm, &qa.plan);
  if (st != SAND_OK) return st;
  if ((e = launch_tmlp(prec, qa, m->num_cu, s)) != hipSuccess) return device_fail(e, "t-mlp launch");
  mark(4);
  return SAND_OK;
}

}  // namespace sand

extern "C" size_t sand_query_workspace_size(int64_t n) { return workspace_layout(n).total; }

extern "C" sand_status sand_query(sand_model m, sand_depthmap dm, const float* xyz, int64_t n,
                                  float* sdf, const sand_query_opts* opts, void* stream) {
  sand_query_opts o;
  if (opts) o = *opts; else sand_query_opts_init(&o);
  sand_status st = check_query("sand_query", m, dm, xyz, n, sdf, o);
  if (st != SAND_OK || n == 0) return st;
  DeviceGuard guard(m->device);
  if (!guard.ok) return fail(SAND_ERR_DEVICE, "sand_query: cannot select device");
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)o.workspace;
  bool owned = false;
  if (o.mode != SAND_FULL && o.mode != SAND_DYNAMIC && !ws) {
    hipError_t e = hipMallocAsync((void**)&ws, workspace_layout(n).total, s);
    if (e != hipSuccess) return fail(SAND_ERR_NOMEM, "sand_query: scratch of %zu bytes",
                                     workspace_layout(n).total);
    owned = true;
  }
  st = run_forward(m, dm, xyz, n, sdf, o, ws, s);
  if (owned) (void)hipFreeAsync(ws, s);
  return st;
}

extern "C" sand_status sand_query_timed(sand_model m, sand_depthmap dm, const float* xyz,
                                        int64_t n, float* sdf, const sand_query_opts* opts,
                                        void* stream, float* phase_ms) {
  if (!phase_ms) return fail(SAND_ERR_INVALID, "sand_query_timed: null phase_ms");
  sand_query_opts o;
  if (opts) o = *opts; else sand_query_opts_init(&o);
  sand_status st = check_query("sand_query_timed", m, dm, xyz, n, sdf, o);
  for (int i = 0; i < 5; ++i) phase_ms[i] = 0.0f;
  if (st != SAND_OK || n == 0) return st;
  DeviceGuard guard(m->device);
  if (!guard.ok) return fail(SAND_ERR_DEVICE, "sand_query_timed: cannot select device");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t ev[5] = {};
  for (int i = 0; i < 5; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) {
      for (int k = 0; k < i; ++k) (void)hipEventDestroy(ev[k]);
      return fail(SAND_ERR_DEVICE, "sand_query_timed: event creation");
    }
  char* ws = (char*)o.workspace;
  bool owned = false;
  if (o.mode != SAND_FULL && o.mode != SAND_DYNAMIC && !ws) {
    if (hipMallocAsync((void**)&ws, workspace_layout(n).total, s) != hipSuccess) {
      for (int k = 0; k < 5; ++k) (void)hipEventDestroy(ev[k]);
      return fail(SAND_ERR_NOMEM, "sand_query_timed: scratch");
    }
    owned = true;
  }
  st = run_forward(m, dm, xyz, n, sdf, o, ws, s, ev);
  if (owned) (void)hipFreeAsync(ws, s);
  if (st == SAND_OK) {
    hipError_t e = hipEventSynchronize(ev[4]);
    if (e != hipSuccess) st = device_fail(e, "sand_query_timed: wait");
    for (int i = 0; i < 4 && st == SAND_OK; ++i) (void)hipEventElapsedTime(&phase_ms[i], ev[i], ev[i + 1]);
    if (st == SAND_OK) (void)hipEventElapsedTime(&phase_ms[4], ev[0], ev[4]);
  }
  for (int k = 0; k < 5; ++k) (void)hipEventDestroy(ev[k]);
  return st;
}

extern "C" size_t sand_query_grad_workspace_size(sand_model m, int64_t n, int32_t precision) {
  if (!m || n <= 0 || precision < 0 || precision > 2) return 0;
  return workspace_layout(n).total + grad_stash_bytes(m, precision);
}

extern "C" sand_status sand_query_grad(sand_model m, sand_depthmap dm, const float* xyz, int64_t n,
                                       const float* dy, float* sdf, float* grad,
                                       const sand_query_opts* opts, void* stream) {
  sand_query_opts o;
  if (opts) o = *opts; else sand_query_opts_init(&o);
  sand_status st = check_query("sand_query_grad", m, dm, xyz, n, grad, o);
  if (st != SAND_OK) return st;
  if (o.mode == SAND_DYNAMIC)
    return fail(SAND_ERR_UNSUPPORTED, "sand_query_grad: dynamic mode has no gradient path "
                "(query with depth_out, then pass the depths in FORCED mode)");
  if (n == 0) return st;
  const size_t need = workspace_layout(n).total + grad_stash_bytes(m, o.precision);
  if (o.workspace && o.workspace_bytes < need)
    return fail(SAND_ERR_INVALID, "sand_query_grad: workspace of %zu bytes, need %zu",
                o.workspace_bytes, need);
  DeviceGuard guard(m->device);
  if (!guard.ok) return fail(SAND_ERR_DEVICE, "sand_query_grad: cannot select device");
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)o.workspace;
  bool owned = false;
  if (!ws) {
    if (hipMallocAsync((void**)&ws, need, s) != hipSuccess)
      return fail(SAND_ERR_NOMEM, "sand_query_grad: scratch of %zu bytes", need);
    owned = true;
  }
  const int prec = o.precision;
  AdjointArgs aa{};
  aa.q.m = m->args[prec];
  aa.q.xyz = xyz;
  aa.q.sdf = sdf;
  aa.q.n = n;
  aa.bwd = m->bwd[prec];
  aa.w1t = m->w1t;
  aa.tails = m->tails;
  aa.dy = dy;
  aa.grad = grad;
  aa.stash = ws + workspace_layout(n).total;
  aa.stash_wg = adjoint_stash_bytes_per_wg(prec, m->WP, m->L);
  hipError_t e = hipSuccess;
  if (o.mode == SAND_FULL) {
    aa.q.full_depth = (o.max_depth > 0 && o.max_depth < m->L) ? o.max_depth : m->L;
    if (o.depth_out) e = launch_fill_u8(o.depth_out, n, (uint8_t)aa.q.full_depth, s);
    if (e != hipSuccess) st = device_fail(e, "depth fill launch");
  } else {
    st = run_bucketing(m, dm, xyz, n, sdf, grad, o, ws, s, adjoint_tile_points(prec), nullptr,
                       &aa.q.perm, &aa.q.plan);
  }
  if (st == SAND_OK) {
    int grid = m->num_cu;
    if (o.mode == SAND_FULL) {
      const int64_t tiles = (n + adjoint_tile_points(prec) - 1) / adjoint_tile_points(prec);
      if (tiles < grid) grid = (int)tiles;
    }
    // the tile counter: the octree lookup's queue lengths, free once bucketing is done
    aa.next_tile = (uint32_t*)(ws + workspace_layout(n).qcount);
    if ((e = launch_fill_u8((uint8_t*)aa.next_tile, 4, 0, s)) != hipSuccess)
      st = device_fail(e, "tile counter fill launch");
    else if ((e = launch_adjoint(prec, aa, grid, s)) != hipSuccess)
      st = device_fail(e, "adjoint launch");
  }
  if (owned) (void)hipFreeAsync(ws, s);
  return st;
}
