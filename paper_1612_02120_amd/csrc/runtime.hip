// Host runtime behind include/emcnn.h: network object, weight packing and
// quantisation, work planning, persistent launches, batched submissions with
// HIP graphs, and the tile-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/emcnn.h"
#include "common.h"
#include "runtime.h"

namespace emcnn {

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return CNN_EHIP;
}

void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

// ------------------------------------------------------------------ number formats

float bf16_rne(float x) {
  // nearest bf16 value; on a tie the one whose last kept bit is 0
  if (!std::isfinite(x)) return x;
  uint32_t u;
  std::memcpy(&u, &x, 4);
  uint32_t lo = u & 0xffff0000u;
  uint32_t hi = lo + 0x10000u;
  float flo, fhi;
  std::memcpy(&flo, &lo, 4);
  std::memcpy(&fhi, &hi, 4);
  double dlo = std::fabs((double)x - (double)flo), dhi = std::fabs((double)fhi - (double)x);
  if (dlo < dhi) return flo;
  if (dhi < dlo) return fhi;
  return ((lo >> 16) & 1u) ? fhi : flo;
}

// All 127 non-negative finite e4m3fn values, ascending (code = index).
static const std::vector<double>& e4m3_table() {
  static std::vector<double> t = [] {
    std::vector<double> v;
    for (int code = 0; code < 127; ++code) {
      int e = (code >> 3) & 15, m = code & 7;
      v.push_back(e == 0 ? std::ldexp((double)m, -9) : std::ldexp(1.0 + m / 8.0, e - 7));
    }
    return v;
  }();
  return t;
}

// e4m3fn code of x: nearest representable value, ties to the even code,
// magnitudes beyond 448 saturate to 448.
uint8_t e4m3_code(double x) {
  const auto& t = e4m3_table();
  uint8_t sign = (x < 0) ? 0x80 : 0;
  double a = std::fabs(x);
  if (a >= 448.0) return sign | 126;
  size_t hi = std::lower_bound(t.begin(), t.end(), a) - t.begin();  // t[hi] >= a
  if (t[hi] == a) return sign | (uint8_t)hi;
  size_t lo = hi - 1;
  double dl = a - t[lo], dh = t[hi] - a;
  size_t pick = dl < dh ? lo : dh < dl ? hi : ((lo & 1) ? hi : lo);
  return sign | (uint8_t)pick;
}

// ------------------------------------------------------------------ spec parsing

static int act_bytes(int prec) { return prec == F32 ? 4 : prec == BF16 ? 2 : 1; }

static std::vector<int> find_first_variants(int prec, int cout, int ks, int maxout, int stride = 1) {
  std::vector<int> v;
  for (int i = 0; i < first_variant_count(); ++i) {
    const FirstInfo* f = first_variant(i);
    if (f->prec_out == prec && f->cout == cout && f->ks == ks && f->maxout == maxout && f->stride == stride)
      v.push_back(i);
  }
  return v;
}

static std::vector<int> find_conv_variants(int prec, int cin, int cout, int ks, int pool, int head, int epi) {
  std::vector<int> v;
  for (int i = 0; i < conv_variant_count(); ++i) {
    const VariantInfo* c = conv_variant(i);
    if (c->prec == prec && c->cin == cin && c->cout == cout && c->ks == ks && c->pool_in == pool &&
        c->head == head && c->epi == epi)
      v.push_back(i);
  }
  return v;
}

static int pack_conv(ExecLayer& L, int variant, const double* w, const double* b, const double* hw, double hb,
                     double in_scale, double next_scale) {
  const VariantInfo* v = conv_variant(variant);
  const int cin = v->cin, cout = v->cout, ks = v->ks, cb = v->cb, chb = v->chb, u = v->u, ngs = v->ngs;
  const int ncb = cin / cb, nchb = cb / chb, nb = cout / 16;
  const int esz = act_bytes(v->prec);
  // flattened K: [cb][s][nb][u][lane]; row reuse: [cb][i][rs][nb][u][lane]. The
  // 16-byte chunk uu of all 64 lanes is contiguous, so each fragment load of a
  // wave reads one contiguous 1 KB block.
  const int nsteps = v->rr ? ks * ngs : ngs;
  const size_t bytes = (size_t)ncb * nsteps * nb * 64 * u * 16;
  std::vector<uint8_t> pk(bytes, 0);
  // quantised weights, [co][ci][i][j]
  const size_t nw = (size_t)cout * cin * ks * ks;
  std::vector<double> wq(nw);
  std::vector<float> osc(cout, 1.0f);
  if (v->prec == F32) {
    for (size_t i = 0; i < nw; ++i) wq[i] = (float)w[i];
  } else if (v->prec == BF16) {
    for (size_t i = 0; i < nw; ++i) wq[i] = bf16_rne((float)w[i]);
  } else {
    const size_t per = (size_t)cin * ks * ks;
    for (int co = 0; co < cout; ++co) {
      double mx = 0.0;
      for (size_t i = 0; i < per; ++i) mx = std::max(mx, std::fabs(w[co * per + i]));
      double sw = mx > 0 ? mx / 448.0 : 1.0;
      for (size_t i = 0; i < per; ++i) wq[co * per + i] = (double)e4m3_code(w[co * per + i] / sw);  // code
      osc[co] = (float)(in_scale * sw);
    }
  }
  for (int c0 = 0; c0 < ncb; ++c0)
    for (int s = 0; s < nsteps; ++s)
      for (int n_b = 0; n_b < nb; ++n_b)
        for (int lane = 0; lane < 64; ++lane) {
          const int n = lane & 15, g = lane >> 4, co = n_b * 16 + n;
          for (int uu = 0; uu < u; ++uu) {
            int i, j, cg;
            if (v->rr) {
              // step s = (filter row i, row-step rs); slot c over the row's (j, chunk) pairs
              i = s / ngs;
              const int c = (4 * (s % ngs) + g) * u + uu;
              if (c >= ks * nchb) continue;
              j = c / nchb;
              cg = c % nchb;
            } else {
              // the kernels' chunk-slot order
              const KSlot k = k_slot(s * 4 * u + 4 * uu + g, ks, nchb, v->rowq != 0);
              if (!k.live) continue;
              i = k.i;
              j = k.j;
              cg = k.cg;
            }
            uint8_t* dst = pk.data() + ((((size_t)(c0 * nsteps + s) * nb + n_b) * u + uu) * 64 + lane) * 16;
            for (int t = 0; t < chb; ++t) {
              const int ci = c0 * cb + cg * chb + t;
              const double val = wq[(((size_t)co * cin + ci) * ks + i) * ks + j];
              if (v->prec == F32) {
                float f = (float)val;
                std::memcpy(dst + t * esz, &f, 4);
              } else if (v->prec == BF16) {
                float f = (float)val;
                uint32_t bits;
                std::memcpy(&bits, &f, 4);
                uint16_t h = (uint16_t)(bits >> 16);
                std::memcpy(dst + t * esz, &h, 2);
              } else {
                dst[t] = (uint8_t)val;
              }
            }
          }
        }
  std::vector<float> bias(b, b + cout);
  hipError_t e;
  void* wdev = nullptr;
  if ((e = hipMalloc(&wdev, bytes)) != hipSuccess) return hip_fail(e, "hipMalloc(weights)");
  L.wpacks.push_back(wdev);
  if ((e = hipMemcpy(wdev, pk.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(weights)");
  if (L.bias) return CNN_OK;  // per-channel data shared by all candidates is already set
  if ((e = hipMalloc(&L.bias, cout * sizeof(float))) != hipSuccess) return hip_fail(e, "hipMalloc(bias)");
  if ((e = hipMemcpy(L.bias, bias.data(), cout * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(bias)");
  if (v->prec == FP8) {
    if ((e = hipMalloc(&L.oscale, cout * sizeof(float))) != hipSuccess) return hip_fail(e, "hipMalloc(scale)");
    if ((e = hipMemcpy(L.oscale, osc.data(), cout * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "hipMemcpy(scale)");
  }
  if (v->head) {
    std::vector<float> h(hw, hw + cout);
    if ((e = hipMalloc(&L.head_w, cout * sizeof(float))) != hipSuccess) return hip_fail(e, "hipMalloc(head)");
    if ((e = hipMemcpy(L.head_w, h.data(), cout * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "hipMemcpy(head)");
    L.head_b = (float)hb;
  }
  L.out_inv_scale = next_scale > 0 ? (float)(1.0 / next_scale) : 1.0f;
  return CNN_OK;
}

// First-layer weights as per-lane MFMA B fragments (see conv_first):
//   FP32 nets: float [step][n-block][lane], lane (n, g) holds tap 4 step + g of
//              channel 16 n-block + n;
//   others:    bf16 [n-block][lane][8], lane (n, g) holds taps 8g .. 8g+7.
// Taps beyond k*k are zero. 1/255 is folded in (the kernel reads raw uint8).
static int pack_first(ExecLayer& L, int variant, const double* w, const double* b, double next_scale) {
  const FirstInfo* f = first_variant(variant);
  const int cout = f->cout, taps = f->ks * f->ks, nb = cout / 16;
  std::vector<unsigned char> pk;
  if (f->prec_out == F32) {
    const int nstep = (taps + 3) / 4;
    std::vector<float> v((size_t)nstep * nb * 64, 0.f);
    for (int s = 0; s < nstep; ++s)
      for (int q = 0; q < nb; ++q)
        for (int lane = 0; lane < 64; ++lane) {
          const int co = q * 16 + (lane & 15), k = 4 * s + (lane >> 4);
          if (k < taps) v[((size_t)s * nb + q) * 64 + lane] = (float)(w[(size_t)co * taps + k] / 255.0);
        }
    pk.resize(v.size() * 4);
    std::memcpy(pk.data(), v.data(), pk.size());
  } else {
    std::vector<uint16_t> v((size_t)nb * 64 * 8, 0);
    for (int q = 0; q < nb; ++q)
      for (int lane = 0; lane < 64; ++lane)
        for (int t = 0; t < 8; ++t) {
          const int co = q * 16 + (lane & 15), k = 8 * (lane >> 4) + t;
          if (k >= taps) continue;
          const float x = bf16_rne((float)(w[(size_t)co * taps + k] / 255.0));
          uint32_t bits;
          std::memcpy(&bits, &x, 4);
          v[((size_t)q * 64 + lane) * 8 + t] = (uint16_t)(bits >> 16);
        }
    pk.resize(v.size() * 2);
    std::memcpy(pk.data(), v.data(), pk.size());
  }
  std::vector<float> bf(b, b + cout);
  hipError_t e;
  void* wdev = nullptr;
  if ((e = hipMalloc(&wdev, pk.size())) != hipSuccess) return hip_fail(e, "hipMalloc(w1)");
  L.wpacks.push_back(wdev);
  if ((e = hipMemcpy(wdev, pk.data(), pk.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(w1)");
  if (L.bias) return CNN_OK;
  if ((e = hipMalloc(&L.bias, cout * sizeof(float))) != hipSuccess) return hip_fail(e, "hipMalloc(b1)");
  if ((e = hipMemcpy(L.bias, bf.data(), cout * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(b1)");
  L.out_inv_scale = next_scale > 0 ? (float)(1.0 / next_scale) : 1.0f;
  return CNN_OK;
}

// Weights of the VALU two-class layer (head_phase). A two-class softmax is
// the sigmoid of the logit difference, so the layer needs only the weight
// difference W[1] - W[0] (taken in FP64, rounded once), as [i][ci / 4][j][ci % 4],
// FP32; the bias is stored padded to 16 floats (the MFMA candidate of the same
// layer reads 16), and the kernel takes b1 - b0.
static int pack_head_valu(ExecLayer& L, int variant, const double* w, const double* b) {
  const VariantInfo* v = conv_variant(variant);
  const int cin = v->cin, ks = v->ks, ncg = cin / 4;
  std::vector<float> pk((size_t)ks * ncg * ks * 4);
  for (int i = 0; i < ks; ++i)
    for (int cg = 0; cg < ncg; ++cg)
      for (int j = 0; j < ks; ++j)
        for (int e = 0; e < 4; ++e) {
          const size_t k0 = (((size_t)0 * cin + 4 * cg + e) * ks + i) * ks + j;
          const size_t k1 = (((size_t)1 * cin + 4 * cg + e) * ks + i) * ks + j;
          pk[(((size_t)i * ncg + cg) * ks + j) * 4 + e] = (float)(w[k1] - w[k0]);
        }
  hipError_t err;
  void* wdev = nullptr;
  if ((err = hipMalloc(&wdev, pk.size() * 4)) != hipSuccess) return hip_fail(err, "hipMalloc(head weights)");
  L.wpacks.push_back(wdev);
  if ((err = hipMemcpy(wdev, pk.data(), pk.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(err, "hipMemcpy(head weights)");
  if (L.bias) return CNN_OK;
  std::vector<float> bf(16, 0.f);
  bf[0] = (float)b[0];
  bf[1] = (float)b[1];
  if ((err = hipMalloc(&L.bias, 16 * sizeof(float))) != hipSuccess) return hip_fail(err, "hipMalloc(head bias)");
  if ((err = hipMemcpy(L.bias, bf.data(), 16 * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(err, "hipMemcpy(head bias)");
  return CNN_OK;
}

// Weights of the two-class layer as a tap GEMM (head_taps): the weight
// difference W[1] - W[0] (FP64, rounded once to the operand type) as MFMA B
// fragments [step t][lane][16 bytes], lane (n16, g) holding tap n16 = KS i + j
// for the CHB channels of 16-byte chunk 4t + g. Bias as for head_phase.
static int pack_head_taps(ExecLayer& L, int variant, const double* w, const double* b) {
  const VariantInfo* v = conv_variant(variant);
  const int cin = v->cin, ks = v->ks, chb = v->chb, esz = act_bytes(v->prec);
  const int nk = cin * esz / 64;
  std::vector<unsigned char> pk((size_t)nk * 64 * 16, 0);
  for (int t = 0; t < nk; ++t)
    for (int lane = 0; lane < 64; ++lane)
      for (int e = 0; e < chb; ++e) {
        const int tap = lane & 15, ch = chb * (4 * t + (lane >> 4)) + e;
        const int i = tap / ks, j = tap % ks;
        const double dw = w[(((size_t)1 * cin + ch) * ks + i) * ks + j] - w[(((size_t)0 * cin + ch) * ks + i) * ks + j];
        unsigned char* dst = pk.data() + ((size_t)t * 64 + lane) * 16 + (size_t)e * esz;
        if (v->prec == F32) {
          const float f = (float)dw;
          std::memcpy(dst, &f, 4);
        } else {
          const float f = bf16_rne((float)dw);
          uint32_t bits;
          std::memcpy(&bits, &f, 4);
          const uint16_t h = (uint16_t)(bits >> 16);
          std::memcpy(dst, &h, 2);
        }
      }
  hipError_t err;
  void* wdev = nullptr;
  if ((err = hipMalloc(&wdev, pk.size())) != hipSuccess) return hip_fail(err, "hipMalloc(head weights)");
  L.wpacks.push_back(wdev);
  if ((err = hipMemcpy(wdev, pk.data(), pk.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(err, "hipMemcpy(head weights)");
  if (L.bias) return CNN_OK;
  std::vector<float> bf(16, 0.f);
  bf[0] = (float)b[0];
  bf[1] = (float)b[1];
  if ((err = hipMalloc(&L.bias, 16 * sizeof(float))) != hipSuccess) return hip_fail(err, "hipMalloc(head bias)");
  if ((err = hipMemcpy(L.bias, bf.data(), 16 * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(err, "hipMemcpy(head bias)");
  return CNN_OK;
}

// Weights of a 1x1 multi-class output conv (head_1x1): W[class][cin] and the
// biases, FP32 as given.
static int pack_head1(ExecLayer& L, int variant, const double* w, const double* b) {
  const VariantInfo* v = conv_variant(variant);
  std::vector<float> pk((size_t)v->cout * v->cin), bf(v->cout);
  for (size_t i = 0; i < pk.size(); ++i) pk[i] = (float)w[i];
  for (int k = 0; k < v->cout; ++k) bf[k] = (float)b[k];
  hipError_t err;
  void* wdev = nullptr;
  if ((err = hipMalloc(&wdev, pk.size() * 4)) != hipSuccess) return hip_fail(err, "hipMalloc(head weights)");
  L.wpacks.push_back(wdev);
  if ((err = hipMemcpy(wdev, pk.data(), pk.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(err, "hipMemcpy(head weights)");
  if (L.bias) return CNN_OK;
  if ((err = hipMalloc(&L.bias, bf.size() * 4)) != hipSuccess) return hip_fail(err, "hipMalloc(head bias)");
  if ((err = hipMemcpy(L.bias, bf.data(), bf.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(err, "hipMemcpy(head bias)");
  return CNN_OK;
}

static void free_layer(ExecLayer& L) {
  for (void* p : L.wpacks)
    if (p) hipFree(p);
  L.wpacks.clear();
  if (L.bias) hipFree(L.bias);
  if (L.oscale) hipFree(L.oscale);
  if (L.head_w) hipFree(L.head_w);
  L.wpack = nullptr;
  L.bias = L.oscale = L.head_w = nullptr;
}

// Nets with stride-2 pools (the FastMemb family, Section 2.2), FP32 or BF16,
// in their dense form: conv(4, 1 -> 64, max-out), then one or more of { 2x2/s2
// pool, conv(4, 32 -> 64, max-out) }, then a 2x2/s2 pool and conv(4, 32 -> 2,
// softmax). Every stride-2 pool becomes a 2x2 max filter at the current
// spacing and doubles the spacing of the later layers. A 2x subsample right
// after the first conv (FastMemb_ss, "A subsampling CNN for 3 nm data") keeps
// one fragment only: the first conv is evaluated at every second row and
// column, and the conv after it runs densely on that half-resolution map with
// no max filter before it. BF16: bf16 weights and stored activations with FP32
// accumulation (the first conv's weights are bf16(w / 255) against exact uint8
// inputs).
static int build_strided(Net* net, const double* weights, const cnn_layer* Lr, int nl) {
  const int prec = net->prec;
  const auto unsupported = [](const std::string& why) {
    return fail(CNN_EUNSUPPORTED, "cnn_create: stride-2 pool nets: " + why);
  };
  const cnn_layer& l0 = Lr[0];
  const bool maps = l0.cin > 1;  // real-valued input maps (MaskExtend) instead of one uint8 channel
  if (l0.kind != CNN_LAYER_CONV || l0.k != 4 || l0.act != CNN_ACT_MAXOUT || (!maps && l0.cout != 64))
    return unsupported("the first layer must be conv(4, C -> 2F, max-out) (C = 1: F = 32)");
  if (maps && prec != CNN_PREC_FP32) return unsupported("nets on real-valued input maps are FP32");
  const bool sub = nl > 1 && Lr[1].kind == CNN_LAYER_SUBSAMPLE2;
  if (sub && maps) return unsupported("a subsample after a multi-channel first layer");
  // layer indices of the convs, and of the pool before each (-1: none)
  std::vector<int> conv_at{0}, pool_at{-1};
  int i = 1;
  if (sub) {
    if (nl < 3 || Lr[2].kind != CNN_LAYER_CONV) return unsupported("a subsample must be followed by a conv");
    conv_at.push_back(2);
    pool_at.push_back(-1);
    i = 3;
  }
  while (i < nl) {
    if (Lr[i].kind == CNN_LAYER_MAXPOOL_S2 && i + 1 < nl && Lr[i + 1].kind == CNN_LAYER_CONV) {
      conv_at.push_back(i + 1);
      pool_at.push_back(i);
      i += 2;
    } else if (i == nl - 1 && Lr[i].kind == CNN_LAYER_CONV && Lr[i].k == 1 && Lr[i].act == CNN_ACT_SOFTMAX0) {
      conv_at.push_back(i);  // a 1x1 multi-class output right after the last conv
      pool_at.push_back(-1);
      i += 1;
    } else {
      return unsupported("after the first conv (and a subsample), expected (stride-2 pool, conv) pairs");
    }
  }
  if (conv_at.size() < 3) return unsupported("expected at least one inner conv before the output conv");
  for (size_t c = 1; c < conv_at.size(); ++c) {
    const cnn_layer& l = Lr[conv_at[c]];
    const bool last = c + 1 == conv_at.size();
    if (last && l.act == CNN_ACT_SOFTMAX0) continue;  // 1x1 output: checked by kernel availability
    if (l.kind != CNN_LAYER_CONV || l.k != 4 ||
        (last ? (l.cin != 32 || l.cout != 2 || l.act != CNN_ACT_SOFTMAX) : l.act != CNN_ACT_MAXOUT))
      return unsupported("inner convs are conv(4, F -> 2F', max-out), the last conv(4, 32 -> 2, softmax) or a "
                         "1x1 softmax over classes");
    if (last && pool_at[c] < 0) return unsupported("the softmax conv must follow a stride-2 pool");
  }
  const double* wp = weights;
  int sp = 1;  // spacing of the current layer's input
  for (size_t c = 0; c < conv_at.size(); ++c) {
    const cnn_layer& l = Lr[conv_at[c]];
    const int64_t nwl = (int64_t)l.cout * l.cin * l.k * l.k;
    const double* w = wp;
    const double* b = wp + nwl;
    wp += nwl + l.cout;
    ExecLayer E;
    E.ks = l.k;
    E.cin = l.cin;
    E.spaced = 1;
    int rc = CNN_OK;
    if (c == 0 && maps) {
      // a spaced conv straight on the caller's NHWC float maps: no max filter, spacing 1
      E.cout = l.cout;
      E.cstore = l.cout / 2;
      E.epi = 1;
      E.pool_in = 0;
      E.pd = 0;
      E.dil = 1;
      E.candidates = find_conv_variants(prec, l.cin, l.cout, l.k, 1, 0, 1);
      E.candidates.erase(std::remove_if(E.candidates.begin(), E.candidates.end(),
                                        [](int v) { return conv_variant(v)->groups != 0; }),
                         E.candidates.end());  // no max filter: no phase groups
      if (E.candidates.empty()) return unsupported("no kernel for a first conv " + std::to_string(l.cin) + " -> " +
                                                   std::to_string(l.cout));
      for (int v : E.candidates)
        if (rc == CNN_OK) rc = pack_conv(E, v, w, b, nullptr, 0.0, 1.0, 0.0);
    } else if (c == 0) {
      E.first = 1;
      E.cout = l.cout;
      E.cstore = l.cout / 2;
      E.epi = 1;
      E.stride = sub ? 2 : 1;
      E.candidates = find_first_variants(prec, l.cout, l.k, 1, E.stride);
      if (E.candidates.empty()) return unsupported("no first-layer kernel");
      for (int v : E.candidates)
        if (rc == CNN_OK) rc = pack_first(E, v, w, b, 0.0);
    } else if (l.act == CNN_ACT_SOFTMAX0) {
      // 1x1 output conv over the classes (row-major input, no spacing)
      E.spaced = 0;
      E.cout = l.cout;
      E.cstore = 1;
      E.epi = 4;
      E.dil = 1;
      E.candidates = find_conv_variants(prec, l.cin, l.cout, 1, 0, 0, 4);
      if (E.candidates.empty()) return unsupported("no kernel for a 1x1 softmax over " + std::to_string(l.cout) +
                                                   " classes from " + std::to_string(l.cin) + " channels");
      for (int v : E.candidates)
        if (rc == CNN_OK) rc = pack_head1(E, v, w, b);
    } else {
      if (pool_at[c] >= 0) {
        E.pool_in = 1;
        E.pd = sp;  // the max filter of the stride-2 pool before this conv
        sp *= 2;
      } else {
        E.pool_in = 0;  // after the subsample: no max filter, dense at spacing 1
        E.pd = 0;
      }
      E.dil = sp;
      if (l.act == CNN_ACT_SOFTMAX) {
        // the two-class layer: first the tap-GEMM kernels (one MFMA column
        // per tap of the weight difference; over phase groups where the max
        // filter before it has half its spacing), then the VALU kernels and the
        // MFMA kernels that run it as 16 columns with zero weights and bias
        // for classes >= 2 (BF16 nets: those two the other way round).
        E.cout = l.cout;
        E.cstore = 1;
        std::vector<int> va = find_conv_variants(prec, l.cin, 2, l.k, 1, 0, 3);
        std::vector<int> mf = find_conv_variants(prec, l.cin, 16, l.k, 1, 0, 2);
        if (prec == CNN_PREC_BF16) va.swap(mf);
        E.candidates.clear();
        if (E.pd >= 1 && 2 * E.pd == E.dil)  // phase groups share the max filter's fragments
          E.candidates = find_conv_variants(prec, l.cin, 2, l.k, 1, 0, 6);
        const std::vector<int> tp = find_conv_variants(prec, l.cin, 2, l.k, 1, 0, 5);
        E.candidates.insert(E.candidates.end(), tp.begin(), tp.end());
        E.candidates.insert(E.candidates.end(), va.begin(), va.end());
        E.candidates.insert(E.candidates.end(), mf.begin(), mf.end());
        if (!E.candidates.empty()) E.epi = conv_variant(E.candidates[0])->epi;
        if (E.candidates.empty()) return unsupported("no kernel for the softmax layer");
        std::vector<double> wpad((size_t)16 * l.cin * l.k * l.k, 0.0), bpad(16, 0.0);
        std::copy(w, w + nwl, wpad.begin());
        std::copy(b, b + l.cout, bpad.begin());
        for (int v : E.candidates) {
          if (rc != CNN_OK) break;
          const int ep = conv_variant(v)->epi;
          rc = ep == 3   ? pack_head_valu(E, v, w, b)
               : ep >= 5 ? pack_head_taps(E, v, w, b)
                         : pack_conv(E, v, wpad.data(), bpad.data(), nullptr, 0.0, 1.0, 0.0);
        }
      } else {
        E.cout = l.cout;
        E.cstore = l.cout / 2;
        E.epi = 1;
        // the spaced kernels take the max filter's spacing from the job: the
        // same kernels serve a conv without a max filter (spacing 0)
        E.candidates = find_conv_variants(prec, l.cin, E.cout, l.k, 1, 0, E.epi);
        if (!(E.pd >= 1 && 2 * E.pd == E.dil))  // phase groups need a max filter at half the spacing
          E.candidates.erase(std::remove_if(E.candidates.begin(), E.candidates.end(),
                                            [](int v) { return conv_variant(v)->groups != 0; }),
                             E.candidates.end());
        if (E.candidates.empty())
          return unsupported("no MFMA kernel for conv " + std::to_string(c) + " (" + std::to_string(l.cin) + " -> " +
                             std::to_string(l.cout) + ")");
        for (int v : E.candidates)
          if (rc == CNN_OK) rc = pack_conv(E, v, w, b, nullptr, 0.0, 1.0, 0.0);
      }
    }
    E.variant = E.candidates[0];
    if (rc == CNN_OK) select_variant(E, E.variant);
    net->layers.push_back(E);
    if (rc != CNN_OK) return rc;
  }
  int off = 0;
  for (auto& E : net->layers) {
    E.in_off = off;
    off += (E.pool_in ? E.pd : 0) + (E.ks - 1) * E.dil;
  }
  if (!sub && off != net->R) return fail(CNN_EINVAL, "cnn_create: internal radius mismatch");
  net->out_stride = sub ? 2 : 1;
  net->in_channels = maps ? l0.cin : 1;
  net->in_elb = maps ? 4 * l0.cin : 1;
  // every map but the output feeds a spaced conv: stored fragment-major modulo its spacing
  for (size_t l = 0; l + 1 < net->layers.size(); ++l) net->layers[l].out_lg = __builtin_ctz(net->layers[l + 1].dil);
  return CNN_OK;
}

int layer_threads(const ExecLayer& L) {
  return L.first ? first_variant(L.variant)->threads : conv_variant(L.variant)->threads;
}
int layer_ty(const ExecLayer& L) { return L.first ? first_variant(L.variant)->ty : conv_variant(L.variant)->ty; }
int layer_tx(const ExecLayer& L) { return L.first ? first_variant(L.variant)->tx : conv_variant(L.variant)->tx; }
bool layer_phase_groups(const ExecLayer& L) { return !L.first && conv_variant(L.variant)->groups != 0; }
const void* layer_fn(const ExecLayer& L) {
  return L.first ? first_variant(L.variant)->fn : conv_variant(L.variant)->fn;
}
const char* layer_name(const ExecLayer& L) {
  return L.first ? first_variant(L.variant)->name : conv_variant(L.variant)->name;
}

bool select_variant(ExecLayer& L, int variant) {
  for (size_t i = 0; i < L.candidates.size(); ++i)
    if (L.candidates[i] == variant && i < L.wpacks.size()) {
      L.variant = variant;
      L.wpack = L.wpacks[i];
      return true;
    }
  return false;
}

bool first_fused(const Net* net) {
  return net->layers.size() > 1 && !net->layers[1].first && conv_variant(net->layers[1].variant)->fused > 0;
}

int persistent_grid(Net* net, const ExecLayer& L, int64_t total_items) {
  int per_cu = 0;
  const void* fn = layer_fn(L);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, layer_threads(L), 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int64_t cap = (int64_t)net->num_cus * per_cu;
  cap = std::max<int64_t>(8, cap / 8 * 8);
  int64_t want = (total_items + 7) / 8 * 8;
  return (int)std::max<int64_t>(8, std::min(cap, want));
}

}  // namespace emcnn

using namespace emcnn;

// ------------------------------------------------------------------ C ABI: create / destroy

extern "C" int cnn_create(const double* weights, int64_t n_weights, const cnn_layer_spec* spec, cnn_net** out) {
  clear_error();
  if (!weights || !spec || !out || !spec->layers || spec->n_layers < 2)
    return fail(CNN_EINVAL, "cnn_create: null argument or fewer than 2 layers");
  *out = nullptr;
  const int prec = spec->precision;
  if (prec != CNN_PREC_FP32 && prec != CNN_PREC_BF16 && prec != CNN_PREC_FP8)
    return fail(CNN_EINVAL, "cnn_create: unknown precision");
  // structural validation; R follows the receptive-field recursion
  // r += (k - 1) j, j *= stride (a 2x2 pool counts as k = 2)
  int64_t expect = 0;
  int R = 0;
  // input channels: one uint8 channel, or real-valued maps (the first conv's cin)
  int C = spec->layers[0].kind == CNN_LAYER_CONV && spec->layers[0].cin > 1 ? spec->layers[0].cin : 1;
  int sp = 1;  // input spacing j of the current layer
  bool strided = false;  // stride-2 pools, max-out or softmax: the FastMemb family
  for (int i = 0; i < spec->n_layers; ++i) {
    const cnn_layer& l = spec->layers[i];
    if (l.kind == CNN_LAYER_CONV) {
      if (l.k < 1 || l.cin != C || l.cout < 1 || (l.act < 0 || l.act > CNN_ACT_SOFTMAX0))
        return fail(CNN_EINVAL, "cnn_create: bad conv layer " + std::to_string(i));
      expect += (int64_t)l.cout * l.cin * l.k * l.k + l.cout;
      R += (l.k - 1) * sp;
      C = l.cout;
      if (l.act == CNN_ACT_MAXOUT) {
        if (l.cout % 2) return fail(CNN_EINVAL, "cnn_create: max-out needs an even channel count");
        C = l.cout / 2;
        strided = true;
      } else if (l.act == CNN_ACT_SOFTMAX) {
        if (l.cout != 2) return fail(CNN_EINVAL, "cnn_create: softmax output needs two classes");
        C = 1;
        strided = true;
      } else if (l.act == CNN_ACT_SOFTMAX0) {
        if (l.cout < 2) return fail(CNN_EINVAL, "cnn_create: a softmax over classes needs two or more");
        C = 1;
        strided = true;
      }
    } else if (l.kind == CNN_LAYER_MAXPOOL || l.kind == CNN_LAYER_MAXPOOL_S2) {
      if (l.k != 2 || i == 0) return fail(CNN_EINVAL, "cnn_create: maxpool must be 2x2 and follow a conv");
      R += sp;
      if (l.kind == CNN_LAYER_MAXPOOL_S2) {
        sp *= 2;
        strided = true;
      }
    } else if (l.kind == CNN_LAYER_SUBSAMPLE2) {
      if (i == 0 || spec->layers[i - 1].kind != CNN_LAYER_CONV)
        return fail(CNN_EINVAL, "cnn_create: a subsample must follow a conv");
      sp *= 2;  // window 1: no growth of the field of view
      strided = true;
    } else {
      return fail(CNN_EINVAL, "cnn_create: bad layer kind at " + std::to_string(i));
    }
  }
  if (expect != n_weights)
    return fail(CNN_EINVAL, "cnn_create: n_weights " + std::to_string(n_weights) + " != " + std::to_string(expect));
  if (C != 1) return fail(CNN_EINVAL, "cnn_create: last layer must have one output channel");
  const cnn_layer* Lr = spec->layers;
  const int nl = spec->n_layers;
  const cnn_layer& hd = Lr[nl - 1];
  if (strided) {
    if (prec != CNN_PREC_FP32 && prec != CNN_PREC_BF16)
      return fail(CNN_EUNSUPPORTED, "cnn_create: stride-2 pool nets are FP32 or BF16");
  } else {
    // supported shape: first conv(5, 1->C, relu) [pool], body convs (relu) [pool], head conv(1, C->1, sigmoid)
    if (Lr[0].kind != CNN_LAYER_CONV || Lr[0].cin != 1 || Lr[0].act != CNN_ACT_RELU)
      return fail(CNN_EUNSUPPORTED, "cnn_create: first layer must be a ReLU conv on one channel");
    if (hd.kind != CNN_LAYER_CONV || hd.k != 1 || hd.cout != 1 || hd.act != CNN_ACT_SIGMOID)
      return fail(CNN_EUNSUPPORTED, "cnn_create: last layer must be a 1x1 conv to one channel with sigmoid");
    if (Lr[nl - 2].kind != CNN_LAYER_CONV)
      return fail(CNN_EUNSUPPORTED, "cnn_create: no pooling directly before the head");
  }

  int dev = 0;
  hipGetDevice(&dev);
  Net* net = new Net();
  net->device = dev;
  net->prec = prec;
  net->R = R;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete net;
    return fail(CNN_EHIP, "cnn_create: hipGetDeviceProperties failed");
  }
  net->num_cus = prop.multiProcessorCount;
  net->arch = prop.gcnArchName;
  if (net->arch.rfind("gfx950", 0) != 0) {
    delete net;
    return fail(CNN_EUNSUPPORTED, "cnn_create: kernels are built for gfx950, device is " + std::string(prop.gcnArchName));
  }
  if (const char* s = std::getenv("EMCNN_WORKSPACE_MB")) net->ws_budget = (size_t)std::atoll(s) << 20;
  if (strided) {
    const int rc = build_strided(net, weights, Lr, nl);
    if (rc != CNN_OK) {
      for (auto& E : net->layers) free_layer(E);
      delete net;
      return rc;
    }
    *out = reinterpret_cast<cnn_net*>(net);
    return CNN_OK;
  }

  // build executed layers; weights pointer walks convs in order
  const double* wp = weights;
  int pending_pool = 0;
  int conv_i = 0;
  int rc = CNN_OK;
  // next FP8 input scale of the conv following layer i
  auto next_conv_scale = [&](int i) -> double {
    for (int k = i + 1; k < nl; ++k)
      if (Lr[k].kind == CNN_LAYER_CONV) {
        const bool is_head = (k == nl - 1);
        return (prec == CNN_PREC_FP8 && !is_head) ? (double)Lr[k].act_scale : 0.0;
      }
    return 0.0;
  };
  for (int i = 0; i < nl && rc == CNN_OK; ++i) {
    const cnn_layer& l = Lr[i];
    if (l.kind == CNN_LAYER_MAXPOOL) {
      if (pending_pool || Lr[i - 1].act != CNN_ACT_RELU) {
        rc = fail(CNN_EUNSUPPORTED, "cnn_create: pooling must follow a ReLU conv, one at a time");
        break;
      }
      pending_pool = 1;
      continue;
    }
    const int64_t nwl = (int64_t)l.cout * l.cin * l.k * l.k;
    const double* w = wp;
    const double* b = wp + nwl;
    wp += nwl + l.cout;
    if (i == nl - 1) break;  // head: fused into the previous conv
    ExecLayer E;
    E.cin = l.cin;
    E.cout = l.cout;
    E.ks = l.k;
    E.pool_in = pending_pool;
    pending_pool = 0;
    const double nxt = next_conv_scale(i);
    if (conv_i == 0) {
      E.first = 1;
      E.candidates = find_first_variants(prec, l.cout, l.k, 0);
      if (E.candidates.empty()) {
        rc = fail(CNN_EUNSUPPORTED, "cnn_create: no first-layer kernel for this shape/precision");
        break;
      }
      E.variant = E.candidates[0];
      for (int c : E.candidates) {
        if (rc == CNN_OK) rc = pack_first(E, c, w, b, nxt);
      }
      if (rc == CNN_OK) select_variant(E, E.variant);
    } else {
      const bool fuse_head = (i == nl - 2);
      if (l.act != CNN_ACT_RELU) {
        rc = fail(CNN_EUNSUPPORTED, "cnn_create: body convs must use ReLU");
        break;
      }
      E.head = fuse_head;
      E.candidates = find_conv_variants(prec, l.cin, l.cout, l.k, E.pool_in, fuse_head, 0);
      {
        // variants that compute the first layer themselves apply only right after it
        const ExecLayer& L0 = net->layers[0];
        std::vector<int> keep;
        for (int c : E.candidates) {
          const int k1 = conv_variant(c)->fused;
          if (k1 == 0 || (conv_i == 1 && L0.first && L0.ks == k1 && L0.cout == l.cin)) keep.push_back(c);
        }
        E.candidates.swap(keep);
      }
      if (E.candidates.empty()) {
        rc = fail(CNN_EUNSUPPORTED, "cnn_create: no MFMA kernel for conv " + std::to_string(i));
        break;
      }
      E.variant = E.candidates[0];
      const double in_scale = (prec == CNN_PREC_FP8) ? (double)l.act_scale : 1.0;
      if (prec == CNN_PREC_FP8 && !(in_scale > 0)) {
        rc = fail(CNN_EINVAL, "cnn_create: FP8 conv " + std::to_string(i) + " needs act_scale > 0");
        break;
      }
      const double* hw = nullptr;
      double hb = 0;
      if (fuse_head) {
        hw = wp;
        hb = wp[hd.cin];
      }
      for (int c : E.candidates) {
        if (rc == CNN_OK) rc = pack_conv(E, c, w, b, hw, hb, in_scale, fuse_head ? 0.0 : nxt);
      }
      if (rc == CNN_OK) select_variant(E, E.variant);
    }
    net->layers.push_back(E);
    ++conv_i;
  }
  if (rc == CNN_OK && (net->layers.size() < 2 || !net->layers.back().head))
    rc = fail(CNN_EUNSUPPORTED, "cnn_create: need at least one body conv to carry the head");
  if (rc != CNN_OK) {
    for (auto& E : net->layers) free_layer(E);
    delete net;
    return rc;
  }
  // storage precision of each layer's output and stored dims offsets
  int off = 0;
  for (auto& E : net->layers) {
    E.in_off = off;  // radius consumed before this layer
    off += (E.pool_in ? E.pd : 0) + (E.ks - 1) * E.dil;
  }
  *out = reinterpret_cast<cnn_net*>(net);
  return CNN_OK;
}

extern "C" int cnn_destroy(cnn_net* h) {
  clear_error();
  if (!h) return CNN_OK;
  Net* net = reinterpret_cast<Net*>(h);
  hipDeviceSynchronize();
  for (auto& E : net->layers) free_layer(E);
  if (net->ws) hipFree(net->ws);
  for (Net::Arena& A : net->arena) {
    if (A.tab_dev) hipFree(A.tab_dev);
    if (A.tab_host) hipHostFree(A.tab_host);
    if (A.graph_exec) hipGraphExecDestroy(A.graph_exec);
    if (A.done) hipEventDestroy(A.done);
  }
  if (net->cap_stream) hipStreamDestroy(net->cap_stream);
  for (auto& t : net->timed) {
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
  }
  for (auto ev : net->event_pool) hipEventDestroy(ev);
  delete net;
  return CNN_OK;
}

extern "C" int cnn_geometry(const cnn_net* h, int32_t* R, int32_t* fov) {
  clear_error();
  if (!h) return fail(CNN_EINVAL, "cnn_geometry: null net");
  const Net* net = reinterpret_cast<const Net*>(h);
  if (R) *R = net->R;
  if (fov) *fov = net->R + 1;
  return CNN_OK;
}

extern "C" const char* cnn_last_error(void) { return last_error(); }

extern "C" int cnn_describe(const cnn_net* h, char* buf, int32_t len) {
  clear_error();
  if (!h || !buf || len < 1) return fail(CNN_EINVAL, "cnn_describe: bad argument");
  const Net* net = reinterpret_cast<const Net*>(h);
  std::string s;
  const bool fused = first_fused(net);
  for (size_t l = 0; l < net->layers.size(); ++l) {
    if (!s.empty()) s += " | ";
    s += layer_name(net->layers[l]);
    if (l == 0 && fused) s += " (computed inside layer 1)";
  }
  // per tile class choices of batched submissions (cnn_autotune_batch)
  for (size_t c = 0; c < net->class_variants.size(); ++c) {
    s += c == 0 ? " || batch classes: " : "; ";
    s += std::to_string(tile_class_side((int)c)) + ":";
    for (size_t l = 0; l < net->layers.size(); ++l) {
      const int v = net->class_variants[c][l];
      s += std::string(l ? " " : " ") + (net->layers[l].first ? first_variant(v)->name : conv_variant(v)->name);
    }
  }
  std::snprintf(buf, len, "%s", s.c_str());
  return CNN_OK;
}
