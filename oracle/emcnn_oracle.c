/*
 * emcnn_oracle.c - plain FP64 CPU reference for dense membrane-probability
 * inference (arXiv 1612.02120, Section 2.2).
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library. It shares no code, header, table
 * or helper with the GPU library; it is written from the definitions below and
 * is deliberately slow and direct.
 *
 * What it computes (Section 2.2, "Accelerating dense computation"): the dense
 * output of a convolution / max-filter network, i.e. one membrane probability
 * per input position whose field of view lies inside the image. Max-pooling is
 * replaced by stride-1 max-filtering, which is what makes the output dense.
 *
 *   input      a0[y][x] = V[y][x] / 255                (one channel per slice)
 *   conv k x k a'[co][y][x] = b[co] + sum_ci sum_i<k sum_j<k W[co][ci][i][j] a[ci][y+i][x+j]
 *              (valid cross-correlation; loops ci, i, j ascending)
 *   relu       max(0, t)
 *   pool       m[c][y][x] = max over i, j in {0,1} of a[c][y+i][x+j]   (2x2, stride 1)
 *   sigmoid    1/(1+e^-t) for t >= 0, e^t/(1+e^t) for t < 0; equal to the
 *              two-class softmax whose outputs are interleaved in Section 2.2.
 *
 * Nets with stride-2 max-pools (FastMemb, Section 2.2: 4x4 convs with 32
 * features, 2x2/s2 max-pools, max-out, a two-class output):
 *   dense form (what the GPU computes; "dilation" d starts at 1)
 *     conv       a'[co][y][x] = b[co] + sum_ci,i,j W[co][ci][i][j] a[ci][y+d i][x+d j]
 *     pool, s=2  m[c][y][x] = max over i, j in {0,1} of a[c][y+d i][x+d j]; then d *= 2
 *   max-out      m[c] = max(a[2c], a[2c+1])      (channel pairs, Goodfellow et al.)
 *   softmax      p = e^{z1} / (e^{z0} + e^{z1}), the class-1 (membrane) output
 *   patch form (the definition the dense form must reproduce): the same net on
 *     one field-of-view window with plain stride-1 convs and stride-2 pools,
 *     which leaves a single output (orc_patch).
 *
 * Subsampling (Section 2.2, "A subsampling CNN for 3 nm data": a pool layer
 * of the net is replaced by a subsampling layer, so that the output map has
 * half the input resolution):
 *   patch form   s[c][y][x] = a[c][2y][2x]  (stride 2, window 1)
 *   dense form, pruned (what the GPU computes; the layer must come before any
 *                stride-2 pool): the map itself is subsampled, a := a[::2, ::2],
 *                and the later layers run densely on it; output (y, x) is the
 *                net on the field-of-view window at input (2y, 2x)
 *   dense form, full (orc_forward_full; the reference the pruned form is pinned
 *                to): the subsample keeps every position and doubles the spacing
 *                d like a stride-2 pool without the max, so that output (Y, X)
 *                is the net on the window at input (Y, X) for every Y, X; the
 *                pruned output is its every second sample in each direction.
 *
 * Multi-channel nets (MaskExtend, Section 3, "MaskExtend: sparse segmentation
 * via CNN": twelve input maps, 4x4 max-out convs with 2x2 stride-2 pools, three
 * output classes) take real-valued input maps as they are (orc_forward_maps,
 * orc_patch_maps), and may end in a softmax over several classes keeping
 * class 0 ("softmax0"): p0 = e^{z0} / sum_c e^{zc}.
 *
 * Fake-quant modes mirror the number formats declared by the GPU forms (the
 * paper states no precision; these are readings):
 *   BF16: first conv uses weights bf16((float)(w/255)) against the raw uint8
 *         value; every later conv except the 1x1 head rounds its weights and its
 *         input activations to bf16 (round to nearest even, via float).
 *   FP8:  first conv as BF16; later convs except the head use e4m3fn codes with
 *         a per-output-channel weight scale sw[co] = max|W[co]| / 448 and a
 *         per-layer input scale s: out = b + s * sw[co] * sum q(w/sw) q(a/s),
 *         q = e4m3fn round-to-nearest-even, saturating at +-448.
 *   The head (last layer, 1x1 to one channel) stays exact in both modes.
 *
 * Student training (BCE on teacher probabilities + Adam, Kingma & Ba) is the
 * plain chain rule through the same definitions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_CONV = 0, ORC_POOL = 1, ORC_POOL2 = 2, ORC_SUB2 = 3 };
enum { ORC_ACT_NONE = 0, ORC_ACT_RELU = 1, ORC_ACT_SIGMOID = 2, ORC_ACT_MAXOUT = 3, ORC_ACT_SOFTMAX = 4,
       ORC_ACT_SOFTMAX0 = 5 };
enum { ORC_Q_EXACT = 0, ORC_Q_BF16 = 1, ORC_Q_FP8 = 2 };

typedef struct {
  int32_t kind, k, cin, cout, act;
} orc_layer;

/* ---------------- scalar definitions ---------------- */

double orc_sigmoid(double t) {
  if (t >= 0.0) return 1.0 / (1.0 + exp(-t));
  double e = exp(t);
  return e / (1.0 + e);
}

/* bf16 round-to-nearest-even of the float value of x. */
double orc_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan unchanged */
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

/* e4m3fn (1 sign, 4 exponent bits, bias 7, 3 mantissa bits, no infinities,
 * largest finite 448, smallest subnormal 2^-9), round to nearest even,
 * saturating to +-448. */
double orc_e4m3(double x) {
  if (x != x) return x;
  double s = x < 0 ? -1.0 : 1.0;
  double a = fabs(x);
  if (a >= 448.0) return s * 448.0;
  if (a == 0.0) return 0.0 * s;
  int e;
  frexp(a, &e);          /* a = f * 2^e, f in [0.5, 1): unbiased exponent e-1 */
  int ue = e - 1;
  if (ue < -6) ue = -6;  /* subnormal range shares the quantum of 2^-6 normals */
  double quantum = ldexp(1.0, ue - 3);
  double q = rint(a / quantum) * quantum; /* rint: nearest, ties to even */
  if (q > 448.0) q = 448.0;
  return s * q;
}

void orc_bf16_array(const double* in, double* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = orc_bf16(in[i]);
}

void orc_e4m3_array(const double* in, double* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = orc_e4m3(in[i]);
}

/* ---------------- layer definitions ---------------- */

/* valid cross-correlation with tap spacing D (D = 1: plain) */
static void conv_valid(const double* in, int C, int H, int W, const double* w,
                       const double* b, int K, int Co, int D, double* out) {
  int Ho = H - (K - 1) * D, Wo = W - (K - 1) * D;
#pragma omp parallel for collapse(2) schedule(static)
  for (int co = 0; co < Co; ++co)
    for (int y = 0; y < Ho; ++y)
      for (int x = 0; x < Wo; ++x) {
        double s = b[co];
        for (int ci = 0; ci < C; ++ci)
          for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j)
              s += w[((co * C + ci) * K + i) * K + j] * in[((int64_t)ci * H + y + i * D) * W + x + j * D];
        out[((int64_t)co * Ho + y) * Wo + x] = s;
      }
}

/* 2x2 max filter with element spacing D (stride 1) */
static void pool2(const double* in, int C, int H, int W, int D, double* out) {
  int Ho = H - D, Wo = W - D;
  for (int c = 0; c < C; ++c)
    for (int y = 0; y < Ho; ++y)
      for (int x = 0; x < Wo; ++x) {
        const double* p = in + ((int64_t)c * H + y) * W + x;
        double m = p[0];
        if (p[D] > m) m = p[D];
        if (p[(int64_t)D * W] > m) m = p[(int64_t)D * W];
        if (p[(int64_t)D * W + D] > m) m = p[(int64_t)D * W + D];
        out[((int64_t)c * Ho + y) * Wo + x] = m;
      }
}

/* 2x2 max-pool with stride 2 (patch form): out[c][y][x] = max of in[c][2y+i][2x+j] */
static void pool2_stride2(const double* in, int C, int H, int W, double* out) {
  int Ho = H / 2, Wo = W / 2;
  for (int c = 0; c < C; ++c)
    for (int y = 0; y < Ho; ++y)
      for (int x = 0; x < Wo; ++x) {
        double m = in[((int64_t)c * H + 2 * y) * W + 2 * x];
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) {
            double v = in[((int64_t)c * H + 2 * y + i) * W + 2 * x + j];
            if (v > m) m = v;
          }
        out[((int64_t)c * Ho + y) * Wo + x] = m;
      }
}

/* Activation of a conv output o (Co x n). Returns the channel count after it
 * (max-out halves it, softmax leaves the class-1 probability); -1 if invalid.
 * logit (nullable) receives the pre-activation output of one-channel convs,
 * and z1 - z0 for the two-class softmax (so that sigmoid(logit) = p). */
static int activate(double* o, int Co, int64_t n, int act, double* logit) {
  if (act == ORC_ACT_MAXOUT) {
    if (Co % 2) return -1;
    for (int c = 0; c < Co / 2; ++c)
      for (int64_t i = 0; i < n; ++i) {
        double a = o[(2 * c) * n + i], b = o[(2 * c + 1) * n + i];
        o[c * n + i] = a > b ? a : b;
      }
    return Co / 2;
  }
  if (act == ORC_ACT_SOFTMAX0) {
    /* softmax over the Co classes; the map keeps class 0's probability */
    if (Co < 2) return -1;
    for (int64_t i = 0; i < n; ++i) {
      double m = o[i];
      for (int c = 1; c < Co; ++c)
        if (o[c * n + i] > m) m = o[c * n + i];
      double den = 0.0;
      for (int c = 0; c < Co; ++c) den += exp(o[c * n + i] - m);
      if (logit) logit[i] = o[i];
      o[i] = exp(o[i] - m) / den;
    }
    return 1;
  }
  if (act == ORC_ACT_SOFTMAX) {
    if (Co != 2) return -1;
    for (int64_t i = 0; i < n; ++i) {
      double z0 = o[i], z1 = o[n + i], m = z0 > z1 ? z0 : z1;
      double e0 = exp(z0 - m), e1 = exp(z1 - m);
      if (logit) logit[i] = z1 - z0;
      o[i] = e1 / (e0 + e1);
    }
    return 1;
  }
  if (logit && Co == 1) memcpy(logit, o, sizeof(double) * n);
  for (int64_t i = 0; i < (int64_t)Co * n; ++i) {
    if (act == ORC_ACT_RELU) o[i] = o[i] > 0.0 ? o[i] : 0.0;
    else if (act == ORC_ACT_SIGMOID) o[i] = orc_sigmoid(o[i]);
  }
  return Co;
}

/* Nets with stride-2 pools, max-out or softmax are defined in exact FP64 only. */
static int strided_net(const orc_layer* L, int nl) {
  for (int l = 0; l < nl; ++l)
    if (L[l].kind == ORC_POOL2 || L[l].kind == ORC_SUB2 || L[l].act == ORC_ACT_MAXOUT || L[l].act == ORC_ACT_SOFTMAX ||
        L[l].act == ORC_ACT_SOFTMAX0)
      return 1;
  return 0;
}

static int param_count(const orc_layer* L, int nl) {
  int n = 0;
  for (int l = 0; l < nl; ++l)
    if (L[l].kind == ORC_CONV) n += L[l].cout * L[l].cin * L[l].k * L[l].k + L[l].cout;
  return n;
}

/* Forward pass of one slice.  trace (nullable) receives, for every layer, a
 * pointer to a malloc'd buffer with that layer's output (caller frees); dims
 * of layer l's output are trace_dims[3l..3l+2] = C, H, W. */
/* img: one uint8 slice (input V / 255), or maps (nullable otherwise): C0 x H x
 * W real-valued input maps taken as they are (multi-channel nets). */
static int forward_slice(const uint8_t* img, const double* maps, int C0, int H, int W, const orc_layer* L, int nl,
                         const double* params, int qmode, const double* act_scale,
                         double* out_prob, double* out_logit, double** trace,
                         int32_t* trace_dims, int full) {
  int C = maps ? C0 : 1, h = H, w = W;
  int dil = 1; /* spacing of the dense form; doubled by every stride-2 pool */
  if (qmode != ORC_Q_EXACT && (strided_net(L, nl) || maps)) return -1;
  double* a = (double*)malloc(sizeof(double) * (size_t)C * H * W);
  if (!a) return -2;
  int first = 1;
  if (maps) {
    memcpy(a, maps, sizeof(double) * (size_t)C * H * W);
  } else {
    for (int64_t i = 0; i < (int64_t)H * W; ++i)
      a[i] = (qmode == ORC_Q_EXACT) ? img[i] / 255.0 : (double)img[i];
  }
  const double* p = params;
  int conv_idx = 0;
  for (int l = 0; l < nl; ++l) {
    const orc_layer* ly = &L[l];
    double* o = NULL;
    if (ly->kind == ORC_CONV) {
      int K = ly->k, Co = ly->cout;
      if (ly->cin != C) { free(a); return -1; }
      int nw = Co * C * K * K;
      const double* wt = p;
      const double* bs = p + nw;
      p += nw + Co;
      int Ho = h - (K - 1) * dil, Wo = w - (K - 1) * dil;
      if (Ho < 1 || Wo < 1) { free(a); return -1; }
      int is_head = (l == nl - 1) && K == 1 && Co == 1;
      double* wq = (double*)malloc(sizeof(double) * nw);
      double* aq = NULL;
      double* osc = NULL; /* per-output-channel rescale (FP8) */
      memcpy(wq, wt, sizeof(double) * nw);
      const double* ain = a;
      if (qmode != ORC_Q_EXACT && !is_head) {
        if (first) {
          for (int i = 0; i < nw; ++i) wq[i] = orc_bf16(wt[i] / 255.0);
        } else if (qmode == ORC_Q_BF16) {
          for (int i = 0; i < nw; ++i) wq[i] = orc_bf16(wt[i]);
          aq = (double*)malloc(sizeof(double) * (size_t)C * h * w);
          for (int64_t i = 0; i < (int64_t)C * h * w; ++i) aq[i] = orc_bf16(a[i]);
          ain = aq;
        } else { /* FP8 */
          double s = act_scale[conv_idx];
          osc = (double*)malloc(sizeof(double) * Co);
          int per = C * K * K;
          for (int co = 0; co < Co; ++co) {
            double mx = 0.0;
            for (int i = 0; i < per; ++i) {
              double v = fabs(wt[co * per + i]);
              if (v > mx) mx = v;
            }
            double sw = mx > 0 ? mx / 448.0 : 1.0;
            for (int i = 0; i < per; ++i) wq[co * per + i] = orc_e4m3(wt[co * per + i] / sw);
            osc[co] = s * sw;
          }
          aq = (double*)malloc(sizeof(double) * (size_t)C * h * w);
          for (int64_t i = 0; i < (int64_t)C * h * w; ++i) aq[i] = orc_e4m3(a[i] / s);
          ain = aq;
        }
      } else if (first && qmode != ORC_Q_EXACT) {
        /* exact head on a raw-uint8 input cannot happen for a 1-layer net we use;
           keep the /255 definition */
        for (int i = 0; i < nw; ++i) wq[i] = wt[i] / 255.0;
      }
      o = (double*)malloc(sizeof(double) * (size_t)Co * Ho * Wo);
      if (osc) {
        double* zb = (double*)calloc(Co, sizeof(double));
        conv_valid(ain, C, h, w, wq, zb, K, Co, dil, o);
        free(zb);
        for (int co = 0; co < Co; ++co)
          for (int64_t i = 0; i < (int64_t)Ho * Wo; ++i)
            o[(int64_t)co * Ho * Wo + i] = bs[co] + osc[co] * o[(int64_t)co * Ho * Wo + i];
      } else {
        conv_valid(ain, C, h, w, wq, bs, K, Co, dil, o);
      }
      free(wq);
      free(aq);
      free(osc);
      first = 0;
      ++conv_idx;
      h = Ho;
      w = Wo;
      C = activate(o, Co, (int64_t)h * w, ly->act, l == nl - 1 ? out_logit : NULL);
      if (C < 0) { free(o); free(a); return -1; }
    } else if (ly->kind == ORC_POOL || ly->kind == ORC_POOL2) {
      if (h <= dil || w <= dil) { free(a); return -1; }
      o = (double*)malloc(sizeof(double) * (size_t)C * (h - dil) * (w - dil));
      pool2(a, C, h, w, dil, o);
      h -= dil;
      w -= dil;
      if (ly->kind == ORC_POOL2) dil *= 2;
    } else if (ly->kind == ORC_SUB2 && full) {
      o = (double*)malloc(sizeof(double) * (size_t)C * h * w);
      memcpy(o, a, sizeof(double) * (size_t)C * h * w);
      dil *= 2;
    } else if (ly->kind == ORC_SUB2) {
      if (dil != 1) { free(a); return -1; }
      const int hs = (h + 1) / 2, ws = (w + 1) / 2;
      o = (double*)malloc(sizeof(double) * (size_t)C * hs * ws);
      for (int c = 0; c < C; ++c)
        for (int y = 0; y < hs; ++y)
          for (int x = 0; x < ws; ++x)
            o[((int64_t)c * hs + y) * ws + x] = a[((int64_t)c * h + 2 * y) * w + 2 * x];
      h = hs;
      w = ws;
    } else {
      free(a);
      return -1;
    }
    free(a);
    a = o;
    if (trace) {
      trace[l] = (double*)malloc(sizeof(double) * (size_t)C * h * w);
      memcpy(trace[l], a, sizeof(double) * (size_t)C * h * w);
      trace_dims[3 * l] = C;
      trace_dims[3 * l + 1] = h;
      trace_dims[3 * l + 2] = w;
    }
  }
  if (C != 1) { free(a); return -1; }
  if (out_prob) memcpy(out_prob, a, sizeof(double) * (size_t)h * w);
  free(a);
  return 0;
}

/* Receptive radius R (field of view R + 1): the recursion r += (k - 1) j,
 * j *= s over the layers, with j the input spacing of a layer (a 2x2 pool is
 * k = 2; stride 2 doubles j). */
int orc_radius(const orc_layer* L, int nl) {
  int R = 0, j = 1;
  for (int l = 0; l < nl; ++l) {
    R += (L[l].kind == ORC_CONV ? L[l].k - 1 : L[l].kind == ORC_SUB2 ? 0 : 1) * j;
    if (L[l].kind == ORC_POOL2 || L[l].kind == ORC_SUB2) j *= 2;
  }
  return R;
}

/* Patch form at one position: the net applied to the (R+1) x (R+1) window of
 * img (H x W) with top-left corner (y, x), using plain stride-1 convs and
 * stride-2 pools, as in a sliding-window classifier. out: the single output
 * (probability); logit (nullable): its logit as orc_forward reports it. */
/* Patch form on one field-of-view window at (y, x): of a uint8 slice (img),
 * or of C0 x H x W real-valued maps (maps, when img is NULL). */
static int patch_any(const uint8_t* img, const double* maps, int C0, int H, int W, const orc_layer* L, int nl,
                     const double* params, int y, int x, double* out, double* logit) {
  int F = orc_radius(L, nl) + 1;
  if (y < 0 || x < 0 || y + F > H || x + F > W) return -1;
  int C = img ? 1 : C0, h = F, w = F;
  double* a = (double*)malloc(sizeof(double) * (size_t)C * F * F);
  if (!a) return -2;
  for (int ch = 0; ch < C; ++ch)
    for (int r = 0; r < F; ++r)
      for (int c = 0; c < F; ++c)
        a[((int64_t)ch * F + r) * F + c] = img ? img[(int64_t)(y + r) * W + x + c] / 255.0
                                              : maps[((int64_t)ch * H + y + r) * W + x + c];
  const double* p = params;
  for (int l = 0; l < nl; ++l) {
    const orc_layer* ly = &L[l];
    double* o = NULL;
    if (ly->kind == ORC_CONV) {
      int K = ly->k, Co = ly->cout, nw = Co * C * K * K;
      if (ly->cin != C || h < K || w < K) { free(a); return -1; }
      o = (double*)malloc(sizeof(double) * (size_t)Co * (h - K + 1) * (w - K + 1));
      conv_valid(a, C, h, w, p, p + nw, K, Co, 1, o);
      p += nw + Co;
      h -= K - 1;
      w -= K - 1;
      C = activate(o, Co, (int64_t)h * w, ly->act, l == nl - 1 ? logit : NULL);
      if (C < 0) { free(o); free(a); return -1; }
    } else if (ly->kind == ORC_POOL) {
      if (h < 2 || w < 2) { free(a); return -1; }
      o = (double*)malloc(sizeof(double) * (size_t)C * (h - 1) * (w - 1));
      pool2(a, C, h, w, 1, o);
      h -= 1;
      w -= 1;
    } else if (ly->kind == ORC_POOL2) {
      if (h < 2 || w < 2) { free(a); return -1; }
      o = (double*)malloc(sizeof(double) * (size_t)C * (h / 2) * (w / 2));
      pool2_stride2(a, C, h, w, o);
      h /= 2;
      w /= 2;
    } else if (ly->kind == ORC_SUB2) {
      const int hs = (h + 1) / 2, ws = (w + 1) / 2;
      o = (double*)malloc(sizeof(double) * (size_t)C * hs * ws);
      for (int c = 0; c < C; ++c)
        for (int r = 0; r < hs; ++r)
          for (int q = 0; q < ws; ++q) o[((int64_t)c * hs + r) * ws + q] = a[((int64_t)c * h + 2 * r) * w + 2 * q];
      h = hs;
      w = ws;
    } else {
      free(a);
      return -1;
    }
    free(a);
    a = o;
  }
  int rc = (C == 1 && h == 1 && w == 1) ? 0 : -1;
  if (!rc && out) *out = a[0];
  free(a);
  return rc;
}

int orc_patch(const uint8_t* img, int H, int W, const orc_layer* L, int nl, const double* params,
              int y, int x, double* out, double* logit) {
  return patch_any(img, NULL, 1, H, W, L, nl, params, y, x, out, logit);
}

int orc_patch_maps(const double* maps, int C, int H, int W, const orc_layer* L, int nl, const double* params,
                   int y, int x, double* out) {
  return patch_any(NULL, maps, C, H, W, L, nl, params, y, x, out, NULL);
}

/* vol: Z x H x W uint8; prob (nullable), logit (nullable): Z x (H-R) x (W-R). */
/* Output dims of the dense form for an H x W slice (full: subsampling layers
 * keep every position). Returns 0, or -1 if the net does not fit. */
int orc_out_dims(const orc_layer* L, int nl, int H, int W, int full, int* Ho, int* Wo) {
  int h = H, w = W, dil = 1;
  for (int l = 0; l < nl; ++l) {
    if (L[l].kind == ORC_CONV) {
      h -= (L[l].k - 1) * dil;
      w -= (L[l].k - 1) * dil;
    } else if (L[l].kind == ORC_POOL || L[l].kind == ORC_POOL2) {
      h -= dil;
      w -= dil;
      if (L[l].kind == ORC_POOL2) dil *= 2;
    } else if (L[l].kind == ORC_SUB2) {
      if (full) {
        dil *= 2;
      } else {
        if (dil != 1) return -1;
        h = (h + 1) / 2;
        w = (w + 1) / 2;
      }
    } else {
      return -1;
    }
    if (h < 1 || w < 1) return -1;
  }
  *Ho = h;
  *Wo = w;
  return 0;
}

static int forward_all(const uint8_t* vol, int Z, int H, int W, const orc_layer* L, int nl, const double* params,
                       int qmode, const double* act_scale, double* prob, double* logit, int nthreads, int full) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int Ho = 0, Wo = 0;
  if (orc_out_dims(L, nl, H, W, full, &Ho, &Wo)) return -1;
  for (int z = 0; z < Z; ++z) {
    int rc = forward_slice(vol + (int64_t)z * H * W, NULL, 1, H, W, L, nl, params, qmode, act_scale,
                           prob ? prob + (int64_t)z * Ho * Wo : NULL,
                           logit ? logit + (int64_t)z * Ho * Wo : NULL, NULL, NULL, full);
    if (rc) return rc;
  }
  return 0;
}

/* Dense output of every slice (Z x Ho x Wo, orc_out_dims; H - R for nets
 * without subsampling). */
int orc_forward(const uint8_t* vol, int Z, int H, int W, const orc_layer* L, int nl,
                const double* params, int qmode, const double* act_scale, double* prob,
                double* logit, int nthreads) {
  return forward_all(vol, Z, H, W, L, nl, params, qmode, act_scale, prob, logit, nthreads, 0);
}

/* Dense output of a multi-channel net on real-valued input maps: maps is
 * Z x C x H x W (each slice's C maps, planar), exact FP64; prob Z x Ho x Wo. */
int orc_forward_maps(const double* maps, int Z, int C, int H, int W, const orc_layer* L, int nl, const double* params,
                     double* prob, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int Ho = 0, Wo = 0;
  if (C < 1 || orc_out_dims(L, nl, H, W, 0, &Ho, &Wo)) return -1;
  for (int z = 0; z < Z; ++z) {
    int rc = forward_slice(NULL, maps + (int64_t)z * C * H * W, C, H, W, L, nl, params, ORC_Q_EXACT, NULL,
                           prob + (int64_t)z * Ho * Wo, NULL, NULL, NULL, 0);
    if (rc) return rc;
  }
  return 0;
}

/* The full dense form (subsampling layers keep every position), exact FP64. */
int orc_forward_full(const uint8_t* vol, int Z, int H, int W, const orc_layer* L, int nl, const double* params,
                     double* prob, int nthreads) {
  return forward_all(vol, Z, H, W, L, nl, params, ORC_Q_EXACT, NULL, prob, NULL, nthreads, 1);
}

/* Every layer's output for one slice; bufs[l] must hold dims given by a first
 * call with bufs == NULL (dims only). */
int orc_trace(const uint8_t* img, int H, int W, const orc_layer* L, int nl,
              const double* params, int qmode, const double* act_scale, int32_t* dims, double** bufs) {
  double** tr = (double**)calloc(nl, sizeof(double*));
  int rc = forward_slice(img, NULL, 1, H, W, L, nl, params, qmode, act_scale, NULL, NULL, tr, dims, 0);
  for (int l = 0; l < nl; ++l) {
    if (bufs && tr[l])
      memcpy(bufs[l], tr[l], sizeof(double) * (size_t)dims[3 * l] * dims[3 * l + 1] * dims[3 * l + 2]);
    free(tr[l]);
  }
  free(tr);
  return rc;
}

/* ---------------- student training ---------------- */

/* Mean BCE-with-logits over all outputs of a batch of patches against teacher
 * probabilities, and its gradient w.r.t. every parameter.
 * Net: convs only (no pooling); ReLU on all but the last conv, whose output is
 * the logit z.  L = (1/N) sum softplus(z) - t z, dL/dz = (sigmoid(z) - t) / N.
 * patches: B x P x P uint8; teacher: B x (P-R) x (P-R). grad has the parameter
 * layout (per conv: W[co][ci][i][j], then b[co]). */
int orc_student_loss_grad(const uint8_t* patches, int B, int P, const double* teacher,
                          const orc_layer* L, int nl, const double* params, double* loss,
                          double* grad) {
  for (int l = 0; l < nl; ++l)
    if (L[l].kind != ORC_CONV) return -1;
  int R = orc_radius(L, nl);
  int Po = P - R;
  int64_t N = (int64_t)B * Po * Po;
  int np = param_count(L, nl);
  memset(grad, 0, sizeof(double) * np);
  double total = 0.0;
  /* per-layer geometry */
  int* hs = (int*)malloc(sizeof(int) * (nl + 1));
  int* cs = (int*)malloc(sizeof(int) * (nl + 1));
  int* poff = (int*)malloc(sizeof(int) * nl);
  hs[0] = P;
  cs[0] = 1;
  int off = 0;
  for (int l = 0; l < nl; ++l) {
    if (L[l].cin != cs[l]) { free(hs); free(cs); free(poff); return -1; }
    hs[l + 1] = hs[l] - L[l].k + 1;
    cs[l + 1] = L[l].cout;
    poff[l] = off;
    off += L[l].cout * L[l].cin * L[l].k * L[l].k + L[l].cout;
  }
  double** act = (double**)calloc(nl + 1, sizeof(double*)); /* post-activation */
  double** pre = (double**)calloc(nl + 1, sizeof(double*)); /* pre-activation */
  for (int l = 0; l <= nl; ++l) {
    act[l] = (double*)malloc(sizeof(double) * (size_t)cs[l] * hs[l] * hs[l]);
    pre[l] = (double*)malloc(sizeof(double) * (size_t)cs[l] * hs[l] * hs[l]);
  }
  for (int bi = 0; bi < B; ++bi) {
    const uint8_t* img = patches + (int64_t)bi * P * P;
    for (int64_t i = 0; i < (int64_t)P * P; ++i) act[0][i] = img[i] / 255.0;
    for (int l = 0; l < nl; ++l) {
      const double* wt = params + poff[l];
      const double* bs = wt + L[l].cout * L[l].cin * L[l].k * L[l].k;
      conv_valid(act[l], cs[l], hs[l], hs[l], wt, bs, L[l].k, cs[l + 1], 1, pre[l + 1]);
      int64_t n = (int64_t)cs[l + 1] * hs[l + 1] * hs[l + 1];
      for (int64_t i = 0; i < n; ++i) {
        double v = pre[l + 1][i];
        act[l + 1][i] = (l == nl - 1) ? v : (v > 0.0 ? v : 0.0);
      }
    }
    /* loss and dL/dz at the head */
    const double* t = teacher + (int64_t)bi * Po * Po;
    double* d = (double*)malloc(sizeof(double) * (size_t)Po * Po);
    for (int64_t i = 0; i < (int64_t)Po * Po; ++i) {
      double z = pre[nl][i];
      double sp = (z > 0 ? z : 0.0) + log1p(exp(-fabs(z)));
      total += sp - t[i] * z;
      d[i] = (orc_sigmoid(z) - t[i]) / (double)N;
    }
    /* back through the convs */
    for (int l = nl - 1; l >= 0; --l) {
      int K = L[l].k, Ci = cs[l], Co = cs[l + 1], Hi = hs[l], Ho = hs[l + 1];
      const double* wt = params + poff[l];
      double* gw = grad + poff[l];
      double* gb = gw + Co * Ci * K * K;
      for (int co = 0; co < Co; ++co)
        for (int y = 0; y < Ho; ++y)
          for (int x = 0; x < Ho; ++x) {
            double g = d[((int64_t)co * Ho + y) * Ho + x];
            gb[co] += g;
            for (int ci = 0; ci < Ci; ++ci)
              for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j)
                  gw[((co * Ci + ci) * K + i) * K + j] +=
                      g * act[l][((int64_t)ci * Hi + y + i) * Hi + x + j];
          }
      if (l == 0) { free(d); break; }
      double* dn = (double*)calloc((size_t)Ci * Hi * Hi, sizeof(double));
      for (int co = 0; co < Co; ++co)
        for (int y = 0; y < Ho; ++y)
          for (int x = 0; x < Ho; ++x) {
            double g = d[((int64_t)co * Ho + y) * Ho + x];
            for (int ci = 0; ci < Ci; ++ci)
              for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j)
                  dn[((int64_t)ci * Hi + y + i) * Hi + x + j] += wt[((co * Ci + ci) * K + i) * K + j] * g;
          }
      for (int64_t i = 0; i < (int64_t)Ci * Hi * Hi; ++i)
        if (!(pre[l][i] > 0.0)) dn[i] = 0.0; /* ReLU gradient: 0 where pre-activation <= 0 */
      free(d);
      d = dn;
    }
  }
  *loss = total / (double)N;
  for (int l = 0; l <= nl; ++l) { free(act[l]); free(pre[l]); }
  free(act); free(pre); free(hs); free(cs); free(poff);
  return 0;
}

/* One Adam step (Kingma & Ba) at step count t >= 1. */
/* One inner conv layer of a ReLU net on a given input map, in the number
 * format of a fake-quant mode (the mode's rule for a conv that is neither the
 * first nor the head): in is C x H x W FP64; with pool the 2x2 stride-1 max
 * filter is applied first; then exact: plain FP64; BF16: weights and inputs
 * rounded to bf16; FP8: weights e4m3(w / sw[co]) with sw[co] = max|W[co]| / 448
 * and inputs e4m3(a / in_scale), rescaled by in_scale * sw[co].
 * out (Co x Ho x Wo) receives b[co] + the scaled sum, the conv output before
 * its activation; absum (nullable, same shape) the scaled sum of the absolute
 * products, which bounds the rounding error of any accumulation order.
 * Returns 0, or -1 for bad sizes. */
int orc_conv_layer(const double* in, int C, int H, int W, int pool, const double* wt, const double* bs, int K,
                   int Co, int qmode, double in_scale, double* out, double* absum) {
  const int h = H - (pool ? 1 : 0), w = W - (pool ? 1 : 0);
  const int Ho = h - (K - 1), Wo = w - (K - 1);
  if (C < 1 || Co < 1 || K < 1 || Ho < 1 || Wo < 1 || (qmode == ORC_Q_FP8 && !(in_scale > 0))) return -1;
  const int per = C * K * K, nw = Co * per;
  double* a = (double*)malloc(sizeof(double) * (size_t)C * h * w);
  double* wq = (double*)malloc(sizeof(double) * nw);
  double* osc = (double*)malloc(sizeof(double) * Co);
  double* zb = (double*)calloc(Co, sizeof(double));
  double* tmp = (double*)malloc(sizeof(double) * (size_t)Co * Ho * Wo);
  if (pool) pool2(in, C, H, W, 1, a);
  else memcpy(a, in, sizeof(double) * (size_t)C * h * w);
  for (int co = 0; co < Co; ++co) {
    double sw = 1.0;
    if (qmode == ORC_Q_FP8) {
      double mx = 0.0;
      for (int i = 0; i < per; ++i)
        if (fabs(wt[co * per + i]) > mx) mx = fabs(wt[co * per + i]);
      sw = mx > 0 ? mx / 448.0 : 1.0;
    }
    for (int i = 0; i < per; ++i) {
      const double v = wt[co * per + i];
      wq[co * per + i] = qmode == ORC_Q_FP8 ? orc_e4m3(v / sw) : qmode == ORC_Q_BF16 ? orc_bf16(v) : v;
    }
    osc[co] = qmode == ORC_Q_FP8 ? in_scale * sw : 1.0;
  }
  for (int64_t i = 0; i < (int64_t)C * h * w; ++i)
    a[i] = qmode == ORC_Q_FP8 ? orc_e4m3(a[i] / in_scale) : qmode == ORC_Q_BF16 ? orc_bf16(a[i]) : a[i];
  conv_valid(a, C, h, w, wq, zb, K, Co, 1, tmp);
  for (int co = 0; co < Co; ++co)
    for (int64_t i = 0; i < (int64_t)Ho * Wo; ++i)
      out[(int64_t)co * Ho * Wo + i] = bs[co] + osc[co] * tmp[(int64_t)co * Ho * Wo + i];
  if (absum) {
    for (int i = 0; i < nw; ++i) wq[i] = fabs(wq[i]);
    for (int64_t i = 0; i < (int64_t)C * h * w; ++i) a[i] = fabs(a[i]);
    conv_valid(a, C, h, w, wq, zb, K, Co, 1, tmp);
    for (int co = 0; co < Co; ++co)
      for (int64_t i = 0; i < (int64_t)Ho * Wo; ++i)
        absum[(int64_t)co * Ho * Wo + i] = osc[co] * tmp[(int64_t)co * Ho * Wo + i];
  }
  free(a);
  free(wq);
  free(osc);
  free(zb);
  free(tmp);
  return 0;
}

void orc_adam(double* theta, double* m, double* v, const double* g, int64_t n, int t, double lr,
              double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    theta[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

int orc_num_threads(void) {
#ifdef _OPENMP
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
#else
  return 1;
#endif
}

/* ---------------- 3-D watershed (Section 2.1, over-segmentation) ----------------
 *
 * The stage after the membrane map: a 3-D watershed over the probability map
 * (membranes high, cell interiors low) yields an over-segmentation. The paper
 * names the algorithm only; the reading implemented here is the watershed by
 * steepest descent ("drop of water") with seeded minima, which has one result:
 *   order   u < v iff p[u] < p[v], or p[u] == p[v] and index(u) < index(v),
 *           index = (z H + y) W + x (a total order: ties broken by index)
 *   seeds   S = { v : p[v] < t }; its 6-connected components, each labelled
 *           1 + the least index in it
 *   descent next(v) = v for v in S, else the least (in the order) of v and
 *           its 6-neighbours inside the volume; following next from v ends at
 *           a fixed point r(v) (the order strictly decreases along the way)
 *   label   the label of r(v)'s seed component if r(v) is in S, else
 *           1 + index(r(v)) (a local minimum that is not a seed)
 * p: Z x H x W float32 (finite values), labels: int32 of the same size;
 * Z H W < 2^31 - 1. Returns 0, -1 for bad sizes, -2 if out of memory. */
int orc_watershed(const float* p, int Z, int H, int W, float t, int32_t* label) {
  if (Z < 1 || H < 1 || W < 1 || (int64_t)Z * H * W >= 2147483647LL) return -1;
  const int64_t N = (int64_t)Z * H * W, HW = (int64_t)H * W;
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * N);
  int32_t* next = (int32_t*)malloc(sizeof(int32_t) * N);
  if (!queue || !next) {
    free(queue);
    free(next);
    return -2;
  }
  for (int64_t v = 0; v < N; ++v) label[v] = 0;
  /* seed components, breadth first from each unlabelled seed in index order:
     the start is the least index of its component */
  for (int64_t v0 = 0; v0 < N; ++v0) {
    if (!(p[v0] < t) || label[v0]) continue;
    int64_t head = 0, tail = 0;
    queue[tail++] = (int32_t)v0;
    label[v0] = (int32_t)(v0 + 1);
    while (head < tail) {
      const int64_t v = queue[head++];
      const int z = (int)(v / HW), y = (int)((v / W) % H), x = (int)(v % W);
      const int64_t nb[6] = {z > 0 ? v - HW : -1, z < Z - 1 ? v + HW : -1, y > 0 ? v - W : -1,
                             y < H - 1 ? v + W : -1, x > 0 ? v - 1 : -1, x < W - 1 ? v + 1 : -1};
      for (int k = 0; k < 6; ++k) {
        const int64_t u = nb[k];
        if (u >= 0 && p[u] < t && !label[u]) {
          label[u] = (int32_t)(v0 + 1);
          queue[tail++] = (int32_t)u;
        }
      }
    }
  }
  /* descent pointers */
  for (int64_t v = 0; v < N; ++v) {
    if (p[v] < t) {
      next[v] = (int32_t)v;
      continue;
    }
    const int z = (int)(v / HW), y = (int)((v / W) % H), x = (int)(v % W);
    const int64_t nb[6] = {z > 0 ? v - HW : -1, z < Z - 1 ? v + HW : -1, y > 0 ? v - W : -1,
                           y < H - 1 ? v + W : -1, x > 0 ? v - 1 : -1, x < W - 1 ? v + 1 : -1};
    int64_t best = v;
    for (int k = 0; k < 6; ++k) {
      const int64_t u = nb[k];
      if (u >= 0 && (p[u] < p[best] || (p[u] == p[best] && u < best))) best = u;
    }
    next[v] = (int32_t)best;
  }
  /* roots: follow next to its fixed point; label[] of a resolved voxel is
     final (seeds already hold theirs), so a walk stops at the first one */
  for (int64_t v0 = 0; v0 < N; ++v0) {
    if (label[v0]) continue;
    int64_t n = 0, v = v0;
    while (!label[v] && next[v] != v) {
      queue[n++] = (int32_t)v;
      v = next[v];
    }
    const int32_t lab = label[v] ? label[v] : (int32_t)(v + 1);
    label[v] = lab;
    for (int64_t i = 0; i < n; ++i) label[queue[i]] = lab;
  }
  free(queue);
  free(next);
  return 0;
}
