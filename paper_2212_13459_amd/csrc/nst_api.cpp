// Host side of libnst: descriptor checks, the tile plan, workspace layout, weight
// packing and the two-pass scheduler of Algorithm 1.  Every device step is a kernel
// of kernels.hip; this file only computes integers and enqueues launches.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/nst.h"
#include "kernels.h"

using namespace nst;

namespace {

// ------------------------------------------------------------------ geometry ---------

struct Geom {
  int n_conv;
  int cin[NST_MAX_CONV], cout[NST_MAX_CONV];
  bool pool[NST_MAX_CONV];      // pool after conv i (only for i < top)
  bool pavg[NST_MAX_CONV];      // that pool averages
  int stride[NST_MAX_CONV];     // cumulative stride of conv i's output
  int S;                        // alignment of windows: stride of the deepest used conv
  int n_style;
  int style[NST_MAX_STYLE];
  int style_of[NST_MAX_CONV];   // style index of conv i, or -1
  int content;                  // -1 if none
  int top;                      // deepest conv the energy uses
  int min_halo;
  int rf_a[NST_MAX_CONV], rf_b[NST_MAX_CONV];   // feature q of conv i sees input rows [s q - a, s q + b]
  int step1_halo;               // margin that makes the owned style / content features exact
};

int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
int ceil_div(int a, int b) { return -floor_div(-a, b); }

bool ok_channels(int c) { return c == 64 || (c > 0 && c % 128 == 0); }

int make_geom(const nst_net_desc *d, Geom *g) {
  if (!d || !g) return NST_EINVAL;
  std::memset(g, 0, sizeof(*g));
  if (d->n_conv < 1 || d->n_conv > NST_MAX_CONV) return NST_EINVAL;
  if (d->n_style < 0 || d->n_style > NST_MAX_STYLE) return NST_EINVAL;
  if ((d->pool_avg & ~d->pool_after) != 0u) return NST_EINVAL;
  g->n_conv = d->n_conv;
  g->n_style = d->n_style;
  g->content = d->content_conv;
  for (int i = 0; i < NST_MAX_CONV; ++i) g->style_of[i] = -1;
  int top = -1;
  for (int k = 0; k < d->n_style; ++k) {
    const int i = d->style_conv[k];
    if (i < 0 || i >= d->n_conv) return NST_EINVAL;
    if (k > 0 && i <= d->style_conv[k - 1]) return NST_EINVAL;
    g->style[k] = i;
    g->style_of[i] = k;
    top = std::max(top, i);
  }
  if (g->content < -1 || g->content >= d->n_conv) return NST_EINVAL;
  top = std::max(top, g->content);
  if (top < 0) return NST_EINVAL;
  g->top = top;
  for (int i = 0; i <= top; ++i) {
    g->cin[i] = d->c_in[i];
    g->cout[i] = d->c_out[i];
    if (i == 0 && g->cin[0] != 3) return NST_EINVAL;
    if (i > 0 && g->cin[i] != g->cout[i - 1]) return NST_EINVAL;
    if (!ok_channels(g->cout[i])) return NST_EINVAL;
    g->pool[i] = (i < top) && ((d->pool_after >> i) & 1u);
    g->pavg[i] = g->pool[i] && ((d->pool_avg >> i) & 1u);
    if (g->pool[i] && g->style_of[i] >= 0) return NST_EINVAL;  // style layer before a pool
  }
  int s = 1, a = 0, b = 0, mh = 0;
  for (int i = 0; i <= top; ++i) {
    g->stride[i] = s;
    a += s;
    b += s;
    g->rf_a[i] = a;
    g->rf_b[i] = b;
    mh = std::max(mh, a + b);
    if (g->pool[i]) {
      b += s;
      s *= 2;
    }
  }
  g->S = g->stride[top];
  g->min_halo = mh;
  // Step 1 only needs the owned features of the style and content layers: a feature whose
  // anchor s q lies in [b0, b1) sees [b0 - a, b1 - 1 + b], inside a window of margin max(a, b)
  g->step1_halo = 0;
  for (int k = 0; k < g->n_style; ++k)
    g->step1_halo = std::max(g->step1_halo, std::max(g->rf_a[g->style[k]], g->rf_b[g->style[k]]));
  if (g->content >= 0)
    g->step1_halo = std::max(g->step1_halo, std::max(g->rf_a[g->content], g->rf_b[g->content]));
  return NST_OK;
}

int validate_sizes(int H, int W, int T, int m) {
  if (H < 1 || W < 1 || T < 1 || m < 0) return NST_ESHAPE;
  if ((long long)H * W > (1LL << 29)) return NST_ESHAPE;   // 3 H W floats indexable, < 2^31
  return NST_OK;
}

void plan_axis(int n, int t, int m, int S, std::vector<int> &b0, std::vector<int> &b1,
               std::vector<int> &e0, std::vector<int> &e1) {
  const int cnt = ceil_div(n, t);
  for (int i = 0; i < cnt; ++i) {
    const int lo = i * t, hi = std::min((i + 1) * t, n);
    b0.push_back(lo);
    b1.push_back(hi);
    e0.push_back(std::max(0, S * floor_div(lo - m, S)));
    e1.push_back(std::min(n, S * ceil_div(hi + m, S)));
  }
}

void build_plan(const Geom &g, int H, int W, int T, int m, std::vector<nst_tile> &out) {
  std::vector<int> rb0, rb1, re0, re1, cb0, cb1, ce0, ce1;
  plan_axis(H, T, m, g.S, rb0, rb1, re0, re1);
  plan_axis(W, T, m, g.S, cb0, cb1, ce0, ce1);
  out.clear();
  for (size_t i = 0; i < rb0.size(); ++i)
    for (size_t j = 0; j < cb0.size(); ++j) {
      nst_tile t;
      std::memset(&t, 0, sizeof(t));
      t.by0 = rb0[i];
      t.by1 = rb1[i];
      t.bx0 = cb0[j];
      t.bx1 = cb1[j];
      t.ey0 = re0[i];
      t.ey1 = re1[i];
      t.ex0 = ce0[j];
      t.ex1 = ce1[j];
      for (int k = 0; k < g.n_conv && k < NST_MAX_CONV; ++k) {
        const int s = k <= g.top ? g.stride[k] : g.stride[g.top];
        const int nh = H / s, nw = W / s;
        t.own[k][0] = std::min(ceil_div(t.by0, s), nh);
        t.own[k][1] = std::min(ceil_div(t.by1, s), nh);
        t.own[k][2] = std::min(ceil_div(t.bx0, s), nw);
        t.own[k][3] = std::min(ceil_div(t.bx1, s), nw);
      }
      out.push_back(t);
    }
}

// ------------------------------------------------------------- workspace ----------

constexpr size_t kAlign = 256;
size_t al(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  int batch = 0;                // tiles per launch
  int nslots = 0;               // tile slots (batch, or every tile of the plan)
  size_t total = 0;
  int hmax = 0, wmax = 0;
  int lh[NST_MAX_CONV] = {}, lw[NST_MAX_CONV] = {};
  int gchunks[NST_MAX_STYLE] = {};
  int cblocks = 0;
  size_t es = 4;
  // global region
  size_t g_gacc = 0, g_dt = 0, g_estyle = 0, g_ec = 0, g_energy = 0, g_tilesum = 0, g_flag = 0;
  size_t g_csum = 0, g_msb = 0;  // channel sums (FP64) and mean/std seed constants (FP32)
  long long total_cc = 0;       // sum over style layers of C_l^2
  long long total_c = 0;        // sum over style layers of C_l
  long long moff[NST_MAX_STYLE] = {};
  long long off_c[NST_MAX_STYLE] = {}, dt_off[NST_MAX_STYLE] = {};
  size_t slots = 0, slot_bytes = 0;
  // per-slot offsets
  size_t s_act[NST_MAX_CONV] = {}, s_pool[NST_MAX_CONV] = {};
  size_t s_d0 = 0, s_d1 = 0, s_rc = 0, s_cpart = 0;
  size_t s_gpart[NST_MAX_STYLE] = {};
  size_t s_mpart[NST_MAX_STYLE] = {};
};

// Element offsets are 64-bit everywhere; the 32-bit quantity is a launch's work-item
// count, at most (window pixels of a layer) x (channels / 4) 16-byte vectors.
int max_window_ok(const Geom &g, const Layout &L) {
  for (int i = 0; i <= g.top; ++i) {
    const long long e = (long long)L.lh[i] * L.lw[i] * (std::max(g.cout[i], g.cin[i]) / 4 + 1);
    if (e >= (1LL << 31)) return NST_ESHAPE;
  }
  return NST_OK;
}

// Layout for a launch batch and a number of tile slots (the batch, or every tile of the
// plan so that activations stay resident from Step 1 to Step 2).  Independent of which
// entry point runs so that one workspace size serves every call on the same (H, W, T, m).
void make_layout(const Geom &g, int precision, const std::vector<nst_tile> &tiles, int batch,
                 int nslots, Layout &L) {
  L = Layout();
  L.batch = batch;
  L.nslots = nslots;
  L.es = elem_size(precision);
  for (const nst_tile &t : tiles) {
    L.hmax = std::max(L.hmax, t.ey1 - t.ey0);
    L.wmax = std::max(L.wmax, t.ex1 - t.ex0);
  }
  for (int i = 0; i <= g.top; ++i) {
    L.lh[i] = L.hmax / g.stride[i];
    L.lw[i] = L.wmax / g.stride[i];
  }
  for (int k = 0; k < g.n_style; ++k) {
    const int i = g.style[k];
    int mx = 0;
    for (const nst_tile &t : tiles) {
      const long long npx = (long long)(t.own[i][1] - t.own[i][0]) * (t.own[i][3] - t.own[i][2]);
      mx = std::max(mx, (int)((npx + kGramChunk - 1) / kGramChunk));
    }
    L.gchunks[k] = mx;
  }
  if (g.content >= 0) {
    const int i = g.content;
    int mx = 0;
    for (const nst_tile &t : tiles) {
      const long long npx = (long long)(t.own[i][1] - t.own[i][0]) * (t.own[i][3] - t.own[i][2]);
      mx = std::max(mx, (int)((npx + kContentBlockPx - 1) / kContentBlockPx));
    }
    L.cblocks = mx;
  }
  // global region
  size_t off = 0;
  long long cc = 0, maxcc = 0;
  for (int k = 0; k < g.n_style; ++k) {
    const int C = g.cout[g.style[k]];
    L.off_c[k] = cc;
    L.dt_off[k] = cc;
    cc += (long long)C * C;
    maxcc = std::max(maxcc, (long long)C * C);
  }
  L.g_gacc = off;
  off = al(off + cc * 8);
  L.g_dt = off;
  off = al(off + cc * L.es);
  L.g_estyle = off;
  off = al(off + NST_MAX_STYLE * 8);
  L.g_ec = off;
  off = al(off + 8);
  L.g_energy = off;
  off = al(off + (2 + NST_MAX_STYLE) * 8);
  L.g_tilesum = off;
  off = al(off + (size_t)batch * maxcc * 8);
  L.g_flag = off;
  off = al(off + 8);
  L.total_cc = cc;
  long long csz = 0;
  for (int k = 0; k < g.n_style; ++k) {
    L.moff[k] = csz;
    csz += g.cout[g.style[k]];
  }
  L.total_c = csz;
  L.g_csum = off;
  off = al(off + csz * 8);
  L.g_msb = off;
  off = al(off + csz * 4);
  L.slots = off;
  // per slot
  size_t so = 0, dmax = 0;
  for (int i = 0; i <= g.top; ++i) {
    L.s_act[i] = so;
    so = al(so + (size_t)L.lh[i] * L.lw[i] * g.cout[i] * L.es);
    if (g.pool[i]) {
      L.s_pool[i] = so;
      so = al(so + (size_t)(L.lh[i] / 2) * (L.lw[i] / 2) * g.cout[i] * L.es);
    }
    dmax = std::max(dmax, (size_t)L.lh[i] * L.lw[i] * std::max(g.cout[i], g.cin[i]) * L.es);
  }
  L.s_d0 = so;
  so = al(so + dmax);
  L.s_d1 = so;
  so = al(so + dmax);
  if (g.content >= 0) {
    const int i = g.content;
    L.s_rc = so;
    so = al(so + (size_t)L.lh[i] * L.lw[i] * g.cout[i] * 4);
    L.s_cpart = so;
    so = al(so + (size_t)L.cblocks * 8);
  }
  for (int k = 0; k < g.n_style; ++k) {
    const int C = g.cout[g.style[k]];
    L.s_gpart[k] = so;
    so = al(so + (size_t)L.gchunks[k] * C * C * 4);
    L.s_mpart[k] = so;
    so = al(so + (size_t)L.gchunks[k] * C * 4);
  }
  L.slot_bytes = so;
  L.total = L.slots + (size_t)nslots * L.slot_bytes;
}

// Launch batch when every tile has a slot: the fewest launches of at most kMaxBatch
// tiles, evenly filled.
int balanced_batch(int nt) {
  const int nb = (nt + kMaxBatch - 1) / kMaxBatch;
  return (nt + nb - 1) / nb;
}

// -------------------------------------------------------------- bf16 pack ----------

uint16_t f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

}  // namespace

// ---------------------------------------------------------------------- ctx ----------

struct ProfRec {
  std::string name;
  double flops, bytes;
  hipEvent_t e0, e1;
};

struct nst_ctx {
  Geom g;
  bool prof_on = false;
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> ev_pool;
  int prec = 0;
  int device = 0;
  void *wf[NST_MAX_CONV] = {};   // forward B operand
  void *wd[NST_MAX_CONV] = {};   // data-gradient B operand
  float *bias[NST_MAX_CONV] = {};
  int padf[NST_MAX_CONV] = {};   // padded N of wf
  int padd[NST_MAX_CONV] = {};   // padded N of wd
};

namespace {

// Pack a float matrix B[k][n] given by a functor into [k/CK][tap][npad][CK] (k = (tap, kc)).
template <typename F>
std::vector<float> pack(int nk, int ntap, int npad, int CK, F val) {
  std::vector<float> p((size_t)nk * ntap * npad, 0.f);
  for (int kc = 0; kc < nk; kc += CK)
    for (int tap = 0; tap < ntap; ++tap)
      for (int n = 0; n < npad; ++n)
        for (int kk = 0; kk < CK && kc + kk < nk; ++kk)
          p[(((size_t)(kc / CK) * ntap + tap) * npad + n) * CK + kk] = val(kc + kk, tap, n);
  return p;
}

int upload(const std::vector<float> &v, int prec, void **out) {
  const size_t n = v.size();
  void *d = nullptr;
  if (prec == NST_BF16) {
    std::vector<uint16_t> b(n);
    for (size_t i = 0; i < n; ++i) b[i] = f2bf(v[i]);
    if (hipMalloc(&d, n * 2) != hipSuccess) return NST_ENOMEM;
    if (hipMemcpy(d, b.data(), n * 2, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d);
      return NST_EHIP;
    }
  } else {
    if (hipMalloc(&d, n * 4) != hipSuccess) return NST_ENOMEM;
    if (hipMemcpy(d, v.data(), n * 4, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d);
      return NST_EHIP;
    }
  }
  *out = d;
  return NST_OK;
}

int bn_of(int cout) { return cout <= 64 ? 64 : 128; }

}  // namespace

extern "C" {

int nst_abi_version(void) { return NST_ABI_VERSION; }

const char *nst_strerror(int st) {
  switch (st) {
    case NST_OK: return "ok";
    case NST_EINVAL: return "invalid argument or unsupported network descriptor";
    case NST_ESHAPE: return "invalid image / tile / margin size";
    case NST_EHALO: return "margin smaller than the receptive field (strict mode)";
    case NST_ENOMEM: return "device allocation failed";
    case NST_EHIP: return "HIP runtime error";
    case NST_ECAPACITY: return "output array too small";
    case NST_EWORKSPACE: return "workspace too small";
    case NST_ENONFINITE: return "non-finite value in an input";
    default: return "unknown status";
  }
}

int nst_net_vgg19(nst_net_desc *out, int tiny, int with_content) {
  if (!out) return NST_EINVAL;
  static const int ch[13][2] = {{3, 64},    {64, 64},   {64, 128},  {128, 128}, {128, 256},
                                {256, 256}, {256, 256}, {256, 256}, {256, 512}, {512, 512},
                                {512, 512}, {512, 512}, {512, 512}};
  std::memset(out, 0, sizeof(*out));
  out->n_conv = tiny ? 5 : 13;
  for (int i = 0; i < out->n_conv; ++i) {
    out->c_in[i] = ch[i][0];
    out->c_out[i] = ch[i][1];
  }
  if (tiny) {
    out->pool_after = (1u << 1) | (1u << 3);
    out->n_style = 3;
    out->style_conv[0] = 0;
    out->style_conv[1] = 2;
    out->style_conv[2] = 4;
    out->content_conv = with_content ? 3 : -1;
  } else {
    out->pool_after = (1u << 1) | (1u << 3) | (1u << 7) | (1u << 11);
    out->n_style = 5;
    const int st[5] = {0, 2, 4, 8, 12};
    for (int k = 0; k < 5; ++k) out->style_conv[k] = st[k];
    out->content_conv = with_content ? 9 : -1;
  }
  return NST_OK;
}

int nst_min_halo(const nst_net_desc *net) {
  Geom g;
  const int st = make_geom(net, &g);
  return st != NST_OK ? st : g.min_halo;
}

int nst_plan(const nst_net_desc *net, int H, int W, int T, int m, nst_tile *out, int cap,
             int *n_tiles) {
  Geom g;
  int st = make_geom(net, &g);
  if (st != NST_OK) return st;
  if (!n_tiles || cap < 0 || (cap > 0 && !out)) return NST_EINVAL;
  if ((st = validate_sizes(H, W, T, m)) != NST_OK) return st;
  std::vector<nst_tile> tiles;
  build_plan(g, H, W, T, m, tiles);
  *n_tiles = (int)tiles.size();
  const int k = std::min(cap, (int)tiles.size());
  if (k > 0) std::memcpy(out, tiles.data(), sizeof(nst_tile) * k);
  return cap < (int)tiles.size() ? NST_ECAPACITY : NST_OK;
}

int nst_workspace_bytes(const nst_net_desc *net, int precision, int H, int W, int T, int m,
                        int tile_batch, size_t *bytes) {
  Geom g;
  int st = make_geom(net, &g);
  if (st != NST_OK) return st;
  if (!bytes || (precision != NST_FP32 && precision != NST_BF16)) return NST_EINVAL;
  if ((st = validate_sizes(H, W, T, m)) != NST_OK) return st;
  if (tile_batch < 1) return NST_EINVAL;
  std::vector<nst_tile> tiles;
  build_plan(g, H, W, T, m, tiles);
  const int nt = (int)tiles.size();
  Layout L;
  if (tile_batch >= nt)
    make_layout(g, precision, tiles, balanced_batch(nt), nt, L);
  else {
    const int b = std::min(tile_batch, kMaxBatch);
    make_layout(g, precision, tiles, b, b, L);
  }
  if ((st = max_window_ok(g, L)) != NST_OK) return st;
  *bytes = L.total;
  return NST_OK;
}

int nst_create(const nst_net_desc *net, const float *const *w, const float *const *b,
               int precision, nst_ctx **out) {
  if (!out || !w) return NST_EINVAL;
  *out = nullptr;
  if (precision != NST_FP32 && precision != NST_BF16) return NST_EINVAL;
  Geom g;
  int st = make_geom(net, &g);
  if (st != NST_OK) return st;
  for (int i = 0; i <= g.top; ++i)
    if (!w[i]) return NST_EINVAL;
  nst_ctx *c = new (std::nothrow) nst_ctx();
  if (!c) return NST_ENOMEM;
  c->g = g;
  c->prec = precision;
  if (hipGetDevice(&c->device) != hipSuccess || scratch_init(c->device) != hipSuccess) {
    delete c;
    return NST_EHIP;
  }
  const int CK = ck_of(precision);
  for (int i = 0; i <= g.top && st == NST_OK; ++i) {
    const float *W = w[i];
    const int ci = g.cin[i], co = g.cout[i];
    // forward operand B[k = (tap, c)][n = o] = W[o][c][ky][kx]
    if (i == 0) {
      c->padf[i] = bn_of(co);
      auto p = pack(32, 1, c->padf[i], CK, [&](int k, int, int n) -> float {
        if (k >= 27 || n >= co) return 0.f;
        const int tap = k / 3, cc = k % 3;
        return W[((size_t)n * ci + cc) * 9 + tap];
      });
      st = upload(p, precision, &c->wf[i]);
    } else {
      c->padf[i] = co;
      auto p = pack(ci, 9, co, CK, [&](int k, int tap, int n) -> float {
        return W[((size_t)n * ci + k) * 9 + tap];
      });
      st = upload(p, precision, &c->wf[i]);
    }
    if (st != NST_OK) break;
    // data-gradient operand B[k = (tap', o)][n = c] = W[o][c][2 - ky'][2 - kx']
    c->padd[i] = (i == 0) ? 32 : ci;
    auto pd = pack(co, 9, c->padd[i], CK, [&](int k, int tap, int n) -> float {
      if (n >= ci) return 0.f;
      return W[((size_t)k * ci + n) * 9 + (8 - tap)];
    });
    st = upload(pd, precision, &c->wd[i]);
    if (st != NST_OK) break;
    std::vector<float> bb(co, 0.f);
    if (b && b[i]) std::memcpy(bb.data(), b[i], sizeof(float) * co);
    void *dbias = nullptr;
    st = upload(bb, NST_FP32, &dbias);
    c->bias[i] = (float *)dbias;
  }
  if (st != NST_OK) {
    nst_destroy(c);
    return st;
  }
  *out = c;
  return NST_OK;
}

void nst_destroy(nst_ctx *c) {
  if (!c) return;
  for (ProfRec &r : c->prof) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (int i = 0; i < NST_MAX_CONV; ++i) {
    if (c->wf[i]) (void)hipFree(c->wf[i]);
    if (c->wd[i]) (void)hipFree(c->wd[i]);
    if (c->bias[i]) (void)hipFree(c->bias[i]);
  }
  delete c;
}

}  // extern "C"

// ------------------------------------------------------------------ runner ----------

namespace {

#define HIPCHK(x)                        \
  do {                                   \
    if ((x) != hipSuccess) return NST_EHIP; \
  } while (0)

using Reg = std::array<int, 4>;

struct Runner {
  nst_ctx *c;
  const Geom &g;
  Layout L;
  bool retain = false;          // every tile has its own slot (activations stay resident)
  std::vector<nst_tile> tiles;  // the plan the calls' windows come from
  int m = 0;                    // the caller's margin (the layout is sized for its plan)
  char *ws;
  hipStream_t s;
  int H, W;

  Runner(nst_ctx *ctx) : c(ctx), g(ctx->g) {}

  hipEvent_t get_event() {
    if (!c->ev_pool.empty()) {
      hipEvent_t e = c->ev_pool.back();
      c->ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  // Enqueue `launch` bracketed by events when profiling is on.
  template <typename F>
  hipError_t prof(const char *name, double flops, double bytes, F &&launch) {
    if (!c->prof_on) return launch();
    ProfRec r{name, flops, bytes, get_event(), get_event()};
    if (!r.e0 || !r.e1) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(r.e0, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(r.e1, s);
    c->prof.push_back(r);
    return e;
  }
  hipError_t conv(int in_mode, int epi, const ConvArgs &a, const Batch &b) {
    double px = 0;
    for (int k = 0; k < b.n; ++k)
      px += (double)std::max(b.a1[k] - b.a0[k], 0) * std::max(b.a3[k] - b.a2[k], 0);
    const double es = (double)L.es;
    double mac, in_b;
    if (in_mode == IN_IMAGE) {
      mac = 27.0;
      in_b = 12.0;
    } else {
      mac = (in_mode == IN_NHWC ? 9.0 * a.cin : 0.0) + (a.in2 ? (double)a.cin2 : 0.0);
      in_b = ((in_mode == IN_NHWC ? a.cin : 0) + (a.in2 ? a.cin2 : 0)) * es;
    }
    const double cout = epi == EPI_STITCH ? 3.0 : (double)a.cout;
    double out_b = epi == EPI_STITCH ? 12.0 : (a.out ? cout * es : 0.0);
    if (a.pool) out_b += 0.25 * cout * es;
    if (a.mask) out_b += cout * es;
    if (a.rc) out_b += cout * 4.0;
    return prof(conv_kernel_name(c->prec, in_mode, epi, a), 2.0 * px * cout * mac,
                px * (in_b + out_b), [&] { return launch_conv(c->prec, in_mode, epi, a, b, s); });
  }

  template <typename T> T *gl(size_t off) const { return (T *)(ws + off); }
  char *slot_base(size_t off) const { return ws + L.slots + off; }
  long long ss(size_t es) const { return (long long)(L.slot_bytes / es); }
  int lh(const nst_tile &t, int i) const { return (t.ey1 - t.ey0) / g.stride[i]; }
  int lw(const nst_tile &t, int i) const { return (t.ex1 - t.ex0) / g.stride[i]; }

  // Batch with window dims/origin of layer i and owned region of layer i.
  Batch base_batch(int first, int n, int i) const {
    Batch b;
    std::memset(&b, 0, sizeof(b));
    b.n = n;
    for (int k = 0; k < n; ++k) {
      const nst_tile &t = tiles[first + k];
      const int s = g.stride[i];
      b.h[k] = lh(t, i);
      b.w[k] = lw(t, i);
      b.gy[k] = t.ey0 / s;
      b.gx[k] = t.ex0 / s;
      b.a0[k] = t.own[i][0] - b.gy[k];
      b.a1[k] = t.own[i][1] - b.gy[k];
      b.a2[k] = t.own[i][2] - b.gx[k];
      b.a3[k] = t.own[i][3] - b.gx[k];
      b.slot[k] = retain ? first + k : k;
    }
    return b;
  }
  static int region_px(const Batch &b, int k) {
    const int r = b.a1[k] - b.a0[k], cc = b.a3[k] - b.a2[k];
    return (r > 0 && cc > 0) ? r * cc : 0;
  }
  void conv_pfx(Batch &b, int in_mode, int epi, int cout) const {
    const int ph = conv_block_rows(c->prec, in_mode, epi, cout);
    const int pw = conv_block_cols(c->prec, in_mode, epi, cout);
    b.pfx[0] = 0;
    for (int k = 0; k < b.n; ++k) {
      // every convolution covers its output region a0..a3 (the image-gradient stitch: the
      // tile's owned pixels; the others: the part of the window the pass needs)
      const int rh = b.a1[k] - b.a0[k];
      const int rw = b.a3[k] - b.a2[k];
      b.pfx[k + 1] = b.pfx[k] + ((std::max(rh, 0) + ph - 1) / ph) * ((std::max(rw, 0) + pw - 1) / pw);
    }
  }
  // Plan with a margin of its own (same blocks, windows no larger than the layout's).
  void replan(int margin) { build_plan(g, H, W, T, std::min(m, margin), tiles); }
  int T = 0;
  void items_pfx(Batch &b, const std::vector<long long> &items, int per_block) const {
    b.pfx[0] = 0;
    for (int k = 0; k < b.n; ++k)
      b.pfx[k + 1] = b.pfx[k] + (int)((items[k] + per_block - 1) / per_block);
  }

  const void *layer_input(int i) const {
    return g.pool[i - 1] ? (const void *)slot_base(L.s_pool[i - 1])
                         : (const void *)slot_base(L.s_act[i - 1]);
  }

  // keep_pooled: also store the full-resolution output of layers that are pooled (the
  // backward needs them; a forward-only pass needs just the pooled maps)
  // regions: per tile k and conv i (index k (top + 1) + i), the output region to compute
  // (window-local rows r0..r1, columns c0..c1 at conv i's resolution)
  int forward(int first, int n, int upto, const float *img, const float *fc, bool keep_pooled,
              const std::vector<Reg> &regions) {
    const size_t es = L.es;
    for (int i = 0; i <= upto; ++i) {
      Batch b = base_batch(first, n, i);
      for (int k = 0; k < n; ++k) {
        const Reg &r = regions[(size_t)k * (g.top + 1) + i];
        b.a0[k] = r[0], b.a1[k] = r[1], b.a2[k] = r[2], b.a3[k] = r[3];
      }
      ConvArgs a;
      std::memset(&a, 0, sizeof(a));
      int in_mode = IN_NHWC;
      if (i == 0) {
        in_mode = IN_IMAGE;
        a.img = img;
        a.img_h = H;
        a.img_w = W;
      } else {
        a.in = layer_input(i);
        a.in_ss = ss(es);
        a.cin = g.cin[i];
      }
      a.wp = c->wf[i];
      a.cout = g.cout[i];
      a.cout_pad = c->padf[i];
      a.bias = c->bias[i];
      a.out = slot_base(L.s_act[i]);
      a.out_ss = ss(es);
      const bool pooled = g.pool[i] && i < upto;
      if (pooled) {
        a.pool = slot_base(L.s_pool[i]);
        a.pool_ss = ss(es);
        a.pool_avg = g.pavg[i] ? 1 : 0;
        if (!keep_pooled) a.out = nullptr;
      }
      if (i == g.content && fc) {
        a.rc = (float *)slot_base(L.s_rc);
        a.rc_ss = ss(4);
        a.fc = fc;
        a.fc_w = W / g.stride[i];
      }
      conv_pfx(b, in_mode, EPI_FWD, a.cout);
      HIPCHK(conv(in_mode, EPI_FWD, a, b));
    }
    return NST_OK;
  }

  // Needed regions of Step 2's data gradients: dE/dZ_i is needed on R_i.  The block's
  // image gradient reads dZ_0 on the block +- 1; dZ_{i-1} on R comes from the data
  // gradient of conv i on R (through a pool: rows r0 / 2 .. (r1 + 1) / 2), which reads
  // dZ_i one pixel further out.  Clipped to the window.
  void backward_regions(int first, int n, std::vector<Reg> &reg) const {
    const int top = g.top;
    reg.assign((size_t)n * (top + 1), Reg{0, 0, 0, 0});
    for (int k = 0; k < n; ++k) {
      const nst_tile &t = tiles[first + k];
      int r0 = t.by0 - t.ey0 - 1, r1 = t.by1 - t.ey0 + 1, c0 = t.bx0 - t.ex0 - 1, c1 = t.bx1 - t.ex0 + 1;
      for (int i = 0; i <= top; ++i) {
        if (i > 0) {
          if (g.pool[i - 1]) {
            r0 = (r0 >> 1) - 1, r1 = ((r1 + 1) >> 1) + 1, c0 = (c0 >> 1) - 1, c1 = ((c1 + 1) >> 1) + 1;
          } else {
            --r0, ++r1, --c0, ++c1;
          }
        }
        r0 = std::max(r0, 0), r1 = std::min(r1, lh(t, i));
        c0 = std::max(c0, 0), c1 = std::min(c1, lw(t, i));
        reg[(size_t)k * (top + 1) + i] = {r0, r1, c0, c1};
      }
    }
  }

  // Regions a forward pass must compute so that the activations of every conv i are
  // exact on seed[i] (per tile and conv; an empty seed asks for nothing): conv i + 1 reads
  // conv i's output one pixel around its own region, through a pool the two rows and
  // columns under each pooled one.  Pooled layers start on even rows and columns (the
  // pooling windows of the whole image).  Clipped to the window.
  void forward_regions(int first, int n, int upto, const std::vector<Reg> &seed,
                       std::vector<Reg> &reg) const {
    const int top = g.top;
    reg.assign((size_t)n * (top + 1), Reg{0, 0, 0, 0});
    for (int k = 0; k < n; ++k) {
      const nst_tile &t = tiles[first + k];
      int r0 = 0, r1 = 0, c0 = 0, c1 = 0;   // empty
      for (int i = upto; i >= 0; --i) {
        if (i < upto && r1 > r0 && c1 > c0) {
          if (g.pool[i]) {
            r0 = 2 * (r0 - 1), r1 = 2 * (r1 + 1), c0 = 2 * (c0 - 1), c1 = 2 * (c1 + 1);
          } else {
            --r0, ++r1, --c0, ++c1;
          }
        }
        const Reg &s = seed[(size_t)k * (top + 1) + i];
        if (s[1] > s[0] && s[3] > s[2]) {
          if (r1 > r0 && c1 > c0) {
            r0 = std::min(r0, s[0]), r1 = std::max(r1, s[1]), c0 = std::min(c0, s[2]), c1 = std::max(c1, s[3]);
          } else {
            r0 = s[0], r1 = s[1], c0 = s[2], c1 = s[3];
          }
        }
        r0 = std::max(r0, 0), r1 = std::min(r1, lh(t, i));
        c0 = std::max(c0, 0), c1 = std::min(c1, lw(t, i));
        if (g.pool[i] && i < upto) r0 &= ~1, c0 &= ~1;
        reg[(size_t)k * (top + 1) + i] = {r0, r1, c0, c1};
      }
    }
  }

  // Forward regions of a pass that needs the owned features of the layers in `layers`
  // (Step 1: style and content layers; nst_layer_feats: one layer).
  void owned_forward_regions(int first, int n, int upto, const bool *layers, std::vector<Reg> &reg) const {
    std::vector<Reg> seed((size_t)n * (g.top + 1), Reg{0, 0, 0, 0});
    for (int k = 0; k < n; ++k) {
      const nst_tile &t = tiles[first + k];
      for (int i = 0; i <= upto; ++i)
        if (layers[i]) {
          const int s = g.stride[i], oy = t.ey0 / s, ox = t.ex0 / s;
          seed[(size_t)k * (g.top + 1) + i] = {t.own[i][0] - oy, t.own[i][1] - oy, t.own[i][2] - ox, t.own[i][3] - ox};
        }
    }
    forward_regions(first, n, upto, seed, reg);
  }

  // Grams of the owned features (and, with means, their channel sums) of tiles first..+n
  int grams(int first, int n, bool means) {
    for (int k = 0; k < g.n_style; ++k) {
      const int i = g.style[k], C = g.cout[i];
      Batch b = base_batch(first, n, i);
      std::vector<long long> items(n);
      for (int t = 0; t < n; ++t) items[t] = region_px(b, t);
      items_pfx(b, items, kGramChunk);
      float *part = (float *)slot_base(L.s_gpart[k]);
      double npx = 0;
      for (int t = 0; t < n; ++t) npx += (double)items[t];
      HIPCHK(prof(c->prec == 1 ? (C >= 128 ? "void nst::k_gram_bf16<128>(__bf16 const*, long long, int, nst::Batch, float*, long long)"
                                           : "void nst::k_gram_bf16<64>(__bf16 const*, long long, int, nst::Batch, float*, long long)")
                               : "void nst::k_gram<float>(float const*, long long, int, nst::Batch, float*, long long)",
                  2.0 * npx * C * C, npx * C * L.es, [&] {
                    return launch_gram(c->prec, slot_base(L.s_act[i]), ss(L.es), C, b, part, ss(4), s);
                  }));
      HIPCHK(launch_gram_tile_reduce(part, ss(4), C, b, gl<double>(L.g_tilesum), s));
      HIPCHK(launch_gram_accum(gl<double>(L.g_tilesum), n, C,
                               gl<double>(L.g_gacc) + L.off_c[k], s));
      if (means)
        HIPCHK(prof(c->prec == 1 ? "void nst::k_chan_partial<__bf16>(__bf16 const*, long long, int, nst::Batch, float*, long long)"
                                 : "void nst::k_chan_partial<float>(float const*, long long, int, nst::Batch, float*, long long)",
                    0.0, npx * C * L.es, [&] {
                      return launch_chan_sums(c->prec, slot_base(L.s_act[i]), ss(L.es), C, b,
                                              (float *)slot_base(L.s_mpart[k]), ss(4),
                                              gl<double>(L.g_csum) + L.moff[k], s);
                    }));
    }
    return NST_OK;
  }

  int content_energy(int first, int n) {
    const int i = g.content, C = g.cout[i];
    Batch b = base_batch(first, n, i);
    std::vector<long long> items(n);
    for (int t = 0; t < n; ++t) items[t] = region_px(b, t);
    items_pfx(b, items, kContentBlockPx);
    double *part = (double *)slot_base(L.s_cpart);
    HIPCHK(launch_content_partial((const float *)slot_base(L.s_rc), ss(4), C, b, part, ss(8), s));
    HIPCHK(launch_content_accum(part, ss(8), b, gl<double>(L.g_ec), s));
    return NST_OK;
  }

  int backward(int first, int n, float two_alpha, bool use_content, bool use_ms, float *grad) {
    const size_t es = L.es;
    const int vec = (int)(16 / es);
    char *cur = slot_base(L.s_d0), *oth = slot_base(L.s_d1);
    const int top = g.top;
    // Needed regions of dE/dZ_i (backward_regions); everything the block's gradient
    // depends on is computed exactly as over the whole window.
    std::vector<Reg> reg;
    backward_regions(first, n, reg);
    // output region of conv i's data gradient: R_{i-1}, or its pooled rows when a pool
    // follows conv i - 1 (pool = true: the pooled region up to the ceiling of the
    // pre-pool rows, for the pool backward; false: the pooled rows that exist)
    auto out_region = [&](Batch &b, int i, bool pool_bwd) {
      for (int k = 0; k < n; ++k) {
        const nst_tile &t = tiles[first + k];
        const Reg &r = reg[(size_t)k * (top + 1) + i - 1];
        if (!g.pool[i - 1]) {
          b.a0[k] = r[0], b.a1[k] = r[1], b.a2[k] = r[2], b.a3[k] = r[3];
        } else {
          const int hh = pool_bwd ? (lh(t, i - 1) + 1) / 2 : lh(t, i);
          const int ww = pool_bwd ? (lw(t, i - 1) + 1) / 2 : lw(t, i);
          b.a0[k] = r[0] >> 1, b.a1[k] = std::min((r[1] + 1) >> 1, hh);
          b.a2[k] = r[2] >> 1, b.a3[k] = std::min((r[3] + 1) >> 1, ww);
        }
      }
    };
    auto fill_seeds = [&](ConvArgs &a, int j) {
      // seeds and mask of conv j's post-ReLU output (Table 1 rows; ReLU'(0) = 0)
      a.mask = slot_base(L.s_act[j]);
      a.mask_ss = ss(es);
      const int k = g.style_of[j];
      if (k >= 0) {
        a.in2 = slot_base(L.s_act[j]);
        a.in2_ss = ss(es);
        a.cin2 = g.cout[j];
        a.wp2 = gl<char>(L.g_dt) + (size_t)L.dt_off[k] * es;
        if (use_ms) a.bias = gl<float>(L.g_msb) + L.moff[k];
      }
      if (j == g.content && use_content) {
        a.rc = (float *)slot_base(L.s_rc);
        a.rc_ss = ss(4);
        a.two_alpha = two_alpha;
      }
    };
    {
      Batch b = base_batch(first, n, top);
      for (int k = 0; k < n; ++k) {
        const Reg &r = reg[(size_t)k * (top + 1) + top];
        b.a0[k] = r[0], b.a1[k] = r[1], b.a2[k] = r[2], b.a3[k] = r[3];
      }
      ConvArgs a;
      std::memset(&a, 0, sizeof(a));
      fill_seeds(a, top);
      a.out = cur;
      a.out_ss = ss(es);
      a.cout = g.cout[top];
      a.cout_pad = g.cout[top];
      conv_pfx(b, IN_NONE, EPI_BWD, a.cout);
      HIPCHK(conv(IN_NONE, EPI_BWD, a, b));
    }
    for (int i = top; i >= 1; --i) {
      Batch b = base_batch(first, n, i);   // conv i's window (its output: dA_{i-1} or the pooled dP)
      out_region(b, i, false);
      ConvArgs a;
      std::memset(&a, 0, sizeof(a));
      a.in = cur;
      a.in_ss = ss(es);
      a.cin = g.cout[i];
      a.wp = c->wd[i];
      a.cout = g.cin[i];
      a.cout_pad = c->padd[i];
      a.out = oth;
      a.out_ss = ss(es);
      if (!g.pool[i - 1]) fill_seeds(a, i - 1);
      conv_pfx(b, IN_NHWC, EPI_BWD, a.cout);
      HIPCHK(conv(IN_NHWC, EPI_BWD, a, b));
      if (g.pool[i - 1]) {
        // oth holds dE/d(pool output); route it back and apply seeds + mask
        Batch bp = base_batch(first, n, i - 1);
        out_region(bp, i, true);
        std::vector<long long> items(n);
        const int C = g.cout[i - 1];
        for (int t = 0; t < n; ++t)
          items[t] = (long long)std::max(bp.a1[t] - bp.a0[t], 0) * std::max(bp.a3[t] - bp.a2[t], 0) * (C / vec);
        items_pfx(bp, items, 256);
        const bool cont = (i - 1) == g.content && use_content;
        double px = 0;   // pre-pool pixels of the region
        for (int t = 0; t < n; ++t) px += 4.0 * std::max(bp.a1[t] - bp.a0[t], 0) * std::max(bp.a3[t] - bp.a2[t], 0);
        HIPCHK(prof(c->prec == 1 ? "void nst::k_pool_bwd<__bf16>(__bf16 const*, long long, __bf16 const*, long long, float const*, long long, float, __bf16*, long long, int, bool, nst::Batch)"
                                 : "void nst::k_pool_bwd<float>(float const*, long long, float const*, long long, float const*, long long, float, float*, long long, int, bool, nst::Batch)",
                    0.0, 2.25 * px * C * es + (cont ? 4.0 * px * C : 0.0), [&] {
                      return launch_pool_bwd(c->prec, oth, ss(es), slot_base(L.s_act[i - 1]), ss(es),
                                             cont ? (const float *)slot_base(L.s_rc) : nullptr, ss(4),
                                             two_alpha, cur, ss(es), C, g.pavg[i - 1], bp, s);
                    }));
      } else {
        std::swap(cur, oth);
      }
    }
    {
      Batch b = base_batch(first, n, 0);
      for (int k = 0; k < n; ++k) {
        const nst_tile &t = tiles[first + k];
        b.a0[k] = t.by0 - t.ey0;
        b.a1[k] = t.by1 - t.ey0;
        b.a2[k] = t.bx0 - t.ex0;
        b.a3[k] = t.bx1 - t.ex0;
      }
      ConvArgs a;
      std::memset(&a, 0, sizeof(a));
      a.in = cur;
      a.in_ss = ss(es);
      a.cin = g.cout[0];
      a.wp = c->wd[0];
      a.cout = 3;
      a.cout_pad = c->padd[0];
      a.grad = grad;
      a.img_h = H;
      a.img_w = W;
      conv_pfx(b, IN_NHWC, EPI_STITCH, 32);
      HIPCHK(conv(IN_NHWC, EPI_STITCH, a, b));
    }
    return NST_OK;
  }
};

int setup(Runner &R, nst_ctx *ctx, int H, int W, int T, int m, void *ws, size_t ws_bytes,
          void *stream, int flags) {
  int st = validate_sizes(H, W, T, m);
  if (st != NST_OK) return st;
  if ((flags & NST_STRICT_HALO) && m < ctx->g.min_halo) return NST_EHALO;
  if (!ws) return NST_EINVAL;
  R.H = H;
  R.W = W;
  R.T = T;
  R.m = m;
  R.ws = (char *)ws;
  R.s = (hipStream_t)stream;
  build_plan(ctx->g, H, W, T, m, R.tiles);
  const int nt = (int)R.tiles.size();
  Layout L1;
  make_layout(ctx->g, ctx->prec, R.tiles, 1, 1, L1);
  if ((st = max_window_ok(ctx->g, L1)) != NST_OK) return st;
  if (ws_bytes < L1.total) return NST_EWORKSPACE;
  if (flags & NST_RESIDENT) {
    // a slot per tile, asked for explicitly: Step 2 then reuses Step 1's activations
    Layout La;
    make_layout(ctx->g, ctx->prec, R.tiles, balanced_batch(nt), nt, La);
    if (La.total > ws_bytes) return NST_EWORKSPACE;
    R.L = La;
    R.retain = true;
    return NST_OK;
  }
  int best = 1;
  for (int b = std::min(nt, kMaxBatch); b > 1; --b) {
    Layout Lb;
    make_layout(ctx->g, ctx->prec, R.tiles, b, b, Lb);
    if (Lb.total <= ws_bytes) {
      best = b;
      break;
    }
  }
  // balance: same number of batches, evenly filled
  const int nb = (nt + best - 1) / best;
  const int bal = (nt + nb - 1) / nb;
  make_layout(ctx->g, ctx->prec, R.tiles, bal, bal, R.L);
  return NST_OK;
}

// Restores the caller's plan when a pass that used a plan of its own returns.
struct PlanScope {
  Runner &R;
  std::vector<nst_tile> saved;
  bool on = false;
  explicit PlanScope(Runner &r) : R(r) {}
  void use(int margin) {
    saved = R.tiles;
    on = true;
    R.replan(margin);
  }
  ~PlanScope() {
    if (on) R.tiles.swap(saved);
  }
};

// keep: also store full-resolution activations of pooled layers (for a Step 2 that
// reuses this pass's activations; the windows are then Step 2's); means: also sum the
// style features' channels.  Otherwise the windows have the Step 1 margin, which is all
// the owned style and content features need.
int step1(Runner &R, const float *x, const float *fc, bool keep, bool means) {
  const Geom &g = R.g;
  PlanScope plan(R);
  if (!keep) plan.use(g.step1_halo);
  HIPCHK(launch_fill_f64(R.gl<double>(R.L.g_gacc), (R.L.g_dt - R.L.g_gacc) / 8, 0.0, R.s));
  HIPCHK(launch_fill_f64(R.gl<double>(R.L.g_ec), 1, 0.0, R.s));
  if (means) HIPCHK(launch_fill_f64(R.gl<double>(R.L.g_csum), (size_t)R.L.total_c, 0.0, R.s));
  int upto = -1;
  for (int k = 0; k < g.n_style; ++k) upto = std::max(upto, g.style[k]);
  if (fc) upto = std::max(upto, g.content);
  const int nt = (int)R.tiles.size();
  for (int first = 0; first < nt; first += R.L.batch) {
    const int n = std::min(R.L.batch, nt - first);
    // the owned style / content features, or (activations kept for Step 2) what Step 2 needs
    std::vector<Reg> regions;
    if (keep) {
      std::vector<Reg> need;
      R.backward_regions(first, n, need);
      R.forward_regions(first, n, upto, need, regions);
    } else {
      bool layers[NST_MAX_CONV] = {};
      for (int k = 0; k < g.n_style; ++k) layers[g.style[k]] = true;
      if (fc) layers[g.content] = true;
      R.owned_forward_regions(first, n, upto, layers, regions);
    }
    int st = R.forward(first, n, upto, x, fc, keep, regions);
    if (st != NST_OK) return st;
    if ((st = R.grams(first, n, means)) != NST_OK) return st;
    if (fc && (st = R.content_energy(first, n)) != NST_OK) return st;
  }
  return NST_OK;
}

// Grams (and channel means) divided by the whole-image n_p (Sec. 3.1, 3.2)
int normalize(Runner &R, double *grams_out, double *means_out) {
  const Geom &g = R.g;
  for (int k = 0; k < g.n_style; ++k) {
    const int i = g.style[k], C = g.cout[i];
    const double np = (double)(R.H / g.stride[i]) * (double)(R.W / g.stride[i]);
    HIPCHK(launch_gram_normalize(R.gl<double>(R.L.g_gacc) + R.L.off_c[k],
                                 grams_out + R.L.off_c[k], (size_t)C * C, np, R.s));
    if (means_out)
      HIPCHK(launch_gram_normalize(R.gl<double>(R.L.g_csum) + R.L.moff[k], means_out + R.L.moff[k],
                                   (size_t)C, np, R.s));
  }
  return NST_OK;
}

}  // namespace

extern "C" {

int nst_profile(nst_ctx *ctx, int enable) {
  if (!ctx) return NST_EINVAL;
  if (enable) {
    for (ProfRec &r : ctx->prof) {
      ctx->ev_pool.push_back(r.e0);
      ctx->ev_pool.push_back(r.e1);
    }
    ctx->prof.clear();
  }
  ctx->prof_on = enable != 0;
  return NST_OK;
}

int nst_profile_read(nst_ctx *ctx, nst_kstat *out, int cap, int *n) {
  if (!ctx || !n || cap < 0 || (cap > 0 && !out)) return NST_EINVAL;
  std::map<std::string, nst_kstat> agg;
  int st = NST_OK;
  for (ProfRec &r : ctx->prof) {
    float ms = 0.f;
    if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess)
      st = NST_EHIP;
    nst_kstat &k = agg[r.name];
    k.launches += 1;
    k.ms += ms;
    k.flops += r.flops;
    k.bytes += r.bytes;
    ctx->ev_pool.push_back(r.e0);
    ctx->ev_pool.push_back(r.e1);
  }
  ctx->prof.clear();
  std::vector<nst_kstat> v;
  for (auto &kv : agg) {
    nst_kstat k = kv.second;
    std::snprintf(k.name, sizeof(k.name), "%s", kv.first.c_str());
    v.push_back(k);
  }
  std::sort(v.begin(), v.end(), [](const nst_kstat &a, const nst_kstat &b) { return a.ms > b.ms; });
  *n = (int)v.size();
  for (int i = 0; i < std::min(cap, (int)v.size()); ++i) out[i] = v[i];
  return st;
}

int nst_style_stats(nst_ctx *ctx, const float *s, int H, int W, int T, int m, double *grams,
                    double *means, void *ws, size_t ws_bytes, void *stream) {
  if (!ctx || !s || !grams) return NST_EINVAL;
  if (ctx->g.n_style == 0) return NST_EINVAL;
  Runner R(ctx);
  int st = setup(R, ctx, H, W, T, m, ws, ws_bytes, stream, 0);
  if (st != NST_OK) return st;
  if ((st = step1(R, s, nullptr, false, means != nullptr)) != NST_OK) return st;
  return normalize(R, grams, means);
}

int nst_style_grams(nst_ctx *ctx, const float *s, int H, int W, int T, int m, double *grams,
                    void *ws, size_t ws_bytes, void *stream) {
  return nst_style_stats(ctx, s, H, W, T, m, grams, nullptr, ws, ws_bytes, stream);
}

int nst_layer_feats(nst_ctx *ctx, const float *img, int H, int W, int T, int m, int conv,
                    float *feats, void *ws, size_t ws_bytes, void *stream) {
  if (!ctx || !img || !feats) return NST_EINVAL;
  if (conv < 0 || conv > ctx->g.top) return NST_EINVAL;
  Runner R(ctx);
  int st = setup(R, ctx, H, W, T, m, ws, ws_bytes, stream, 0);
  if (st != NST_OK) return st;
  R.replan(std::max(ctx->g.rf_a[conv], ctx->g.rf_b[conv]));   // owned features of conv only
  const int nt = (int)R.tiles.size();
  const int vec = (int)(16 / R.L.es);
  for (int first = 0; first < nt; first += R.L.batch) {
    const int n = std::min(R.L.batch, nt - first);
    bool layers[NST_MAX_CONV] = {};
    layers[conv] = true;
    std::vector<Reg> regions;
    R.owned_forward_regions(first, n, conv, layers, regions);
    if ((st = R.forward(first, n, conv, img, nullptr, false, regions)) != NST_OK) return st;
    Batch b = R.base_batch(first, n, conv);
    std::vector<long long> items(n);
    for (int t = 0; t < n; ++t) items[t] = (long long)Runner::region_px(b, t) * (ctx->g.cout[conv] / vec);
    R.items_pfx(b, items, 256);
    HIPCHK(launch_stitch_feats(ctx->prec, R.slot_base(R.L.s_act[conv]), R.ss(R.L.es),
                               ctx->g.cout[conv], b, feats, W / ctx->g.stride[conv], R.s));
  }
  return NST_OK;
}

int nst_content_feats(nst_ctx *ctx, const float *c, int H, int W, int T, int m, float *feats,
                      void *ws, size_t ws_bytes, void *stream) {
  if (!ctx) return NST_EINVAL;
  if (ctx->g.content < 0) return NST_EINVAL;
  return nst_layer_feats(ctx, c, H, W, T, m, ctx->g.content, feats, ws, ws_bytes, stream);
}

int nst_loss_grad_ms(nst_ctx *ctx, const float *x, int H, int W, const double *target_grams,
                     const float *content_feats, const double *w_style, double alpha,
                     const nst_mean_std *ms, int T, int m, int flags, double *grams_x,
                     double *energy, float *grad, void *ws, size_t ws_bytes, void *stream) {
  if (!ctx || !x || !grams_x) return NST_EINVAL;
  if ((flags & ~(NST_BOTH | NST_STRICT_HALO | NST_RESIDENT | NST_CHECK_FINITE)) != 0 ||
      (flags & NST_BOTH) == 0)
    return NST_EINVAL;
  const Geom &g = ctx->g;
  const bool s1 = flags & NST_STEP1, s2 = flags & NST_STEP2;
  const bool use_c = g.content >= 0 && alpha != 0.0;
  if (use_c && !content_feats) return NST_EINVAL;
  if (g.n_style > 0 && (!target_grams || !w_style)) return NST_EINVAL;
  if (s2 && !grad) return NST_EINVAL;
  const bool use_ms = ms != nullptr && g.n_style > 0;
  if (use_ms && (!ms->w_mean || !ms->w_std || !ms->target_means || !ms->means_x)) return NST_EINVAL;
  Runner R(ctx);
  int st = setup(R, ctx, H, W, T, m, ws, ws_bytes, stream, flags);
  if (st != NST_OK) return st;
  const float *fc = use_c ? content_feats : nullptr;
  if (flags & NST_CHECK_FINITE) {
    // count non-finite inputs on the device, then wait for the count (a host sync)
    unsigned *cnt = R.gl<unsigned>(R.L.g_flag);
    HIPCHK(launch_fill_u32(cnt, 1, 0u, R.s));
    HIPCHK(launch_count_nonfinite_f32(x, (size_t)3 * H * W, cnt, R.s));
    if (fc) {
      const int i = g.content;
      const size_t n = (size_t)(H / g.stride[i]) * (W / g.stride[i]) * g.cout[i];
      HIPCHK(launch_count_nonfinite_f32(fc, n, cnt, R.s));
    }
    if (g.n_style > 0) HIPCHK(launch_count_nonfinite_f64(target_grams, (size_t)R.L.total_cc, cnt, R.s));
    if (!s1) HIPCHK(launch_count_nonfinite_f64(grams_x, (size_t)R.L.total_cc, cnt, R.s));
    if (use_ms) {
      HIPCHK(launch_count_nonfinite_f64(ms->target_means, (size_t)R.L.total_c, cnt, R.s));
      if (!s1) HIPCHK(launch_count_nonfinite_f64(ms->means_x, (size_t)R.L.total_c, cnt, R.s));
    }
    unsigned host_cnt = 0;
    HIPCHK(hipMemcpyAsync(&host_cnt, cnt, sizeof(unsigned), hipMemcpyDeviceToHost, R.s));
    HIPCHK(hipStreamSynchronize(R.s));
    if (host_cnt != 0) return NST_ENONFINITE;
    for (int k = 0; k < g.n_style; ++k) {
      if (!std::isfinite(w_style[k])) return NST_ENONFINITE;
      if (use_ms && (!std::isfinite(ms->w_mean[k]) || !std::isfinite(ms->w_std[k]))) return NST_ENONFINITE;
    }
    if (!std::isfinite(alpha)) return NST_ENONFINITE;
  }

  StyleTermsArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.n_style = g.n_style;
  for (int k = 0; k < g.n_style; ++k) {
    const int i = g.style[k];
    sa.C[k] = g.cout[i];
    sa.off[k] = R.L.off_c[k];
    sa.dt_off[k] = R.L.dt_off[k];
    sa.w[k] = w_style[k];
    sa.inv_np[k] = 1.0 / ((double)(H / g.stride[i]) * (double)(W / g.stride[i]));
    sa.moff[k] = R.L.moff[k];
    if (use_ms) {
      sa.w1[k] = ms->w_mean[k];
      sa.w2[k] = ms->w_std[k];
    }
  }
  if (use_ms) {
    sa.mx = ms->means_x;
    sa.mt = ms->target_means;
    sa.msb = R.gl<float>(R.L.g_msb);
  }

  if (s1) {
    if ((st = step1(R, x, fc, R.retain && s2, use_ms)) != NST_OK) return st;
    if ((st = normalize(R, grams_x, use_ms ? ms->means_x : nullptr)) != NST_OK) return st;
  } else {
    HIPCHK(launch_fill_f64(R.gl<double>(R.L.g_ec), 1, 0.0, R.s));
  }
  if (g.n_style > 0)
    HIPCHK(launch_style_terms(ctx->prec, grams_x, target_grams, sa, R.gl<char>(R.L.g_dt),
                              R.gl<double>(R.L.g_estyle), R.s));
  if (s2) {
    const int nt = (int)R.tiles.size();
    for (int first = 0; first < nt; first += R.L.batch) {
      const int n = std::min(R.L.batch, nt - first);
      // Step 1 of this call left every tile's activations (and content difference) in its
      // slot when each tile has one; otherwise Step 2 recomputes them (Algorithm 1)
      if (!(s1 && R.retain)) {
        // the forward on what the data gradients read (masks, residual operands, pools)
        std::vector<Reg> need, regions;
        R.backward_regions(first, n, need);
        R.forward_regions(first, n, g.top, need, regions);
        if ((st = R.forward(first, n, g.top, x, fc, true, regions)) != NST_OK) return st;
      }
      if (!s1 && fc && (st = R.content_energy(first, n)) != NST_OK) return st;
      if ((st = R.backward(first, n, (float)(2.0 * alpha), use_c, use_ms, grad)) != NST_OK) return st;
    }
  }
  HIPCHK(launch_energy_total(R.gl<double>(R.L.g_ec), R.gl<double>(R.L.g_estyle), g.n_style,
                             use_c ? alpha : 0.0, R.gl<double>(R.L.g_energy), R.s));
  if (energy) {
    HIPCHK(hipMemcpyAsync(energy, R.gl<double>(R.L.g_energy), sizeof(double) * (2 + g.n_style),
                          hipMemcpyDeviceToHost, R.s));
    HIPCHK(hipStreamSynchronize(R.s));
  }
  return NST_OK;
}

int nst_loss_grad(nst_ctx *ctx, const float *x, int H, int W, const double *target_grams,
                  const float *content_feats, const double *w_style, double alpha, int T, int m,
                  int flags, double *grams_x, double *energy, float *grad, void *ws,
                  size_t ws_bytes, void *stream) {
  return nst_loss_grad_ms(ctx, x, H, W, target_grams, content_feats, w_style, alpha, nullptr, T, m,
                          flags, grams_x, energy, grad, ws, ws_bytes, stream);
}

size_t nst_scratch_bytes(void) { return kScratchBytes; }

int nst_loss_grad_noalloc(nst_ctx *ctx, const float *x, int H, int W, const double *target_grams,
                          const float *content_feats, const double *w_style, double alpha, int T,
                          int m, int flags, double *grams_x, double *energy, float *grad,
                          void *stream) {
  if (!ctx) return NST_EINVAL;
  void *ws = scratch_ptr(ctx->device);
  if (!ws) return NST_EHIP;
  // the same run as nst_loss_grad on the device's static scratch; sizes whose smallest
  // tile batch does not fit are refused with NST_EWORKSPACE before any launch
  return nst_loss_grad_ms(ctx, x, H, W, target_grams, content_feats, w_style, alpha, nullptr, T, m,
                          flags, grams_x, energy, grad, ws, kScratchBytes, stream);
}

}  // extern "C"
