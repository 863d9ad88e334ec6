// C ABI of libsimnet.so (declared in include/simnet.h): validation, context
// and device-state ownership, weight re-layout, dispatch to the kernels.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/simnet.h"
#include "simnet_internal.h"

using namespace simnet;

struct sim_ctx {
  sim_config cfg;
  int32_t n_sub = 0;
  int64_t n_instr = 0;
  const float* feat = nullptr;
  int net = -1;  // 0 NetSmall, 1 NetC3
  int C = 0;
  uint32_t relu = 0;
  bool weights = false;
  bool completed = false;
  int64_t max_pos = 0, n_pred = 0, n_meas = 0;
  float* logits_out = nullptr;
  hipStream_t stream = nullptr;
  void* dev_block = nullptr;  // state + table
  float* dev_weights = nullptr;
  int64_t* dev_total = nullptr;
  DevState st{};
  DevWeights w{};
  std::string err;
};

namespace {

int fail(sim_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(sim_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

int hip_fail(sim_ctx* c, hipError_t e, const char* what) {
  return fail(c, SIM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Window shapes with a kernel: (n_feat, n_slot) -> net id.
int window_net(int32_t n_feat, int32_t n_slot) {
  if (n_feat == NetSmall::D && n_slot == NetSmall::L) return 0;
  if (n_feat == NetC3::D && n_slot == NetC3::L) return 1;
  return -1;
}

int check_cfg(const sim_config* cfg, const sim_trace* tr, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return SIM_EINVAL;
  };
  if (!cfg || !tr) return bad("null config or trace");
  if (cfg->n_feat < 1 || cfg->n_slot < 2) return bad("n_feat must be >= 1 and n_slot >= 2");
  if (cfg->n_out != 2) return bad("n_out must be 2 (fetch, execution)");
  if (cfg->retire_width < 1 || cfg->retire_width > WMAX) return bad("retire_width must be 1..16");
  const int32_t cols[3] = {cfg->col_res, cfg->col_exe, cfg->col_sto};
  for (int i = 0; i < 3; ++i) {
    if (cols[i] < -1 || cols[i] >= cfg->n_feat) return bad("dynamic column out of range");
    for (int j = 0; j < i; ++j)
      if (cols[i] >= 0 && cols[i] == cols[j]) return bad("dynamic columns must differ");
  }
  if (cfg->lat_max < 1) return bad("lat_max must be >= 1");
  if (cfg->prec < SIM_FP32 || cfg->prec > SIM_FP8E4M3) return bad("unknown precision");
  if (cfg->reserved != 0) return bad("reserved field must be 0");
  if (!tr->feat) return bad("feat is NULL");
  if (tr->feat_dtype != SIM_FEAT_F32) return bad("unknown feat_dtype");
  if (tr->n_instr < 1 || tr->n_instr >= (int64_t)1 << 31) return bad("n_instr must be in [1, 2^31)");
  if (tr->n_sub < 1) return bad("n_sub must be >= 1");
  if (!tr->start || !tr->len || !tr->warm) return bad("sub-trace table is NULL");
  for (int32_t k = 0; k < tr->n_sub; ++k) {
    if (tr->len[k] < 1) return bad("every sub-trace needs len >= 1");
    if (tr->warm[k] < 0 || tr->warm[k] > tr->start[k]) return bad("warm must be in [0, start]");
    if (tr->start[k] < 0 || tr->start[k] + tr->len[k] > tr->n_instr)
      return bad("sub-trace outside the trace");
  }
  return SIM_OK;
}

// B[k][n] packed per (k-group of 16, n-tile of 16) as 64 lanes x 4 floats:
// lane holds B[kg*16 + 4*(lane/16) + s][nt*16 + lane%16], s = 0..3.
template <class F>
void pack_b(int K, int N, F&& B, float* out) {
  const int KG = K / 16, NTL = N / 16;
  for (int kg = 0; kg < KG; ++kg)
    for (int nt = 0; nt < NTL; ++nt)
      for (int lane = 0; lane < 64; ++lane)
        for (int s = 0; s < 4; ++s)
          out[(((size_t)kg * NTL + nt) * 64 + lane) * 4 + s] =
              B(kg * 16 + 4 * (lane / 16) + s, nt * 16 + lane % 16);
}

struct Expect {
  int32_t kind, c_in, c_out;
};

template <class Net>
std::vector<Expect> expected_layers() {
  std::vector<Expect> v;
  v.push_back({0, Net::D, Net::CH1});
  v.push_back({0, Net::CH1, Net::CH2});
  if (Net::NCONV == 3) v.push_back({0, Net::CH2, Net::CH3});
  if (Net::HID > 0) {
    v.push_back({1, Net::CHL * Net::NB, Net::HID});
    v.push_back({1, Net::HID, Net::NOUT});
  } else {
    v.push_back({1, Net::CHL * Net::NB, Net::NOUT});
  }
  return v;
}

// Re-lay-out PyTorch-order parameters for one network; returns the floats.
template <class Net>
std::vector<float> relayout(const float* params, size_t* offs_out /*[12]*/) {
  std::vector<const float*> w, b;
  size_t off = 0;
  for (const Expect& e : expected_layers<Net>()) {
    const size_t nw = (size_t)e.c_out * e.c_in * (e.kind == 0 ? 2 : 1);
    w.push_back(params + off);
    off += nw;
    b.push_back(params + off);
    off += e.c_out;
  }
  const int chp[4] = {Net::CH0, Net::CH1, Net::CH2, Net::CH3};
  const int chr[4] = {Net::D, Net::CH1, Net::CH2, Net::CH3};
  std::vector<float> out;
  auto reserve = [&](size_t n) {  // 256-byte aligned sections
    const size_t at = (out.size() + 63) / 64 * 64;
    out.resize(at + n, 0.f);
    return at;
  };
  for (int l = 0; l < Net::NCONV; ++l) {
    const int K = 2 * chp[l], N = chp[l + 1], cin = chr[l];
    const float* wl = w[l];
    const size_t at = reserve((size_t)K * N);
    pack_b(K, N,
           [&](int k, int n) {
             const int t = k / chp[l], c = k % chp[l];
             return c < cin ? wl[((size_t)n * cin + c) * 2 + t] : 0.f;
           },
           out.data() + at);
    offs_out[2 * l] = at;
    const size_t bt = reserve(N);
    std::copy(b[l], b[l] + N, out.begin() + bt);
    offs_out[2 * l + 1] = bt;
  }
  const int li = Net::NCONV;
  if (Net::HID > 0) {
    const int K = Net::CHL, N = Net::HID, NB = Net::NB;
    const float* W1 = w[li];
    const size_t per = (size_t)K * N;
    const size_t at = reserve(per * NB);
    for (int j = 0; j < NB; ++j)
      pack_b(K, N, [&](int c, int n) { return W1[(size_t)n * (K * NB) + c * NB + j]; },
             out.data() + at + per * j);
    offs_out[6] = at;
    const size_t bt = reserve(N);
    std::copy(b[li], b[li] + N, out.begin() + bt);
    offs_out[7] = bt;
    const size_t lt = reserve((size_t)Net::NOUT * N);
    std::copy(w[li + 1], w[li + 1] + (size_t)Net::NOUT * N, out.begin() + lt);
    offs_out[8] = lt;
    const size_t lb = reserve(Net::NOUT);
    std::copy(b[li + 1], b[li + 1] + Net::NOUT, out.begin() + lb);
    offs_out[9] = lb;
  } else {
    const int K = Net::CHL, NB = Net::NB;
    const float* Wf = w[li];
    const size_t lt = reserve((size_t)NB * Net::NOUT * K);
    for (int j = 0; j < NB; ++j)
      for (int o = 0; o < Net::NOUT; ++o)
        for (int c = 0; c < K; ++c)
          out[lt + ((size_t)j * Net::NOUT + o) * K + c] = Wf[(size_t)o * (K * NB) + c * NB + j];
    offs_out[6] = offs_out[7] = 0;
    offs_out[8] = lt;
    const size_t lb = reserve(Net::NOUT);
    std::copy(b[li], b[li] + Net::NOUT, out.begin() + lb);
    offs_out[9] = lb;
  }
  return out;
}

template <class Net>
size_t param_count() {
  size_t n = 0;
  for (const Expect& e : expected_layers<Net>())
    n += (size_t)e.c_out * e.c_in * (e.kind == 0 ? 2 : 1) + e.c_out;
  return n;
}

template <class Net>
bool layers_match(const sim_layer* layers, int32_t n) {
  const std::vector<Expect> ex = expected_layers<Net>();
  if ((size_t)n != ex.size()) return false;
  for (int32_t i = 0; i < n; ++i)
    if (layers[i].kind != ex[i].kind || layers[i].c_in != ex[i].c_in ||
        layers[i].c_out != ex[i].c_out)
      return false;
  return true;
}

}  // namespace

extern "C" {

int sim_validate_config(const sim_config* cfg, const sim_trace* trace) {
  return check_cfg(cfg, trace, nullptr);
}

int sim_init(const sim_config* cfg, const sim_trace* tr, sim_ctx** out) {
  if (!out) return SIM_EINVAL;
  *out = nullptr;
  sim_ctx* c = new (std::nothrow) sim_ctx();
  if (!c) return SIM_ENOMEM;
  std::string why;
  int rc = check_cfg(cfg, tr, &why);
  if (rc != SIM_OK) {
    fprintf(stderr, "sim_init: %s\n", why.c_str());
    delete c;
    return rc;
  }
  c->net = window_net(cfg->n_feat, cfg->n_slot);
  if (c->net < 0 || cfg->prec != SIM_FP32) {
    fprintf(stderr, "sim_init: no kernel for window %dx%d at precision %d\n", cfg->n_slot,
            cfg->n_feat, cfg->prec);
    delete c;
    return SIM_EUNSUPPORTED;
  }
  c->cfg = *cfg;
  c->C = cfg->n_slot - 1;
  c->n_sub = tr->n_sub;
  c->n_instr = tr->n_instr;
  c->feat = static_cast<const float*>(tr->feat);
  c->stream = static_cast<hipStream_t>(cfg->stream);

  const int32_t K = tr->n_sub, C = c->C;
  std::vector<int64_t> first(K), npos(K), poff(K);
  std::vector<int32_t> warm(K);
  int64_t acc = 0;
  for (int32_t k = 0; k < K; ++k) {
    first[k] = tr->start[k] - tr->warm[k];
    npos[k] = tr->warm[k] + tr->len[k];
    warm[k] = tr->warm[k];
    poff[k] = acc;
    acc += npos[k];
    c->n_meas += tr->len[k];
    c->max_pos = std::max(c->max_pos, npos[k]);
  }
  c->n_pred = acc;

  // one device block: table + state + results + counters + total
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) / 256 * 256;
    return at;
  };
  const size_t o_first = take(8 * K), o_npos = take(8 * K), o_warm = take(4 * K),
               o_poff = take(8 * K), o_cur = take(8 * K), o_tw = take(8 * K),
               o_rp = take(8 * K), o_pos = take(8 * K), o_head = take(4 * K),
               o_cnt = take(4 * K), o_rw = take(8 * (size_t)K * WMAX),
               o_qi = take(4 * (size_t)K * C), o_qe = take(4 * (size_t)K * C),
               o_qt = take(8 * (size_t)K * C), o_qr = take(8 * (size_t)K * C),
               o_fe = take(8 * K), o_dr = take(8 * K), o_fi = take(8 * K), o_wt = take(8 * K),
               o_ctr = take(8 * NCOUNTERS), o_tot = take(8);
  hipError_t e = hipMalloc(&c->dev_block, off);
  if (e != hipSuccess) {
    fprintf(stderr, "sim_init: hipMalloc(%zu): %s\n", off, hipGetErrorString(e));
    delete c;
    return e == hipErrorOutOfMemory ? SIM_ENOMEM : SIM_EDEVICE;
  }
  char* base = static_cast<char*>(c->dev_block);
  DevState& s = c->st;
  s.first = reinterpret_cast<int64_t*>(base + o_first);
  s.n_pos = reinterpret_cast<int64_t*>(base + o_npos);
  s.warm = reinterpret_cast<int32_t*>(base + o_warm);
  s.pred_off = reinterpret_cast<int64_t*>(base + o_poff);
  s.cur = reinterpret_cast<int64_t*>(base + o_cur);
  s.t_w = reinterpret_cast<int64_t*>(base + o_tw);
  s.r_prev = reinterpret_cast<int64_t*>(base + o_rp);
  s.pos = reinterpret_cast<int64_t*>(base + o_pos);
  s.head = reinterpret_cast<int32_t*>(base + o_head);
  s.count = reinterpret_cast<int32_t*>(base + o_cnt);
  s.rw = reinterpret_cast<int64_t*>(base + o_rw);
  s.q_idx = reinterpret_cast<int32_t*>(base + o_qi);
  s.q_e = reinterpret_cast<int32_t*>(base + o_qe);
  s.q_t = reinterpret_cast<int64_t*>(base + o_qt);
  s.q_r = reinterpret_cast<int64_t*>(base + o_qr);
  s.fetch = reinterpret_cast<int64_t*>(base + o_fe);
  s.drain = reinterpret_cast<int64_t*>(base + o_dr);
  s.final_tick = reinterpret_cast<int64_t*>(base + o_fi);
  s.warm_tick = reinterpret_cast<int64_t*>(base + o_wt);
  s.counters = reinterpret_cast<unsigned long long*>(base + o_ctr);
  c->dev_total = reinterpret_cast<int64_t*>(base + o_tot);

  hipError_t e1 = hipMemcpyAsync(base + o_first, first.data(), 8 * K, hipMemcpyHostToDevice, c->stream);
  hipError_t e2 = hipMemcpyAsync(base + o_npos, npos.data(), 8 * K, hipMemcpyHostToDevice, c->stream);
  hipError_t e3 = hipMemcpyAsync(base + o_warm, warm.data(), 4 * K, hipMemcpyHostToDevice, c->stream);
  hipError_t e4 = hipMemcpyAsync(base + o_poff, poff.data(), 8 * K, hipMemcpyHostToDevice, c->stream);
  hipError_t e5 = launch_reset(s, K, C, c->stream);
  hipError_t e6 = hipStreamSynchronize(c->stream);  // host vectors die at return
  for (hipError_t x : {e1, e2, e3, e4, e5, e6})
    if (x != hipSuccess) {
      fprintf(stderr, "sim_init: %s\n", hipGetErrorString(x));
      (void)hipFree(c->dev_block);
      delete c;
      return SIM_EDEVICE;
    }
  *out = c;
  return SIM_OK;
}

int sim_load_weights(sim_ctx* c, const sim_layer* layers, int32_t n_layers, const float* params,
                     int32_t on_device) {
  if (!c) return SIM_EINVAL;
  if (!layers || n_layers < 1 || !params) return fail(c, SIM_EINVAL, "null layers or params");
  const bool ok = c->net == 0 ? layers_match<NetSmall>(layers, n_layers)
                              : layers_match<NetC3>(layers, n_layers);
  if (!ok) return fail(c, SIM_EUNSUPPORTED, "no kernel for this layer list");
  if (layers[n_layers - 1].relu)
    return fail(c, SIM_EUNSUPPORTED, "the output layer must not have ReLU");
  const size_t np = c->net == 0 ? param_count<NetSmall>() : param_count<NetC3>();
  std::vector<float> host(np);
  if (on_device) {
    hipError_t e = hipMemcpy(host.data(), params, np * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "copy params to host");
  } else {
    memcpy(host.data(), params, np * 4);
  }
  for (size_t i = 0; i < np; ++i)
    if (!isfinite(host[i])) return fail(c, SIM_ENONFINITE, "parameter %zu is not finite", i);
  size_t offs[12] = {0};
  std::vector<float> packed =
      c->net == 0 ? relayout<NetSmall>(host.data(), offs) : relayout<NetC3>(host.data(), offs);
  uint32_t relu = 0;
  for (int32_t i = 0; i < n_layers; ++i)
    if (layers[i].relu) relu |= 1u << i;
  float* dw = nullptr;
  hipError_t e = hipMalloc(&dw, packed.size() * 4);
  if (e != hipSuccess) return hip_fail(c, e, "hipMalloc weights");
  e = hipMemcpy(dw, packed.data(), packed.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dw);
    return hip_fail(c, e, "upload weights");
  }
  if (c->dev_weights) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->dev_weights);
  }
  c->dev_weights = dw;
  DevWeights& w = c->w;
  const int nconv = c->net == 0 ? NetSmall::NCONV : NetC3::NCONV;
  for (int l = 0; l < 3; ++l) {
    w.conv_w[l] = l < nconv ? dw + offs[2 * l] : nullptr;
    w.conv_b[l] = l < nconv ? dw + offs[2 * l + 1] : nullptr;
  }
  const bool hid = c->net == 1;
  w.hid_w = hid ? dw + offs[6] : nullptr;
  w.hid_b = hid ? dw + offs[7] : nullptr;
  w.last_w = dw + offs[8];
  w.last_b = dw + offs[9];
  c->relu = relu;
  c->weights = true;
  return sim_reset(c);
}

int sim_reset(sim_ctx* c) {
  if (!c) return SIM_EINVAL;
  hipError_t e = launch_reset(c->st, c->n_sub, c->C, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "reset");
  c->completed = false;
  return SIM_OK;
}

int sim_record_logits(sim_ctx* c, float* logits) {
  if (!c) return SIM_EINVAL;
  c->logits_out = logits;
  return SIM_OK;
}

static int step_launch(sim_ctx* c, int64_t n_steps, int32_t mode, const int32_t* table) {
  if (mode < SIM_LAT_PREDICT || mode > SIM_LAT_SHADOW) return fail(c, SIM_EINVAL, "bad lat_mode");
  if (mode != SIM_LAT_PREDICT && !table) return fail(c, SIM_EINVAL, "lat_table required");
  if (mode != SIM_LAT_INJECT && !c->weights) return fail(c, SIM_ESTATE, "weights not loaded");
  if (c->completed) return fail(c, SIM_ESTATE, "run completed; call sim_reset");
  StepParams p{};
  p.feat = c->feat;
  p.n_sub = c->n_sub;
  p.W = c->cfg.retire_width;
  p.col_res = c->cfg.col_res;
  p.col_exe = c->cfg.col_exe;
  p.col_sto = c->cfg.col_sto;
  p.lat_max = c->cfg.lat_max;
  p.lat_mode = mode;
  p.lat_table = table;
  p.logits_out = c->logits_out;
  p.n_steps = (int32_t)std::min<int64_t>(n_steps, INT32_MAX);
  hipError_t e = launch_step(c->net, c->w, c->relu, c->st, p, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "step launch");
  return SIM_OK;
}

int sim_step(sim_ctx* c, int32_t n_steps, int32_t mode, const int32_t* table) {
  if (!c) return SIM_EINVAL;
  if (n_steps < 0) return fail(c, SIM_EINVAL, "n_steps < 0");
  if (n_steps == 0) return SIM_OK;
  return step_launch(c, n_steps, mode, table);
}

int sim_run(sim_ctx* c, int32_t mode, const int32_t* table, sim_result* res) {
  if (!c) return SIM_EINVAL;
  if (!res) return fail(c, SIM_EINVAL, "null result");
  int rc = step_launch(c, c->max_pos, mode, table);
  if (rc != SIM_OK) return rc;
  hipError_t e = launch_total(c->st, c->n_sub, c->dev_total, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "total launch");
  int64_t total = 0;
  unsigned long long ctr[NCOUNTERS] = {0};
  e = hipMemcpyAsync(&total, c->dev_total, 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctr, c->st.counters, sizeof ctr, hipMemcpyDeviceToHost, c->stream);
  const size_t kb = 8 * (size_t)c->n_sub;
  if (e == hipSuccess && res->fetch_cycles)
    e = hipMemcpyAsync(res->fetch_cycles, c->st.fetch, kb, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && res->drain_cycles)
    e = hipMemcpyAsync(res->drain_cycles, c->st.drain, kb, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && res->final_tick)
    e = hipMemcpyAsync(res->final_tick, c->st.final_tick, kb, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && res->warm_tick)
    e = hipMemcpyAsync(res->warm_tick, c->st.warm_tick, kb, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "sim_run results");
  res->total_cycles = total;
  res->measured_instr = c->n_meas;
  res->predicted_instr = c->n_pred;
  res->n_clamped = (int64_t)ctr[0];
  res->n_nonfinite = (int64_t)ctr[1];
  res->n_shadow_mismatch = (int64_t)ctr[2];
  c->completed = true;
  return SIM_OK;
}

int predictor_fwd(sim_ctx* c, const void* x, int64_t B, float* logits, void* save_or_null) {
  if (!c) return SIM_EINVAL;
  if (!c->weights) return fail(c, SIM_ESTATE, "weights not loaded");
  if (save_or_null) return fail(c, SIM_EUNSUPPORTED, "save buffer not supported");
  if (B < 0 || (B > 0 && (!x || !logits))) return fail(c, SIM_EINVAL, "bad batch arguments");
  if (B == 0) return SIM_OK;
  if ((B + MT - 1) / MT > INT32_MAX) return fail(c, SIM_EINVAL, "batch too large");
  hipError_t e = launch_forward(c->net, c->w, c->relu, static_cast<const float*>(x), B, logits,
                                c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "forward launch");
  return SIM_OK;
}

void sim_destroy(sim_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->dev_weights) (void)hipFree(c->dev_weights);
  if (c->dev_block) (void)hipFree(c->dev_block);
  delete c;
}

const char* sim_last_error(const sim_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
