// Host side of the learned form: the DeepSets surrogate (parameters, Adam
// state, training batches) and the 1-NN search engine that uses it to order
// candidates, with the RWMD lower bound (Alg. 1) for pruning and the full
// method (Alg. 3) as the judge.  The NN problem is Problem NN of Sec. 6.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/w1approx.h"
#include "ctx.h"
#include "surrogate.h"

namespace w1 {

// Packed features of a list of diagrams on the device.
struct DiagSet {
  DBuf X, dstart;
  std::vector<int64_t> h_start;  // D + 1
  int64_t D = 0;
  void release() {
    for (DBuf* b : {&X, &dstart})
      if (b->p) (void)hipFree(b->p), b->p = nullptr, b->cap = 0;
  }
  int64_t count(int64_t i) const { return h_start[(size_t)i + 1] - h_start[(size_t)i]; }
};

struct Surrogate {
  int device = 0;
  DBuf params, m1, m2, grad, w1op, w2op, w2t;
  DBuf hbuf, pool, emb, gp, lpart, demb, dpool, cnt2, h1, h1t, mask2, xb, dz2, dz2t, dh1, part, stage;
  DiagSet set;
  int64_t step = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double last[3] = {0, 0, 0};
  DsOperands ops() { return DsOperands{(uint16_t*)w1op.p, (uint16_t*)w2op.p, (uint16_t*)w2t.p}; }
  std::vector<DBuf*> bufs() {
    return {&params, &m1, &m2, &grad, &w1op, &w2op, &w2t, &hbuf, &pool, &emb, &gp, &lpart, &demb, &dpool,
            &cnt2, &h1, &h1t, &mask2, &xb, &dz2, &dz2t, &dh1, &part, &stage};
  }
};

struct NNIndex {
  int device = 0;
  int dtype = W1_F32;
  int64_t m = 0;
  DBuf raw, emb;
  std::vector<w1_pd> views;  // device views of the database diagrams
  std::vector<double> stats; // m x NN_NSTATS dual-bound sums
  bool has_emb = false;
};

namespace {

inline uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline double unif(uint64_t& x) { return (double)(splitmix64(x) >> 11) * 0x1.0p-53; }

void init_params(std::vector<float>& p, uint64_t seed) {
  p.assign(DS_NPARAM, 0.f);
  uint64_t st = seed;
  auto fill = [&](int off, int n, double a) {
    for (int i = 0; i < n; ++i) p[(size_t)(off + i)] = (float)((2.0 * unif(st) - 1.0) * a);
  };
  fill(DS_OFF_W1, DS_H * 2, std::sqrt(6.0 / 2.0));
  fill(DS_OFF_B1, DS_H, 0.1);
  fill(DS_OFF_W2, DS_H * DS_H, std::sqrt(6.0 / DS_H));
  fill(DS_OFF_W3, DS_E * DS_H, 2e-3);
}

void upload_params(Ctx& c, Surrogate& s, const float* h) {
  upload(c, s.params.p, h, sizeof(float) * DS_NPARAM);
  fill_u32((uint32_t*)s.m1.p, 0, DS_NPARAM, c.st);
  fill_u32((uint32_t*)s.m2.p, 0, DS_NPARAM, c.st);
  ds_prep((const float*)s.params.p, s.ops(), c.st);
  check(c, hipGetLastError());
  check(c, hipStreamSynchronize(c.st));
  s.step = 0;
}

int check_pds(const w1_pd* d, int64_t k, int* dtype, int64_t* total) {
  if (k < 0 || (k > 0 && !d)) return W1_EINVAL;
  int dt = -1;
  int64_t tot = 0;
  for (int64_t i = 0; i < k; ++i) {
    if (d[i].n < 0 || (d[i].n > 0 && !d[i].xy) || (d[i].dtype != W1_F32 && d[i].dtype != W1_F64) || d[i].reserved)
      return W1_EINVAL;
    if (dt < 0) dt = d[i].dtype;
    if (d[i].dtype != dt) return W1_EINVAL;
    tot += d[i].n;
  }
  if (tot >= (int64_t(1) << 31)) return W1_EINVAL;
  *dtype = dt < 0 ? W1_F32 : dt;
  *total = tot;
  return W1_OK;
}

// Validate, drop diagonal points and pack (birth, persistence) of k diagrams
// into S (device).  Throws StageError.
void pack(Ctx& c, const w1_pd* d, int64_t k, bool dev_in, DBuf& stage, DiagSet& S) {
  int dtype;
  int64_t total;
  if (check_pds(d, k, &dtype, &total) != W1_OK) throw StageError{W1_EINVAL};
  const size_t esz = dtype == W1_F32 ? 4 : 8;
  std::vector<SegDesc> segs((size_t)k);
  char* st = (!dev_in && total > 0) ? need<char>(c, stage, total * 2 * (int64_t)esz) : nullptr;
  int64_t off = 0;
  for (int64_t i = 0; i < k; ++i) {
    const void* ptr = d[i].xy;
    if (!dev_in && d[i].n > 0) {
      check(c, hipMemcpyAsync(st + off * 2 * esz, d[i].xy, (size_t)d[i].n * 2 * esz, hipMemcpyHostToDevice, c.st));
      ptr = st + off * 2 * esz;
    }
    segs[(size_t)i] = SegDesc{ptr, d[i].n, off, (int32_t)i, 0};
    off += d[i].n;
  }
  S.D = k;
  S.h_start.assign((size_t)k + 1, 0);
  int64_t* dstart = need<int64_t>(c, S.dstart, k + 1);
  if (total == 0) {
    upload(c, dstart, S.h_start.data(), sizeof(int64_t) * (size_t)(k + 1));
    need<float2>(c, S.X, 1);
    return;
  }
  SegDesc* dsegs = need<SegDesc>(c, c.segs, k);
  upload(c, dsegs, segs.data(), segs.size() * sizeof(SegDesc));
  uint32_t* flag = need<uint32_t>(c, c.head, total + 1);
  uint32_t* pos = need<uint32_t>(c, c.idx, total + 1);
  int32_t* err = need<int32_t>(c, c.err, 1);
  fill_u32((uint32_t*)err, 0, 1, c.st);
  ds_flags(dsegs, (int)k, total, dtype, flag, err, c.st);
  scan_u32(flag, pos, total + 1, need<char>(c, c.scantmp, (int64_t)scan_tmp_bytes(total + 1, 4)), c.st);
  ds_seg_starts(dsegs, (int)k, pos, total, dstart, c.st);
  check(c, hipGetLastError());
  int32_t herr = 0;
  readback(c, err, &herr, 1);
  if (herr) throw StageError{W1_EINVAL};
  readback(c, dstart, S.h_start.data(), k + 1);
  float2* X = need<float2>(c, S.X, std::max<int64_t>(S.h_start[(size_t)k], 1));
  ds_scatter(dsegs, (int)k, total, dtype, flag, pos, X, c.st);
  check(c, hipGetLastError());
}

// Forward and backward over one batch: diagrams dl (indices into S), pairs
// (pa, pb) in batch-local indices, labels w.  Leaves the gradient in s.grad
// and returns the loss.
double grad_batch(Ctx& c, Surrogate& s, const DiagSet& S, const std::vector<int32_t>& dl,
                  const std::vector<int32_t>& pa, const std::vector<int32_t>& pb, const std::vector<double>& w) {
  const int64_t D = (int64_t)dl.size(), P = (int64_t)pa.size();
  std::vector<int64_t> roff((size_t)D + 1, 0);
  for (int64_t i = 0; i < D; ++i) roff[(size_t)i + 1] = roff[(size_t)i] + ((S.count(dl[(size_t)i]) + 31) & ~int64_t(31));
  const int64_t rows = roff[(size_t)D];
  std::vector<int32_t> occ_start((size_t)D + 1, 0), occ((size_t)(2 * P));
  for (int64_t j = 0; j < P; ++j) {
    ++occ_start[(size_t)pa[(size_t)j] + 1];
    ++occ_start[(size_t)pb[(size_t)j] + 1];
  }
  for (int64_t i = 0; i < D; ++i) occ_start[(size_t)i + 1] += occ_start[(size_t)i];
  {
    std::vector<int32_t> cur(occ_start.begin(), occ_start.end() - 1);
    for (int64_t j = 0; j < P; ++j) {
      occ[(size_t)cur[(size_t)pa[(size_t)j]]++] = (int32_t)(2 * j);
      occ[(size_t)cur[(size_t)pb[(size_t)j]]++] = (int32_t)(2 * j + 1);
    }
  }
  // one upload: roff | w | dl | pa | pb | occ_start | occ
  std::vector<char> h;
  auto put = [&](const void* src, size_t bytes) {
    const size_t at = (h.size() + 15) & ~size_t(15);
    h.resize(at + bytes);
    if (bytes) std::memcpy(h.data() + at, src, bytes);
    return at;
  };
  const size_t o_roff = put(roff.data(), roff.size() * 8);
  const size_t o_w = put(w.data(), w.size() * 8);
  const size_t o_dl = put(dl.data(), dl.size() * 4);
  const size_t o_pa = put(pa.data(), pa.size() * 4);
  const size_t o_pb = put(pb.data(), pb.size() * 4);
  const size_t o_os = put(occ_start.data(), occ_start.size() * 4);
  const size_t o_oc = put(occ.data(), occ.size() * 4);
  char* hd = need<char>(c, s.hbuf, (int64_t)h.size());
  upload(c, hd, h.data(), h.size());
  const int64_t* d_roff = (const int64_t*)(hd + o_roff);
  const double* d_w = (const double*)(hd + o_w);
  const int32_t* d_dl = (const int32_t*)(hd + o_dl);

  const float* prm = (const float*)s.params.p;
  float* grad = (float*)s.grad.p;
  float* pool = need<float>(c, s.pool, D * DS_H);
  float* emb = need<float>(c, s.emb, D * DS_E);
  int32_t* cnt2 = need<int32_t>(c, s.cnt2, D * DS_H);
  DsTrainRows tr;
  tr.roff = d_roff;
  tr.rows = rows;
  tr.h1 = need<uint16_t>(c, s.h1, rows * DS_H);
  tr.h1t = need<uint16_t>(c, s.h1t, rows * DS_H);
  tr.m2 = need<uint32_t>(c, s.mask2, rows * 4);
  tr.xb = need<float2>(c, s.xb, rows);
  tr.cnt2 = cnt2;
  float* gp = need<float>(c, s.gp, P * DS_E);
  double* lpart = need<double>(c, s.lpart, P);
  float* demb = need<float>(c, s.demb, D * DS_E);
  float* dpool = need<float>(c, s.dpool, D * DS_H);
  uint16_t* dz2 = need<uint16_t>(c, s.dz2, rows * DS_H);
  uint16_t* dz2t = need<uint16_t>(c, s.dz2t, rows * DS_H);
  float* dh1 = need<float>(c, s.dh1, rows * DS_H);
  const int64_t SL2 = 2048, SL1 = 1024;
  const int64_t nz2 = std::max<int64_t>(1, ceil_div(rows, SL2)), nz1 = std::max<int64_t>(1, ceil_div(rows, SL1));
  float* part = need<float>(c, s.part, std::max(nz2 * DS_H * DS_H, nz1 * 384));

  ds_embed((const float2*)S.X.p, (const int64_t*)S.dstart.p, d_dl, D, prm, s.ops(), pool, emb, &tr, c.st);
  ds_loss(emb, (const int32_t*)(hd + o_pa), (const int32_t*)(hd + o_pb), d_w, P, gp, lpart, c.st);
  ds_demb(gp, (const int32_t*)(hd + o_os), (const int32_t*)(hd + o_oc), D, demb, c.st);
  ds_dW3(demb, pool, D, grad, c.st);
  ds_dpool(demb, prm, D, dpool, c.st);
  ds_db2(dpool, cnt2, D, grad, c.st);
  if (rows > 0) {
    ds_dz2(tr.m2, dpool, d_roff, D, rows, dz2, dz2t, c.st);
    ds_gemm_nt(dz2t, tr.h1t, part, DS_H, DS_H, rows, SL2, c.st);
    ds_sum_slices(part, nz2, DS_H * DS_H, grad + DS_OFF_W2, c.st);
    ds_gemm_nt(dz2, (const uint16_t*)s.w2t.p, dh1, rows, DS_H, DS_H, DS_H, c.st);
    ds_dlayer1(dh1, tr.h1, tr.xb, rows, SL1, part, c.st);
    ds_sum_slices(part, nz1, 384, grad + DS_OFF_W1, c.st);
  } else {
    fill_u32((uint32_t*)(grad + DS_OFF_W1), 0, DS_OFF_B2 - DS_OFF_W1, c.st);
  }
  check(c, hipGetLastError());
  std::vector<double> hl((size_t)P);
  readback(c, lpart, hl.data(), P);
  double loss = 0.0;
  for (double v : hl) loss += v;
  return loss;
}

// Embed every diagram of S into emb (device, D x 64) in descending size
// order (long diagrams start first), timing the forward kernel.
void embed_set(Ctx& c, Surrogate& s, const DiagSet& S, float* emb) {
  std::vector<int32_t> order((size_t)S.D);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return S.count(a) > S.count(b); });
  int32_t* dl = need<int32_t>(c, s.hbuf, std::max<int64_t>(S.D, 1));
  upload(c, dl, order.data(), order.size() * 4);
  float* pool = need<float>(c, s.pool, std::max<int64_t>(S.D, 1) * DS_H);
  check(c, hipEventRecord(s.e0, c.st));
  ds_embed((const float2*)S.X.p, (const int64_t*)S.dstart.p, dl, S.D, (const float*)s.params.p, s.ops(), pool, emb,
           nullptr, c.st);
  check(c, hipEventRecord(s.e1, c.st));
  check(c, hipGetLastError());
  check(c, hipEventSynchronize(s.e1));
  float ms = 0.f;
  check(c, hipEventElapsedTime(&ms, s.e0, s.e1));
  s.last[0] = ms;
  s.last[1] = (double)S.h_start[(size_t)S.D];
  s.last[2] = (double)S.D;
}

// Dual-bound sums of k device-resident diagrams (host out, k x NN_NSTATS).
void dual_stats(Ctx& c, const w1_pd* v, int64_t k, int dtype, std::vector<double>& out) {
  out.assign((size_t)(k * NN_NSTATS), 0.0);
  if (k <= 0) return;
  std::vector<SegDesc> segs((size_t)k);
  for (int64_t i = 0; i < k; ++i) segs[(size_t)i] = SegDesc{v[i].xy, v[i].n, 0, (int32_t)i, 0};
  SegDesc* dsegs = need<SegDesc>(c, c.segs, k);
  upload(c, dsegs, segs.data(), segs.size() * sizeof(SegDesc));
  double* S = need<double>(c, c.lt, k * NN_NSTATS);
  int32_t* err = need<int32_t>(c, c.err, 1);
  fill_u32((uint32_t*)err, 0, 1, c.st);
  nn_stats(dsegs, (int)k, dtype, S, err, c.st);
  check(c, hipGetLastError());
  int32_t herr = 0;
  readback(c, err, &herr, 1);
  if (herr) throw StageError{W1_EINVAL};
  readback(c, S, out.data(), k * NN_NSTATS);
}

// Lower bound on W1(A, B) from the dual sums, reduced by their rounding margin.
double dual_bound(const double* sa, const double* sb) {
  double lb = 0.0;
  for (int j = 0; j < NN_NSTATS; ++j) lb = std::max(lb, std::fabs(sa[j] - sb[j]) - 1e-8 * (sa[j] + sb[j]));
  return lb;
}

template <typename F>
int guarded(Ctx* c, void* stream, F&& f) {
  if (hipSetDevice(c->device) != hipSuccess) return W1_EHIP;
  c->st = (hipStream_t)stream;
  try {
    return f();
  } catch (const StageError& e) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize((hipStream_t)stream);
    return e.code;
  } catch (const std::bad_alloc&) {
    return W1_ENOMEM;
  }
}

int check_pairs(int64_t k, const int64_t* pa, const int64_t* pb, const double* w, int64_t P) {
  if (P <= 0 || !pa || !pb || !w || P >= (int64_t(1) << 29)) return W1_EINVAL;
  for (int64_t j = 0; j < P; ++j)
    if (pa[j] < 0 || pa[j] >= k || pb[j] < 0 || pb[j] >= k || !(w[j] > 0.0) || !std::isfinite(w[j]))
      return W1_EINVAL;
  return W1_OK;
}

}  // namespace
}  // namespace w1

using namespace w1;

struct w1_surrogate : Surrogate {};
struct w1_nn_index : NNIndex {};

extern "C" {

int w1_surrogate_create(w1_ctx* c, uint64_t seed, w1_surrogate** out) {
  if (!c || !out) return W1_EINVAL;
  *out = nullptr;
  w1_surrogate* s = new (std::nothrow) w1_surrogate();
  if (!s) return W1_ENOMEM;
  s->device = c->device;
  const int rc = guarded(c, nullptr, [&]() {
    need<float>(*c, s->params, DS_NPARAM);
    need<float>(*c, s->m1, DS_NPARAM);
    need<float>(*c, s->m2, DS_NPARAM);
    need<float>(*c, s->grad, DS_NPARAM);
    need<uint16_t>(*c, s->w1op, 8 * 64 * 8);
    need<uint16_t>(*c, s->w2op, 8 * 4 * 64 * 8);
    need<uint16_t>(*c, s->w2t, DS_H * DS_H);
    check(*c, hipEventCreate(&s->e0));
    check(*c, hipEventCreate(&s->e1));
    std::vector<float> h;
    init_params(h, seed);
    upload_params(*c, *s, h.data());
    return W1_OK;
  });
  if (rc != W1_OK) {
    w1_surrogate_destroy(s);
    return rc;
  }
  *out = s;
  return W1_OK;
}

int w1_surrogate_destroy(w1_surrogate* s) {
  if (!s) return W1_EINVAL;
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  for (DBuf* b : s->bufs())
    if (b->p) (void)hipFree(b->p);
  s->set.release();
  if (s->e0) (void)hipEventDestroy(s->e0);
  if (s->e1) (void)hipEventDestroy(s->e1);
  delete s;
  return W1_OK;
}

int w1_surrogate_get_params(const w1_surrogate* s, float* out, int64_t n) {
  if (!s || !out || n != DS_NPARAM) return W1_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return W1_EHIP;
  if (hipDeviceSynchronize() != hipSuccess) return W1_EHIP;
  if (hipMemcpy(out, s->params.p, sizeof(float) * DS_NPARAM, hipMemcpyDeviceToHost) != hipSuccess) return W1_EHIP;
  return W1_OK;
}

int w1_surrogate_set_params(w1_surrogate* s, const float* in, int64_t n) {
  if (!s || !in || n != DS_NPARAM) return W1_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(in[i])) return W1_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return W1_EHIP;
  if (hipDeviceSynchronize() != hipSuccess) return W1_EHIP;
  if (hipMemcpy(s->params.p, in, sizeof(float) * DS_NPARAM, hipMemcpyHostToDevice) != hipSuccess) return W1_EHIP;
  if (hipMemset(s->m1.p, 0, sizeof(float) * DS_NPARAM) != hipSuccess) return W1_EHIP;
  if (hipMemset(s->m2.p, 0, sizeof(float) * DS_NPARAM) != hipSuccess) return W1_EHIP;
  ds_prep((const float*)s->params.p, s->ops(), nullptr);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return W1_EHIP;
  s->step = 0;
  return W1_OK;
}

int w1_surrogate_embed(w1_ctx* c, w1_surrogate* s, const w1_pd* d, int64_t k, uint32_t flags, void* stream,
                       float* emb_out) {
  if (!c || !s || !emb_out || k <= 0 || !d || s->device != c->device) return W1_EINVAL;
  return guarded(c, stream, [&]() {
    pack(*c, d, k, (flags & W1_INPUT_DEVICE) != 0, s->stage, s->set);
    float* emb = need<float>(*c, s->emb, k * DS_E);
    embed_set(*c, *s, s->set, emb);
    readback(*c, emb, emb_out, k * DS_E);
    return W1_OK;
  });
}

int w1_surrogate_grad(w1_ctx* c, w1_surrogate* s, const w1_pd* d, int64_t k, const int64_t* pa, const int64_t* pb,
                      const double* w, int64_t npairs, uint32_t flags, void* stream, double* loss_out,
                      float* grad_out) {
  if (!c || !s || !d || k <= 0 || s->device != c->device || (!loss_out && !grad_out)) return W1_EINVAL;
  if (check_pairs(k, pa, pb, w, npairs) != W1_OK) return W1_EINVAL;
  return guarded(c, stream, [&]() {
    pack(*c, d, k, (flags & W1_INPUT_DEVICE) != 0, s->stage, s->set);
    std::vector<int32_t> dl((size_t)k), a((size_t)npairs), b((size_t)npairs);
    std::iota(dl.begin(), dl.end(), 0);
    for (int64_t j = 0; j < npairs; ++j) a[(size_t)j] = (int32_t)pa[j], b[(size_t)j] = (int32_t)pb[j];
    std::vector<double> wl(w, w + npairs);
    const double loss = grad_batch(*c, *s, s->set, dl, a, b, wl);
    if (loss_out) *loss_out = loss;
    if (grad_out) readback(*c, (const float*)s->grad.p, grad_out, DS_NPARAM);
    return W1_OK;
  });
}

int w1_surrogate_train(w1_ctx* c, w1_surrogate* s, const w1_pd* d, int64_t k, const int64_t* pa, const int64_t* pb,
                       const double* w, int64_t npairs, const w1_train_params* tp, uint32_t flags, void* stream,
                       double* epoch_loss_out) {
  if (!c || !s || !d || k <= 0 || !tp || s->device != c->device) return W1_EINVAL;
  if (tp->epochs < 0 || tp->batch_pairs <= 0) return W1_EINVAL;
  if (check_pairs(k, pa, pb, w, npairs) != W1_OK) return W1_EINVAL;
  const float lr = tp->lr > 0 ? tp->lr : 1e-3f, b1 = tp->beta1 > 0 ? tp->beta1 : 0.9f,
              b2 = tp->beta2 > 0 ? tp->beta2 : 0.999f, ae = tp->adam_eps > 0 ? tp->adam_eps : 1e-8f;
  return guarded(c, stream, [&]() {
    pack(*c, d, k, (flags & W1_INPUT_DEVICE) != 0, s->stage, s->set);
    std::vector<int64_t> order((size_t)npairs);
    std::iota(order.begin(), order.end(), 0);
    std::vector<int32_t> slot((size_t)k, -1), stamp((size_t)k, -1);
    uint64_t rng = tp->seed;
    int32_t batch_id = 0;
    for (int ep = 0; ep < tp->epochs; ++ep) {
      for (int64_t i = npairs - 1; i > 0; --i) {
        const int64_t j = (int64_t)(splitmix64(rng) % (uint64_t)(i + 1));
        std::swap(order[(size_t)i], order[(size_t)j]);
      }
      double ep_loss = 0.0;
      for (int64_t b0 = 0; b0 < npairs; b0 += tp->batch_pairs) {
        const int64_t b1e = std::min<int64_t>(npairs, b0 + tp->batch_pairs);
        std::vector<int32_t> dl, la, lb;
        std::vector<double> lw;
        auto local = [&](int64_t g) {
          if (stamp[(size_t)g] != batch_id) {
            stamp[(size_t)g] = batch_id;
            slot[(size_t)g] = (int32_t)dl.size();
            dl.push_back((int32_t)g);
          }
          return slot[(size_t)g];
        };
        for (int64_t t = b0; t < b1e; ++t) {
          const int64_t j = order[(size_t)t];
          la.push_back(local(pa[j]));
          lb.push_back(local(pb[j]));
          lw.push_back(w[j]);
        }
        ++batch_id;
        const double loss = grad_batch(*c, *s, s->set, dl, la, lb, lw);
        ep_loss += loss * (double)(b1e - b0) / (double)npairs;
        ++s->step;
        const float bc1 = 1.f - std::pow(b1, (float)s->step), bc2 = 1.f - std::pow(b2, (float)s->step);
        ds_adam((float*)s->params.p, (const float*)s->grad.p, (float*)s->m1.p, (float*)s->m2.p, DS_NPARAM, lr, b1, b2,
                ae, bc1, bc2, c->st);
        ds_prep((const float*)s->params.p, s->ops(), c->st);
        check(*c, hipGetLastError());
      }
      if (epoch_loss_out) epoch_loss_out[ep] = ep_loss;
    }
    check(*c, hipStreamSynchronize(c->st));
    return W1_OK;
  });
}

int w1_surrogate_last_times(const w1_surrogate* s, double* out, int n) {
  if (!s || !out || n < 3) return W1_EINVAL;
  for (int i = 0; i < 3; ++i) out[i] = s->last[i];
  return W1_OK;
}

int w1_nn_build(w1_ctx* c, w1_surrogate* s, const w1_pd* db, int64_t m, uint32_t flags, void* stream,
                w1_nn_index** out) {
  if (!c || !out || !db || m <= 0 || (s && s->device != c->device)) return W1_EINVAL;
  *out = nullptr;
  int dtype;
  int64_t total;
  if (check_pds(db, m, &dtype, &total) != W1_OK) return W1_EINVAL;
  w1_nn_index* x = new (std::nothrow) w1_nn_index();
  if (!x) return W1_ENOMEM;
  x->device = c->device;
  x->dtype = dtype;
  x->m = m;
  const bool dev_in = (flags & W1_INPUT_DEVICE) != 0;
  const int rc = guarded(c, stream, [&]() {
    const size_t row = dtype == W1_F32 ? 8 : 16;
    char* raw = need<char>(*c, x->raw, std::max<int64_t>(total, 1) * (int64_t)row);
    x->views.resize((size_t)m);
    int64_t off = 0;
    for (int64_t i = 0; i < m; ++i) {
      if (db[i].n > 0)
        check(*c, hipMemcpyAsync(raw + off * row, db[i].xy, (size_t)db[i].n * row,
                                 dev_in ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->st));
      x->views[(size_t)i] = w1_pd{raw + off * row, db[i].n, dtype, 0};
      off += db[i].n;
    }
    check(*c, hipStreamSynchronize(c->st));
    dual_stats(*c, x->views.data(), m, dtype, x->stats);
    if (s) {
      pack(*c, x->views.data(), m, true, s->stage, s->set);
      float* emb = need<float>(*c, x->emb, m * DS_E);
      embed_set(*c, *s, s->set, emb);
      x->has_emb = true;
    }
    return W1_OK;
  });
  if (rc != W1_OK) {
    w1_nn_destroy(x);
    return rc;
  }
  *out = x;
  return W1_OK;
}

int w1_nn_destroy(w1_nn_index* x) {
  if (!x) return W1_EINVAL;
  (void)hipSetDevice(x->device);
  (void)hipDeviceSynchronize();
  if (x->raw.p) (void)hipFree(x->raw.p);
  if (x->emb.p) (void)hipFree(x->emb.p);
  delete x;
  return W1_OK;
}

int w1_nn_query(w1_ctx* c, w1_nn_index* x, w1_surrogate* s, const w1_pd* q, int64_t nq, const w1_nn_params* p,
                uint32_t flags, void* stream, int64_t* nn_out, double* w1_out, int64_t* verif_out,
                w1_nn_stats* stats) {
  if (!c || !x || !p || nq < 0 || (nq > 0 && (!q || !nn_out)) || x->device != c->device) return W1_EINVAL;
  if (p->seed_k < 0 || p->keep < 0 || p->reserved != 0 || p->mode < W1_NN_RWMD || p->mode > W1_NN_PIPELINE ||
      !(p->eps > 0.0 && p->eps <= 1.0))
    return W1_EINVAL;
  if (p->mode == W1_NN_SURROGATE && (!s || !x->has_emb || s->device != c->device)) return W1_EINVAL;
  int dtype;
  int64_t total;
  if (check_pds(q, nq, &dtype, &total) != W1_OK) return W1_EINVAL;
  if (nq > 0 && dtype != x->dtype) return W1_EINVAL;
  w1_nn_stats st{};
  if (nq == 0) {
    if (stats) *stats = st;
    return W1_OK;
  }
  const int64_t m = x->m;
  using clk = std::chrono::steady_clock;
  auto ms_since = [](clk::time_point t0) { return std::chrono::duration<double, std::milli>(clk::now() - t0).count(); };
  const auto t_start = clk::now();
  const bool dev_in = (flags & W1_INPUT_DEVICE) != 0;
  DBuf qraw;
  std::vector<w1_pd> qv((size_t)nq);
  std::vector<double> qstats;
  int rc = guarded(c, stream, [&]() {
    const size_t row = dtype == W1_F32 ? 8 : 16;
    char* raw = need<char>(*c, qraw, std::max<int64_t>(total, 1) * (int64_t)row);
    int64_t off = 0;
    for (int64_t i = 0; i < nq; ++i) {
      if (q[i].n > 0)
        check(*c, hipMemcpyAsync(raw + off * row, q[i].xy, (size_t)q[i].n * row,
                                 dev_in ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->st));
      qv[(size_t)i] = w1_pd{raw + off * row, q[i].n, dtype, 0};
      off += q[i].n;
    }
    check(*c, hipStreamSynchronize(c->st));
    dual_stats(*c, qv.data(), nq, dtype, qstats);  // also validates the queries
    return W1_OK;
  });

  std::vector<double> L((size_t)(nq * m), -1.0);
  // RWMD bounds of the listed (query, candidate) pairs, batched.
  auto rwmd = [&](const std::vector<std::vector<int32_t>>& lists) {
    const auto t0 = clk::now();
    std::vector<w1_pd> A, B;
    std::vector<int64_t> slot;
    std::vector<double> val;
    int64_t pts = 0;
    int r = W1_OK;
    auto flush = [&]() {
      if (A.empty() || r != W1_OK) return;
      val.assign(A.size(), 0.0);
      r = w1_rwmd(c, A.data(), B.data(), (int64_t)A.size(), W1_INPUT_DEVICE, stream, val.data());
      if (r == W1_OK)
        for (size_t t = 0; t < slot.size(); ++t) L[(size_t)slot[t]] = val[t];
      A.clear();
      B.clear();
      slot.clear();
      pts = 0;
    };
    for (int64_t i = 0; i < nq && r == W1_OK; ++i)
      for (int32_t j : lists[(size_t)i]) {
        const w1_pd& a = qv[(size_t)i];
        const w1_pd& b = x->views[(size_t)j];
        if (!A.empty() && (pts + a.n + b.n >= (int64_t(1) << 27) || (int64_t)A.size() >= (int64_t(1) << 16))) flush();
        A.push_back(a);
        B.push_back(b);
        slot.push_back(i * m + j);
        pts += a.n + b.n;
        ++st.rwmd_evals;
      }
    flush();
    st.t_rwmd_ms += ms_since(t0);
    return r;
  };

  std::vector<double> best_w((size_t)nq, INFINITY);
  std::vector<int64_t> best_i((size_t)nq, -1), nver((size_t)nq, 0);
  std::vector<char> done((size_t)(nq * m), 0);
  // Verification rounds over per-query candidate lists.  policy 0: verify
  // all; 1: skip candidates whose RWMD exceeds the best; 2: as 1, and stop
  // at the first such candidate (lists sorted by RWMD).
  auto verify = [&](const std::vector<std::vector<int32_t>>& lists, int policy) {
    const auto t0 = clk::now();
    std::vector<int64_t> cur((size_t)nq, 0);
    std::vector<char> live((size_t)nq, 1);
    // verifications solve the network without its diagonal-dominated pairs:
    // the same optimum, hence the same w1, with a smaller flow problem
    w1_params wp{p->eps, 0.1, 0, W1_INPUT_DEVICE | W1_PRUNE, 0};
    int r = W1_OK;
    for (;;) {
      std::vector<int64_t> who, cand;
      for (int64_t i = 0; i < nq; ++i) {
        if (!live[(size_t)i]) continue;
        const std::vector<int32_t>& o = lists[(size_t)i];
        int64_t& k = cur[(size_t)i];
        int64_t pick = -1;
        while (k < (int64_t)o.size()) {
          const int32_t j = o[(size_t)k];
          if (done[(size_t)(i * m + j)]) {
            ++k;
            continue;
          }
          if (policy > 0 && L[(size_t)(i * m + j)] > best_w[(size_t)i]) {
            if (policy == 2) k = (int64_t)o.size();  // sorted: all later ones are ruled out
            else ++k;
            continue;
          }
          pick = j;
          ++k;
          break;
        }
        if (pick < 0) {
          live[(size_t)i] = 0;
          continue;
        }
        who.push_back(i);
        cand.push_back(pick);
      }
      if (who.empty()) break;
      std::vector<w1_pd> A, B;
      for (size_t t = 0; t < who.size(); ++t) {
        A.push_back(qv[(size_t)who[t]]);
        B.push_back(x->views[(size_t)cand[t]]);
      }
      std::vector<w1_result> res(who.size());
      std::memset(res.data(), 0, res.size() * sizeof(w1_result));
      r = w1_approx_batch(c, A.data(), B.data(), (int64_t)who.size(), &wp, stream, res.data());
      for (size_t t = 0; t < who.size() && r == W1_OK; ++t)
        if (res[t].status < 0) r = res[t].status;
      if (r == W1_OK)
        for (size_t t = 0; t < who.size(); ++t) {
          const int64_t i = who[t], j = cand[t];
          const double v = res[t].w1;
          ++nver[(size_t)i];
          done[(size_t)(i * m + j)] = 1;
          if (v < best_w[(size_t)i] || (v == best_w[(size_t)i] && j < best_i[(size_t)i])) {
            best_w[(size_t)i] = v;
            best_i[(size_t)i] = j;
          }
        }
      for (auto& rr : res) w1_result_free(&rr);
      ++st.rounds;
      if (r != W1_OK) break;
    }
    st.t_verify_ms += ms_since(t0);
    return r;
  };
  // The method at s = 1 on the paper's grid for s = 1 (Alg. 2: eps_c = 1) for
  // the listed pairs, batched: an upper bound on W1 that orders candidates.
  std::vector<double> S1((size_t)(nq * m), INFINITY);
  auto sparse = [&](const std::vector<std::vector<int32_t>>& lists) {
    const auto t0 = clk::now();
    w1_params sp{p->eps, 0.1, 1, W1_INPUT_DEVICE | W1_PRUNE | W1_PAPER_GRID, 0};
    std::vector<w1_pd> A, B;
    std::vector<int64_t> slot;
    int64_t pts = 0;
    int r = W1_OK;
    auto flush = [&]() {
      if (A.empty() || r != W1_OK) return;
      std::vector<w1_result> res(A.size());
      std::memset(res.data(), 0, res.size() * sizeof(w1_result));
      r = w1_approx_batch(c, A.data(), B.data(), (int64_t)A.size(), &sp, stream, res.data());
      for (size_t t = 0; t < res.size() && r == W1_OK; ++t)
        if (res[t].status < 0) r = res[t].status;
      if (r == W1_OK)
        for (size_t t = 0; t < slot.size(); ++t) S1[(size_t)slot[t]] = res[t].w1;
      for (auto& rr : res) w1_result_free(&rr);
      A.clear();
      B.clear();
      slot.clear();
      pts = 0;
    };
    for (int64_t i = 0; i < nq && r == W1_OK; ++i)
      for (int32_t j : lists[(size_t)i]) {
        const w1_pd& a = qv[(size_t)i];
        const w1_pd& b = x->views[(size_t)j];
        if (!A.empty() && (pts + a.n + b.n >= (int64_t(1) << 24) || (int64_t)A.size() >= 4096)) flush();
        A.push_back(a);
        B.push_back(b);
        slot.push_back(i * m + j);
        pts += a.n + b.n;
        ++st.sparse_evals;
      }
    flush();
    st.t_sparse_ms += ms_since(t0);
    return r;
  };
  auto sort_by_L = [&](std::vector<std::vector<int32_t>>& lists) {
    for (int64_t i = 0; i < nq; ++i) {
      const double* Li = L.data() + i * m;
      std::stable_sort(lists[(size_t)i].begin(), lists[(size_t)i].end(),
                       [&](int32_t a, int32_t b) { return Li[a] < Li[b]; });
    }
  };

  std::vector<std::vector<int32_t>> all((size_t)nq);
  for (auto& o : all) {
    o.resize((size_t)m);
    std::iota(o.begin(), o.end(), 0);
  }
  if (rc == W1_OK && p->mode == W1_NN_EXHAUSTIVE) {
    rc = verify(all, 0);
  } else if (rc == W1_OK && (p->mode == W1_NN_SPARSE || p->mode == W1_NN_PIPELINE)) {
    // RWMD for every pair, the s = 1 stage on the `keep` nearest by RWMD,
    // then the seed_k best of those verified (the pipeline stops there)
    const bool pipeline = p->mode == W1_NN_PIPELINE;
    const int64_t keep = std::min<int64_t>(m, p->keep > 0 ? p->keep : 15);
    const int64_t c2 = std::min<int64_t>(keep, p->seed_k > 0 ? p->seed_k : (pipeline ? 3 : 1));
    rc = rwmd(all);
    std::vector<std::vector<int32_t>> head((size_t)nq);
    if (rc == W1_OK) {
      sort_by_L(all);
      for (int64_t i = 0; i < nq; ++i) head[(size_t)i].assign(all[(size_t)i].begin(), all[(size_t)i].begin() + keep);
      rc = sparse(head);
    }
    if (rc == W1_OK) {
      for (int64_t i = 0; i < nq; ++i) {
        const double* si = S1.data() + i * m;
        std::vector<int32_t>& o = head[(size_t)i];
        std::stable_sort(o.begin(), o.end(), [&](int32_t a, int32_t b) { return si[a] < si[b]; });
        o.resize((size_t)c2);
      }
      rc = verify(head, 0);
    }
    if (rc == W1_OK && !pipeline) rc = verify(all, 2);
  } else if (rc == W1_OK && p->mode == W1_NN_RWMD) {
    rc = rwmd(all);
    if (rc == W1_OK) {
      sort_by_L(all);
      rc = verify(all, 2);
    }
  } else if (rc == W1_OK) {
    // surrogate ranking, seeds, dual-bound gate, RWMD on the survivors
    const auto t0 = clk::now();
    std::vector<float> score((size_t)(nq * m));
    rc = guarded(c, stream, [&]() {
      pack(*c, qv.data(), nq, true, s->stage, s->set);
      float* eq = need<float>(*c, s->emb, nq * DS_E);
      embed_set(*c, *s, s->set, eq);
      float* sc = need<float>(*c, s->gp, nq * m);
      ds_scores(eq, nq, (const float*)x->emb.p, m, sc, c->st);
      check(*c, hipGetLastError());
      readback(*c, sc, score.data(), nq * m);
      return W1_OK;
    });
    const int64_t k = std::min<int64_t>(m, p->seed_k > 0 ? p->seed_k : 1);
    std::vector<std::vector<int32_t>> seeds((size_t)nq);
    for (int64_t i = 0; i < nq; ++i) {
      std::vector<int32_t>& o = all[(size_t)i];
      const float* si = score.data() + i * m;
      std::partial_sort(o.begin(), o.begin() + k, o.end(),
                        [&](int32_t a, int32_t b) { return si[a] < si[b] || (si[a] == si[b] && a < b); });
      seeds[(size_t)i].assign(o.begin(), o.begin() + k);
    }
    st.t_embed_ms += ms_since(t0);
    if (rc == W1_OK) rc = verify(seeds, 0);
    if (rc == W1_OK) {
      const auto t1 = clk::now();
      std::vector<std::vector<int32_t>> live((size_t)nq);
      for (int64_t i = 0; i < nq; ++i) {
        const double* sq = qstats.data() + i * NN_NSTATS;
        for (int64_t j = 0; j < m; ++j)
          if (!done[(size_t)(i * m + j)] && dual_bound(sq, x->stats.data() + j * NN_NSTATS) <= best_w[(size_t)i])
            live[(size_t)i].push_back((int32_t)j);
      }
      st.t_embed_ms += ms_since(t1);
      rc = rwmd(live);
      if (rc == W1_OK) {
        sort_by_L(live);
        rc = verify(live, 2);
      }
    }
  }
  if (rc == W1_OK)
    for (int64_t i = 0; i < nq; ++i) {
      nn_out[i] = best_i[(size_t)i];
      if (w1_out) w1_out[i] = best_w[(size_t)i];
      if (verif_out) verif_out[i] = nver[(size_t)i];
      st.verifications += nver[(size_t)i];
    }
  if (qraw.p) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(qraw.p);
  }
  st.t_total_ms = ms_since(t_start);
  if (stats) *stats = st;
  return rc;
}

}  // extern "C"
