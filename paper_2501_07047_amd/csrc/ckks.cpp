// CKKS operations of the C ABI: polynomial product, basis conversion, hybrid
// key switching (ModUp / inner product / ModDown), HE-Mult and Rotate.
//
// The paper (arXiv 2501.07047) evaluates HE-Mult and Rotate with dnum-digit
// hybrid key switching (Tab. perf_cmp, Sec. Evaluation latency breakdown) and
// maps its BConv onto the matrix engine with BAT (App. "Basis Conversion");
// it cites rather than defines the key switch, so the steps follow the usual
// hybrid form: digits of alpha = ceil(L/dnum) consecutive limbs; ModUp = INTT,
// BConv of each digit to all other limbs, NTT; inner product with the
// evaluation key; ModDown = INTT of the special limbs, BConv to Q, NTT,
// (x - y) * P^-1.  All buffers are in NTT form; limbs are ordered Q then P.
#include <cstring>
#include <memory>
#include <string>

#include "context.h"
#include "params.h"
#include "ckks_plan.h"

#include <algorithm>

namespace cross {

namespace {

LimbMod limb_mod(uint32_t q) {
  LimbMod m{};
  int k = 0;
  while ((1ull << k) <= q) ++k;           // bit length
  m.q = q;
  m.bar_k = (uint32_t)k;
  m.bar_m = (uint32_t)(((unsigned __int128)1 << (2 * k)) / q);
  return m;
}

uint32_t shoup(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }

StreamMod stream_mod(uint32_t q) {
  const LimbMod l = limb_mod(q);
  StreamMod m{};
  m.q = q;
  m.bar_m = l.bar_m;
  m.bar_k = l.bar_k;
  m.qneg = (uint32_t)(0u - inv_mod_2_32(q));
  for (int i = 0; i < 4; ++i) m.pow2[i] = powmod(2, 32 + 8 * i, q);
  return m;
}

// Balanced base-256 digits of v: v = sum_i d_i 256^i, d_i in [-128, 127] (v within
// [-128 * 0x1010101, 127 * 0x1010101]).
void balanced_digits4(int64_t v, int8_t (&d)[4]) {
  for (int i = 0; i < 4; ++i) {
    int64_t r = ((v % 256) + 256) % 256;
    if (r >= 128) r -= 256;
    d[i] = (int8_t)r;
    v = (v - r) / 256;
  }
}

// Fragment-ordered BAT table of the BConv matrix [qhat_i]_t (see bconv_kernel).
// Narrow primes: 7-bit chunks ii of ([qhat_i]_t 2^32 2^(7j)) mod t.  With a wide
// prime among sources or targets: balanced signed 8-bit digits ii of the
// representative of ([qhat_i]_t 2^32 2^(8j)) mod t in [-128 * 0x1010101, 127 * 0x1010101],
// followed by the int32 correction 128 * (sum of the row's digits) of every output
// row (mblocks x 32), which undoes the operand bias b - 128.
std::vector<int8_t> bconv_table(const std::vector<uint32_t>& src, const std::vector<uint32_t>& dst, bool wide) {
  const int ns = (int)src.size(), nd = (int)dst.size();
  const int kb = (ns + 7) / 8, mb = (nd + 7) / 8;
  std::vector<int8_t> out((size_t)mb * kb * 1024 + (wide ? (size_t)mb * 32 * 4 : 0), 0);
  // Montgomery-form [qhat_i]_t
  std::vector<uint32_t> qh((size_t)nd * ns);
  for (int t = 0; t < nd; ++t) {
    const uint32_t p = dst[t];
    for (int i = 0; i < ns; ++i) {
      uint64_t h = 1;
      for (int i2 = 0; i2 < ns; ++i2)
        if (i2 != i) h = h * (src[i2] % p) % p;
      qh[(size_t)t * ns + i] = (uint32_t)(h * (((uint64_t)1 << 32) % p) % p);
    }
  }
  std::vector<int64_t> rowsum((size_t)mb * 32, 0);
  const int64_t hi = 127 * (int64_t)0x1010101;
  for (int m = 0; m < mb; ++m)
    for (int k = 0; k < kb; ++k)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 16; ++e) {
          const int row = m * 32 + (lane & 31);
          const int t = row / 4, ii = row % 4;
          const int i = k * 8 + (lane >> 5) * 4 + e / 4, j = e % 4;
          int8_t v = 0;
          if (t < nd && i < ns) {
            const uint32_t p = dst[t];
            if (wide) {
              const uint64_t x = ((uint64_t)qh[(size_t)t * ns + i] << (8 * j)) % p;
              int8_t dg[4];
              balanced_digits4((int64_t)x > hi ? (int64_t)x - (int64_t)p : (int64_t)x, dg);
              v = dg[ii];
            } else {
              const uint64_t x = ((uint64_t)qh[(size_t)t * ns + i] << (kChunkBits * j)) % p;
              v = (int8_t)((x >> (kChunkBits * ii)) & 0x7f);
            }
          }
          out[((size_t)(m * kb + k) * 1024) + lane * 16 + e] = v;
          rowsum[row] += v;
        }
  if (wide)
    for (int r = 0; r < mb * 32; ++r) {
      const int32_t c = (int32_t)(128 * rowsum[r]);
      std::memcpy(&out[(size_t)mb * kb * 1024 + 4 * (size_t)r], &c, 4);
    }
  return out;
}

cross_status make_bconv(cross_ctx ctx, const std::vector<uint32_t>& sp, const std::vector<uint64_t>& soff,
                        const std::vector<uint32_t>& dp, const std::vector<uint64_t>& doff,
                        BconvStatic* out) {
  std::vector<BconvSrc> s(sp.size());
  for (size_t i = 0; i < sp.size(); ++i) {
    uint64_t h = 1;
    for (size_t i2 = 0; i2 < sp.size(); ++i2)
      if (i2 != i) h = h * (sp[i2] % sp[i]) % sp[i];
    uint32_t w = powmod(h, sp[i] - 2, sp[i]);
    s[i] = BconvSrc{soff[i], sp[i], w, shoup(w, sp[i]), 0};
  }
  std::vector<BconvDst> d(dp.size());
  for (size_t t = 0; t < dp.size(); ++t) d[t] = BconvDst{doff[t], dp[t], inv_mod_2_32(dp[t])};
  bool wide = false;
  for (uint32_t q : sp) wide = wide || wide_prime(q);
  for (uint32_t q : dp) wide = wide || wide_prime(q);
  std::vector<int8_t> tab = bconv_table(sp, dp, wide);
  void *a = nullptr, *b = nullptr, *c = nullptr;
  cross_status st = cached_device_copy(ctx, s.data(), s.size() * sizeof(BconvSrc), &a);
  if (st == CROSS_OK) st = cached_device_copy(ctx, d.data(), d.size() * sizeof(BconvDst), &b);
  if (st == CROSS_OK) st = cached_device_copy(ctx, tab.data(), tab.size(), &c);
  if (st != CROSS_OK) return st;
  out->src = (const BconvSrc*)a;
  out->dst = (const BconvDst*)b;
  out->table = (const int8_t*)c;
  out->nsrc = (int)sp.size();
  out->ndst = (int)dp.size();
  out->wide = wide ? 1 : 0;
  return CROSS_OK;
}

hipError_t run_bconv(cross_ctx ctx, const BconvStatic& bs, const uint32_t* in, uint64_t in_stride,
                     uint32_t* out, uint64_t out_stride, int npoly, int log_n, hipStream_t s) {
  BconvLaunch g{bs.src, bs.dst, bs.table, bs.nsrc, bs.ndst, in, out, in_stride, out_stride, npoly, log_n, bs.wide};
  ProfScope ps(ctx, "bconv", s);
  return launch_bconv(g, s);
}




cross_status validate_primes(cross_ctx ctx, const uint32_t* p, uint32_t n, uint32_t log_n, bool wide_ok = false) {
  for (uint32_t i = 0; i < n; ++i) {
    cross_status st = check_prime(ctx, p[i], log_n, wide_ok);
    if (st != CROSS_OK) return st;
    for (uint32_t j = 0; j < i; ++j)
      if (p[j] == p[i]) return fail(ctx, CROSS_EINVAL, "primes must be pairwise distinct");
  }
  return CROSS_OK;
}

}  // namespace

cross_status get_ckks_plan(cross_ctx ctx, const cross_ckks_params* prm, CkksPlan** out) {
  if (!prm || !prm->primes) return fail(ctx, CROSS_EINVAL, "null params");
  if (prm->log_n < 5 || prm->log_n > CROSS_MAX_LOG_N) return fail(ctx, CROSS_EINVAL, "log_n out of range [5, 16]");
  if (prm->L < 1 || prm->K < 1 || prm->dnum < 1 || prm->L + prm->K > CROSS_MAX_LIMBS)
    return fail(ctx, CROSS_EINVAL, "need L >= 1, K >= 1, dnum >= 1, L + K <= 64");
  const int L = (int)prm->L, K = (int)prm->K, dnum = (int)prm->dnum;
  const int alpha = (L + dnum - 1) / dnum;
  if (alpha > 32 || K > 32) return fail(ctx, CROSS_EUNSUPPORTED, "digit or special basis above 32 limbs");
  std::string key((const char*)prm->primes, (L + K) * 4);
  key += std::to_string(prm->log_n) + "/" + std::to_string(L) + "/" + std::to_string(K) + "/" +
         std::to_string(dnum) + "/" + std::to_string(split_of(ctx, (int)prm->log_n));
  {
    int lr = 0, lc1 = 0;
    effective_split(ctx, (int)prm->log_n, true, &lr, &lc1);
    key += "/" + std::to_string(lr) + "x" + std::to_string(lc1);
  }
  auto it = ctx->ext_plans.find(key);
  if (it != ctx->ext_plans.end()) {
    *out = static_cast<CkksPlan*>(it->second.get());
    return CROSS_OK;
  }
  cross_status st = validate_primes(ctx, prm->primes, L + K, prm->log_n, true);
  if (st != CROSS_OK) return st;
  std::shared_ptr<CkksPlan> holder = std::make_shared<CkksPlan>();
  CkksPlan* c = holder.get();
  for (int i = 0; i < L + K; ++i) c->wide = c->wide || wide_prime(prm->primes[i]);
  c->log_n = (int)prm->log_n;
  c->L = L;
  c->K = K;
  c->dnum = dnum;
  c->alpha = alpha;
  c->ndig = (L + alpha - 1) / alpha;
  c->primes.assign(prm->primes, prm->primes + L + K);
  const uint64_t N = 1ull << prm->log_n;
  for (int i = 0; i < L + K; ++i) {
    Plan* p = nullptr;
    st = get_plan(ctx, c->primes[i], c->log_n, &p);
    if (st != CROSS_OK) return st;
    c->plans.push_back(p);
    Plan* p2 = nullptr;
    st = get_plan(ctx, c->primes[i], c->log_n, &p2, false);
    if (st != CROSS_OK) return st;
    c->plans2.push_back(p2);
  }
  std::vector<LimbMod> mods(L + K);
  for (int i = 0; i < L + K; ++i) mods[i] = limb_mod(c->primes[i]);
  uint64_t P = 1;
  std::vector<TailConst> tail(L);
  for (int i = 0; i < L; ++i) {
    const uint32_t q = c->primes[i];
    uint64_t pm = 1;
    for (int k = 0; k < K; ++k) pm = pm * (c->primes[L + k] % q) % q;
    uint32_t pinv = powmod(pm, q - 2, q);
    tail[i] = TailConst{q, pinv, shoup(pinv, q), 0};
  }
  (void)P;
  void *dm = nullptr, *dt = nullptr;
  st = cached_device_copy(ctx, mods.data(), mods.size() * sizeof(LimbMod), &dm);
  if (st == CROSS_OK) st = cached_device_copy(ctx, tail.data(), tail.size() * sizeof(TailConst), &dt);
  if (st != CROSS_OK) return st;
  c->mods = (const LimbMod*)dm;
  c->tail = (const TailConst*)dt;
  // ModUp BConvs: digit j (limbs [lo, hi) of x [L][N]) -> ext[j][t] for t outside the digit
  std::vector<uint64_t> csrc, cdst;
  for (int j = 0; j < c->ndig; ++j) {
    const int lo = j * alpha, hi = std::min(L, (j + 1) * alpha);
    std::vector<uint32_t> sp, dp;
    std::vector<uint64_t> so, dof;
    std::vector<int> tg;
    for (int i = lo; i < hi; ++i) {
      sp.push_back(c->primes[i]);
      so.push_back((uint64_t)i * N);
      csrc.push_back((uint64_t)i * N);
      cdst.push_back(((uint64_t)j * (L + K) + i) * N);
    }
    for (int t = 0; t < L + K; ++t) {
      if (t >= lo && t < hi) continue;
      dp.push_back(c->primes[t]);
      dof.push_back(((uint64_t)j * (L + K) + t) * N);
      tg.push_back(t);
    }
    BconvStatic bs;
    st = make_bconv(ctx, sp, so, dp, dof, &bs);
    if (st != CROSS_OK) return st;
    c->modup.push_back(bs);
    c->targets.push_back(tg);
  }
  void *a = nullptr, *b = nullptr;
  st = cached_device_copy(ctx, csrc.data(), csrc.size() * 8, &a);
  if (st == CROSS_OK) st = cached_device_copy(ctx, cdst.data(), cdst.size() * 8, &b);
  if (st != CROSS_OK) return st;
  c->copy_src = (const uint64_t*)a;
  c->copy_dst = (const uint64_t*)b;
  // ModDown BConv: P limbs (coefficient form, [K][N] per poly) -> Q limbs ([L][N] per poly)
  {
    std::vector<uint32_t> sp(c->primes.begin() + L, c->primes.end()), dp(c->primes.begin(), c->primes.begin() + L);
    std::vector<uint64_t> so(K), dof(L);
    for (int k = 0; k < K; ++k) so[k] = (uint64_t)(L + k) * N;
    for (int i = 0; i < L; ++i) dof[i] = (uint64_t)i * N;
    st = make_bconv(ctx, sp, so, dp, dof, &c->moddown);
    if (st != CROSS_OK) return st;
  }
  ctx->ext_plans[key] = holder;
  *out = c;
  return CROSS_OK;
}

cross_status perm_table(cross_ctx ctx, int log_n, uint32_t g, const uint32_t** out) {
  // one device table per (N, g), looked up by that key: building and hashing the
  // N-entry permutation on every call would cost more than the automorphism itself
  const std::string key = "perm:" + std::to_string(log_n) + ":" + std::to_string(g);
  auto it = ctx->const_cache.find(key);
  if (it != ctx->const_cache.end()) {
    *out = (const uint32_t*)it->second;
    return CROSS_OK;
  }
  const uint32_t N = 1u << log_n;
  std::vector<uint32_t> perm(N);
  for (uint32_t p = 0; p < N; ++p) {
    uint64_t e = (2ull * bitrev(p, log_n) + 1) * g % (2ull * N);
    perm[p] = bitrev((uint32_t)((e - 1) / 2), log_n);
  }
  void* d = nullptr;
  if (hipMalloc(&d, perm.size() * 4) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, CROSS_ENOMEM, "hipMalloc of the automorphism table failed");
  }
  if (hipMemcpy(d, perm.data(), perm.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return fail(ctx, CROSS_EDEVICE, "automorphism table upload failed");
  }
  ctx->const_cache[key] = d;
  *out = (const uint32_t*)d;
  return CROSS_OK;
}

namespace {

// Debug mode: residue-range check of an input (no-op unless enabled on the context).
#define CHECK_IN(...)                                                                   \
  do {                                                                                  \
    cross_status _c = check_residues(ctx, __VA_ARGS__);                                 \
    if (_c != CROSS_OK) return _c;                                                      \
  } while (0)

#define HIPCHK(expr, what)                                                              \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string(what) + ": " + hipGetErrorString(_e)); \
  } while (0)

// NTT/INTT of a list of limbs (by index into c->plans) at given offsets.
cross_status ntt_list(cross_ctx ctx, const CkksPlan* c, const std::vector<int>& limb,
                      const std::vector<uint64_t>& offs, uint32_t* data, uint64_t stride, int npoly,
                      bool inverse, uint32_t* tmp, hipStream_t s) {
  std::vector<Plan*> pl(limb.size());
  for (size_t i = 0; i < limb.size(); ++i) pl[i] = c->plans[limb[i]];
  return ntt_limbs(ctx, pl, offs, data, stride, npoly, inverse, tmp, s);
}

// ModUp of d (NTT form, [B][L][N]) into ext [B][dnum][L+K][N].  `tmp` holds
// B*dnum*(L+K)*N words.  Without x, d is overwritten (its INTT runs in place) and ext
// receives every limb of every digit (a digit's own limbs copied from d, inactive
// digits zero).  With x ([B][L][N] scratch), d is kept, its INTT goes to x, and ext
// receives only the converted limbs (t outside digit j): the key-switch inner
// product then reads a digit's own limbs from d.
// With conv (x given), the converted limbs are left in coefficient form and their
// (limb, offset) lists returned for a fused NTT + inner product.
struct ConvLimbs {
  std::vector<int> limb;
  std::vector<uint64_t> off;
};

cross_status modup_core(cross_ctx ctx, const CkksPlan* c, uint32_t* d, uint32_t* ext, int B,
                        uint32_t* tmp, hipStream_t s, uint32_t* x = nullptr, ConvLimbs* conv = nullptr) {
  const int L = c->L, K = c->K, LK = L + K;
  const uint64_t N = 1ull << c->log_n;
  const uint64_t ext_stride = (uint64_t)c->dnum * LK * N;
  // 1. digit limbs are copied unchanged (NTT form)
  if (!x) {
    ProfScope ps(ctx, "limb_copy", s);
    HIPCHK(launch_limb_copy(d, (uint64_t)L * N, c->copy_src, ext, ext_stride, c->copy_dst, L, c->log_n, B, s),
           "modup copy");
  }
  // inactive digits are zero
  if (!x && c->ndig < c->dnum) {
    std::vector<uint64_t> zo;
    for (int j = c->ndig; j < c->dnum; ++j)
      for (int t = 0; t < LK; ++t) zo.push_back(((uint64_t)j * LK + t) * N);
    void* dz = nullptr;
    cross_status st = cached_device_copy(ctx, zo.data(), zo.size() * 8, &dz);
    if (st != CROSS_OK) return st;
    HIPCHK(launch_limb_copy(nullptr, 0, (const uint64_t*)dz, ext, ext_stride, (const uint64_t*)dz,
                            (int)zo.size(), c->log_n, B, s), "modup zero");
  }
  // 2. coefficient form of d
  std::vector<uint64_t> lo(L);
  for (int i = 0; i < L; ++i) lo[i] = (uint64_t)i * N;
  std::vector<Plan*> pl(L);
  for (int i = 0; i < L; ++i) pl[i] = c->plans[i];
  cross_status st = ntt_limbs(ctx, pl, lo, d, (uint64_t)L * N, B, true, tmp, s, x);
  if (st != CROSS_OK) return st;
  const uint32_t* coef = x ? x : d;
  // 3. BConv of each digit to the other limbs (all digits in one launch), then 4. NTT of
  // all converted limbs in one launch
  std::vector<int> nl;
  std::vector<uint64_t> no;
  std::vector<BconvLaunch> gs;
  for (int j = 0; j < c->ndig; ++j) {
    const BconvStatic& bs = c->modup[j];
    gs.push_back(BconvLaunch{bs.src, bs.dst, bs.table, bs.nsrc, bs.ndst, coef, ext, (uint64_t)L * N, ext_stride, B,
                             c->log_n, bs.wide});
    for (int t : c->targets[j]) {
      nl.push_back(t);
      no.push_back(((uint64_t)j * LK + t) * N);
    }
  }
  {
    ProfScope ps(ctx, "bconv", s);
    HIPCHK(launch_bconv_multi(gs.data(), (int)gs.size(), s), "modup bconv");
  }
  // the converted limbs target-major: the digits' transforms of one prime are
  // neighbours in the launch, so its step-2 twiddles are fetched into one L2
  {
    std::vector<size_t> ord(nl.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return nl[x] < nl[y]; });
    std::vector<int> nl2(nl.size());
    std::vector<uint64_t> no2(no.size());
    for (size_t i = 0; i < ord.size(); ++i) {
      nl2[i] = nl[ord[i]];
      no2[i] = no[ord[i]];
    }
    nl.swap(nl2);
    no.swap(no2);
  }
  if (conv) {
    conv->limb = nl;
    conv->off = no;
    return CROSS_OK;
  }
  return ntt_list(ctx, c, nl, no, ext, ext_stride, B, false, tmp, s);
}

// ModDown of acc ([npoly][L+K][N], NTT form; its P limbs are overwritten) into out
// ([npoly][L][N]): out = base + (acc_Q - NTT(BConv(INTT(acc_P)))) * P^-1.
cross_status moddown_core(cross_ctx ctx, const CkksPlan* c, uint32_t* acc, int npoly, uint32_t* z,
                          const uint32_t* base, bool base_only_even, uint32_t* out, uint32_t* tmp,
                          hipStream_t s) {
  const int L = c->L, K = c->K, LK = L + K;
  const uint64_t N = 1ull << c->log_n;
  std::vector<int> pl(K);
  std::vector<uint64_t> po(K);
  for (int k = 0; k < K; ++k) {
    pl[k] = L + k;
    po[k] = (uint64_t)(L + k) * N;
  }
  cross_status st = ntt_list(ctx, c, pl, po, acc, (uint64_t)LK * N, npoly, true, tmp, s);
  if (st != CROSS_OK) return st;
  HIPCHK(run_bconv(ctx, c->moddown, acc, (uint64_t)LK * N, z, (uint64_t)L * N, npoly, c->log_n, s), "moddown bconv");
  std::vector<int> ql(L);
  std::vector<uint64_t> qo(L);
  std::vector<Plan*> qp(L);
  for (int i = 0; i < L; ++i) {
    ql[i] = i;
    qo[i] = (uint64_t)i * N;
    qp[i] = c->plans[i];
  }
  if (ntt_tail_fusable(ctx, qp)) {
    // the NTT's row kernel writes out = base + (acc - NTT(z)) * P^-1 directly
    const RowsTail t{acc, (uint64_t)LK * N, base, out, (uint64_t)L * N, c->tail, base_only_even ? 1 : 0};
    return ntt_limbs_tail(ctx, qp, qo, z, (uint64_t)L * N, npoly, tmp, t, s);
  }
  st = ntt_list(ctx, c, ql, qo, z, (uint64_t)L * N, npoly, false, tmp, s);
  if (st != CROSS_OK) return st;
  ProfScope ps(ctx, "moddown_tail", s);
  HIPCHK(launch_moddown_tail(acc, (uint64_t)LK * N, z, base, out, (uint64_t)L * N, c->tail, L, c->log_n,
                             npoly, base_only_even, s), "moddown tail");
  return CROSS_OK;
}

// Rescale by the last `drop` primes: the CKKS plan with those primes as P
// (NTT plans, ModDown tail constants) plus a conversion and copy offsets for a
// compact [npoly][drop][N] scratch holding the dropped limbs.
struct RescalePlan {
  CkksPlan* c = nullptr;
  BconvStatic bconv;                      // dropped limbs (scratch layout) -> kept limbs
  const uint64_t* copy_src = nullptr;     // dropped limbs within an input polynomial
  const uint64_t* copy_dst = nullptr;     // and within the scratch
};

cross_status get_rescale_plan(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                              uint32_t drop, RescalePlan** out) {
  const uint32_t Lk = L - drop;
  // the digit split is unused here; alpha <= 32 keeps the plan within its limits
  cross_ckks_params prm{log_n, Lk, drop, (Lk + 31) / 32, primes};
  CkksPlan* c = nullptr;
  cross_status st = get_ckks_plan(ctx, &prm, &c);
  if (st != CROSS_OK) return st;
  const std::string key = "rescale/" + std::to_string(reinterpret_cast<uintptr_t>(c));
  auto it = ctx->ext_plans.find(key);
  if (it != ctx->ext_plans.end()) {
    *out = static_cast<RescalePlan*>(it->second.get());
    return CROSS_OK;
  }
  std::shared_ptr<RescalePlan> holder = std::make_shared<RescalePlan>();
  RescalePlan* r = holder.get();
  r->c = c;
  const uint64_t N = 1ull << log_n;
  std::vector<uint32_t> sp(primes + Lk, primes + L), dp(primes, primes + Lk);
  std::vector<uint64_t> so(drop), cs(drop), dof(Lk);
  for (uint32_t k = 0; k < drop; ++k) {
    so[k] = (uint64_t)k * N;
    cs[k] = (uint64_t)(Lk + k) * N;
  }
  for (uint32_t i = 0; i < Lk; ++i) dof[i] = (uint64_t)i * N;
  if ((st = make_bconv(ctx, sp, so, dp, dof, &r->bconv)) != CROSS_OK) return st;
  void *a = nullptr, *b = nullptr;
  st = cached_device_copy(ctx, cs.data(), cs.size() * 8, &a);
  if (st == CROSS_OK) st = cached_device_copy(ctx, so.data(), so.size() * 8, &b);
  if (st != CROSS_OK) return st;
  r->copy_src = (const uint64_t*)a;
  r->copy_dst = (const uint64_t*)b;
  ctx->ext_plans[key] = holder;
  *out = r;
  return CROSS_OK;
}

struct KsWork {
  uint32_t *d, *ext, *tmp, *acc, *z;
};

cross_status ks_workspace(cross_ctx ctx, const CkksPlan* c, int B, hipStream_t s, KsWork* w) {
  const uint64_t N = 1ull << c->log_n;
  const uint64_t LK = c->L + c->K;
  const uint64_t nd = (uint64_t)B * c->L * N, next = (uint64_t)B * c->dnum * LK * N;
  const uint64_t nacc = (uint64_t)B * 2 * LK * N, nz = (uint64_t)B * 2 * c->L * N;
  const uint64_t ntmp = std::max(std::max(next, nacc), std::max(nz, nd));
  void* base = nullptr;
  cross_status st = workspace(ctx, s, (nd + next + ntmp + nacc + nz) * 4, &base);
  if (st != CROSS_OK) return st;
  uint32_t* p = (uint32_t*)base;
  w->d = p;
  w->ext = p + nd;
  w->tmp = w->ext + next;
  w->acc = w->tmp + ntmp;
  w->z = w->acc + nacc;
  return CROSS_OK;
}

cross_status begin(cross_ctx ctx) {
  if (!ctx) return CROSS_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, CROSS_EDEVICE, "hipSetDevice failed");
  return CROSS_OK;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Byte ranges [a, a + na) and [b, b + nb) share at least one byte.
bool overlaps(const void* a, uint64_t na, const void* b, uint64_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

// Key switch of d (NTT form, [B][L][N], in workspace w.d): ModUp, inner product with key, ModDown
// of both accumulators into out0/out1 of out [B][2][L][N] with optional base.
cross_status keyswitch_into(cross_ctx ctx, const CkksPlan* c, const uint32_t* key, int B, KsWork& w,
                            uint32_t* out, const uint32_t* base, bool base_only_even, hipStream_t s) {
  // the coefficient form of d goes to w.z, free until the ModDown
  const int LK = c->L + c->K;
  const uint64_t N = 1ull << c->log_n, ext_stride = (uint64_t)c->dnum * LK * N;
  std::vector<Plan*> all(c->plans.begin(), c->plans.begin() + LK);
  if (ntt_tail_fusable(ctx, all)) {
    // ModUp NTT and inner product fused: the row-side step of the converted limbs,
    // then one row kernel that finishes each transform and accumulates its key products
    ConvLimbs cv;
    cross_status st = modup_core(ctx, c, w.d, w.ext, B, w.tmp, s, w.z, &cv);
    if (st != CROSS_OK) return st;
    std::vector<Plan*> cp(cv.limb.size());
    for (size_t i = 0; i < cv.limb.size(); ++i) cp[i] = c->plans[cv.limb[i]];
    if ((st = ntt_rowside_forward(ctx, cp, cv.off, w.ext, ext_stride, B, w.tmp, s)) != CROSS_OK) return st;
    std::vector<IpLimb> lm(LK);
    const std::vector<int> order = ip_limb_order(c->L, c->K);
    for (int pos = 0; pos < LK; ++pos) {
      const int t = order[pos];
      const Plan* p = c->plans[t];
      const LimbMod m = limb_mod(p->q);
      lm[pos] = IpLimb{p->row_fwd_b, p->row_fwd_t3_mont, p->q, p->qinv, m.bar_m, m.bar_k,
                       t < c->L ? t / c->alpha : -1, t};
    }
    void* dl = nullptr;
    if ((st = cached_device_copy(ctx, lm.data(), lm.size() * sizeof(IpLimb), &dl)) != CROSS_OK) return st;
    const RowsIp rp{(const IpLimb*)dl, w.tmp, w.d, key, w.acc, ext_stride, LK, c->L, B, c->ndig,
                    all[0]->log_r - 3};
    {
      ProfScope ps(ctx, "ntt_rows_ip", s);
      HIPCHK(launch_ntt_rows_ip(rp, s), "fused ModUp NTT and inner product");
    }
    return moddown_core(ctx, c, w.acc, 2 * B, w.z, base, base_only_even, out, w.tmp, s);
  }
  cross_status st = modup_core(ctx, c, w.d, w.ext, B, w.tmp, s, w.z);
  if (st != CROSS_OK) return st;
  {
    ProfScope ps(ctx, "inner_product", s);
    HIPCHK(launch_inner_product(w.ext, key, w.acc, c->mods, c->L + c->K, c->dnum, c->ndig, c->log_n, B, s, w.d,
                                c->L, c->alpha, c->wide),
           "inner product");
  }
  return moddown_core(ctx, c, w.acc, 2 * B, w.z, base, base_only_even, out, w.tmp, s);
}


}  // namespace

}  // namespace cross

using namespace cross;

extern "C" {

cross_status cross_poly_mul(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                            uint32_t batch, const uint32_t* a, const uint32_t* b, uint32_t* out,
                            void* stream) {
  cross_status st = begin(ctx);
  if (st != CROSS_OK) return st;
  if (!primes || !a || !b || !out || !aligned(a) || !aligned(b) || !aligned(out))
    return fail(ctx, CROSS_EINVAL, "null or misaligned pointer");
  if (log_n < CROSS_MIN_LOG_N || log_n > CROSS_MAX_LOG_N || L < 1 || L > CROSS_MAX_LIMBS || batch < 1)
    return fail(ctx, CROSS_EINVAL, "bad shape");
  for (uint32_t i = 0; i < L; ++i) {
    st = check_prime(ctx, primes[i], log_n);
    if (st != CROSS_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  const uint64_t N = 1ull << log_n, tot = (uint64_t)batch * L * N;
  std::vector<Plan*> plans(L);
  std::vector<uint64_t> offs(L);
  std::vector<LimbMod> mods(L);
  for (uint32_t i = 0; i < L; ++i) {
    st = get_plan(ctx, primes[i], (int)log_n, &plans[i]);
    if (st != CROSS_OK) return st;
    offs[i] = i * N;
    mods[i] = limb_mod(primes[i]);
  }
  void *ws = nullptr, *dm = nullptr;
  st = workspace(ctx, s, tot * 2 * 4, &ws);
  if (st == CROSS_OK) st = cached_device_copy(ctx, mods.data(), mods.size() * sizeof(LimbMod), &dm);
  if (st != CROSS_OK) return st;
  uint32_t* wb = (uint32_t*)ws;
  uint32_t* tmp = wb + tot;
  CHECK_IN("a", a, (uint64_t)L * N, (int)batch, primes, (int)L, (int)log_n, s);
  CHECK_IN("b", b, (uint64_t)L * N, (int)batch, primes, (int)L, (int)log_n, s);
  HIPCHK(hipMemcpyAsync(wb, b, tot * 4, hipMemcpyDeviceToDevice, s), "copy b");   // b first: out may alias b
  HIPCHK(hipMemcpyAsync(out, a, tot * 4, hipMemcpyDeviceToDevice, s), "copy a");
  const uint64_t stride = (uint64_t)L * N;
  auto ntt = [&](uint32_t* d, bool inv) -> cross_status {
    return ntt_limbs(ctx, plans, offs, d, stride, (int)batch, inv, tmp, s);
  };
  if ((st = ntt(out, false)) != CROSS_OK) return st;
  if ((st = ntt(wb, false)) != CROSS_OK) return st;
  {
    ProfScope ps(ctx, "pointwise_mul", s);
    HIPCHK(launch_pointwise_mul(out, wb, out, (const LimbMod*)dm, (int)L, (int)log_n, (int)batch, s), "pointwise");
  }
  return ntt(out, true);
}

cross_status cross_bconv(cross_ctx ctx, uint32_t log_n, const uint32_t* src_primes, uint32_t l,
                         const uint32_t* dst_primes, uint32_t lp, const uint32_t* in, uint32_t* out,
                         uint32_t batch, void* stream) {
  cross_status st = begin(ctx);
  if (st != CROSS_OK) return st;
  if (!src_primes || !dst_primes || !in || !out || !aligned(in) || !aligned(out))
    return fail(ctx, CROSS_EINVAL, "null or misaligned pointer");
  if (log_n < 5 || log_n > CROSS_MAX_LOG_N || l < 1 || l > 32 || lp < 1 || lp > CROSS_MAX_LIMBS || batch < 1)
    return fail(ctx, CROSS_EINVAL, "bad shape (1 <= l <= 32, 1 <= lp <= 64, 5 <= log_n <= 16)");
  st = validate_primes(ctx, src_primes, l, 0, true);
  if (st != CROSS_OK) return st;
  for (uint32_t j = 0; j < lp; ++j) {
    st = check_prime(ctx, dst_primes[j], 0, true);
    if (st != CROSS_OK) return st;
  }
  const uint64_t N = 1ull << log_n;
  if (overlaps(in, (uint64_t)batch * l * N * 4, out, (uint64_t)batch * lp * N * 4))
    return fail(ctx, CROSS_EINVAL, "out must not overlap in");
  std::vector<uint32_t> sp(src_primes, src_primes + l), dp(dst_primes, dst_primes + lp);
  std::vector<uint64_t> so(l), dof(lp);
  for (uint32_t i = 0; i < l; ++i) so[i] = i * N;
  for (uint32_t j = 0; j < lp; ++j) dof[j] = j * N;
  BconvStatic bs;
  st = make_bconv(ctx, sp, so, dp, dof, &bs);
  if (st != CROSS_OK) return st;
  CHECK_IN("in", in, (uint64_t)l * N, (int)batch, src_primes, (int)l, (int)log_n, (hipStream_t)stream);
  HIPCHK(run_bconv(ctx, bs, in, (uint64_t)l * N, out, (uint64_t)lp * N, (int)batch, (int)log_n, (hipStream_t)stream),
         "bconv");
  return CROSS_OK;
}

cross_status cross_keyswitch_modup(cross_ctx ctx, const cross_ckks_params* prm, const uint32_t* in,
                                   uint32_t* out, uint32_t batch, void* stream) {
  cross_status st = begin(ctx);
  if (st != CROSS_OK) return st;
  CkksPlan* c = nullptr;
  if ((st = get_ckks_plan(ctx, prm, &c)) != CROSS_OK) return st;
  if (!in || !out || !aligned(in) || !aligned(out) || batch < 1) return fail(ctx, CROSS_EINVAL, "bad buffer or batch");
  hipStream_t s = (hipStream_t)stream;
  KsWork w;
  if ((st = ks_workspace(ctx, c, (int)batch, s, &w)) != CROSS_OK) return st;
  const uint64_t N = 1ull << c->log_n;
  CHECK_IN("in", in, (uint64_t)c->L * N, (int)batch, c->primes.data(), c->L, c->log_n, s);
  HIPCHK(hipMemcpyAsync(w.d, in, (uint64_t)batch * c->L * N * 4, hipMemcpyDeviceToDevice, s), "copy in");
  return modup_core(ctx, c, w.d, out, (int)batch, w.tmp, s);
}

cross_status cross_keyswitch_moddown(cross_ctx ctx, const cross_ckks_params* prm, const uint32_t* in,
                                     uint32_t* out, uint32_t batch, void* stream) {
  cross_status st = begin(ctx);
  if (st != CROSS_OK) return st;
  CkksPlan* c = nullptr;
  if ((st = get_ckks_plan(ctx, prm, &c)) != CROSS_OK) return st;
  if (!in || !out || !aligned(in) || !aligned(out) || batch < 1) return fail(ctx, CROSS_EINVAL, "bad buffer or batch");
  hipStream_t s = (hipStream_t)stream;
  KsWork w;
  if ((st = ks_workspace(ctx, c, (int)batch, s, &w)) != CROSS_OK) return st;
  const uint64_t N = 1ull << c->log_n, LK = c->L + c->K;
  CHECK_IN("in", in, LK * N, (int)batch, c->primes.data(), (int)LK, c->log_n, s);
  HIPCHK(hipMemcpyAsync(w.acc, in, (uint64_t)batch * LK * N * 4, hipMemcpyDeviceToDevice, s), "copy in");
  return moddown_core(ctx, c, w.acc, (int)batch, w.z, nullptr, false, out, w.tmp, s);
}

cross_status cross_he_mult(cross_ctx ctx, const cross_ckks_params* prm, const uint32_t* ct_a,
                           const uint32_t* ct_b, const uint32_t* relin_key, uint32_t* out,
                           uint32_t batch, void* stream) {
  cross_status st = begin(ctx);
  if (st != CROSS_OK) return st;
  CkksPlan* c = nullptr;
  if ((st = get_ckks_plan(ctx, prm, &c)) != CROSS_OK) return st;
  if (!ct_a || !ct_b || !relin_key || !out || !aligned(ct_a) || !aligned(ct_b) || !aligned(relin_key) ||
      !aligned(out) || batch < 1)
    return fail(ctx, CROSS_EINVAL, "bad buffer or batch");
  {
    const uint64_t N = 1ull << c->log_n, ct_bytes = (uint64_t)batch * 2 * c->L * N * 4,
                   key_bytes = (uint64_t)c->dnum * 2 * (c->L + c->K) * N * 4;
    if (overlaps(out, ct_bytes, ct_a, ct_bytes) || overlaps(out, ct_bytes, ct_b, ct_bytes) ||
        overlaps(out, ct_bytes, relin_key, key_bytes))
      return fail(ctx, CROSS_EINVAL, "out must not overlap ct_a, ct_b or relin_key");
  }
  hipStream_t s = (hipStream_t)stream;
  KsWork w;
  if ((st = ks_workspace(ctx, c, (int)batch, s, &w)) != CROSS_OK) return st;
  {
    const uint64_t N = 1ull << c->log_n;
    CHECK_IN("ct_a", ct_a, (uint64_t)c->L * N, 2 * (int)batch, c->primes.data(), c->L, c->log_n, s);
    CHECK_IN("ct_b", ct_b, (uint64_t)c->L * N, 2 * (int)batch, c->primes.data(), c->L, c->log_n, s);
    CHECK_IN("relin_key", relin_key, (uint64_t)(c->L + c->K) * N, 2 * c->dnum, c->primes.data(), c->L + c->K,
             c->log_n, s);
  }
  {
    ProfScope ps(ctx, "tensor", s);
    HIPCHK(launch_tensor(ct_a, ct_b, out, w.d, c->mods, c->L, c->log_n, (int)batch, s, c->wide), "tensor");
  }
  return keyswitch_into(ctx, c, relin_key, (int)batch, w, out, out, false, s);
}

cross_status cross_he_add(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                          uint32_t npoly, const uint32_t* a, const uint32_t* b, uint32_t* out,
                          void* stream) {
  cross_status st = begin(ctx);
  if (st != CROSS_OK) return st;
  if (!primes || !a || !b || !out || !aligned(a) || !aligned(b) || !aligned(out))
    return fail(ctx, CROSS_EINVAL, "null or misaligned pointer");
  if (log_n < CROSS_MIN_LOG_N || log_n > CROSS_MAX_LOG_N || L < 1 || L > CROSS_MAX_LIMBS || npoly < 1)
    return fail(ctx, CROSS_EINVAL, "bad shape");
  std::vector<LimbMod> mods(L);
  for (uint32_t i = 0; i < L; ++i) {
    if ((st = check_prime(ctx, primes[i], log_n)) != CROSS_OK) return st;
    mods[i] = limb_mod(primes[i]);
  }
  void* dm = nullptr;
  if ((st = cached_device_copy(ctx, mods.data(), mods.size() * sizeof(LimbMod), &dm)) != CROSS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  CHECK_IN("a", a, (uint64_t)L << log_n, (int)npoly, primes, (int)L, (int)log_n, s);
  CHECK_IN("b", b, (uint64_t)L << log_n, (int)npoly, primes, (int)L, (int)log_n, s);
  ProfScope ps(ctx, "he_add", s);
  HIPCHK(launch_pointwise_add(a, b, out, (const LimbMod*)dm, (int)L, (int)log_n, (int)npoly, s), "he_add");
  return CROSS_OK;
}

cross_status cross_rescale(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                           uint32_t drop, uint32_t npoly, const uint32_t* in, uint32_t* out,
                           void* stream) {
  cross_status st = begin(ctx);
  if (st != CROSS_OK) return st;
  if (!primes || !in || !out || !aligned(in) || !aligned(out))
    return fail(ctx, CROSS_EINVAL, "null or misaligned pointer");
  if (log_n < 5 || log_n > CROSS_MAX_LOG_N || L < 2 || L > CROSS_MAX_LIMBS || drop < 1 || drop >= L ||
      drop > 32 || npoly < 1)
    return fail(ctx, CROSS_EINVAL, "bad shape (5 <= log_n <= 16, 1 <= drop < L <= 64, drop <= 32)");
  const uint64_t N = 1ull << log_n, Lk = L - drop;
  const uintptr_t i0 = reinterpret_cast<uintptr_t>(in), o0 = reinterpret_cast<uintptr_t>(out);
  if (i0 < o0 + (uint64_t)npoly * Lk * N * 4 && o0 < i0 + (uint64_t)npoly * L * N * 4)
    return fail(ctx, CROSS_EINVAL, "out must not overlap in");
  RescalePlan* r = nullptr;
  if ((st = get_rescale_plan(ctx, log_n, primes, L, drop, &r)) != CROSS_OK) return st;
  CHECK_IN("in", in, (uint64_t)L * N, (int)npoly, primes, (int)L, (int)log_n, (hipStream_t)stream);
  const CkksPlan* c = r->c;
  hipStream_t s = (hipStream_t)stream;
  const uint64_t ny = (uint64_t)npoly * drop * N, nz = (uint64_t)npoly * Lk * N;
  void* base = nullptr;
  if ((st = workspace(ctx, s, (ny + nz + std::max(ny, nz)) * 4, &base)) != CROSS_OK) return st;
  uint32_t* y = (uint32_t*)base;
  uint32_t* z = y + ny;
  uint32_t* tmp = z + nz;
  {
    ProfScope ps(ctx, "limb_copy", s);
    HIPCHK(launch_limb_copy(in, (uint64_t)L * N, r->copy_src, y, (uint64_t)drop * N, r->copy_dst, (int)drop,
                            (int)log_n, (int)npoly, s), "rescale copy");
  }
  std::vector<int> pl(drop), ql(Lk);
  std::vector<uint64_t> po(drop), qo(Lk);
  for (uint32_t k = 0; k < drop; ++k) {
    pl[k] = (int)(Lk + k);
    po[k] = (uint64_t)k * N;
  }
  for (uint32_t i = 0; i < Lk; ++i) {
    ql[i] = (int)i;
    qo[i] = (uint64_t)i * N;
  }
  if ((st = ntt_list(ctx, c, pl, po, y, (uint64_t)drop * N, (int)npoly, true, tmp, s)) != CROSS_OK) return st;
  HIPCHK(run_bconv(ctx, r->bconv, y, (uint64_t)drop * N, z, Lk * N, (int)npoly, (int)log_n, s), "rescale bconv");
  {
    std::vector<Plan*> qp(Lk);
    for (uint32_t i = 0; i < Lk; ++i) qp[i] = c->plans[i];
    if (ntt_tail_fusable(ctx, qp)) {
      // the NTT's row kernel writes out = (in - NTT(z)) * P^-1 directly
      const RowsTail t{in, (uint64_t)L * N, nullptr, out, Lk * N, c->tail, 0};
      return ntt_limbs_tail(ctx, qp, qo, z, Lk * N, (int)npoly, tmp, t, s);
    }
  }
  if ((st = ntt_list(ctx, c, ql, qo, z, Lk * N, (int)npoly, false, tmp, s)) != CROSS_OK) return st;
  ProfScope ps(ctx, "rescale_tail", s);
  HIPCHK(launch_moddown_tail(in, (uint64_t)L * N, z, nullptr, out, Lk * N, c->tail, (int)Lk, (int)log_n,
                             (int)npoly, false, s), "rescale tail");
  return CROSS_OK;
}

cross_status cross_rotate(cross_ctx ctx, const cross_ckks_params* prm, int32_t steps, const uint32_t* ct,
                          const uint32_t* rot_key, uint32_t* out, uint32_t batch, void* stream) {
  cross_status st = begin(ctx);
  if (st != CROSS_OK) return st;
  CkksPlan* c = nullptr;
  if ((st = get_ckks_plan(ctx, prm, &c)) != CROSS_OK) return st;
  if (!ct || !rot_key || !out || !aligned(ct) || !aligned(rot_key) || !aligned(out) || batch < 1)
    return fail(ctx, CROSS_EINVAL, "bad buffer or batch");
  hipStream_t s = (hipStream_t)stream;
  const uint64_t N = 1ull << c->log_n;
  {
    const uint64_t ct_bytes = (uint64_t)batch * 2 * c->L * N * 4,
                   key_bytes = (uint64_t)c->dnum * 2 * (c->L + c->K) * N * 4;
    if (overlaps(out, ct_bytes, ct, ct_bytes) || overlaps(out, ct_bytes, rot_key, key_bytes))
      return fail(ctx, CROSS_EINVAL, "out must not overlap ct or rot_key");
  }
  const int64_t half = (int64_t)N / 2;
  const uint64_t r = (uint64_t)((((int64_t)steps % half) + half) % half);
  const uint32_t g = powmod(5, r, (uint32_t)(2 * N));
  const uint32_t* perm = nullptr;
  if ((st = perm_table(ctx, c->log_n, g, &perm)) != CROSS_OK) return st;
  KsWork w;
  if ((st = ks_workspace(ctx, c, (int)batch, s, &w)) != CROSS_OK) return st;
  const uint64_t L = c->L;
  CHECK_IN("ct", ct, L * N, 2 * (int)batch, c->primes.data(), c->L, c->log_n, s);
  CHECK_IN("rot_key", rot_key, (uint64_t)(c->L + c->K) * N, 2 * c->dnum, c->primes.data(), c->L + c->K, c->log_n, s);
  {
    ProfScope ps(ctx, "automorphism", s);
    // sigma(c0) -> out[b][0] (the ModDown base of the first component); sigma(c1) -> workspace
    HIPCHK(launch_automorphism(ct, 2 * L * N, out, 2 * L * N, perm, c->log_n, (int)L, (int)batch, s), "sigma c0");
    HIPCHK(launch_automorphism(ct + L * N, 2 * L * N, w.d, L * N, perm, c->log_n, (int)L, (int)batch, s), "sigma c1");
  }
  return keyswitch_into(ctx, c, rot_key, (int)batch, w, out, out, true, s);
}

}  // extern "C"

/* ---- chunked forms of the key-switching streams (stream ablation) ---- */

namespace {

cross_status stream_mods(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L, const StreamMod** out) {
  std::vector<StreamMod> m(L);
  for (uint32_t i = 0; i < L; ++i) {
    cross_status st = check_prime(ctx, primes[i], log_n);
    if (st != CROSS_OK) return st;
    m[i] = stream_mod(primes[i]);
  }
  void* d = nullptr;
  cross_status st = cached_device_copy(ctx, m.data(), m.size() * sizeof(StreamMod), &d);
  *out = (const StreamMod*)d;
  return st;
}

}  // namespace

extern "C" {

cross_status cross_evk_bat_prepare(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t LK,
                                   uint32_t dnum, const uint32_t* key, uint32_t* key_bat, void* stream) {
  cross_status st = begin(ctx);
  if (st != CROSS_OK) return st;
  if (!primes || !key || !key_bat || !aligned(key) || !aligned(key_bat))
    return fail(ctx, CROSS_EINVAL, "null or misaligned pointer");
  if (log_n < CROSS_MIN_LOG_N || log_n > CROSS_MAX_LOG_N || LK < 1 || LK > CROSS_MAX_LIMBS || dnum < 1 || dnum > 64)
    return fail(ctx, CROSS_EINVAL, "bad shape");
  const uint64_t n = ((uint64_t)dnum * 2 * LK) << log_n;
  if (overlaps(key, n * 4, key_bat, n * 16)) return fail(ctx, CROSS_EINVAL, "key_bat must not overlap key");
  const StreamMod* m = nullptr;
  if ((st = stream_mods(ctx, log_n, primes, LK, &m)) != CROSS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  CHECK_IN("key", key, (uint64_t)LK << log_n, 2 * (int)dnum, primes, (int)LK, (int)log_n, s);
  ProfScope ps(ctx, "evk_bat_prepare", s);
  HIPCHK(launch_evk_bat_prepare(key, key_bat, m, (int)LK, (int)dnum, (int)log_n, s), "evk_bat_prepare");
  return CROSS_OK;
}

cross_status cross_keyswitch_inner_product(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t LK,
                                           uint32_t dnum, uint32_t batch, int form, const uint32_t* ext,
                                           const uint32_t* key, uint32_t* out, void* stream) {
  cross_status st = begin(ctx);
  if (st != CROSS_OK) return st;
  if (!primes || !ext || !key || !out || !aligned(ext) || !aligned(key) || !aligned(out))
    return fail(ctx, CROSS_EINVAL, "null or misaligned pointer");
  if (log_n < CROSS_MIN_LOG_N || log_n > CROSS_MAX_LOG_N || LK < 1 || LK > CROSS_MAX_LIMBS || dnum < 1 ||
      dnum > 64 || batch < 1)
    return fail(ctx, CROSS_EINVAL, "bad shape");
  if (form != CROSS_STREAM_VALU && form != CROSS_STREAM_CHUNKED) return fail(ctx, CROSS_EINVAL, "unknown form");
  const uint64_t N = 1ull << log_n;
  const uint64_t n_ext = (uint64_t)batch * dnum * LK * N, n_out = (uint64_t)batch * 2 * LK * N;
  const uint64_t n_key = (uint64_t)dnum * 2 * LK * N * (form == CROSS_STREAM_CHUNKED ? 4 : 1);
  if (overlaps(out, n_out * 4, ext, n_ext * 4) || overlaps(out, n_out * 4, key, n_key * 4))
    return fail(ctx, CROSS_EINVAL, "out must not overlap ext or key");
  hipStream_t s = (hipStream_t)stream;
  CHECK_IN("ext", ext, LK * N, (int)(batch * dnum), primes, (int)LK, (int)log_n, s);
  if (form == CROSS_STREAM_VALU) CHECK_IN("key", key, LK * N, 2 * (int)dnum, primes, (int)LK, (int)log_n, s);
  if (form == CROSS_STREAM_CHUNKED) {
    const StreamMod* m = nullptr;
    if ((st = stream_mods(ctx, log_n, primes, LK, &m)) != CROSS_OK) return st;
    ProfScope ps(ctx, "inner_product_bat", s);
    HIPCHK(launch_inner_product_bat(ext, key, out, m, (int)LK, (int)dnum, (int)log_n, (int)batch, s),
           "inner_product_bat");
    return CROSS_OK;
  }
  if (log_n < 2) return fail(ctx, CROSS_EINVAL, "bad shape");
  std::vector<LimbMod> mods(LK);
  for (uint32_t i = 0; i < LK; ++i) {
    if ((st = check_prime(ctx, primes[i], log_n)) != CROSS_OK) return st;
    mods[i] = limb_mod(primes[i]);
  }
  void* dm = nullptr;
  if ((st = cached_device_copy(ctx, mods.data(), mods.size() * sizeof(LimbMod), &dm)) != CROSS_OK) return st;
  ProfScope ps(ctx, "inner_product", s);
  HIPCHK(launch_inner_product(ext, key, out, (const LimbMod*)dm, (int)LK, (int)dnum, (int)dnum, (int)log_n,
                              (int)batch, s),
         "inner_product");
  return CROSS_OK;
}

cross_status cross_tensor(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L, uint32_t batch,
                          int form, const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t* d2,
                          void* stream) {
  cross_status st = begin(ctx);
  if (st != CROSS_OK) return st;
  if (!primes || !a || !b || !out || !d2 || !aligned(a) || !aligned(b) || !aligned(out) || !aligned(d2))
    return fail(ctx, CROSS_EINVAL, "null or misaligned pointer");
  if (log_n < CROSS_MIN_LOG_N || log_n > CROSS_MAX_LOG_N || L < 1 || L > CROSS_MAX_LIMBS || batch < 1)
    return fail(ctx, CROSS_EINVAL, "bad shape");
  if (form != CROSS_STREAM_VALU && form != CROSS_STREAM_CHUNKED) return fail(ctx, CROSS_EINVAL, "unknown form");
  const uint64_t N = 1ull << log_n, n_ct = (uint64_t)batch * 2 * L * N, n_d2 = (uint64_t)batch * L * N;
  if (overlaps(out, n_ct * 4, a, n_ct * 4) || overlaps(out, n_ct * 4, b, n_ct * 4) ||
      overlaps(d2, n_d2 * 4, a, n_ct * 4) || overlaps(d2, n_d2 * 4, b, n_ct * 4) ||
      overlaps(d2, n_d2 * 4, out, n_ct * 4))
    return fail(ctx, CROSS_EINVAL, "out and d2 must not overlap each other or the inputs");
  hipStream_t s = (hipStream_t)stream;
  CHECK_IN("a", a, (uint64_t)L * N, 2 * (int)batch, primes, (int)L, (int)log_n, s);
  CHECK_IN("b", b, (uint64_t)L * N, 2 * (int)batch, primes, (int)L, (int)log_n, s);
  if (form == CROSS_STREAM_CHUNKED) {
    const StreamMod* m = nullptr;
    if ((st = stream_mods(ctx, log_n, primes, L, &m)) != CROSS_OK) return st;
    ProfScope ps(ctx, "tensor_conv", s);
    HIPCHK(launch_tensor_conv(a, b, out, d2, m, (int)L, (int)log_n, (int)batch, s), "tensor_conv");
    return CROSS_OK;
  }
  std::vector<LimbMod> mods(L);
  for (uint32_t i = 0; i < L; ++i) {
    if ((st = check_prime(ctx, primes[i], log_n)) != CROSS_OK) return st;
    mods[i] = limb_mod(primes[i]);
  }
  void* dm = nullptr;
  if ((st = cached_device_copy(ctx, mods.data(), mods.size() * sizeof(LimbMod), &dm)) != CROSS_OK) return st;
  ProfScope ps(ctx, "tensor", s);
  HIPCHK(launch_tensor(a, b, out, d2, (const LimbMod*)dm, (int)L, (int)log_n, (int)batch, s), "tensor");
  return CROSS_OK;
}

}  // extern "C"
