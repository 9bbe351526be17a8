// Plan files: the analysis, the rewrite and the tuned schedules of a handle
// written to a file and read back into another handle, so that a process can
// solve without analysing, rewriting or tuning again (rewriting is a one-off
// preprocessing step whose output any later solve can use, Sec. II.B).
//
// Layout (little-endian, as the host writes it): an 8-byte magic, a u32
// version, then sections {u32 tag, u32 element size, u64 count, bytes}, and a
// final section holding the FNV-1a-64 hash of every byte before it. The
// window images, work vectors and graphs are not stored: they are rebuilt from
// the stored schedules by the first solve (or sptrsv_prepare).
#include <cstdio>
#include <cstring>
#include <memory>

#include "common.h"
#include "sync.h"

namespace {

constexpr char kMagic[8] = {'S', 'P', 'T', 'R', 'S', 'V', 'P', 'L'};
constexpr uint32_t kVersion = 4;
constexpr uint32_t kTagHash = 0xffffffffu;

uint64_t fnv1a(const unsigned char *p, size_t n, uint64_t h = 1469598103934665603ull) {
  for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}

struct Writer {
  std::vector<unsigned char> buf;
  void raw(const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    buf.insert(buf.end(), c, c + n);
  }
  template <class T>
  void pod(uint32_t tag, const T &v) {
    section(tag, sizeof(T), 1, &v);
  }
  void section(uint32_t tag, uint32_t esize, uint64_t count, const void *p) {
    raw(&tag, 4);
    raw(&esize, 4);
    raw(&count, 8);
    if (count) raw(p, (size_t)esize * count);
  }
  template <class T>
  void vec(uint32_t tag, const std::vector<T> &v) {
    section(tag, sizeof(T), v.size(), v.data());
  }
};

struct Reader {
  const unsigned char *p;
  size_t n, at = 0;
  bool ok = true;
  // next section: its tag must be `tag` and its element size `esize`
  const unsigned char *section(uint32_t tag, uint32_t esize, uint64_t *count) {
    if (!ok || n - at < 16) return fail();
    uint32_t t, e;
    uint64_t c;
    std::memcpy(&t, p + at, 4);
    std::memcpy(&e, p + at + 4, 4);
    std::memcpy(&c, p + at + 8, 8);
    at += 16;
    if (t != tag || e != esize || (e && c > (n - at) / e)) return fail();
    const unsigned char *d = p + at;
    at += (size_t)e * c;
    *count = c;
    return d;
  }
  template <class T>
  bool pod(uint32_t tag, T *v) {
    uint64_t c = 0;
    const unsigned char *d = section(tag, sizeof(T), &c);
    if (!d || c != 1) return fail(), false;
    std::memcpy(v, d, sizeof(T));
    return true;
  }
  template <class T>
  bool vec(uint32_t tag, std::vector<T> *v) {
    uint64_t c = 0;
    const unsigned char *d = section(tag, sizeof(T), &c);
    if (!d) return false;
    v->resize(c);
    if (c) std::memcpy(v->data(), d, sizeof(T) * c);
    return true;
  }
  const unsigned char *fail() {
    ok = false;
    return nullptr;
  }
};

// Device array <-> section. Arrays are stored with their used length, which
// the reader checks against the sizes it derives from the plan header.
template <class T>
sptrsv_status_t put(sptrsv_ctx *h, Writer &w, uint32_t tag, const DArr<T> &a, size_t count) {
  std::vector<T> tmp(count);
  if (count) HIPCHK(h, hipMemcpy(tmp.data(), a.p, sizeof(T) * count, hipMemcpyDeviceToHost));
  w.vec(tag, tmp);
  return SPTRSV_OK;
}

template <class T>
sptrsv_status_t get(sptrsv_ctx *h, Reader &r, uint32_t tag, DArr<T> &a, size_t count) {
  uint64_t c = 0;
  const unsigned char *d = r.section(tag, sizeof(T), &c);
  if (!d || c != count) return set_err(h, SPTRSV_ERR_ARG, "plan file: section %u missing or of the wrong size", tag);
  HIPCHK(h, a.alloc(std::max<size_t>(count, 1)));
  if (count) HIPCHK(h, hipMemcpy(a.p, d, sizeof(T) * count, hipMemcpyHostToDevice));
  return SPTRSV_OK;
}

struct PlanHead {
  int32_t present, n, nlev, rev_io, has_t, n_tpos, t_lanes, pad;
  int64_t nnz, nnz_t_off, total_cost;
  double avg_cost;
  sptrsv_schedule_t sched;
};

struct TunedEntry {
  int32_t nrhs;
  sptrsv_schedule_t sched;
};

sptrsv_status_t put_plan(sptrsv_ctx *h, Writer &w, uint32_t base, const Plan &P) {
  PlanHead hd{};
  hd.present = P.ready ? 1 : 0;
  if (P.ready) {
    hd.n = P.n, hd.nlev = P.nlev, hd.rev_io = P.rev_io, hd.has_t = P.has_t, hd.n_tpos = P.n_tpos;
    hd.t_lanes = P.t_lanes, hd.nnz = P.nnz, hd.nnz_t_off = P.nnz_t_off, hd.total_cost = P.total_cost;
    hd.avg_cost = P.avg_cost, hd.sched = P.sched;
  }
  w.pod(base, hd);
  if (!P.ready) return SPTRSV_OK;
  const size_t n = (size_t)P.n, nl = (size_t)P.nlev, noff = (size_t)(P.nnz - P.n);
  STCHK(put(h, w, base + 1, P.level_ptr, nl + 1));
  STCHK(put(h, w, base + 2, P.perm, n));
  STCHK(put(h, w, base + 3, P.iperm, n));
  STCHK(put(h, w, base + 4, P.row_level, n));
  STCHK(put(h, w, base + 5, P.srp, n + 1));
  STCHK(put(h, w, base + 6, P.sci, noff));
  STCHK(put(h, w, base + 7, P.sva, noff));
  STCHK(put(h, w, base + 8, P.sdg, n));
  STCHK(put(h, w, base + 9, P.lv_rows, nl));
  STCHK(put(h, w, base + 10, P.lv_nnz, nl));
  STCHK(put(h, w, base + 11, P.lv_cost, nl));
  STCHK(put(h, w, base + 12, P.ell_c, n));
  STCHK(put(h, w, base + 13, P.ell_v, 2 * n));
  w.vec(base + 14, P.h_xh);
  w.vec(base + 15, P.h_level_ptr);
  w.vec(base + 16, P.h_lv_nnz);
  std::vector<TunedEntry> tuned;
  for (const auto &kv : P.tuned) tuned.push_back(TunedEntry{kv.first, kv.second});
  w.vec(base + 17, tuned);
  if (P.rev_io) {
    STCHK(put(h, w, base + 18, P.perm_io, n));
    STCHK(put(h, w, base + 19, P.iperm_io, n));
  }
  if (P.has_t) {
    STCHK(put(h, w, base + 20, P.trp, n + 1));
    STCHK(put(h, w, base + 21, P.tci, (size_t)P.nnz_t_off));
    STCHK(put(h, w, base + 22, P.tva, (size_t)P.nnz_t_off));
    w.vec(base + 23, P.h_tpos);
    w.vec(base + 24, P.h_lv_tnnz);
  }
  return SPTRSV_OK;
}

sptrsv_status_t get_plan(sptrsv_ctx *h, Reader &r, uint32_t base, Plan &P) {
  PlanHead hd{};
  if (!r.pod(base, &hd)) return set_err(h, SPTRSV_ERR_ARG, "plan file: plan header %u", base);
  P = Plan{};
  if (!hd.present) return SPTRSV_OK;
  if (hd.n < 0 || hd.nlev < 0 || hd.nlev > hd.n || hd.nnz < hd.n || hd.nnz_t_off < 0 || hd.n_tpos < 0 ||
      hd.n_tpos > hd.n)
    return set_err(h, SPTRSV_ERR_ARG, "plan file: inconsistent plan sizes");
  P.n = hd.n, P.nlev = hd.nlev, P.rev_io = hd.rev_io != 0, P.has_t = hd.has_t != 0, P.n_tpos = hd.n_tpos;
  P.t_lanes = hd.t_lanes, P.nnz = hd.nnz, P.nnz_t_off = hd.nnz_t_off, P.total_cost = hd.total_cost;
  P.avg_cost = hd.avg_cost, P.sched = hd.sched;
  const size_t n = (size_t)P.n, nl = (size_t)P.nlev, noff = (size_t)(P.nnz - P.n);
  STCHK(get(h, r, base + 1, P.level_ptr, nl + 1));
  STCHK(get(h, r, base + 2, P.perm, n));
  STCHK(get(h, r, base + 3, P.iperm, n));
  STCHK(get(h, r, base + 4, P.row_level, n));
  STCHK(get(h, r, base + 5, P.srp, n + 1));
  STCHK(get(h, r, base + 6, P.sci, noff));
  STCHK(get(h, r, base + 7, P.sva, noff));
  STCHK(get(h, r, base + 8, P.sdg, n));
  STCHK(get(h, r, base + 9, P.lv_rows, nl));
  STCHK(get(h, r, base + 10, P.lv_nnz, nl));
  STCHK(get(h, r, base + 11, P.lv_cost, nl));
  STCHK(get(h, r, base + 12, P.ell_c, n));
  STCHK(get(h, r, base + 13, P.ell_v, 2 * n));
  std::vector<TunedEntry> tuned;
  if (!r.vec(base + 14, &P.h_xh) || !r.vec(base + 15, &P.h_level_ptr) || !r.vec(base + 16, &P.h_lv_nnz) ||
      !r.vec(base + 17, &tuned) || P.h_xh.size() != nl * kExtraBuckets || P.h_level_ptr.size() != nl + 1 ||
      P.h_lv_nnz.size() != nl)
    return set_err(h, SPTRSV_ERR_ARG, "plan file: host tables of plan %u", base);
  for (size_t l = 0; l < nl; ++l)
    if (P.h_level_ptr[l] > P.h_level_ptr[l + 1]) return set_err(h, SPTRSV_ERR_ARG, "plan file: level bounds");
  if (P.h_level_ptr[0] != 0 || P.h_level_ptr[nl] != P.n) return set_err(h, SPTRSV_ERR_ARG, "plan file: level bounds");
  for (const TunedEntry &e : tuned) P.tuned[e.nrhs] = e.sched;
  if (P.rev_io) {
    STCHK(get(h, r, base + 18, P.perm_io, n));
    STCHK(get(h, r, base + 19, P.iperm_io, n));
  }
  if (P.has_t) {
    STCHK(get(h, r, base + 20, P.trp, n + 1));
    STCHK(get(h, r, base + 21, P.tci, (size_t)P.nnz_t_off));
    STCHK(get(h, r, base + 22, P.tva, (size_t)P.nnz_t_off));
    if (!r.vec(base + 23, &P.h_tpos) || !r.vec(base + 24, &P.h_lv_tnnz) || P.h_tpos.size() != (size_t)P.n_tpos ||
        P.h_lv_tnnz.size() != nl)
      return set_err(h, SPTRSV_ERR_ARG, "plan file: b-transform tables");
    HIPCHK(h, P.tpos.alloc(std::max<size_t>(P.h_tpos.size(), 1)));
    if (!P.h_tpos.empty())
      HIPCHK(h, hipMemcpy(P.tpos.p, P.h_tpos.data(), sizeof(int32_t) * P.h_tpos.size(), hipMemcpyHostToDevice));
  }
  // per-launch control words start at zero, as build_plan leaves them
  HIPCHK(h, P.wbar.alloc(kGridBarWords));
  HIPCHK(h, hipMemset(P.wbar.p, 0, kGridBarWords * sizeof(unsigned)));
  HIPCHK(h, P.tp.alloc(4));
  HIPCHK(h, hipMemset(P.tp.p, 0, 4 * sizeof(unsigned)));
  HIPCHK(h, P.sf_ticket.alloc(1));
  P.ready = true;
  return SPTRSV_OK;
}

struct HandleHead {
  int32_t form, n, has_rewrite, pad;
  int64_t nnz;
  sptrsv_rewrite_stats_t rstats;
};

}  // namespace

extern "C" {

sptrsv_status_t sptrsv_plan_save(sptrsv_handle_t h, const char *path) {
  if (!h || !path) return SPTRSV_ERR_ARG;
  h->last_error.clear();
  if (!h->orig.ready) return set_err(h, SPTRSV_ERR_STATE, "plan_save: matrix not analysed");
  HIPCHK(h, hipDeviceSynchronize());
  Writer w;
  w.raw(kMagic, 8);
  w.raw(&kVersion, 4);
  HandleHead hh{};
  hh.form = h->form, hh.n = h->n, hh.has_rewrite = h->has_rewrite ? 1 : 0, hh.nnz = h->nnz, hh.rstats = h->rstats;
  w.pod(1, hh);
  const size_t n = (size_t)h->n, nnz = (size_t)h->nnz;
  STCHK(put(h, w, 2, h->rp, n + 1));
  STCHK(put(h, w, 3, h->ci, nnz));
  STCHK(put(h, w, 4, h->va, nnz));
  STCHK(put_plan(h, w, 100, h->orig));
  if (h->has_rewrite) {
    const size_t a = (size_t)h->rstats.nnz_Lp, b = (size_t)h->rstats.nnz_T;
    STCHK(put(h, w, 10, h->lp_rp, n + 1));
    STCHK(put(h, w, 11, h->lp_ci, a));
    STCHK(put(h, w, 12, h->lp_va, a));
    STCHK(put(h, w, 13, h->t_rp, n + 1));
    STCHK(put(h, w, 14, h->t_ci, b));
    STCHK(put(h, w, 15, h->t_va, b));
    STCHK(put(h, w, 16, h->target, n));
    STCHK(put_plan(h, w, 200, h->rew));
  }
  const uint64_t hash = fnv1a(w.buf.data(), w.buf.size());
  w.pod(kTagHash, hash);
  std::unique_ptr<FILE, int (*)(FILE *)> f(std::fopen(path, "wb"), &std::fclose);
  if (!f) return set_err(h, SPTRSV_ERR_ARG, "plan_save: cannot open %s for writing", path);
  if (std::fwrite(w.buf.data(), 1, w.buf.size(), f.get()) != w.buf.size())
    return set_err(h, SPTRSV_ERR_ARG, "plan_save: short write to %s", path);
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_plan_load(sptrsv_handle_t h, const char *path) {
  if (!h || !path) return SPTRSV_ERR_ARG;
  h->last_error.clear();
  std::vector<unsigned char> buf;
  {
    std::unique_ptr<FILE, int (*)(FILE *)> f(std::fopen(path, "rb"), &std::fclose);
    if (!f) return set_err(h, SPTRSV_ERR_ARG, "plan_load: cannot open %s", path);
    unsigned char chunk[1 << 16];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof(chunk), f.get())) > 0) buf.insert(buf.end(), chunk, chunk + got);
  }
  // magic, version and the trailing hash section (16 + 8 bytes) before anything else
  if (buf.size() < 12 + 24 || std::memcmp(buf.data(), kMagic, 8) != 0)
    return set_err(h, SPTRSV_ERR_ARG, "plan_load: %s is not a plan file", path);
  uint32_t ver = 0;
  std::memcpy(&ver, buf.data() + 8, 4);
  if (ver != kVersion) return set_err(h, SPTRSV_ERR_ARG, "plan_load: version %u, expected %u", ver, kVersion);
  const size_t body = buf.size() - 24;
  {
    Reader tail{buf.data(), buf.size(), body};
    uint64_t stored = 0;
    if (!tail.pod(kTagHash, &stored) || stored != fnv1a(buf.data(), body))
      return set_err(h, SPTRSV_ERR_ARG, "plan_load: %s is truncated or corrupt (hash mismatch)", path);
  }
  Reader r{buf.data(), body, 12};
  HandleHead hh{};
  if (!r.pod(1, &hh) || hh.n < 0 || hh.nnz < hh.n || hh.form < SPTRSV_LOWER || hh.form > SPTRSV_UPPER_TRANS)
    return set_err(h, SPTRSV_ERR_ARG, "plan_load: bad handle header");
  // replace the handle's state only once the whole file has been read
  HIPCHK(h, hipDeviceSynchronize());
  h->orig.ready = h->rew.ready = false;
  h->has_rewrite = false;
  for (Graph &g : h->graphs) {  // graphs captured the old plan's buffers
    if (g.ge) (void)hipGraphExecDestroy(g.ge);
    if (g.g) (void)hipGraphDestroy(g.g);
  }
  h->graphs.clear();
  const size_t n = (size_t)hh.n, nnz = (size_t)hh.nnz;
  STCHK(get(h, r, 2, h->rp, n + 1));
  STCHK(get(h, r, 3, h->ci, nnz));
  STCHK(get(h, r, 4, h->va, nnz));
  Plan orig;
  STCHK(get_plan(h, r, 100, orig));
  if (!orig.ready || orig.n != hh.n) return set_err(h, SPTRSV_ERR_ARG, "plan_load: no analysis in %s", path);
  Plan rew;
  if (hh.has_rewrite) {
    const size_t a = (size_t)hh.rstats.nnz_Lp, b = (size_t)hh.rstats.nnz_T;
    if (hh.rstats.nnz_Lp < hh.n || hh.rstats.nnz_T < hh.n) return set_err(h, SPTRSV_ERR_ARG, "plan_load: sizes");
    STCHK(get(h, r, 10, h->lp_rp, n + 1));
    STCHK(get(h, r, 11, h->lp_ci, a));
    STCHK(get(h, r, 12, h->lp_va, a));
    STCHK(get(h, r, 13, h->t_rp, n + 1));
    STCHK(get(h, r, 14, h->t_ci, b));
    STCHK(get(h, r, 15, h->t_va, b));
    STCHK(get(h, r, 16, h->target, n));
    STCHK(get_plan(h, r, 200, rew));
    if (!rew.ready || rew.n != hh.n) return set_err(h, SPTRSV_ERR_ARG, "plan_load: rewritten plan missing");
  }
  if (r.at != body) return set_err(h, SPTRSV_ERR_ARG, "plan_load: trailing data in %s", path);
  h->form = hh.form;
  h->n = hh.n;
  h->nnz = hh.nnz;
  h->orig = std::move(orig);
  if (hh.has_rewrite) {
    h->rew = std::move(rew);
    h->rstats = hh.rstats;
    h->has_rewrite = true;
  }
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_get_info(sptrsv_handle_t h, sptrsv_info_t *out, sptrsv_rewrite_stats_t *st) {
  if (!h || !out) return SPTRSV_ERR_ARG;
  if (!h->orig.ready) return set_err(h, SPTRSV_ERR_STATE, "get_info: matrix not analysed");
  out->form = h->form;
  out->n = h->n;
  out->nlev = h->orig.nlev;
  out->has_rewrite = h->has_rewrite ? 1 : 0;
  out->nnz = h->nnz;
  if (st) *st = h->has_rewrite ? h->rstats : sptrsv_rewrite_stats_t{};
  return SPTRSV_OK;
}

}  // extern "C"
