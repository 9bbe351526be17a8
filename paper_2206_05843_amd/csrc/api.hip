// C ABI of libsptrsv: handle, analysis, plans, schedules and the solve.
#include <algorithm>
#include <cstdarg>
#include <cstring>

#include "common.h"
#include "sync.h"

sptrsv_status_t status_from_bits(int bits) {
  if (bits & EB_ARG) return SPTRSV_ERR_ARG;
  if (bits & EB_NOT_LOWER) return SPTRSV_ERR_NOT_LOWER;
  if (bits & EB_UNSORTED) return SPTRSV_ERR_UNSORTED;
  if (bits & EB_MISSING_DIAG) return SPTRSV_ERR_MISSING_DIAG;
  if (bits & EB_ZERO_PIVOT) return SPTRSV_ERR_ZERO_PIVOT;
  if (bits & EB_NONFINITE) return SPTRSV_ERR_NONFINITE;
  if (bits & EB_OVERFLOW) return SPTRSV_ERR_OVERFLOW;
  if (bits & EB_TIMEOUT) return SPTRSV_ERR_TIMEOUT;
  return SPTRSV_OK;
}

sptrsv_status_t set_err(sptrsv_ctx *h, sptrsv_status_t st, const char *fmt, ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    h->last_error = std::string(sptrsv_status_name(st)) + ": " + buf;
  }
  return st;
}

namespace {

int bit_width(int64_t v) {
  int b = 0;
  while (v > 0) {
    ++b;
    v >>= 1;
  }
  return b;
}

}  // namespace

// Overlapped transposes: at most kMaxSegments segments of the level chain,
// used from kOverlapMin work-vector entries on.
#ifndef SPTRSV_OVERLAP_MIN_LOG2
#define SPTRSV_OVERLAP_MIN_LOG2 22
#endif
#ifndef SPTRSV_MAX_SEGMENTS
#define SPTRSV_MAX_SEGMENTS 16
#endif
constexpr int32_t kMaxSegments = SPTRSV_MAX_SEGMENTS;
constexpr int64_t kOverlapMin = (int64_t)1 << SPTRSV_OVERLAP_MIN_LOG2;

sptrsv_schedule_t default_schedule() {
  sptrsv_schedule_t s{};
  s.mode = 0;
  s.thin_rows = 4096;
  s.wg_threads = 512;
  s.wide_threads = 256;
  s.lanes_per_row = 1;
  s.wide_grid = 0;
  s.overlap = 0;
  s.thin_cols = 0;
  return s;
}

namespace {

bool same_sched(const sptrsv_schedule_t &a, const sptrsv_schedule_t &b) {
  return a.mode == b.mode && a.thin_rows == b.thin_rows && a.wg_threads == b.wg_threads &&
         a.wide_threads == b.wide_threads && a.lanes_per_row == b.lanes_per_row && a.wide_grid == b.wide_grid &&
         a.overlap == b.overlap && a.thin_cols == b.thin_cols;
}

sptrsv_status_t check_sched(sptrsv_ctx *h, const sptrsv_schedule_t &s) {
  if (s.mode < 0 || s.mode > 4) return set_err(h, SPTRSV_ERR_ARG, "schedule mode %d", s.mode);
  if (s.mode == 4 && s.wide_threads != 128 && s.wide_threads != 256 && s.wide_threads != 512)
    return set_err(h, SPTRSV_ERR_ARG, "wide_threads %d: a dataflow run takes 128, 256 or 512", s.wide_threads);
  if (s.wg_threads != 256 && s.wg_threads != 512 && s.wg_threads != 1024)
    return set_err(h, SPTRSV_ERR_ARG, "wg_threads %d", s.wg_threads);
  if (s.wide_threads < 64 || s.wide_threads > 1024 || s.wide_threads % 64)
    return set_err(h, SPTRSV_ERR_ARG, "wide_threads %d", s.wide_threads);
  const int g = s.lanes_per_row;
  if (g != 1 && g != 2 && g != 4 && g != 8 && g != 16 && g != 32)
    return set_err(h, SPTRSV_ERR_ARG, "lanes_per_row %d", g);
  if (s.thin_rows < 0) return set_err(h, SPTRSV_ERR_ARG, "thin_rows %d", s.thin_rows);
  if (s.wide_grid < 0 || s.wide_grid > 65536) return set_err(h, SPTRSV_ERR_ARG, "wide_grid %d", s.wide_grid);
  if (s.overlap != 0 && s.overlap != 1) return set_err(h, SPTRSV_ERR_ARG, "overlap %d", s.overlap);
  if (s.thin_cols < 0) return set_err(h, SPTRSV_ERR_ARG, "thin_cols %d", s.thin_cols);
  if (s.mode == 3 && s.wide_grid > 2048)
    return set_err(h, SPTRSV_ERR_ARG, "wide_grid %d: the synchronisation-free launch takes at most 2048 workgroups",
                   s.wide_grid);
  return SPTRSV_OK;
}

}  // namespace

// The schedule actually used for (P, nrhs): a tuned one if present, else the
// handle's knobs.
sptrsv_schedule_t effective_sched(const Plan &P, int32_t nrhs) {
  auto it = P.tuned.find(nrhs);
  return it != P.tuned.end() ? it->second : P.sched;
}

static int64_t win_bytes(int64_t rows, int64_t ents, int64_t nl, int32_t nrhs) {
  return thin_window_bytes(rows, ents, nl, nrhs);
}

// Wide levels whose rows have at least kLongRow off-diagonals on average are
// solved with a workgroup per row when there are 2 to 256 right-hand sides:
// a (row, column) item alone would sum them one after another.
constexpr int64_t kLongRow = 16;
bool long_rows(const Plan &P, int32_t l, int32_t nrhs) {
  if (nrhs < 2 || nrhs > 256 || P.h_lv_nnz.size() <= (size_t)l) return false;
  const int64_t rows = P.h_level_ptr[(size_t)l + 1] - P.h_level_ptr[(size_t)l];
  return rows > 0 && P.h_lv_nnz[(size_t)l] - rows >= kLongRow * rows;
}

// Right-hand sides per thin-run workgroup under schedule sc: thin_cols when
// it divides nrhs (and is smaller), else all of them.
int32_t thin_width(const sptrsv_schedule_t &sc, int32_t nrhs) {
  const int32_t c = sc.thin_cols;
  return c > 0 && c < nrhs && nrhs % c == 0 ? c : nrhs;
}

// A level alone in a window reads all its dependencies from earlier windows,
// so it needs no overflow records.
bool level_fits_window(const Plan &P, int32_t l, int32_t nrhs) {
  const int64_t rows = P.h_level_ptr[l + 1] - P.h_level_ptr[l];
  return win_bytes(rows, 0, 1, nrhs) <= thin_win_bytes();
}

// Upper bound on the overflow records of level l's rows in a window that
// starts at level ws: dependencies (beyond each row's two at the highest
// levels) at most l - ws levels up, counted by whole distance buckets.
static int64_t extras_in(const Plan &P, int32_t l, int32_t ws) {
  const int32_t d = l - ws;
  const int32_t *hx = P.h_xh.data() + (size_t)l * kExtraBuckets;
  int64_t e = 0;
  for (int b = 0; b < kExtraBuckets && kExtraLo[b] <= d; ++b) e += hx[b];
  return e;
}

// Cut levels [l0, l1) into LDS windows; flag windows whose levels fit one wave
// (bit 0) or one item per thread of a workgroup of wg threads (bit 1), and
// give each window its bound on overflow records. Appends the windows and a
// terminator holding l1; returns the number of windows.
int32_t cut_windows(const Plan &P, int32_t l0, int32_t l1, int32_t nrhs, int32_t wg, std::vector<int4> &out) {
  const int64_t cap = thin_win_bytes();
  const size_t first = out.size();
  int32_t ws = l0;
  int64_t rows = 0, ents = 0, maxit = 0;
  auto flags = [&]() { return (maxit <= 64 ? 1 : 0) | (maxit <= wg ? 2 : 0); };
  for (int32_t l = l0; l < l1; ++l) {
    const int64_t rl = P.h_level_ptr[l + 1] - P.h_level_ptr[l];
    int64_t el = extras_in(P, l, ws);
    if (l > ws && win_bytes(rows + rl, ents + el, l - ws + 1, nrhs) > cap) {
      out.push_back(int4{ws, flags(), (int32_t)ents, 0});
      ws = l;
      rows = ents = maxit = 0;
      el = 0;
    }
    rows += rl;
    ents += el;
    maxit = std::max<int64_t>(maxit, rl * nrhs);
  }
  out.push_back(int4{ws, flags(), (int32_t)ents, 0});
  const int32_t nw = (int32_t)(out.size() - first);
  out.push_back(int4{l1, -1, 0, 0});
  return nw;
}

// Static images of every window in P.h_win (entries with y >= 0; the others
// end a run): exact overflow counts replace the host bounds in .z, image
// offsets (16-byte units) go to .w, and the table is uploaded.
sptrsv_status_t build_images(sptrsv_ctx *h, Plan &P, hipStream_t s) {
  const int32_t nent = (int32_t)P.h_win.size();
  if (nent == 0 || P.n == 0) return SPTRSV_OK;
  std::vector<int32_t> lvl_win((size_t)P.nlev, -1);
  for (int32_t e = 0; e < nent; ++e) {
    if (P.h_win[(size_t)e].y < 0) continue;
    for (int32_t l = P.h_win[(size_t)e].x; l < P.h_win[(size_t)e + 1].x; ++l) lvl_win[(size_t)l] = e;
  }
  const int32_t n = P.n;
  DArr<int32_t> d_lw;
  DArr<long long> ocnt, oex, ecnt, eex, wpre;
  HIPCHK(h, d_lw.alloc((size_t)P.nlev));
  HIPCHK(h, ocnt.alloc(n));
  HIPCHK(h, oex.alloc(n));
  HIPCHK(h, ecnt.alloc(n));
  HIPCHK(h, eex.alloc(n));
  HIPCHK(h, wpre.alloc((size_t)nent));
  if (P.win.n < (size_t)nent) HIPCHK(h, P.win.alloc((size_t)nent));
  HIPCHK(h, hipMemcpyAsync(d_lw.p, lvl_win.data(), sizeof(int32_t) * (size_t)P.nlev, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(P.win.p, P.h_win.data(), sizeof(int4) * (size_t)nent, hipMemcpyHostToDevice, s));
  HIPCHK(h, launch_img_count(n, P.level_ptr.p, P.nlev, d_lw.p, P.win.p, P.srp.p, P.sci.p, ocnt.p, ecnt.p, s));
  const size_t scr = scan_scratch_elems(n) + 16;
  if (h->scan_tmp.n < scr) HIPCHK(h, h->scan_tmp.alloc(scr));
  HIPCHK(h, launch_scan_i64(ocnt.p, oex.p, n, h->scan_tmp.p, s));
  HIPCHK(h, launch_scan_i64(ecnt.p, eex.p, n, h->scan_tmp.p, s));
  int32_t *aux = h->d_aux.p;
  HIPCHK(h, hipMemsetAsync(aux + 1, 0, sizeof(int32_t), s));
  HIPCHK(h, P.ext_ptr.reserve((size_t)n + 1));
  HIPCHK(h, launch_ptr_from_scan(eex.p, ecnt.p, n, P.ext_ptr.p, aux + 1, s));
  HIPCHK(h, launch_win_prefix(nent, P.win.p, P.level_ptr.p, n, oex.p, ocnt.p, wpre.p, s));
  std::vector<long long> hpre((size_t)nent);
  int32_t next = 0, bits = 0;
  HIPCHK(h, hipMemcpyAsync(hpre.data(), wpre.p, sizeof(long long) * (size_t)nent, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(&next, P.ext_ptr.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(&bits, aux + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (bits) return set_err(h, SPTRSV_ERR_OVERFLOW, "dependencies before LDS windows exceed int32 indexing");
  int64_t units = 0;
  for (int32_t e = 0; e < nent; ++e) {
    int4 &W = P.h_win[(size_t)e];
    if (W.y < 0) continue;
    const long long no = hpre[(size_t)e + 1] - hpre[(size_t)e];
    if (no > W.z)  // the host bound is an upper bound by construction
      return set_err(h, SPTRSV_ERR_ARG, "window %d: %lld overflow records exceed the bound %d", e, no, W.z);
    const int64_t R = P.h_level_ptr[(size_t)P.h_win[(size_t)e + 1].x] - P.h_level_ptr[(size_t)W.x];
    W.z = (int32_t)no;
    W.w = (int32_t)units;
    units += window_image_units(R, no);
    if (units >= ((int64_t)1 << 31)) return set_err(h, SPTRSV_ERR_OVERFLOW, "window images exceed int32 indexing");
  }
  HIPCHK(h, P.img.reserve((size_t)units));
  HIPCHK(h, P.ext.reserve((size_t)next));
  HIPCHK(h, hipMemcpyAsync(P.win.p, P.h_win.data(), sizeof(int4) * (size_t)nent, hipMemcpyHostToDevice, s));
  HIPCHK(h, launch_img_fill(n, P.level_ptr.p, P.nlev, d_lw.p, P.win.p, P.srp.p, P.sci.p, P.sva.p, P.sdg.p, oex.p,
                            P.ext_ptr.p, P.img.p, P.ext.p, io_perm(P), s));
  HIPCHK(h, hipStreamSynchronize(s));
  return SPTRSV_OK;
}

// Chunk tables of the dataflow runs (schedule mode 4): each level of a flow
// run is cut into chunks of one workgroup's items (rows_per_chunk rows); a
// chunk's list holds the distinct chunks of the same run that hold the rows
// its rows depend on. Built on the host from the level-ordered pattern, which
// the plan keeps a host copy of after the first build.
static sptrsv_status_t build_flow(sptrsv_ctx *h, Plan &P, int32_t nrhs, const sptrsv_schedule_t &sc,
                                  hipStream_t s) {
  const int32_t n = P.n;
  if (P.h_srp.empty()) {
    P.h_srp.resize((size_t)n + 1);
    P.h_sci.resize((size_t)std::max<int64_t>(P.nnz - n, 1));
    HIPCHK(h, hipMemcpyAsync(P.h_srp.data(), P.srp.p, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, s));
    if (P.nnz > n)
      HIPCHK(h, hipMemcpyAsync(P.h_sci.data(), P.sci.p, sizeof(int32_t) * (size_t)(P.nnz - n), hipMemcpyDeviceToHost,
                               s));
    HIPCHK(h, hipStreamSynchronize(s));
  }
  const int32_t rpc = std::max(1, sc.wide_threads * flow_items_per_thread() / nrhs);
  std::vector<int32_t> cpos, dptr, dlist, lcs, chunk_of((size_t)n, -1), stamp;
  int32_t nflags = 0;
  for (Run &r : P.runs) {
    if (!r.flow) continue;
    r.cp = (int32_t)cpos.size();
    r.fl = nflags;
    r.lc = (int32_t)lcs.size();
    r.max_chunks = 0;
    const int32_t pbeg = P.h_level_ptr[(size_t)r.l0], pend = P.h_level_ptr[(size_t)r.l1];
    for (int32_t l = r.l0; l < r.l1; ++l) {
      const int32_t first = (int32_t)cpos.size() - r.cp;
      lcs.push_back(first);
      for (int32_t p = P.h_level_ptr[(size_t)l]; p < P.h_level_ptr[(size_t)l + 1]; p += rpc) {
        const int32_t k = (int32_t)cpos.size() - r.cp;
        const int32_t pe = std::min(p + rpc, P.h_level_ptr[(size_t)l + 1]);
        for (int32_t q = p; q < pe; ++q) chunk_of[(size_t)q] = k;
        cpos.push_back(p);
      }
      r.max_chunks = std::max(r.max_chunks, (int32_t)cpos.size() - r.cp - first);
    }
    r.nchunk = (int32_t)cpos.size() - r.cp;
    lcs.push_back(r.nchunk);
    cpos.push_back(pend);
    // dptr has one entry per chunk and a terminator, aligned with cpos (same offsets)
    dptr.resize(cpos.size() - 1 - r.nchunk);
    stamp.assign((size_t)r.nchunk, -1);
    for (int32_t k = 0; k < r.nchunk; ++k) {
      dptr.push_back((int32_t)dlist.size());
      for (int32_t p = cpos[(size_t)(r.cp + k)]; p < cpos[(size_t)(r.cp + k + 1)]; ++p)
        for (int32_t q = P.h_srp[(size_t)p]; q < P.h_srp[(size_t)p + 1]; ++q) {
          const int32_t d = P.h_sci[(size_t)q];
          if (d < pbeg) continue;  // finished by an earlier launch
          const int32_t dc = chunk_of[(size_t)d];
          if (stamp[(size_t)dc] != k) {
            stamp[(size_t)dc] = k;
            dlist.push_back(dc);
          }
        }
    }
    dptr.push_back((int32_t)dlist.size());
    nflags += r.nchunk;
  }
  if (dlist.empty()) dlist.push_back(0);
  HIPCHK(h, P.flow_pos.alloc(cpos.size()));
  HIPCHK(h, P.flow_dptr.alloc(dptr.size()));
  HIPCHK(h, P.flow_dlist.alloc(dlist.size()));
  HIPCHK(h, P.flow_lc.alloc(std::max<size_t>(lcs.size(), 1)));
  if (!lcs.empty())
    HIPCHK(h, hipMemcpy(P.flow_lc.p, lcs.data(), sizeof(int32_t) * lcs.size(), hipMemcpyHostToDevice));
  HIPCHK(h, P.flow_flags.alloc((size_t)std::max(nflags, 1)));
  HIPCHK(h, P.flow_ctl.alloc(4));
  HIPCHK(h, hipMemcpy(P.flow_pos.p, cpos.data(), sizeof(int32_t) * cpos.size(), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(P.flow_dptr.p, dptr.data(), sizeof(int32_t) * dptr.size(), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(P.flow_dlist.p, dlist.data(), sizeof(int32_t) * dlist.size(), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemset(P.flow_flags.p, 0, sizeof(unsigned) * (size_t)std::max(nflags, 1)));
  HIPCHK(h, hipMemset(P.flow_ctl.p, 0, 4 * sizeof(unsigned)));
  return SPTRSV_OK;
}

// Segments of the level chain and the tile groups of the overlapped
// transposes (Plan::ovl): used when the vectors are large (n * nrhs >= 2^22)
// and the chain has several runs; segments end at run boundaries, at about
// equal shares of the positions.

static sptrsv_status_t build_overlap(sptrsv_ctx *h, Plan &P, int32_t nrhs, const sptrsv_schedule_t &sc,
                                     hipStream_t s) {
  P.ovl = false;
  P.seg_run.clear();
  const int32_t nruns = (int32_t)P.runs.size();
  if (!sc.overlap || sc.mode == 3 || (int64_t)P.n * nrhs < kOverlapMin || nruns < 4 || !h->side) return SPTRSV_OK;
  const int32_t K = std::min(kMaxSegments, nruns);
  P.seg_run.push_back(0);
  for (int32_t k = 1; k < K; ++k) {
    const int64_t target = (int64_t)P.n * k / K;
    int32_t r = P.seg_run.back() + 1;
    while (r < nruns && P.h_level_ptr[(size_t)P.runs[(size_t)r].l0] < target) ++r;
    if (r >= nruns) break;
    P.seg_run.push_back(r);
  }
  P.seg_run.push_back(nruns);
  const int32_t nseg = (int32_t)P.seg_run.size() - 1;
  if (nseg < 2) {
    P.seg_run.clear();
    return SPTRSV_OK;
  }
  std::vector<int32_t> seg_pos((size_t)nseg + 1);
  for (int32_t k = 0; k < nseg; ++k) seg_pos[(size_t)k] = P.h_level_ptr[(size_t)P.runs[(size_t)P.seg_run[(size_t)k]].l0];
  seg_pos[(size_t)nseg] = P.n;
  const int32_t ntiles = (P.n + 63) / 64;
  DArr<int32_t> first, last;
  HIPCHK(h, first.alloc((size_t)ntiles));
  HIPCHK(h, last.alloc((size_t)ntiles));
  HIPCHK(h, launch_tile_span(P.n, io_iperm(P), first.p, last.p, s));
  std::vector<int32_t> hf((size_t)ntiles), hl((size_t)ntiles);
  HIPCHK(h, hipMemcpyAsync(hf.data(), first.p, sizeof(int32_t) * (size_t)ntiles, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(hl.data(), last.p, sizeof(int32_t) * (size_t)ntiles, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  auto seg_of = [&](int32_t pos) {
    return (int32_t)(std::upper_bound(seg_pos.begin(), seg_pos.end(), pos) - seg_pos.begin()) - 1;
  };
  // counting sort of the tiles by the segment of their first / last position
  auto group = [&](const std::vector<int32_t> &key, std::vector<int32_t> &off, std::vector<int32_t> &out) {
    off.assign((size_t)nseg + 1, 0);
    std::vector<int32_t> g((size_t)ntiles);
    for (int32_t t = 0; t < ntiles; ++t) {
      g[(size_t)t] = seg_of(key[(size_t)t]);
      ++off[(size_t)g[(size_t)t] + 1];
    }
    for (int32_t k = 0; k < nseg; ++k) off[(size_t)k + 1] += off[(size_t)k];
    out.assign((size_t)ntiles, 0);
    std::vector<int32_t> at(off.begin(), off.end() - 1);
    for (int32_t t = 0; t < ntiles; ++t) out[(size_t)at[(size_t)g[(size_t)t]]++] = t;
  };
  std::vector<int32_t> gt, st;
  group(hf, P.g_off, gt);
  group(hl, P.s_off, st);
  HIPCHK(h, P.g_tiles.reserve((size_t)ntiles));
  HIPCHK(h, P.s_tiles.reserve((size_t)ntiles));
  HIPCHK(h, hipMemcpy(P.g_tiles.p, gt.data(), sizeof(int32_t) * (size_t)ntiles, hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(P.s_tiles.p, st.data(), sizeof(int32_t) * (size_t)ntiles, hipMemcpyHostToDevice));
  P.t_off.assign((size_t)nseg + 1, 0);
  for (int32_t k = 0; k <= nseg; ++k)
    P.t_off[(size_t)k] = (int32_t)(std::lower_bound(P.h_tpos.begin(), P.h_tpos.end(), seg_pos[(size_t)k]) -
                                   P.h_tpos.begin());
  if ((int32_t)h->ovl_ev.size() < 2 * nseg + 2) return set_err(h, SPTRSV_ERR_STATE, "overlap events missing");
  P.ovl = true;
  return SPTRSV_OK;
}

sptrsv_status_t make_runs(sptrsv_ctx *h, Plan &P, int32_t nrhs, const sptrsv_schedule_t &sc, hipStream_t s) {
  P.runs.clear();
  P.h_win.clear();
  const int64_t cap = thin_win_bytes();
  const int64_t thr = sc.thin_rows;
  auto rows_of = [&](int32_t l) -> int64_t { return P.h_level_ptr[l + 1] - P.h_level_ptr[l]; };
  const bool flow = sc.mode == 4;
  const int32_t gw = thin_width(sc, nrhs);  // columns per thin-run workgroup
  for (int32_t l = 0; l < P.nlev; ++l) {
    const int64_t rows = rows_of(l);
    bool thin = sc.mode == 2 || ((sc.mode == 0 || flow) && rows <= thr);
    if (win_bytes(rows, 0, 1, gw) > cap) thin = false;  // must fit one window alone
    // a wide level whose rows average many dependencies, with several
    // right-hand sides, is a launch of its own with a workgroup per row
    const bool longr = !thin && long_rows(P, l, nrhs);
    // consecutive thin levels share a run; so do consecutive wide levels of a persistent or dataflow launch
    if (!longr && !P.runs.empty() && P.runs.back().thin == thin && !P.runs.back().longr &&
        P.runs.back().l1 == l && (thin || sc.wide_grid > 0 || flow))
      P.runs.back().l1 = l + 1;
    else
      P.runs.push_back(Run{l, l + 1, thin});
    if (!thin) P.runs.back().flow = flow && !longr;
    P.runs.back().longr = longr;
  }
  // with the transposes overlapped, long dataflow runs are cut into pieces of
  // about n / kMaxSegments positions so that the chain has segment boundaries
  if (flow && sc.overlap && (int64_t)P.n * nrhs >= kOverlapMin) {
    std::vector<Run> cut;
    const int64_t piece = std::max<int64_t>(1, P.n / kMaxSegments);
    for (const Run &r : P.runs) {
      if (!r.flow) {
        cut.push_back(r);
        continue;
      }
      int32_t a = r.l0;
      for (int32_t l = r.l0; l < r.l1; ++l)
        if (P.h_level_ptr[(size_t)l + 1] - P.h_level_ptr[(size_t)a] >= piece || l + 1 == r.l1) {
          Run q{a, l + 1, false};
          q.flow = true;
          cut.push_back(q);
          a = l + 1;
        }
    }
    P.runs.swap(cut);
  }
  for (Run &r : P.runs) {
    if (!r.thin) continue;
    r.wi = (int32_t)P.h_win.size();
    r.nw = cut_windows(P, r.l0, r.l1, gw, sc.wg_threads, P.h_win);
  }
  P.runs_nrhs = -1;  // until the images are built
  STCHK(build_images(h, P, s));
  if (flow) STCHK(build_flow(h, P, nrhs, sc, s));
  STCHK(build_overlap(h, P, nrhs, sc, s));
  P.runs_nrhs = nrhs;
  P.runs_sched = sc;
  return SPTRSV_OK;
}

sptrsv_status_t ensure_work(sptrsv_ctx *h, Plan &P, int32_t nrhs) {
  const size_t need = (size_t)P.n * (size_t)nrhs;
  if (P.bp.n < need || !P.bp.p) HIPCHK(h, P.bp.alloc(need));
  if (P.xp.n < need || !P.xp.p) HIPCHK(h, P.xp.alloc(need));
  P.work_nrhs = std::max(P.work_nrhs, nrhs);
  return SPTRSV_OK;
}

// ---------------------------------------------------------------------------
// Plan construction: levels (longest path), stable bucketing of rows by level,
// level-ordered copy, optional T, statistics.
sptrsv_status_t build_plan(sptrsv_ctx *h, Plan &P, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                           const double *va, const int32_t *trp, const int32_t *tci, const double *tva,
                           hipStream_t s, bool rev_io) {
  sptrsv_schedule_t keep_sched = P.ready ? P.sched : default_schedule();
  P = Plan{};
  P.sched = keep_sched;
  P.n = n;
  P.nnz = nnz;
  HIPCHK(h, P.level_ptr.alloc((size_t)n + 1));
  HIPCHK(h, P.perm.alloc(n));
  HIPCHK(h, P.iperm.alloc(n));
  HIPCHK(h, P.row_level.alloc(n));
  HIPCHK(h, P.srp.alloc((size_t)n + 1));
  if (n == 0) {
    HIPCHK(h, hipMemsetAsync(P.level_ptr.p, 0, sizeof(int32_t), s));
    HIPCHK(h, hipMemsetAsync(P.srp.p, 0, sizeof(int32_t), s));
    HIPCHK(h, P.sci.alloc(1));
    HIPCHK(h, P.sva.alloc(1));
    HIPCHK(h, P.sdg.alloc(1));
    HIPCHK(h, hipStreamSynchronize(s));
    P.h_level_ptr.assign(1, 0);
    P.ready = true;
    return SPTRSV_OK;
  }
  DArr<int32_t> lev1, keys, ktmp, vtmp, hist;
  DArr<long long> cnt, ex, hist64;
  HIPCHK(h, lev1.alloc(n));
  HIPCHK(h, keys.alloc(n));
  HIPCHK(h, ktmp.alloc(n));
  HIPCHK(h, vtmp.alloc(n));
  HIPCHK(h, cnt.alloc(n));
  HIPCHK(h, ex.alloc(n));
  const size_t hn = radix_hist_elems(n);
  HIPCHK(h, hist.alloc(hn));
  HIPCHK(h, hist64.alloc(hn));
  const size_t scr = std::max(scan_scratch_elems((int64_t)hn), scan_scratch_elems(n)) + 16;
  if (h->scan_tmp.n < scr) HIPCHK(h, h->scan_tmp.alloc(scr));
  int32_t *aux = h->d_aux.p;  // [0] ticket, [1] error bits, [2] max level+1, [3..4] total cost
  HIPCHK(h, hipMemsetAsync(aux, 0, 8 * sizeof(int32_t), s));
  HIPCHK(h, hipMemsetAsync(lev1.p, 0, sizeof(int32_t) * (size_t)n, s));
  HIPCHK(h, launch_levels(n, rp, ci, lev1.p, reinterpret_cast<unsigned *>(aux), aux + 1, s));
  HIPCHK(h, launch_max(lev1.p, n, aux + 2, s));
  int32_t haux[8];
  HIPCHK(h, hipMemcpyAsync(haux, aux, sizeof(haux), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (haux[1]) return set_err(h, status_from_bits(haux[1]), "level construction failed (bits 0x%x)", haux[1]);
  const int32_t nlev = haux[2];
  P.nlev = nlev;
  // rows sorted stably by level -> level_rows (= perm), level_ptr
  HIPCHK(h, hipMemcpyAsync(keys.p, lev1.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, launch_iota(P.perm.p, n, s));
  HIPCHK(h, launch_radix_by_key(keys.p, P.perm.p, ktmp.p, vtmp.p, n, bit_width(nlev), hist.p, hist64.p,
                                h->scan_tmp.p, s));
  HIPCHK(h, launch_level_ptr_from_sorted(keys.p, n, P.level_ptr.p, nlev, s));
  HIPCHK(h, launch_invert_perm(P.perm.p, n, P.iperm.p, s));
  if (rev_io) {
    P.rev_io = true;
    HIPCHK(h, P.perm_io.alloc(n));
    HIPCHK(h, P.iperm_io.alloc(n));
    HIPCHK(h, launch_rev_io(n, P.perm.p, P.iperm.p, P.perm_io.p, P.iperm_io.p, s));
  }
  HIPCHK(h, launch_sub1(lev1.p, n, P.row_level.p, s));
  // level-ordered copy of the off-diagonals
  HIPCHK(h, launch_count_off(P.perm.p, rp, n, cnt.p, s));
  HIPCHK(h, launch_scan_i64(cnt.p, ex.p, n, h->scan_tmp.p, s));
  HIPCHK(h, launch_ptr_from_scan(ex.p, cnt.p, n, P.srp.p, aux + 1, s));
  const int64_t noff = nnz - n;
  HIPCHK(h, P.sci.alloc((size_t)std::max<int64_t>(noff, 1)));
  HIPCHK(h, P.sva.alloc((size_t)std::max<int64_t>(noff, 1)));
  HIPCHK(h, P.sdg.alloc(n));
  HIPCHK(h, launch_fill_solve(n, P.perm.p, P.iperm.p, rp, ci, va, P.srp.p, P.sci.p, P.sva.p, P.sdg.p, s));
  HIPCHK(h, P.ell_c.alloc(n));
  HIPCHK(h, P.ell_v.alloc((size_t)2 * n));
  HIPCHK(h, launch_fill_ell(n, P.srp.p, P.sci.p, P.sva.p, P.ell_c.p, P.ell_v.p, s));
  HIPCHK(h, P.wbar.alloc(kGridBarWords));
  HIPCHK(h, hipMemsetAsync(P.wbar.p, 0, kGridBarWords * sizeof(unsigned), s));
  HIPCHK(h, P.tp.alloc(4));
  HIPCHK(h, hipMemsetAsync(P.tp.p, 0, 4 * sizeof(unsigned), s));
  HIPCHK(h, P.sf_ticket.alloc(1));
  if (trp) {
    P.has_t = true;
    HIPCHK(h, P.trp.alloc((size_t)n + 1));
    HIPCHK(h, launch_count_off(P.perm.p, trp, n, cnt.p, s));
    HIPCHK(h, launch_scan_i64(cnt.p, ex.p, n, h->scan_tmp.p, s));
    HIPCHK(h, launch_ptr_from_scan(ex.p, cnt.p, n, P.trp.p, aux + 1, s));
    int32_t tn = 0;
    HIPCHK(h, hipMemcpyAsync(&tn, P.trp.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    P.nnz_t_off = tn;
    HIPCHK(h, P.tci.alloc((size_t)std::max(tn, 1)));
    HIPCHK(h, P.tva.alloc((size_t)std::max(tn, 1)));
    HIPCHK(h, launch_fill_t(n, P.perm.p, trp, tci, tva, P.trp.p, P.tci.p, P.tva.p, rev_io, s));
  }
  // statistics of the cost model
  HIPCHK(h, P.lv_rows.alloc(nlev));
  HIPCHK(h, P.lv_nnz.alloc(nlev));
  HIPCHK(h, P.lv_cost.alloc(nlev));
  HIPCHK(h, launch_level_stats(nlev, P.level_ptr.p, P.srp.p, P.lv_rows.p, P.lv_nnz.p, P.lv_cost.p,
                               reinterpret_cast<long long *>(aux + 4), s));
  P.h_level_ptr.resize((size_t)nlev + 1);
  HIPCHK(h, hipMemcpyAsync(P.h_level_ptr.data(), P.level_ptr.p, sizeof(int32_t) * ((size_t)nlev + 1),
                           hipMemcpyDeviceToHost, s));
  P.h_lv_nnz.resize((size_t)nlev);
  HIPCHK(h, hipMemcpyAsync(P.h_lv_nnz.data(), P.lv_nnz.p, sizeof(int64_t) * (size_t)nlev, hipMemcpyDeviceToHost, s));
  std::vector<int32_t> htrp;
  if (P.has_t) {
    htrp.resize((size_t)n + 1);
    HIPCHK(h, hipMemcpyAsync(htrp.data(), P.trp.p, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(h, hipMemcpyAsync(haux, aux, sizeof(haux), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (haux[1]) return set_err(h, status_from_bits(haux[1]), "plan construction failed (bits 0x%x)", haux[1]);
  STCHK(build_extra_hist(h, P, s));
  if (P.has_t) {
    P.h_lv_tnnz.resize((size_t)nlev);
    for (int32_t l = 0; l < nlev; ++l)
      P.h_lv_tnnz[(size_t)l] = htrp[(size_t)P.h_level_ptr[l + 1]] - htrp[(size_t)P.h_level_ptr[l]];
    // positions whose row of T has off-diagonals: the only rows b' = T b changes
    std::vector<int32_t> tpos;
    for (int32_t p = 0; p < n; ++p)
      if (htrp[(size_t)p + 1] > htrp[(size_t)p]) tpos.push_back(p);
    P.n_tpos = (int32_t)tpos.size();
    P.h_tpos = tpos;
    // lanes per row of T: enough that a group's reads of a row coalesce, few
    // enough that most lanes hold an entry
    const double avg_t = P.n_tpos > 0 ? (double)P.nnz_t_off / (double)P.n_tpos : 0.0;
    P.t_lanes = avg_t >= 48.0 ? 64 : avg_t >= 12.0 ? 16 : avg_t >= 3.0 ? 4 : 1;
    HIPCHK(h, P.tpos.alloc(std::max<size_t>(tpos.size(), 1)));
    if (!tpos.empty())
      HIPCHK(h, hipMemcpy(P.tpos.p, tpos.data(), sizeof(int32_t) * tpos.size(), hipMemcpyHostToDevice));
  }
  long long tot;
  std::memcpy(&tot, haux + 4, sizeof(tot));
  P.total_cost = tot;
  P.avg_cost = nlev > 0 ? (double)tot / (double)nlev : 0.0;
  P.ready = true;
  return SPTRSV_OK;
}

// Algorithmic bytes of solving levels [l0, l1), the levels' share of the
// compulsory traffic of a solve: every nonzero once as value + column (12 B,
// the diagonal included), per row its pointer and level map entry (8 B; 12 B
// with the row pointer of T for a rewritten matrix), b read and x written
// once per right-hand side, and the level pointers. T's entries are the
// gather's share (T b is applied there).
static double run_bytes(const Plan &P, int32_t l0, int32_t l1, int32_t nrhs) {
  double b = 4.0 * (l1 - l0 + 1);
  const double per_row = P.has_t ? 12.0 : 8.0;
  for (int32_t l = l0; l < l1; ++l) {
    const double rows = P.h_level_ptr[l + 1] - P.h_level_ptr[l];
    b += 12.0 * (double)P.h_lv_nnz[l] + per_row * rows + 16.0 * rows * nrhs;
  }
  return b;
}

// Live profile: an event pair around one launch (class cls).
static int prof_begin(sptrsv_ctx *h, int cls, double bytes, hipStream_t s) {
  if (!h->prof || h->prof_used + 2 > h->prof_ev.size()) return -1;
  const int slot = (int)(h->prof_used / 2);
  if (hipEventRecord(h->prof_ev[h->prof_used], s) != hipSuccess) return -1;
  h->prof_used += 2;
  h->prof_cls[(size_t)slot] = cls;
  h->prof_bytes[(size_t)slot] = bytes;
  return slot;
}
static void prof_end(sptrsv_ctx *h, int slot, hipStream_t s) {
  if (slot >= 0) (void)hipEventRecord(h->prof_ev[(size_t)slot * 2 + 1], s);
}

ThinArgs thin_args(const Plan &P) { return thin_args(P, P.bp.p, P.xp.p); }
ThinArgs thin_args(const Plan &P, double *bp, double *xp) {
  return ThinArgs{P.level_ptr.p, P.sdg.p, P.img.p, P.ext_ptr.p, P.ext.p, bp, xp, P.tp.p};
}

// The level-distance histogram of the dependencies that need overflow records
// (host copy, for cutting LDS windows).
sptrsv_status_t build_extra_hist(sptrsv_ctx *h, Plan &P, hipStream_t s) {
  P.h_xh.assign((size_t)P.nlev * kExtraBuckets, 0);
  if (P.n == 0 || P.nlev == 0) return SPTRSV_OK;
  DArr<int32_t> lop, hist;
  HIPCHK(h, lop.alloc(P.n));
  HIPCHK(h, hist.alloc(P.h_xh.size()));
  HIPCHK(h, hipMemsetAsync(hist.p, 0, sizeof(int32_t) * P.h_xh.size(), s));
  HIPCHK(h, launch_extra_hist(P.n, P.level_ptr.p, P.nlev, P.srp.p, P.sci.p, lop.p, hist.p, s));
  HIPCHK(h, hipMemcpyAsync(P.h_xh.data(), hist.p, sizeof(int32_t) * P.h_xh.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return SPTRSV_OK;
}

// b (caller's layout) -> bp (level order, interleaved); for the rewritten
// system b' = T b, where only the rows of T with off-diagonals differ from b:
// those are recomputed from the caller's b after the plain gather.
sptrsv_status_t gather_b(sptrsv_ctx *h, Plan &P, int32_t nrhs, const double *b, int64_t ldb, double *bp,
                         hipStream_t s) {
  HIPCHK(h, launch_gather(P.n, nrhs, b, ldb, io_iperm(P), bp, s));
  if (P.has_t && P.n_tpos > 0)
    HIPCHK(h, launch_apply_t(P.n_tpos, nrhs, P.t_lanes, P.tpos.p, io_perm(P), P.trp.p, P.tci.p, P.tva.p, b, 1, ldb,
                             bp, s));
  return SPTRSV_OK;
}

// One solve over the plan's runs, built for (nrhs, its schedule), with the
// work vectors bp and xp (n * nrhs doubles each). Allocates nothing.
// One run of the level chain (not the synchronisation-free executor).
static sptrsv_status_t launch_run(sptrsv_ctx *h, Plan &P, const Run &r, int32_t nrhs, const ThinArgs &ta, double *bp,
                                  double *xp, hipStream_t s) {
  const sptrsv_schedule_t &sc = P.runs_sched;
  int *err = h->d_err.p;
  const int slot = h->prof ? prof_begin(h, r.thin ? 1 : 2, run_bytes(P, r.l0, r.l1, nrhs), s) : -1;
  if (r.thin) {
    HIPCHK(h, launch_thin_run(sc.wg_threads, P.win.p + r.wi, r.nw, nrhs, ta, err, s, nullptr, 0.f,
                              thin_width(sc, nrhs)));
  } else if (r.longr) {
    const int64_t rows = P.h_level_ptr[r.l1] - P.h_level_ptr[r.l0];
    const int32_t avg = (int32_t)std::min<int64_t>((P.h_lv_nnz[(size_t)r.l0] - rows) / std::max<int64_t>(rows, 1),
                                                   1 << 20);
    HIPCHK(h, launch_wide_long(P.h_level_ptr[r.l0], P.h_level_ptr[r.l1], nrhs, avg, P.srp.p, P.sci.p, P.sva.p,
                               P.sdg.p, bp, xp, err, s, ta.rio));
  } else if (r.flow) {
    const FlowArgs fa{P.flow_pos.p + r.cp, P.flow_dptr.p + r.cp, P.flow_dlist.p, P.flow_lc.p + r.lc,
                      P.flow_flags.p + r.fl, P.flow_ctl.p, P.srp.p, P.sci.p, P.sva.p, P.sdg.p, P.ell_c.p,
                      P.ell_v.p, bp, xp};
    HIPCHK(h, launch_flow_run(sc.wide_threads, sc.wide_grid, fa, r.l1 - r.l0, r.max_chunks, nrhs, err,
                              wait_limit(h), s));
  } else if (sc.wide_grid > 0) {
    HIPCHK(h, launch_wide_run(sc.wide_grid, sc.wide_threads, r.l0, r.l1, P.level_ptr.p, nrhs, P.srp.p, P.sci.p,
                              P.sva.p, P.sdg.p, P.ell_c.p, P.ell_v.p, bp, xp, P.wbar.p, err, wait_limit(h), s,
                              ta.rio));
  } else {
    HIPCHK(h, launch_wide_level(sc.wide_threads, sc.lanes_per_row, P.h_level_ptr[r.l0], P.h_level_ptr[r.l1], nrhs,
                                P.srp.p, P.sci.p, P.sva.p, P.sdg.p, P.ell_c.p, P.ell_v.p, bp, xp, err, s, ta.rio));
  }
  prof_end(h, slot, s);
  return SPTRSV_OK;
}

// The solve with the transposes beside the level chain: the side stream
// gathers segment k's tiles (and applies T to its rows) before the chain
// reaches segment k, and scatters the tiles that end in segment k while later
// segments run; the caller's stream waits for the side stream at the end.
static sptrsv_status_t solve_overlapped(sptrsv_ctx *h, Plan &P, int32_t nrhs, const double *b, int64_t ldb,
                                        double *x, int64_t ldx, double *bp, double *xp, hipStream_t s) {
  const int32_t nseg = (int32_t)P.seg_run.size() - 1;
  hipStream_t side = h->side;
  hipEvent_t *ev = h->ovl_ev.data();  // [0] fork, [1 + k] gathered, [1 + nseg + k] solved, [1 + 2 nseg] join
  const int32_t *iperm = io_iperm(P);
  HIPCHK(h, hipEventRecord(ev[0], s));
  HIPCHK(h, hipStreamWaitEvent(side, ev[0], 0));
  // segment k's b (and b-transform) on the side stream, then its event
  auto gather_seg = [&](int32_t k) -> sptrsv_status_t {
    HIPCHK(h, launch_gather_tiles(P.n, nrhs, b, ldb, iperm, P.g_tiles.p + P.g_off[(size_t)k],
                                  P.g_off[(size_t)k + 1] - P.g_off[(size_t)k], bp, side));
    const int32_t t0 = P.t_off[(size_t)k], t1 = P.t_off[(size_t)k + 1];
    if (P.has_t && t1 > t0)
      HIPCHK(h, launch_apply_t(t1 - t0, nrhs, P.t_lanes, P.tpos.p + t0, io_perm(P), P.trp.p, P.tci.p, P.tva.p, b,
                               1, ldb, bp, side));
    HIPCHK(h, hipEventRecord(ev[1 + k], side));
    return SPTRSV_OK;
  };
  // The side stream runs at most two segments ahead of the chain: segments 0
  // and 1 first, then, after segment k is solved, the scatter of k and the
  // gather of k + 2. The transposes are spread over the chain instead of
  // taking the memory system from its first segments all at once.
  STCHK(gather_seg(0));
  if (nseg > 1) STCHK(gather_seg(1));
  const ThinArgs ta = thin_args(P, bp, xp);
  for (int32_t k = 0; k < nseg; ++k) {
    HIPCHK(h, hipStreamWaitEvent(s, ev[1 + k], 0));
    for (int32_t ri = P.seg_run[(size_t)k]; ri < P.seg_run[(size_t)k + 1]; ++ri)
      STCHK(launch_run(h, P, P.runs[(size_t)ri], nrhs, ta, bp, xp, s));
    const int32_t n_sc = P.s_off[(size_t)k + 1] - P.s_off[(size_t)k];
    if (k + 1 < nseg) {
      HIPCHK(h, hipEventRecord(ev[1 + nseg + k], s));
      HIPCHK(h, hipStreamWaitEvent(side, ev[1 + nseg + k], 0));
      HIPCHK(h, launch_scatter_tiles(P.n, nrhs, xp, iperm, P.s_tiles.p + P.s_off[(size_t)k], n_sc, x, ldx, side));
      if (k + 2 < nseg) STCHK(gather_seg(k + 2));
    } else {
      HIPCHK(h, launch_scatter_tiles(P.n, nrhs, xp, iperm, P.s_tiles.p + P.s_off[(size_t)k], n_sc, x, ldx, s));
    }
  }
  HIPCHK(h, hipEventRecord(ev[1 + 2 * nseg], side));
  HIPCHK(h, hipStreamWaitEvent(s, ev[1 + 2 * nseg], 0));
  return SPTRSV_OK;
}

sptrsv_status_t solve_runs(sptrsv_ctx *h, Plan &P, int32_t nrhs, const double *b, int64_t ldb, double *x,
                           int64_t ldx, double *bp, double *xp, hipStream_t s) {
  if (P.n == 0) return SPTRSV_OK;
  const sptrsv_schedule_t sc = P.runs_sched;
  if (P.ovl && !h->prof) return solve_overlapped(h, P, nrhs, b, ldb, x, ldx, bp, xp, s);
  int *err = h->d_err.p;
  const double vec_bytes = 16.0 * (double)P.n * nrhs + 4.0 * P.n;
  int slot = prof_begin(h, 0, vec_bytes + (P.has_t ? 12.0 * (double)P.nnz_t_off + 4.0 * P.n : 0.0), s);
  STCHK(gather_b(h, P, nrhs, b, ldb, bp, s));
  prof_end(h, slot, s);
  if (sc.mode == 3) {  // synchronisation-free: one launch for the whole solve (profiled with the wide class)
    slot = h->prof ? prof_begin(h, 2, run_bytes(P, 0, P.nlev, nrhs), s) : -1;
    HIPCHK(h, launch_syncfree(P.n, nrhs, P.srp.p, P.sci.p, P.sva.p, P.sdg.p, bp, xp, P.sf_ticket.p, err,
                              sc.wide_grid, wait_limit(h), s));
    prof_end(h, slot, s);
  }
  const ThinArgs ta = thin_args(P, bp, xp);
  for (const Run &r : P.runs) {
    if (sc.mode == 3) break;
    STCHK(launch_run(h, P, r, nrhs, ta, bp, xp, s));
  }
  slot = prof_begin(h, 3, vec_bytes, s);
  HIPCHK(h, launch_scatter(P.n, nrhs, xp, io_iperm(P), x, ldx, s));
  prof_end(h, slot, s);
  return SPTRSV_OK;
}

bool runs_ready(const Plan &P, int32_t nrhs) {
  return P.runs_nrhs == nrhs && same_sched(effective_sched(P, nrhs), P.runs_sched);
}

sptrsv_status_t plan_solve(sptrsv_ctx *h, Plan &P, int32_t nrhs, const double *b, int64_t ldb, double *x,
                           int64_t ldx, hipStream_t s) {
  if (P.n == 0) return SPTRSV_OK;
  STCHK(ensure_work(h, P, nrhs));
  if (!runs_ready(P, nrhs)) STCHK(make_runs(h, P, nrhs, effective_sched(P, nrhs), s));
  return solve_runs(h, P, nrhs, b, ldb, x, ldx, P.bp.p, P.xp.p, s);
}

// The flags of the rows of T with off-diagonals, for solves by rows.
// And the dependencies of every position as caller rows (the first four in
// ell_r, all in sci_r).
sptrsv_status_t ensure_rows(sptrsv_ctx *h, Plan &P, hipStream_t s) {
  if (P.rows_ready || P.n == 0) return SPTRSV_OK;
  if (P.has_t) {
    HIPCHK(h, P.tflag.alloc((size_t)P.n));
    HIPCHK(h, launch_tflag(P.n, P.n_tpos, P.tpos.p, P.tflag.p, s));
  }
  HIPCHK(h, P.ell_r.alloc((size_t)P.n));
  HIPCHK(h, launch_map_ell(P.n, P.ell_c.p, io_perm(P), P.ell_r.p, s));
  const int64_t noff = P.nnz - P.n;
  HIPCHK(h, P.sci_r.alloc((size_t)std::max<int64_t>(noff, 1)));
  HIPCHK(h, launch_map_cols(noff, P.sci.p, io_perm(P), P.sci_r.p, s));
  P.rows_ready = true;
  return SPTRSV_OK;
}

// A solve with the right-hand sides stored by rows (entry (i, c) of b and x
// at i * nrhs + c; nrhs > 1). Thin runs and one launch per wide level read b
// and write x through the level order themselves (the b-transform writes only
// the rows of T with off-diagonals into the work vector); the other schedules
// copy b into the work vector and x out of it by rows.
sptrsv_status_t solve_rows(sptrsv_ctx *h, Plan &P, int32_t nrhs, const double *b, double *x, hipStream_t s) {
  if (P.n == 0) return SPTRSV_OK;
  STCHK(ensure_work(h, P, nrhs));
  if (!runs_ready(P, nrhs)) STCHK(make_runs(h, P, nrhs, effective_sched(P, nrhs), s));
  STCHK(ensure_rows(h, P, s));
  const sptrsv_schedule_t sc = P.runs_sched;
  double *bp = P.bp.p, *xp = P.xp.p;
  const int32_t *perm = io_perm(P);
  const bool t = P.has_t && P.n_tpos > 0;
  if (sc.mode != 3 && sc.mode != 4) {
    if (t)
      HIPCHK(h, launch_apply_t(P.n_tpos, nrhs, P.t_lanes, P.tpos.p, perm, P.trp.p, P.tci.p, P.tva.p, b, nrhs, 1, bp,
                               s));
    ThinArgs ta = thin_args(P, bp, xp);
    ta.rio = RowsIO{b, x, perm, P.has_t ? P.tflag.p : nullptr, P.ell_r.p, P.sci_r.p};
    for (const Run &r : P.runs) STCHK(launch_run(h, P, r, nrhs, ta, bp, xp, s));
    return SPTRSV_OK;
  }
  HIPCHK(h, launch_gather_rows(P.n, nrhs, b, perm, bp, s));
  if (t)
    HIPCHK(h, launch_apply_t(P.n_tpos, nrhs, P.t_lanes, P.tpos.p, perm, P.trp.p, P.tci.p, P.tva.p, b, nrhs, 1, bp, s));
  if (sc.mode == 3) {
    HIPCHK(h, launch_syncfree(P.n, nrhs, P.srp.p, P.sci.p, P.sva.p, P.sdg.p, bp, xp, P.sf_ticket.p, h->d_err.p,
                              sc.wide_grid, wait_limit(h), s));
  } else {
    const ThinArgs ta = thin_args(P, bp, xp);
    for (const Run &r : P.runs) STCHK(launch_run(h, P, r, nrhs, ta, bp, xp, s));
  }
  HIPCHK(h, launch_scatter_rows(P.n, nrhs, xp, perm, x, s));
  return SPTRSV_OK;
}

// ------------------------------------------------------------------- ABI
// The plan a solve-side entry point addresses (the analysed matrix or its rewrite).
Plan *plan_of(sptrsv_ctx *h, int which) {
  if (which == SPTRSV_ORIGINAL) return &h->orig;
  if (which == SPTRSV_REWRITTEN) return &h->rew;
  return nullptr;
}

// Plans whose schedule can be set, read and tuned (the batched one as well).
Plan *sched_plan_of(sptrsv_ctx *h, int which) {
  if (which == SPTRSV_BATCH) return h->b_ready ? &h->bat : nullptr;
  return plan_of(h, which);
}

extern "C" {

const char *sptrsv_status_name(sptrsv_status_t s) {
  switch (s) {
    case SPTRSV_OK: return "SPTRSV_OK";
    case SPTRSV_ERR_ARG: return "SPTRSV_ERR_ARG";
    case SPTRSV_ERR_STATE: return "SPTRSV_ERR_STATE";
    case SPTRSV_ERR_NOT_LOWER: return "SPTRSV_ERR_NOT_LOWER";
    case SPTRSV_ERR_UNSORTED: return "SPTRSV_ERR_UNSORTED";
    case SPTRSV_ERR_MISSING_DIAG: return "SPTRSV_ERR_MISSING_DIAG";
    case SPTRSV_ERR_ZERO_PIVOT: return "SPTRSV_ERR_ZERO_PIVOT";
    case SPTRSV_ERR_NONFINITE: return "SPTRSV_ERR_NONFINITE";
    case SPTRSV_ERR_OVERFLOW: return "SPTRSV_ERR_OVERFLOW";
    case SPTRSV_ERR_ALLOC: return "SPTRSV_ERR_ALLOC";
    case SPTRSV_ERR_HIP: return "SPTRSV_ERR_HIP";
    case SPTRSV_ERR_TIMEOUT: return "SPTRSV_ERR_TIMEOUT";
  }
  return "SPTRSV_UNKNOWN";
}

sptrsv_status_t sptrsv_create(sptrsv_handle_t *out) {
  if (!out) return SPTRSV_ERR_ARG;
  *out = nullptr;
  sptrsv_ctx *h = new (std::nothrow) sptrsv_ctx();
  if (!h) return SPTRSV_ERR_ALLOC;
  if (hipGetDevice(&h->dev) != hipSuccess || h->d_err.alloc(4) != hipSuccess || h->d_aux.alloc(512) != hipSuccess ||
      hipMemset(h->d_err.p, 0, 4 * sizeof(int32_t)) != hipSuccess ||
      hipMemset(h->d_aux.p, 0, 512 * sizeof(int32_t)) != hipSuccess) {
    delete h;
    return SPTRSV_ERR_HIP;
  }
  static bool inited = false;
  if (!inited) {
    solve_kernels_init();
    inited = true;
  }
  const hipError_t ne = noalloc_init(h->dev);
  if (ne != hipSuccess) {
    delete h;
    return SPTRSV_ERR_HIP;
  }
  // side stream and events of the overlapped transposes (default priority)
  bool ok = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) == hipSuccess;
  h->ovl_ev.assign(2 * kMaxSegments + 2, nullptr);
  for (auto &e : h->ovl_ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)sptrsv_destroy(h);
    return SPTRSV_ERR_HIP;
  }
  h->orig.sched = default_schedule();
  h->rew.sched = default_schedule();
  *out = h;
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_destroy(sptrsv_handle_t h) {
  if (!h) return SPTRSV_OK;
  (void)hipDeviceSynchronize();
  for (Graph &g : h->graphs) {
    if (g.ge) (void)hipGraphExecDestroy(g.ge);
    if (g.g) (void)hipGraphDestroy(g.g);
  }
  for (hipEvent_t e : h->ovl_ev)
    if (e) (void)hipEventDestroy(e);
  if (h->side) (void)hipStreamDestroy(h->side);
  delete h;
  return SPTRSV_OK;
}

const char *sptrsv_last_error(sptrsv_handle_t h) { return h ? h->last_error.c_str() : "null handle"; }

}  // extern "C"

namespace {

bool form_reversed(int32_t f) { return f == SPTRSV_UPPER || f == SPTRSV_LOWER_TRANS; }

// Transpose of a CSR with sorted rows (stable sort of the entries by column).
sptrsv_status_t transpose_csr(sptrsv_ctx *h, int32_t n, int32_t nnz, const int32_t *rp, const int32_t *ci,
                              const double *va, int32_t *orp, int32_t *oci, double *ova, hipStream_t s) {
  DArr<int32_t> keys, order, ktmp, vtmp, row_of, hist;
  DArr<long long> hist64;
  HIPCHK(h, keys.alloc(nnz));
  HIPCHK(h, order.alloc(nnz));
  HIPCHK(h, ktmp.alloc(nnz));
  HIPCHK(h, vtmp.alloc(nnz));
  HIPCHK(h, row_of.alloc(nnz));
  const size_t hn = radix_hist_elems(nnz);
  HIPCHK(h, hist.alloc(hn));
  HIPCHK(h, hist64.alloc(hn));
  const size_t scr = std::max(scan_scratch_elems((int64_t)hn), scan_scratch_elems(nnz)) + 16;
  if (h->scan_tmp.n < scr) HIPCHK(h, h->scan_tmp.alloc(scr));
  HIPCHK(h, hipMemcpyAsync(keys.p, ci, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, launch_iota(order.p, nnz, s));
  HIPCHK(h, launch_radix_by_key(keys.p, order.p, ktmp.p, vtmp.p, nnz, bit_width(n), hist.p, hist64.p,
                                h->scan_tmp.p, s));
  HIPCHK(h, launch_ptr_from_sorted(keys.p, nnz, n, orp, s));
  HIPCHK(h, launch_row_of_entry(n, rp, row_of.p, s));
  HIPCHK(h, launch_take_entries(nnz, order.p, row_of.p, va, oci, ova, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return SPTRSV_OK;
}

// Validate the input in its own triangular form and store its lower form in
// the handle: L as is; J U J; J L^T J; U^T (see k_form.hip).
sptrsv_status_t analyze_form(sptrsv_ctx *h, int32_t form, int32_t n, int32_t nnz, const int32_t *d_row_ptr,
                             const int32_t *d_col, const double *d_val, hipStream_t s, int32_t *nlevels_out) {
  if (!h) return SPTRSV_ERR_ARG;
  h->last_error.clear();
  if (form < SPTRSV_LOWER || form > SPTRSV_UPPER_TRANS) return set_err(h, SPTRSV_ERR_ARG, "analyze: form %d", form);
  if (n < 0 || nnz < 0 || !d_row_ptr || (nnz > 0 && (!d_col || !d_val)))
    return set_err(h, SPTRSV_ERR_ARG, "analyze: n=%d nnz=%d", n, nnz);
  if (nnz < n) return set_err(h, SPTRSV_ERR_MISSING_DIAG, "analyze: nnz %d < n %d", nnz, n);
  h->orig.ready = false;
  h->rew.ready = false;
  h->has_rewrite = false;
  const bool upper_in = form == SPTRSV_UPPER || form == SPTRSV_UPPER_TRANS;
  const bool trans = form == SPTRSV_LOWER_TRANS || form == SPTRSV_UPPER_TRANS;
  // the input as a lower matrix: itself, or its reversal for an upper input
  DArr<int32_t> r_rp, r_ci;
  DArr<double> r_va;
  const int32_t *lrp = d_row_ptr, *lci = d_col;
  const double *lva = d_val;
  if (upper_in) {
    HIPCHK(h, r_rp.alloc((size_t)n + 1));
    HIPCHK(h, r_ci.alloc((size_t)std::max(nnz, 1)));
    HIPCHK(h, r_va.alloc((size_t)std::max(nnz, 1)));
    HIPCHK(h, launch_rev_entries(n, nnz, d_row_ptr, d_col, d_val, r_rp.p, r_ci.p, r_va.p, s));
    lrp = r_rp.p;
    lci = r_ci.p;
    lva = r_va.p;
  }
  int32_t *aux = h->d_aux.p;
  HIPCHK(h, hipMemsetAsync(aux + 1, 0, sizeof(int32_t), s));
  HIPCHK(h, launch_validate(n, nnz, lrp, lci, lva, aux + 1, s));
  int32_t bits = 0;
  HIPCHK(h, hipMemcpyAsync(&bits, aux + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (bits)
    return set_err(h, status_from_bits(bits), "analyze: invalid %s matrix (bits 0x%x)",
                   upper_in ? "upper-triangular" : "lower-triangular", bits);
  h->n = n;
  h->nnz = nnz;
  h->form = form;
  HIPCHK(h, h->rp.alloc((size_t)n + 1));
  HIPCHK(h, h->ci.alloc((size_t)std::max(nnz, 1)));
  HIPCHK(h, h->va.alloc((size_t)std::max(nnz, 1)));
  if (!trans) {
    HIPCHK(h, hipMemcpyAsync(h->rp.p, lrp, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s));
    if (nnz) {
      HIPCHK(h, hipMemcpyAsync(h->ci.p, lci, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
      HIPCHK(h, hipMemcpyAsync(h->va.p, lva, sizeof(double) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
    }
  } else if (n > 0) {
    // (lower)^T is upper; its reversal is the lower form
    DArr<int32_t> t_rp, t_ci;
    DArr<double> t_va;
    HIPCHK(h, t_rp.alloc((size_t)n + 1));
    HIPCHK(h, t_ci.alloc((size_t)std::max(nnz, 1)));
    HIPCHK(h, t_va.alloc((size_t)std::max(nnz, 1)));
    STCHK(transpose_csr(h, n, nnz, lrp, lci, lva, t_rp.p, t_ci.p, t_va.p, s));
    HIPCHK(h, launch_rev_entries(n, nnz, t_rp.p, t_ci.p, t_va.p, h->rp.p, h->ci.p, h->va.p, s));
  } else {
    HIPCHK(h, hipMemsetAsync(h->rp.p, 0, sizeof(int32_t), s));
  }
  STCHK(build_plan(h, h->orig, n, nnz, h->rp.p, h->ci.p, h->va.p, nullptr, nullptr, nullptr, s, form_reversed(form)));
  if (nlevels_out) *nlevels_out = h->orig.nlev;
  return SPTRSV_OK;
}

}  // namespace

// Longest-path membership of the rows of the handle's lower matrix (row
// constraints of Sec. III.A): heights by a sweep over the plan's levels from
// the last to the first (launch_heights), then oncrit[r] = level(r) +
// height(r) == nlev - 1.
sptrsv_status_t crit_rows(sptrsv_ctx *h, const Plan &P, uint8_t *oncrit, hipStream_t s) {
  const int32_t n = P.n;
  if (n == 0) return SPTRSV_OK;
  DArr<int32_t> hp;
  HIPCHK(h, hp.alloc((size_t)n));
  HIPCHK(h, hipMemsetAsync(hp.p, 0, sizeof(int32_t) * (size_t)n, s));
  HIPCHK(h, launch_heights(n, P.nlev, P.level_ptr.p, P.h_level_ptr.data(), P.srp.p, P.sci.p, hp.p, s));
  HIPCHK(h, launch_crit_from_heights(n, P.nlev, P.perm.p, P.row_level.p, hp.p, oncrit, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return SPTRSV_OK;
}

extern "C" {

sptrsv_status_t sptrsv_analyze(sptrsv_handle_t h, int32_t n, int32_t nnz, const int32_t *d_row_ptr,
                               const int32_t *d_col, const double *d_val, hipStream_t s, int32_t *nlevels_out) {
  return analyze_form(h, SPTRSV_LOWER, n, nnz, d_row_ptr, d_col, d_val, s, nlevels_out);
}

sptrsv_status_t sptrsv_analyze_form(sptrsv_handle_t h, int32_t form, int32_t n, int32_t nnz, const int32_t *d_row_ptr,
                                    const int32_t *d_col, const double *d_val, hipStream_t s, int32_t *nlevels_out) {
  return analyze_form(h, form, n, nnz, d_row_ptr, d_col, d_val, s, nlevels_out);
}


sptrsv_status_t sptrsv_get_levels(sptrsv_handle_t h, int which, int32_t *d_level_ptr, int32_t *d_level_rows,
                                  int32_t *d_row_level, hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  Plan *P = plan_of(h, which);
  if (!P) return set_err(h, SPTRSV_ERR_ARG, "which=%d", which);
  if (!P->ready) return set_err(h, SPTRSV_ERR_STATE, "matrix not analysed");
  if (d_level_ptr)
    HIPCHK(h, hipMemcpyAsync(d_level_ptr, P->level_ptr.p, sizeof(int32_t) * ((size_t)P->nlev + 1),
                             hipMemcpyDeviceToDevice, s));
  if (P->n && d_level_rows)
    HIPCHK(h, hipMemcpyAsync(d_level_rows, P->perm.p, sizeof(int32_t) * (size_t)P->n, hipMemcpyDeviceToDevice, s));
  if (P->n && d_row_level)
    HIPCHK(h,
           hipMemcpyAsync(d_row_level, P->row_level.p, sizeof(int32_t) * (size_t)P->n, hipMemcpyDeviceToDevice, s));
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_level_stats(sptrsv_handle_t h, int which, int64_t *d_rows, int64_t *d_nnz, int64_t *d_cost,
                                   int64_t *h_total_cost, double *h_avg_level_cost, hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  Plan *P = plan_of(h, which);
  if (!P) return set_err(h, SPTRSV_ERR_ARG, "which=%d", which);
  if (!P->ready) return set_err(h, SPTRSV_ERR_STATE, "matrix not analysed");
  const size_t b = sizeof(int64_t) * (size_t)P->nlev;
  if (P->nlev && d_rows) HIPCHK(h, hipMemcpyAsync(d_rows, P->lv_rows.p, b, hipMemcpyDeviceToDevice, s));
  if (P->nlev && d_nnz) HIPCHK(h, hipMemcpyAsync(d_nnz, P->lv_nnz.p, b, hipMemcpyDeviceToDevice, s));
  if (P->nlev && d_cost) HIPCHK(h, hipMemcpyAsync(d_cost, P->lv_cost.p, b, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (h_total_cost) *h_total_cost = P->total_cost;
  if (h_avg_level_cost) *h_avg_level_cost = P->avg_cost;
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_prepare(sptrsv_handle_t h, int which, int32_t nrhs, hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  Plan *P = plan_of(h, which);
  if (!P) return set_err(h, SPTRSV_ERR_ARG, "which=%d", which);
  if (!P->ready) return set_err(h, SPTRSV_ERR_STATE, "matrix not analysed/rewritten");
  if (nrhs < 1) return set_err(h, SPTRSV_ERR_ARG, "nrhs=%d", nrhs);
  STCHK(ensure_work(h, *P, nrhs));
  const sptrsv_schedule_t sc = effective_sched(*P, nrhs);
  STCHK(make_runs(h, *P, nrhs, sc, s));
  STCHK(ensure_rows(h, *P, s));
  return SPTRSV_OK;
}

}  // extern "C"

// Arguments of a solve entry point: the plan they address, or an error.
Plan *solve_plan(sptrsv_ctx *h, int which, int32_t nrhs, const double *d_b, int64_t ldb, const double *d_x,
                 int64_t ldx, sptrsv_status_t *st) {
  *st = SPTRSV_OK;
  Plan *P = plan_of(h, which);
  if (!P) {
    *st = set_err(h, SPTRSV_ERR_ARG, "which=%d", which);
    return nullptr;
  }
  if (!P->ready) {
    *st = set_err(h, SPTRSV_ERR_STATE, which == SPTRSV_REWRITTEN ? "no rewrite yet" : "matrix not analysed");
    return nullptr;
  }
  const int64_t n = P->n;
  if (nrhs < 1 || ldb < n || ldx < n || (n > 0 && (!d_b || !d_x))) {
    *st = set_err(h, SPTRSV_ERR_ARG, "solve: nrhs=%d ldb=%lld ldx=%lld", nrhs, (long long)ldb, (long long)ldx);
    return nullptr;
  }
  if (n > 0) {
    const char *b0 = reinterpret_cast<const char *>(d_b);
    const char *b1 = b0 + sizeof(double) * (size_t)(ldb * (nrhs - 1) + n);
    const char *x0 = reinterpret_cast<const char *>(d_x);
    const char *x1 = x0 + sizeof(double) * (size_t)(ldx * (nrhs - 1) + n);
    if (b0 < x1 && x0 < b1) {
      *st = set_err(h, SPTRSV_ERR_ARG, "b and x overlap");
      return nullptr;
    }
  }
  return P;
}

extern "C" {

sptrsv_status_t sptrsv_solve(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, int64_t ldb,
                             double *d_x, int64_t ldx, hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  sptrsv_status_t st;
  Plan *P = solve_plan(h, which, nrhs, d_b, ldb, d_x, ldx, &st);
  if (!P) return st;
  return plan_solve(h, *P, nrhs, d_b, ldb, d_x, ldx, s);
}

sptrsv_status_t sptrsv_solve_rows(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, double *d_x,
                                  hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  const Plan *Q = plan_of(h, which);
  const int64_t n = Q ? Q->n : 0;
  sptrsv_status_t st;
  Plan *P = solve_plan(h, which, nrhs, d_b, n, d_x, n, &st);  // the same extent as n x nrhs column-major
  if (!P) return st;
  if (nrhs == 1) return plan_solve(h, *P, 1, d_b, n, d_x, n, s);  // one column: the same layout
  return solve_rows(h, *P, nrhs, d_b, d_x, s);
}

sptrsv_status_t sptrsv_check(sptrsv_handle_t h, hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  int32_t bits = 0;
  HIPCHK(h, hipMemcpyAsync(&bits, h->d_err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (bits) {
    HIPCHK(h, hipMemsetAsync(h->d_err.p, 0, sizeof(int32_t), s));
    HIPCHK(h, hipStreamSynchronize(s));
    return set_err(h, status_from_bits(bits), "device reported error bits 0x%x", bits);
  }
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_set_schedule(sptrsv_handle_t h, int which, const sptrsv_schedule_t *sched) {
  if (!h || !sched) return SPTRSV_ERR_ARG;
  Plan *P = sched_plan_of(h, which);
  if (!P) return set_err(h, SPTRSV_ERR_ARG, "which=%d", which);
  STCHK(check_sched(h, *sched));
  P->sched = *sched;
  P->tuned.clear();
  P->runs_nrhs = -1;
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_get_schedule(sptrsv_handle_t h, int which, int32_t nrhs, sptrsv_schedule_t *sched) {
  if (!h || !sched) return SPTRSV_ERR_ARG;
  Plan *P = sched_plan_of(h, which);
  if (!P) return set_err(h, SPTRSV_ERR_ARG, "which=%d", which);
  if (nrhs < 1) return set_err(h, SPTRSV_ERR_ARG, "nrhs=%d", nrhs);
  *sched = effective_sched(*P, nrhs);
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_profile(sptrsv_handle_t h, int enable, sptrsv_kernel_profile_t *out, hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  constexpr size_t kPairs = 16384;
  if (enable) {
    if (h->prof_ev.empty()) {
      h->prof_ev.resize(2 * kPairs);
      for (auto &e : h->prof_ev) HIPCHK(h, hipEventCreate(&e));
      h->prof_cls.assign(kPairs, 0);
      h->prof_bytes.assign(kPairs, 0.0);
    }
    h->prof_used = 0;
    h->prof = true;
    return SPTRSV_OK;
  }
  h->prof = false;
  HIPCHK(h, hipStreamSynchronize(s));
  sptrsv_kernel_profile_t acc[4] = {};
  for (size_t i = 0; i < h->prof_used / 2; ++i) {
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, h->prof_ev[2 * i], h->prof_ev[2 * i + 1]));
    const int c = h->prof_cls[i];
    acc[c].launches += 1;
    acc[c].ms += ms;
    acc[c].bytes += h->prof_bytes[i];
  }
  if (out)
    for (int c = 0; c < 4; ++c) out[c] = acc[c];
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_level_floor(sptrsv_handle_t h, int which, int32_t nrhs, int32_t flags,
                                   const sptrsv_level_costs_t *c, double *floor_us) {
  if (!h || !c || !floor_us) return SPTRSV_ERR_ARG;
  Plan *P = plan_of(h, which);
  if (!P) return set_err(h, SPTRSV_ERR_ARG, "which=%d", which);
  if (!P->ready) return set_err(h, SPTRSV_ERR_STATE, "matrix not analysed/rewritten");
  if (nrhs < 1) return set_err(h, SPTRSV_ERR_ARG, "nrhs=%d", nrhs);
  *floor_us = 0.0;
  if (P->n == 0) return SPTRSV_OK;
  if (!runs_ready(*P, nrhs)) STCHK(make_runs(h, *P, nrhs, effective_sched(*P, nrhs), nullptr));
  const sptrsv_schedule_t sc = P->runs_sched;
  if (flags & ~(SPTRSV_FLOOR_GRAPH | SPTRSV_FLOOR_ROWS)) return set_err(h, SPTRSV_ERR_ARG, "flags=%d", flags);
  const double launch = (flags & SPTRSV_FLOOR_GRAPH) ? c->graph_node_ns : c->launch_ns;
  // gather, b-transform, scatter; right-hand sides by rows read and written
  // through the level order skip the gather and the scatter where the runs
  // are thin runs and per-level wide launches
  const bool direct = (flags & SPTRSV_FLOOR_ROWS) && sc.mode != 3 && sc.mode != 4;
  double ns = launch * ((direct ? 0 : 2) + (P->has_t && P->n_tpos > 0 ? 1 : 0));
  if (sc.mode == 3) {
    ns += 2 * launch + (double)P->nlev * c->flag_hop_ns;  // fill of x, the solve; a hop per level
  } else {
    for (const Run &r : P->runs) {
      if (r.thin) {
        ns += launch;
        for (int32_t w = 0; w < r.nw; ++w) {
          const int4 W = P->h_win[(size_t)(r.wi + w)];
          const int32_t nl = P->h_win[(size_t)(r.wi + w + 1)].x - W.x;
          ns += (double)nl * ((W.y & 1) ? c->thin_wave_level_ns : c->thin_level_ns);
        }
      } else if (r.flow) {
        ns += launch + (double)(r.l1 - r.l0 - 1) * c->flag_hop_ns;
      } else if (sc.wide_grid > 0) {
        ns += launch + (double)(r.l1 - r.l0 - 1) * c->grid_barrier_ns;
      } else {
        ns += (double)(r.l1 - r.l0) * launch;
      }
    }
  }
  *floor_us = ns * 1e-3;
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_residual(sptrsv_handle_t h, int32_t nrhs, const double *d_b, int64_t ldb, const double *d_x,
                                int64_t ldx, double *h_out, hipStream_t s) {
  if (!h || !h_out) return SPTRSV_ERR_ARG;
  if (!h->orig.ready) return set_err(h, SPTRSV_ERR_STATE, "matrix not analysed");
  if (nrhs < 1 || nrhs > 56 || ldb < h->n || ldx < h->n) return set_err(h, SPTRSV_ERR_ARG, "residual args");
  unsigned long long *out = reinterpret_cast<unsigned long long *>(h->d_aux.p + 128);
  HIPCHK(h, hipMemsetAsync(out, 0, sizeof(unsigned long long) * (size_t)nrhs, s));
  HIPCHK(h, launch_residual(h->n, nrhs, h->rp.p, h->ci.p, h->va.p, d_b, ldb, d_x, ldx, out, h->orig.rev_io, s));
  std::vector<unsigned long long> hv((size_t)nrhs);
  HIPCHK(h, hipMemcpyAsync(hv.data(), out, sizeof(unsigned long long) * (size_t)nrhs, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  for (int c = 0; c < nrhs; ++c) std::memcpy(&h_out[c], &hv[(size_t)c], sizeof(double));
  return SPTRSV_OK;
}

}  // extern "C"
