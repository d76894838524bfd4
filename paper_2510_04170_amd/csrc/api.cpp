// C-ABI entry points of librfmnewton: problem description, layout building and
// the stage calls.  Every entry point catches rfm::Error and returns its status.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>

#include "rfm_internal.h"

namespace rfm {

static thread_local std::string g_last_error;

void set_last_error(const std::string& m) { g_last_error = m; }

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

void copy_in(Problem& P, double* dst, const double* src, size_t count) {
  if (count == 0) return;
  RFM_HIP(hipMemcpyAsync(dst, src, count * sizeof(double),
                         is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, P.stream));
}

void copy_out(Problem& P, double* dst, const double* src, size_t count) {
  if (count == 0) return;
  bool dev = is_device_ptr(dst);
  RFM_HIP(hipMemcpyAsync(dst, src, count * sizeof(double), dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         P.stream));
  if (!dev) RFM_HIP(hipStreamSynchronize(P.stream));
}

// host copy of a caller array that may live on the device
static std::vector<double> host_doubles(const double* src, size_t count) {
  std::vector<double> v(count);
  if (count == 0) return v;
  if (is_device_ptr(src))
    RFM_HIP(hipMemcpy(v.data(), src, count * sizeof(double), hipMemcpyDeviceToHost));
  else
    std::memcpy(v.data(), src, count * sizeof(double));
  return v;
}

Problem::~Problem() {}

int Profiler::slot_of(const char* name) {
  for (size_t i = 0; i < names.size(); ++i)
    if (names[i] == name) return (int)i;
  names.emplace_back(name);
  stats.emplace_back();
  return (int)names.size() - 1;
}

void Profiler::begin(hipStream_t s, hipEvent_t* a) {
  if (pool.empty()) {
    hipEvent_t e;
    RFM_HIP(hipEventCreate(&e));
    pool.push_back(e);
  }
  *a = pool.back();
  pool.pop_back();
  RFM_HIP(hipEventRecord(*a, s));
}

void Profiler::end(hipStream_t s, hipEvent_t a, const char* name, double flops, double bytes) {
  hipEvent_t b;
  if (pool.empty()) {
    RFM_HIP(hipEventCreate(&b));
  } else {
    b = pool.back();
    pool.pop_back();
  }
  RFM_HIP(hipEventRecord(b, s));
  pending.push_back(PendingEv{a, b, slot_of(name), flops, bytes});
  if (pending.size() >= 4096) resolve();
}

void Profiler::resolve() {
  for (auto& pe : pending) {
    RFM_HIP(hipEventSynchronize(pe.b));
    float ms = 0.f;
    RFM_HIP(hipEventElapsedTime(&ms, pe.a, pe.b));
    KStat& k = stats[pe.slot];
    k.launches += 1;
    k.seconds += 1e-3 * ms;
    k.flops += pe.flops;
    k.bytes += pe.bytes;
    pool.push_back(pe.a);
    pool.push_back(pe.b);
  }
  pending.clear();
}

Profiler::~Profiler() {
  for (auto& pe : pending) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

static void set_device(Problem& P) { RFM_HIP(hipSetDevice(P.device)); }

static bool all_finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

// box geometry: identical arithmetic to the description (lo + i h, + h)
static void box_centre_halfwidth(const GeomDesc& g, int e, double* mu, double* sig) {
  int rem = e;
  for (int a = 0; a < g.dim; ++a) {
    int i = rem % g.nsub[a];
    rem /= g.nsub[a];
    double h = (g.hi[a] - g.lo[a]) / g.nsub[a];
    double blo = g.lo[a] + i * h;
    double bhi = blo + h;
    mu[a] = 0.5 * (blo + bhi);
    sig[a] = 0.5 * (bhi - blo);
  }
}

const OpDesc* device_op(Problem& P) {
  if (!P.have_d_op || std::memcmp(&P.op, &P.op_on_device, sizeof(OpDesc)) != 0) {
    P.d_op.resize(1);
    RFM_HIP(hipStreamSynchronize(P.stream));  // no kernel still reads the old copy
    RFM_HIP(hipMemcpy(P.d_op.p, &P.op, sizeof(OpDesc), hipMemcpyHostToDevice));
    std::memcpy(&P.op_on_device, &P.op, sizeof(OpDesc));  // bytes, padding included, for the memcmp
    P.have_d_op = true;
  }
  return P.d_op.p;
}

// a derivative selector RFM_D_* valid for the problem's dimension
static bool deriv_ok(const Problem& P, int d) {
  return d == RFM_D_ID || (d >= RFM_D_X0 && d < RFM_D_X0 + P.dim) || d == RFM_D_LAPLACE ||
         (d == RFM_D_LAPLACE_SPACE && P.dim >= 2);
}

static int row_width_of_group(const Problem& P, const GroupH& g) {
  if (g.kind == RFM_PDE) return P.ncomp * P.J;
  if (g.kind == RFM_CONTINUITY) return 2 * P.J;
  return P.J;
}

// Build rows, tiles and the column-block contribution lists, then upload.
static void finalize(Problem& P) {
  if (P.finalized) return;
  RFM_CHECK(P.have_partition, RFM_EINVAL, "rfm_finalize: partition not set");
  RFM_CHECK(P.have_features, RFM_EINVAL, "rfm_finalize: features not set");
  RFM_CHECK(P.have_operator, RFM_EINVAL, "rfm_finalize: operator not set");
  RFM_CHECK(!P.groups.empty(), RFM_EINVAL, "rfm_finalize: no points");
  const int K = P.ncomp, J = P.J;
  const bool smooth = P.geom.pou == RFM_POU_SMOOTH;
  for (const auto& g : P.groups) {
    RFM_CHECK(!(smooth && g.kind == RFM_CONTINUITY), RFM_EINVAL,
              "rfm_finalize: no continuity rows with the smooth partition of unity");
    const int segs = smooth ? (1 << P.dim) : 1;
    RFM_CHECK((int64_t)row_width_of_group(P, g) * segs <= kMaxRowWidth, RFM_EINVAL, "row wider than 16384 values");
  }

  // rows
  std::vector<RowDesc> rows;
  rows.reserve(P.m);
  for (auto& g : P.groups) {
    g.row0 = (int64_t)rows.size();
    int nsel = g.comp < 0 ? K : 1;
    int nord = g.kind == RFM_CONTINUITY ? g.cont_order : 1;
    for (int k = 0; k < nsel; ++k) {
      int sel = g.comp < 0 ? k : g.comp;
      for (int s = 0; s < nord; ++s)
        for (int64_t p = 0; p < g.npts; ++p) {
          RowDesc r;
          r.pt = (int32_t)(g.pt0 + p);
          r.owner = g.owner;
          r.neighbor = g.neighbor;
          r.kind = (uint8_t)g.kind;
          r.sel = (uint8_t)sel;
          r.order = (uint8_t)s;
          r.pad = 0;
          rows.push_back(r);
        }
    }
    g.nrows = (int64_t)rows.size() - g.row0;
  }
  P.m = (int64_t)rows.size();
  RFM_CHECK(P.m > 0 && P.m < (int64_t)INT32_MAX, RFM_EINVAL, "row count out of range");
  RFM_CHECK((int64_t)P.rowdata.size() == P.m, RFM_EINVAL, "internal: row data size");

  // tiles: runs of rows with the same support, at most kTileRows rows
  P.tiles_h.clear();
  int64_t voff = 0, poff = 0;
  auto add_run = [&](int64_t r0, int64_t nr, int colA, int wA, int colB, int wB) {
    for (int64_t t0 = 0; t0 < nr; t0 += kTileRows) {
      TileDesc t{};
      t.row0 = (int32_t)(r0 + t0);
      t.nrows = (int32_t)std::min<int64_t>(kTileRows, nr - t0);
      t.colA = colA;
      t.wA = wA;
      t.colB = colB;
      t.wB = wB;
      t.val_off = voff;
      t.part_off = poff;
      t.nseg = wB ? 2 : 1;
      t.wseg = wA;
      t.seg_col[0] = colA;
      t.seg_col[1] = colB;
      voff += (int64_t)t.nrows * (wA + wB);
      poff += wA + wB;
      P.tiles_h.push_back(t);
    }
  };
  // smooth partition: a run of rows whose points lie in the supports of the same boxes; segment s holds
  // the columns (box boxes[s], component c0 .. c0 + wseg / J - 1)
  auto add_run_smooth = [&](int64_t r0, int64_t nr, const std::vector<int>& boxes, int c0, int wseg) {
    for (int64_t t0 = 0; t0 < nr; t0 += kTileRows) {
      TileDesc t{};
      t.row0 = (int32_t)(r0 + t0);
      t.nrows = (int32_t)std::min<int64_t>(kTileRows, nr - t0);
      t.nseg = (int32_t)boxes.size();
      t.wseg = wseg;
      for (int k = 0; k < t.nseg; ++k) t.seg_col[k] = (boxes[k] * K + c0) * J;
      t.colA = t.seg_col[0];
      t.wA = t.nseg * wseg;
      t.colB = 0;
      t.wB = 0;
      t.val_off = voff;
      t.part_off = poff;
      voff += (int64_t)t.nrows * t.wA;
      poff += t.wA;
      P.tiles_h.push_back(t);
    }
  };
  // the boxes whose smooth partition function is non-zero at point pt, ascending (|l_a(x)| < 5/4 on every
  // axis among the owner's neighbours; points lie in the domain, where a flat side reaches no further)
  auto cover = [&](int64_t pt, int owner) {
    std::vector<int> out;
    int idx[kMaxDim], rem = owner;
    for (int a = 0; a < P.dim; ++a) {
      idx[a] = rem % P.geom.nsub[a];
      rem /= P.geom.nsub[a];
    }
    int ncand = 1;
    for (int a = 0; a < P.dim; ++a) ncand *= 3;
    for (int k = 0; k < ncand; ++k) {
      int kk = k, e = 0, stride = 1;
      bool ok = true;
      for (int a = 0; a < P.dim && ok; ++a) {
        const int ia = idx[a] + kk % 3 - 1;
        kk /= 3;
        if (ia < 0 || ia >= P.geom.nsub[a]) {
          ok = false;
          break;
        }
        const double h = (P.geom.hi[a] - P.geom.lo[a]) / P.geom.nsub[a];
        const double mu = P.geom.lo[a] + (ia + 0.5) * h, sig = 0.5 * h;
        const double y = (P.px[(size_t)pt * P.dim + a] - mu) / sig;
        if (!(std::fabs(y) < 1.25)) ok = false;
        e += ia * stride;
        stride *= P.geom.nsub[a];
      }
      if (ok) out.push_back(e);
    }
    std::sort(out.begin(), out.end());
    return out;
  };
  if (smooth) {
    for (const auto& g : P.groups) {
      if (g.npts == 0) continue;
      const int nsel = g.comp < 0 ? K : 1;
      const bool pde = g.kind == RFM_PDE;  // PDE rows touch all components of their boxes
      for (int k = 0; k < nsel; ++k) {
        const int c = g.comp < 0 ? k : g.comp;
        const int64_t rbase = g.row0 + (int64_t)k * g.npts;
        int64_t p0 = 0;
        std::vector<int> cur = cover(g.pt0, g.owner);
        for (int64_t p = 1; p <= g.npts; ++p) {
          std::vector<int> nxt;
          if (p < g.npts) nxt = cover(g.pt0 + p, g.owner);
          if (p == g.npts || nxt != cur) {
            RFM_CHECK(!cur.empty() && (int)cur.size() <= kMaxSeg, RFM_EINVAL, "internal: partition cover");
            add_run_smooth(rbase + p0, p - p0, cur, pde ? 0 : c, pde ? K * J : J);
            p0 = p;
            cur.swap(nxt);
          }
        }
      }
    }
  }
  for (const auto& g : P.groups) {
    if (g.npts == 0 || smooth) continue;
    int nsel = g.comp < 0 ? K : 1;
    if (g.kind == RFM_PDE) {
      add_run(g.row0, g.nrows, g.owner * K * J, K * J, 0, 0);
    } else if (g.kind == RFM_CONTINUITY) {
      for (int k = 0; k < nsel; ++k) {
        int c = g.comp < 0 ? k : g.comp;
        add_run(g.row0 + (int64_t)k * g.cont_order * g.npts, (int64_t)g.cont_order * g.npts,
                (g.owner * K + c) * J, J, (g.neighbor * K + c) * J, J);
      }
    } else {
      for (int k = 0; k < nsel; ++k) {
        int c = g.comp < 0 ? k : g.comp;
        add_run(g.row0 + (int64_t)k * g.npts, g.npts, (g.owner * K + c) * J, J, 0, 0);
      }
    }
  }
  P.ntiles = (int)P.tiles_h.size();
  P.max_tile_w = 0;
  for (const auto& t : P.tiles_h) P.max_tile_w = std::max(P.max_tile_w, t.wA + t.wB);
  P.nvals = voff;
  P.npart = poff;

  // column blocks (e, c) of J columns each: contributing (tile, offset) in tile order
  const int nblk = P.geom.nbox * K;
  std::vector<std::vector<std::pair<int, int>>> contrib(nblk);
  for (int t = 0; t < P.ntiles; ++t) {
    const TileDesc& td = P.tiles_h[t];
    for (int sg = 0; sg < td.nseg; ++sg)
      for (int o = 0; o < td.wseg; o += J) contrib[(td.seg_col[sg] + o) / J].push_back({t, sg * td.wseg + o});
  }
  P.cb_ptr_h.assign(nblk + 1, 0);
  P.cb_tile_h.clear();
  P.cb_off_h.clear();
  for (int bk = 0; bk < nblk; ++bk) {
    for (auto& pr : contrib[bk]) {
      P.cb_tile_h.push_back(pr.first);
      P.cb_off_h.push_back(pr.second);
    }
    P.cb_ptr_h[bk + 1] = (int32_t)P.cb_tile_h.size();
  }
  // FP64 sketch: for each column block the rows touching it (tile order, which is ascending row order)
  // with the d_J offset of each row's segment in the block
  P.sk_ptr_h.assign(nblk + 1, 0);
  P.sk_row_h.clear();
  P.sk_off_h.clear();
  for (int bk = 0; bk < nblk; ++bk) {
    for (auto& pr : contrib[bk]) {
      const TileDesc& td = P.tiles_h[pr.first];
      const int w = td.wA + td.wB;
      for (int rr = 0; rr < td.nrows; ++rr) {
        P.sk_row_h.push_back(td.row0 + rr);
        P.sk_off_h.push_back(td.val_off + (int64_t)rr * w + pr.second);
      }
    }
    P.sk_ptr_h[bk + 1] = (int64_t)P.sk_row_h.size();
  }
  // low-precision sketch operand: for each column block the 32-row groups (rows 32 g .. 32 g + 31) that hold a
  // row touching it, ascending, padded with empty groups to a multiple of 4; per slot the d_J offset of each row's
  // segment in the block (-1 where the row does not touch it)
  P.cbs_ptr_h.assign(nblk + 1, 0);
  P.slot_group_h.clear();
  std::vector<int64_t>& slot_rowoff = P.slot_rowoff_h;
  slot_rowoff.clear();
  for (int bk = 0; bk < nblk; ++bk) {
    std::map<int64_t, std::array<int64_t, 32>> grp;
    for (auto& pr : contrib[bk]) {
      const TileDesc& td = P.tiles_h[pr.first];
      const int w = td.wA + td.wB;
      for (int r = 0; r < td.nrows; ++r) {
        const int64_t gr = (int64_t)td.row0 + r;
        auto it = grp.find(gr / 32);
        if (it == grp.end()) {
          std::array<int64_t, 32> a;
          a.fill(-1);
          it = grp.emplace(gr / 32, a).first;
        }
        it->second[gr % 32] = td.val_off + (int64_t)r * w + pr.second;
      }
    }
    for (auto& kv : grp) {
      P.slot_group_h.push_back((int32_t)kv.first);
      slot_rowoff.insert(slot_rowoff.end(), kv.second.begin(), kv.second.end());
    }
    while ((P.slot_group_h.size() - (size_t)P.cbs_ptr_h[bk]) % 4) {
      P.slot_group_h.push_back(-1);
      slot_rowoff.insert(slot_rowoff.end(), 32, (int64_t)-1);
    }
    P.cbs_ptr_h[bk + 1] = (int32_t)P.slot_group_h.size();
  }
  P.nslots = (int64_t)P.slot_group_h.size();

  std::vector<int32_t> rowtile(P.m);
  for (int t = 0; t < P.ntiles; ++t)
    for (int r = 0; r < P.tiles_h[t].nrows; ++r) rowtile[P.tiles_h[t].row0 + r] = t;

  // feature table
  const int dim = P.dim;
  const int64_t nf = (int64_t)P.geom.nbox * K * J;
  std::vector<double> ft((size_t)(2 * dim + 3) * nf);
  for (int e = 0; e < P.geom.nbox; ++e) {
    double mu[kMaxDim], sig[kMaxDim];
    box_centre_halfwidth(P.geom, e, mu, sig);
    for (int c = 0; c < K; ++c)
      for (int j = 0; j < J; ++j) {
        int64_t f = ((int64_t)e * K + c) * J + j;
        double s2 = 0, s2s = 0;
        for (int a = 0; a < dim; ++a) {
          double w = P.W[(size_t)f * dim + a];
          double ws = w / sig[a];
          ft[(size_t)a * nf + f] = w;
          ft[(size_t)(dim + a) * nf + f] = ws;
          s2 += ws * ws;
          if (a < dim - 1) s2s += ws * ws;
        }
        ft[(size_t)(2 * dim) * nf + f] = P.b[f];
        ft[(size_t)(2 * dim + 1) * nf + f] = s2;
        ft[(size_t)(2 * dim + 2) * nf + f] = s2s;
      }
  }

  // upload
  P.d_px.resize(P.px.size());
  RFM_HIP(hipMemcpy(P.d_px.p, P.px.data(), P.px.size() * sizeof(double), hipMemcpyHostToDevice));
  P.d_pnormal.resize(P.pnormal.size());
  RFM_HIP(hipMemcpy(P.d_pnormal.p, P.pnormal.data(), P.pnormal.size() * sizeof(double), hipMemcpyHostToDevice));
  P.d_rowdata.resize(P.m);
  RFM_HIP(hipMemcpy(P.d_rowdata.p, P.rowdata.data(), P.m * sizeof(double), hipMemcpyHostToDevice));
  P.d_feat.resize(ft.size());
  RFM_HIP(hipMemcpy(P.d_feat.p, ft.data(), ft.size() * sizeof(double), hipMemcpyHostToDevice));
  for (int a = 0; a < kMaxDim; ++a) {
    P.feat.W[a] = a < dim ? P.d_feat.p + (size_t)a * nf : nullptr;
    P.feat.WS[a] = a < dim ? P.d_feat.p + (size_t)(dim + a) * nf : nullptr;
  }
  P.feat.b = P.d_feat.p + (size_t)(2 * dim) * nf;
  P.feat.S2 = P.d_feat.p + (size_t)(2 * dim + 1) * nf;
  P.feat.S2s = P.d_feat.p + (size_t)(2 * dim + 2) * nf;
  P.d_rows.resize(P.m);
  RFM_HIP(hipMemcpy(P.d_rows.p, rows.data(), P.m * sizeof(RowDesc), hipMemcpyHostToDevice));
  P.d_tiles.resize(P.ntiles);
  RFM_HIP(hipMemcpy(P.d_tiles.p, P.tiles_h.data(), P.ntiles * sizeof(TileDesc), hipMemcpyHostToDevice));
  P.d_cbs_ptr.resize(P.cbs_ptr_h.size());
  RFM_HIP(hipMemcpy(P.d_cbs_ptr.p, P.cbs_ptr_h.data(), P.cbs_ptr_h.size() * 4, hipMemcpyHostToDevice));
  P.d_slot_group.resize(std::max<int64_t>(1, P.nslots));
  P.d_slot_rowoff.resize(std::max<int64_t>(32, 32 * P.nslots));
  if (P.nslots) {
    RFM_HIP(hipMemcpy(P.d_slot_group.p, P.slot_group_h.data(), P.nslots * 4, hipMemcpyHostToDevice));
    RFM_HIP(hipMemcpy(P.d_slot_rowoff.p, slot_rowoff.data(), slot_rowoff.size() * 8, hipMemcpyHostToDevice));
  }
  P.d_cb_ptr.resize(P.cb_ptr_h.size());
  RFM_HIP(hipMemcpy(P.d_cb_ptr.p, P.cb_ptr_h.data(), P.cb_ptr_h.size() * 4, hipMemcpyHostToDevice));
  P.d_cb_tile.resize(std::max<size_t>(1, P.cb_tile_h.size()));
  P.d_cb_off.resize(std::max<size_t>(1, P.cb_off_h.size()));
  if (!P.cb_tile_h.empty()) {
    RFM_HIP(hipMemcpy(P.d_cb_tile.p, P.cb_tile_h.data(), P.cb_tile_h.size() * 4, hipMemcpyHostToDevice));
    RFM_HIP(hipMemcpy(P.d_cb_off.p, P.cb_off_h.data(), P.cb_off_h.size() * 4, hipMemcpyHostToDevice));
  }
  P.d_rowtile.resize(P.m);
  RFM_HIP(hipMemcpy(P.d_rowtile.p, rowtile.data(), P.m * 4, hipMemcpyHostToDevice));
  P.d_sk_ptr.resize(P.sk_ptr_h.size());
  RFM_HIP(hipMemcpy(P.d_sk_ptr.p, P.sk_ptr_h.data(), P.sk_ptr_h.size() * 8, hipMemcpyHostToDevice));
  P.d_sk_row.resize(std::max<size_t>(1, P.sk_row_h.size()));
  P.d_sk_off.resize(std::max<size_t>(1, P.sk_off_h.size()));
  if (!P.sk_row_h.empty()) {
    RFM_HIP(hipMemcpy(P.d_sk_row.p, P.sk_row_h.data(), P.sk_row_h.size() * 4, hipMemcpyHostToDevice));
    RFM_HIP(hipMemcpy(P.d_sk_off.p, P.sk_off_h.data(), P.sk_off_h.size() * 8, hipMemcpyHostToDevice));
  }

  // working storage sized by m and n
  P.d_J.resize(P.nvals);
  P.d_DF.resize(P.m);
  P.d_D.resize(P.m);
  P.d_part.resize(std::max<int64_t>(1, P.npart));
  P.d_u.resize(P.n);
  P.d_du.resize(P.n);
  P.d_vec.resize(6 * std::max(P.m, P.n));
  P.d_red.resize(65536);
  P.d_scal.resize(64);
  P.d_lsab.resize((size_t)P.m * (2 + 2 * K + 2 * kMaxQ));
  P.d_lsqr.resize(1);
  P.d_sync.resize(1 << 16);
  RFM_HIP(hipMemset(P.d_sync.p, 0, P.d_sync.n * sizeof(int32_t)));
  RFM_HIP(hipDeviceSynchronize());
  P.finalized = true;
}

static Problem& get(rfm_problem* p) {
  RFM_CHECK(p != nullptr, RFM_EINVAL, "null problem");
  Problem& P = *reinterpret_cast<Problem*>(p);
  set_device(P);
  return P;
}

static Problem& ready(rfm_problem* p) {
  Problem& P = get(p);
  finalize(P);
  return P;
}

}  // namespace rfm

using namespace rfm;

extern "C" {

const char* rfm_last_error(void) { return g_last_error.c_str(); }

rfm_status rfm_create(rfm_problem** out, int32_t dim, int32_t ncomp, int32_t device, void* hip_stream) {
  return guarded([&] {
    RFM_CHECK(out != nullptr, RFM_EINVAL, "rfm_create: out is NULL");
    *out = nullptr;
    RFM_CHECK(dim >= 1 && dim <= kMaxDim, RFM_EINVAL, "rfm_create: dim must be 1..4");
    RFM_CHECK(ncomp >= 1 && ncomp <= kMaxComp, RFM_EINVAL, "rfm_create: ncomp must be 1..4");
    int ndev = 0;
    RFM_HIP(hipGetDeviceCount(&ndev));
    RFM_CHECK(device >= 0 && device < ndev, RFM_EINVAL, "rfm_create: no such device");
    RFM_HIP(hipSetDevice(device));
    (void)noalloc_scratch(device);  // device address of the fixed scratch of rfm_jtmul_noalloc, once per device
    auto* P = new Problem();
    P->dim = dim;
    P->ncomp = ncomp;
    P->device = device;
    P->stream = reinterpret_cast<hipStream_t>(hip_stream);
    P->geom.dim = dim;
    P->geom.ncomp = ncomp;
    *out = reinterpret_cast<rfm_problem*>(P);
  });
}

void rfm_destroy(rfm_problem* p) {
  if (!p) return;
  Problem* P = reinterpret_cast<Problem*>(p);
  (void)hipSetDevice(P->device);
  (void)hipStreamSynchronize(P->stream);
  if (P->proj) rfm_destroy(P->proj);
  delete P;
}

rfm_status rfm_set_partition(rfm_problem* p, const double* lo, const double* hi, const int32_t* nsub) {
  return guarded([&] {
    Problem& P = get(p);
    RFM_CHECK(!P.finalized, RFM_EINVAL, "rfm_set_partition: problem already finalized");
    RFM_CHECK(lo && hi && nsub, RFM_EINVAL, "rfm_set_partition: NULL argument");
    int64_t nbox = 1;
    for (int a = 0; a < P.dim; ++a) {
      RFM_CHECK(std::isfinite(lo[a]) && std::isfinite(hi[a]) && hi[a] > lo[a], RFM_EINVAL,
                "rfm_set_partition: need finite lo < hi");
      RFM_CHECK(nsub[a] >= 1, RFM_EINVAL, "rfm_set_partition: nsub must be >= 1");
      P.geom.lo[a] = lo[a];
      P.geom.hi[a] = hi[a];
      P.geom.nsub[a] = nsub[a];
      nbox *= nsub[a];
    }
    RFM_CHECK(nbox < (1 << 24), RFM_EINVAL, "rfm_set_partition: too many boxes");
    P.geom.nbox = (int)nbox;
    P.have_partition = true;
  });
}

rfm_status rfm_set_partition_of_unity(rfm_problem* p, int32_t kind) {
  return guarded([&] {
    Problem& P = get(p);
    RFM_CHECK(!P.finalized, RFM_EINVAL, "rfm_set_partition_of_unity: problem already finalized");
    RFM_CHECK(kind == RFM_POU_INDICATOR || kind == RFM_POU_SMOOTH, RFM_EINVAL,
              "rfm_set_partition_of_unity: unknown kind");
    P.geom.pou = kind;
  });
}

rfm_status rfm_set_features(rfm_problem* p, int32_t J, const double* W, const double* b) {
  return guarded([&] {
    Problem& P = get(p);
    RFM_CHECK(!P.finalized, RFM_EINVAL, "rfm_set_features: problem already finalized");
    RFM_CHECK(P.have_partition, RFM_EINVAL, "rfm_set_features: set the partition first");
    RFM_CHECK(J >= 1 && J <= 8192, RFM_EINVAL, "rfm_set_features: J must be 1..8192");
    RFM_CHECK((int64_t)P.ncomp * J <= kMaxRowWidth, RFM_EINVAL, "rfm_set_features: ncomp*J exceeds 16384");
    RFM_CHECK(W && b, RFM_EINVAL, "rfm_set_features: NULL argument");
    const size_t nf = (size_t)P.geom.nbox * P.ncomp * J;
    RFM_CHECK(nf < (size_t)INT32_MAX, RFM_EINVAL, "rfm_set_features: nbox*ncomp*J out of range");
    P.W = host_doubles(W, nf * P.dim);
    P.b = host_doubles(b, nf);
    RFM_CHECK(all_finite(P.W) && all_finite(P.b), RFM_ENUMERIC, "rfm_set_features: non-finite weights");
    P.J = J;
    P.geom.J = J;
    P.n = (int64_t)nf;
    P.have_features = true;
  });
}

rfm_status rfm_add_points(rfm_problem* p, int32_t kind, int64_t npts, const double* x, int32_t owner,
                          int32_t neighbor, const double* normal, int32_t comp, int32_t cont_order,
                          const double* data) {
  return guarded([&] {
    Problem& P = get(p);
    RFM_CHECK(!P.finalized, RFM_EINVAL, "rfm_add_points: problem already finalized");
    RFM_CHECK(P.have_partition, RFM_EINVAL, "rfm_add_points: set the partition first");
    RFM_CHECK(kind >= RFM_PDE && kind <= RFM_CONTINUITY, RFM_EINVAL, "rfm_add_points: bad kind");
    RFM_CHECK(npts >= 0, RFM_EINVAL, "rfm_add_points: npts < 0");
    RFM_CHECK(owner >= 0 && owner < P.geom.nbox, RFM_EINVAL, "rfm_add_points: owner out of range");
    RFM_CHECK(comp >= -1 && comp < P.ncomp, RFM_EINVAL, "rfm_add_points: comp out of range");
    if (kind == RFM_CONTINUITY) {
      RFM_CHECK(neighbor >= 0 && neighbor < P.geom.nbox && neighbor != owner, RFM_EINVAL,
                "rfm_add_points: continuity needs a different neighbour box");
      RFM_CHECK(cont_order == 1 || cont_order == 2, RFM_EINVAL, "rfm_add_points: cont_order must be 1 or 2");
      RFM_CHECK(data == nullptr, RFM_EINVAL, "rfm_add_points: continuity rows take no data");
    } else {
      RFM_CHECK(data != nullptr || npts == 0, RFM_EINVAL, "rfm_add_points: data required");
    }
    if (kind == RFM_NEUMANN || kind == RFM_CONTINUITY)
      RFM_CHECK(normal != nullptr || npts == 0, RFM_EINVAL, "rfm_add_points: normal required");
    if (npts == 0) return;
    RFM_CHECK(x != nullptr, RFM_EINVAL, "rfm_add_points: x is NULL");
    RFM_CHECK(P.npts + npts < (int64_t)INT32_MAX, RFM_EINVAL, "rfm_add_points: too many points");
    const int dim = P.dim;
    std::vector<double> xh = host_doubles(x, (size_t)npts * dim);
    RFM_CHECK(all_finite(xh), RFM_ENUMERIC, "rfm_add_points: non-finite coordinates");
    std::vector<double> nh((size_t)npts * dim, 0.0);
    if (normal) {
      nh = host_doubles(normal, (size_t)npts * dim);
      RFM_CHECK(all_finite(nh), RFM_ENUMERIC, "rfm_add_points: non-finite normals");
    }
    const int nsel = comp < 0 ? P.ncomp : 1;
    std::vector<double> dh;
    if (data) {
      dh = host_doubles(data, (size_t)npts * nsel);
      RFM_CHECK(all_finite(dh), RFM_ENUMERIC, "rfm_add_points: non-finite data");
    }
    GroupH g;
    g.kind = kind;
    g.owner = owner;
    g.neighbor = kind == RFM_CONTINUITY ? neighbor : -1;
    g.comp = comp;
    g.cont_order = kind == RFM_CONTINUITY ? cont_order : 1;
    g.pt0 = P.npts;
    g.npts = npts;
    g.row0 = 0;
    g.nrows = 0;
    P.px.insert(P.px.end(), xh.begin(), xh.end());
    P.pnormal.insert(P.pnormal.end(), nh.begin(), nh.end());
    P.npts += npts;
    // data per row in row order (selection, order, point)
    int nord = g.cont_order;
    for (int k = 0; k < nsel; ++k)
      for (int s = 0; s < nord; ++s)
        for (int64_t q = 0; q < npts; ++q) P.rowdata.push_back(data ? dh[(size_t)q * nsel + k] : 0.0);
    P.groups.push_back(g);
  });
}

rfm_status rfm_set_operator(rfm_problem* p, const rfm_lin_term* lin, int32_t nlin, const rfm_poly_term* nl,
                            int32_t nnl) {
  return guarded([&] {
    Problem& P = get(p);
    RFM_CHECK(nlin >= 0 && nlin <= kMaxLin && nnl >= 0 && nnl <= kMaxPoly, RFM_EINVAL,
              "rfm_set_operator: at most 16 linear and 8 polynomial terms");
    RFM_CHECK((nlin == 0 || lin) && (nnl == 0 || nl), RFM_EINVAL, "rfm_set_operator: NULL terms");
    OpDesc op = P.op;  // keeps the pointwise terms
    op.nlin = 0;
    op.npoly = 0;
    op.nlin = nlin;
    for (int i = 0; i < nlin; ++i) {
      const auto& t = lin[i];
      RFM_CHECK(t.eq >= 0 && t.eq < P.ncomp && t.comp >= 0 && t.comp < P.ncomp, RFM_EINVAL,
                "rfm_set_operator: term index out of range");
      RFM_CHECK(deriv_ok(P, t.deriv), RFM_EINVAL, "rfm_set_operator: bad derivative selector");
      RFM_CHECK(std::isfinite(t.coeff), RFM_ENUMERIC, "rfm_set_operator: non-finite coefficient");
      op.lin_eq[i] = t.eq;
      op.lin_comp[i] = t.comp;
      op.lin_deriv[i] = t.deriv;
      op.lin_coeff[i] = t.coeff;
    }
    op.npoly = nnl;
    for (int i = 0; i < nnl; ++i) {
      const auto& t = nl[i];
      RFM_CHECK(t.eq >= 0 && t.eq < P.ncomp, RFM_EINVAL, "rfm_set_operator: term index out of range");
      RFM_CHECK(std::isfinite(t.coeff), RFM_ENUMERIC, "rfm_set_operator: non-finite coefficient");
      op.poly_eq[i] = t.eq;
      op.poly_coeff[i] = t.coeff;
      for (int c = 0; c < kMaxComp; ++c) {
        int pw = c < P.ncomp ? t.pow[c] : 0;
        RFM_CHECK(pw >= 0 && pw <= 8, RFM_EINVAL, "rfm_set_operator: powers must be 0..8");
        op.poly_pow[i][c] = pw;
      }
    }
    P.op = op;
    P.have_operator = true;
  });
}

rfm_status rfm_set_fn_terms(rfm_problem* p, const rfm_fn_term* terms, int32_t n) {
  return guarded([&] {
    Problem& P = get(p);
    RFM_CHECK(n >= 0 && n <= kMaxFn, RFM_EINVAL, "rfm_set_fn_terms: at most 8 terms");
    RFM_CHECK(n == 0 || terms, RFM_EINVAL, "rfm_set_fn_terms: NULL terms");
    OpDesc op = P.op;
    op.nfn = n;
    for (int i = 0; i < n; ++i) {
      const auto& t = terms[i];
      RFM_CHECK(t.eq >= 0 && t.eq < P.ncomp && t.comp >= 0 && t.comp < P.ncomp, RFM_EINVAL,
                "rfm_set_fn_terms: term index out of range");
      RFM_CHECK(t.fn == RFM_FN_COSH || t.fn == RFM_FN_SINH || t.fn == RFM_FN_EXP, RFM_EINVAL,
                "rfm_set_fn_terms: unknown function");
      RFM_CHECK(std::isfinite(t.coeff), RFM_ENUMERIC, "rfm_set_fn_terms: non-finite coefficient");
      op.fn_eq[i] = t.eq;
      op.fn_comp[i] = t.comp;
      op.fn_kind[i] = t.fn;
      op.fn_coeff[i] = t.coeff;
    }
    P.op = op;
  });
}

rfm_status rfm_set_prod_terms(rfm_problem* p, const rfm_prod_term* terms, int32_t n) {
  return guarded([&] {
    Problem& P = get(p);
    RFM_CHECK(n >= 0 && n <= kMaxProd, RFM_EINVAL, "rfm_set_prod_terms: at most 8 terms");
    RFM_CHECK(n == 0 || terms, RFM_EINVAL, "rfm_set_prod_terms: NULL terms");
    OpDesc op = P.op;
    op.nprod = n;
    op.nq = 0;
    for (int i = 0; i < n; ++i) {
      const auto& t = terms[i];
      RFM_CHECK(t.eq >= 0 && t.eq < P.ncomp, RFM_EINVAL, "rfm_set_prod_terms: equation out of range");
      RFM_CHECK(t.nfac >= 1 && t.nfac <= kMaxFac, RFM_EINVAL, "rfm_set_prod_terms: 1..4 factors per term");
      RFM_CHECK(std::isfinite(t.coeff), RFM_ENUMERIC, "rfm_set_prod_terms: non-finite coefficient");
      op.prod_eq[i] = t.eq;
      op.prod_nfac[i] = t.nfac;
      op.prod_coeff[i] = t.coeff;
      for (int k = 0; k < kMaxFac; ++k) {
        op.prod_q[i][k] = 0;
        op.prod_pow[i][k] = 0;
      }
      for (int k = 0; k < t.nfac; ++k) {
        const rfm_factor& f = t.fac[k];
        RFM_CHECK(f.comp >= 0 && f.comp < P.ncomp, RFM_EINVAL, "rfm_set_prod_terms: component out of range");
        RFM_CHECK(deriv_ok(P, f.deriv), RFM_EINVAL, "rfm_set_prod_terms: bad derivative selector");
        RFM_CHECK(f.pow >= 1 && f.pow <= 8, RFM_EINVAL, "rfm_set_prod_terms: powers 1..8");
        int q = 0;
        while (q < op.nq && !(op.q_comp[q] == f.comp && op.q_deriv[q] == f.deriv)) ++q;
        if (q == op.nq) {
          RFM_CHECK(op.nq < kMaxQ, RFM_EINVAL, "rfm_set_prod_terms: more than 8 distinct field derivatives");
          op.q_comp[q] = f.comp;
          op.q_deriv[q] = f.deriv;
          ++op.nq;
        }
        op.prod_q[i][k] = q;
        op.prod_pow[i][k] = f.pow;
      }
    }
    P.op = op;
  });
}

rfm_status rfm_set_group_data(rfm_problem* p, int32_t group, const double* data) {
  return guarded([&] {
    Problem& P = get(p);
    RFM_CHECK(group >= 0 && group < (int32_t)P.groups.size(), RFM_EINVAL, "rfm_set_group_data: no such group");
    const GroupH& g = P.groups[group];
    RFM_CHECK(g.kind != RFM_CONTINUITY, RFM_EINVAL, "rfm_set_group_data: continuity rows take no data");
    RFM_CHECK(data != nullptr || g.npts == 0, RFM_EINVAL, "rfm_set_group_data: data is NULL");
    const int nsel = g.comp < 0 ? P.ncomp : 1;
    int64_t off = 0;
    for (int32_t k = 0; k < group; ++k) {
      const GroupH& h = P.groups[k];
      off += h.npts * (h.comp < 0 ? P.ncomp : 1) * h.cont_order;
    }
    const std::vector<double> dh = host_doubles(data, (size_t)g.npts * nsel);
    RFM_CHECK(all_finite(dh), RFM_ENUMERIC, "rfm_set_group_data: non-finite data");
    for (int k = 0; k < nsel; ++k)
      for (int64_t q = 0; q < g.npts; ++q) P.rowdata[off + k * g.npts + q] = dh[(size_t)q * nsel + k];
    if (P.finalized && g.npts) {
      RFM_HIP(hipMemcpyAsync(P.d_rowdata.p + off, P.rowdata.data() + off, (size_t)nsel * g.npts * sizeof(double),
                             hipMemcpyHostToDevice, P.stream));
      RFM_HIP(hipStreamSynchronize(P.stream));
    }
  });
}

rfm_status rfm_finalize(rfm_problem* p) {
  return guarded([&] { finalize(get(p)); });
}

int64_t rfm_num_unknowns(const rfm_problem* p) {
  if (!p) return -1;
  const Problem& P = *reinterpret_cast<const Problem*>(p);
  return P.have_features ? P.n : -1;
}

int64_t rfm_num_rows(const rfm_problem* p) {
  if (!p) return -1;
  const Problem& P = *reinterpret_cast<const Problem*>(p);
  return P.finalized ? P.m : -1;
}

int64_t rfm_num_jacobian_values(const rfm_problem* p) {
  if (!p) return -1;
  const Problem& P = *reinterpret_cast<const Problem*>(p);
  return P.finalized ? P.nvals : -1;
}

rfm_status rfm_stage_count_sketch(rfm_problem* p, double gamma, uint64_t seed, uint64_t jac_index) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_J, RFM_EINVAL, "no Jacobian assembled");
    RFM_CHECK(gamma > 1.0 && std::isfinite(gamma), RFM_EINVAL, "gamma must be > 1");
    const int64_t s = (int64_t)std::ceil(gamma * (double)P.n);
    RFM_CHECK(s >= P.n && s < (int64_t)INT32_MAX, RFM_EINVAL, "sketch size out of range");
    P.s = s;
    launch_count_sketch(P, seed, jac_index);
    P.have_B = true;
    P.have_R = false;
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_sketch_table(int32_t prec, double* out) {
  return guarded([&] {
    RFM_CHECK(prec == RFM_PREC_BF16 || prec == RFM_PREC_FP8, RFM_EINVAL, "table precision must be BF16 or FP8");
    RFM_CHECK(out != nullptr, RFM_EINVAL, "NULL argument");
    sketch_table(prec, out);
  });
}

int64_t rfm_sketch_operand_slots(rfm_problem* p, int32_t block) {
  if (!p) return -1;
  Problem& P = *reinterpret_cast<Problem*>(p);
  if (!P.finalized || block < 0 || block >= P.geom.nbox * P.ncomp) return -1;
  return P.cbs_ptr_h[block + 1] - P.cbs_ptr_h[block];
}

rfm_status rfm_get_sketch_operand(rfm_problem* p, int32_t piece, int32_t block, int64_t slot0, int64_t nslots,
                                  double* out, int32_t* groups, int32_t* scale_exp) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(out != nullptr, RFM_EINVAL, "NULL argument");
    get_sketch_operand(P, piece, block, slot0, nslots, out, groups, scale_exp);
  });
}

int64_t rfm_sketch_rows(const rfm_problem* p) {
  if (!p) return -1;
  return reinterpret_cast<const Problem*>(p)->s;
}

// ---------------------------------------------------------------------------
// stage calls
// ---------------------------------------------------------------------------

rfm_status rfm_stage_assemble(rfm_problem* p, const double* u, double row_scale_c) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(u != nullptr, RFM_EINVAL, "rfm_stage_assemble: u is NULL");
    RFM_CHECK(row_scale_c > 0 && std::isfinite(row_scale_c), RFM_EINVAL, "rfm_stage_assemble: c must be > 0");
    copy_in(P, P.d_u.p, u, P.n);
    launch_assemble(P, P.d_u.p, row_scale_c);
    P.have_J = true;
    P.have_J32 = false;
    P.pan_prec = -1;
    P.cur_c = row_scale_c;
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_get_scaled_residual(rfm_problem* p, double* DF) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_J, RFM_EINVAL, "no Jacobian assembled");
    RFM_CHECK(DF, RFM_EINVAL, "NULL output");
    copy_out(P, DF, P.d_DF.p, P.m);
  });
}

rfm_status rfm_get_row_scale(rfm_problem* p, double* D) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_J, RFM_EINVAL, "no Jacobian assembled");
    RFM_CHECK(D, RFM_EINVAL, "NULL output");
    copy_out(P, D, P.d_D.p, P.m);
  });
}

rfm_status rfm_get_jacobian_rows(rfm_problem* p, int64_t r0, int64_t nrows, double* out) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_J, RFM_EINVAL, "no Jacobian assembled");
    RFM_CHECK(out && r0 >= 0 && nrows >= 0 && r0 + nrows <= P.m, RFM_EINVAL, "row range out of bounds");
    RFM_CHECK((double)nrows * P.n < 4e9, RFM_EINVAL, "too many rows requested at once");
    if (nrows == 0) return;
    DBuf<double> tmp;
    tmp.resize((size_t)nrows * P.n);
    launch_jacobian_rows(P, r0, nrows, tmp.p);
    copy_out(P, out, tmp.p, (size_t)nrows * P.n);
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_jmul(rfm_problem* p, const double* x, double* y) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_J, RFM_EINVAL, "no Jacobian assembled");
    RFM_CHECK(x && y, RFM_EINVAL, "NULL argument");
    double* dx = P.d_vec.p;
    double* dy = P.d_vec.p + std::max(P.m, P.n);
    copy_in(P, dx, x, P.n);
    launch_jmul(P, P.d_J.p, dx, dy, nullptr, nullptr, nullptr);
    copy_out(P, y, dy, P.m);
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_jtmul(rfm_problem* p, const double* y, double* x) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_J, RFM_EINVAL, "no Jacobian assembled");
    RFM_CHECK(x && y, RFM_EINVAL, "NULL argument");
    double* dy = P.d_vec.p;
    double* dx = P.d_vec.p + std::max(P.m, P.n);
    copy_in(P, dy, y, P.m);
    launch_jtmul(P, P.d_J.p, dy, dx, nullptr);
    copy_out(P, x, dx, P.n);
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_jtmul_noalloc(rfm_problem* p, const double* y, double* x) {
  return guarded([&] {
    RFM_CHECK(p != nullptr, RFM_EINVAL, "rfm_jtmul_noalloc: NULL problem");
    Problem& P = *reinterpret_cast<Problem*>(p);
    RFM_CHECK(P.finalized && P.have_J, RFM_EINVAL,
              "rfm_jtmul_noalloc: the problem needs rfm_finalize and an assembled Jacobian first");
    RFM_CHECK(y && x && is_device_ptr(y) && is_device_ptr(x), RFM_EINVAL,
              "rfm_jtmul_noalloc: y and x must be device pointers");
    RFM_CHECK((size_t)P.npart <= noalloc_scratch_doubles(), RFM_EINVAL,
              "rfm_jtmul_noalloc: the Jacobian's tile partials (" + std::to_string(P.npart) +
                  " values) exceed the fixed scratch (" + std::to_string(noalloc_scratch_doubles()) + " values)");
    RFM_HIP(hipSetDevice(P.device));
    launch_jtmul_noalloc(P, y, x, noalloc_scratch(P.device));
  });
}

rfm_status rfm_stage_sketch(rfm_problem* p, double gamma, uint64_t seed, uint64_t jac_index, int32_t prec,
                            int32_t pieces) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_J, RFM_EINVAL, "no Jacobian assembled");
    RFM_CHECK(gamma > 1.0 && std::isfinite(gamma), RFM_EINVAL, "gamma must be > 1");
    RFM_CHECK(prec == RFM_PREC_F64 || prec == RFM_PREC_BF16 || prec == RFM_PREC_FP8, RFM_EINVAL,
              "sketch precision must be F64, BF16 or FP8");
    int64_t s = (int64_t)std::ceil(gamma * (double)P.n);
    RFM_CHECK(s >= P.n && s < (int64_t)INT32_MAX, RFM_EINVAL, "sketch size out of range");
    RFM_CHECK(pieces >= 0 && pieces <= kMaxPieces, RFM_EINVAL, "sketch pieces must be 0..16");
    P.s = s;
    if (prec == RFM_PREC_F64)
      launch_sketch(P, seed, jac_index, prec);
    else
      launch_sketch_lowp(P, seed, jac_index, prec, pieces);
    P.have_B = true;
    P.have_R = false;
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_get_sketch_cols(rfm_problem* p, int64_t c0, int64_t ncols, double* out) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_B, RFM_EINVAL, "no sketch (or it was factorised)");
    RFM_CHECK(out && c0 >= 0 && ncols >= 0 && c0 + ncols <= P.n, RFM_EINVAL, "column range out of bounds");
    copy_out(P, out, P.d_B.p + (size_t)c0 * P.s, (size_t)ncols * P.s);
  });
}

rfm_status rfm_stage_qr(rfm_problem* p) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_B, RFM_EINVAL, "no sketch to factorise");
    P.have_B = false;
    qr_factor(P);
    P.have_R = true;
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_stage_sketch_qr_streamed(rfm_problem* p, double gamma, uint64_t seed, uint64_t jac_index,
                                        int32_t prec, int32_t pieces, int64_t rows_per_pass) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_J, RFM_EINVAL, "no Jacobian assembled");
    RFM_CHECK(gamma > 1.0 && std::isfinite(gamma), RFM_EINVAL, "gamma must be > 1");
    RFM_CHECK(prec == RFM_PREC_F64 || prec == RFM_PREC_BF16 || prec == RFM_PREC_FP8, RFM_EINVAL,
              "sketch precision must be F64, BF16 or FP8");
    RFM_CHECK(pieces >= 0 && pieces <= kMaxPieces, RFM_EINVAL, "sketch pieces must be 0..16");
    RFM_CHECK(rows_per_pass >= 0 && (rows_per_pass == 0 || rows_per_pass >= 128), RFM_EINVAL,
              "rows_per_pass must be 0 or at least 128");
    const int64_t s = (int64_t)std::ceil(gamma * (double)P.n);
    RFM_CHECK(s >= P.n && s < (int64_t)INT32_MAX, RFM_EINVAL, "sketch size out of range");
    P.s = s;
    P.have_B = false;
    P.have_R = false;
    streamed_sketch_qr(P, seed, jac_index, prec, pieces, rows_per_pass);
    P.have_R = true;
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_stage_count_sketch_qr_streamed(rfm_problem* p, double gamma, uint64_t seed, uint64_t jac_index,
                                              int64_t rows_per_pass) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_J, RFM_EINVAL, "no Jacobian assembled");
    RFM_CHECK(gamma > 1.0 && std::isfinite(gamma), RFM_EINVAL, "gamma must be > 1");
    RFM_CHECK(rows_per_pass >= 0 && (rows_per_pass == 0 || rows_per_pass >= 128), RFM_EINVAL,
              "rows_per_pass must be 0 or at least 128");
    const int64_t s = (int64_t)std::ceil(gamma * (double)P.n);
    RFM_CHECK(s >= P.n && s < (int64_t)INT32_MAX, RFM_EINVAL, "sketch size out of range");
    P.s = s;
    P.have_B = false;
    P.have_R = false;
    streamed_count_sketch_qr(P, seed, jac_index, rows_per_pass);
    P.have_R = true;
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_get_r_cols(rfm_problem* p, int64_t c0, int64_t ncols, double* out) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_R, RFM_EINVAL, "no R factor");
    RFM_CHECK(out && c0 >= 0 && ncols >= 0 && c0 + ncols <= P.n, RFM_EINVAL, "column range out of bounds");
    if (ncols == 0) return;
    DBuf<double> tmp;
    tmp.resize((size_t)ncols * P.n);
    launch_get_r_cols(P, c0, ncols, tmp.p);
    copy_out(P, out, tmp.p, (size_t)ncols * P.n);
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_r_solve(rfm_problem* p, const double* y, double* x) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_R, RFM_EINVAL, "no R factor");
    RFM_CHECK(x && y, RFM_EINVAL, "NULL argument");
    double* dy = P.d_vec.p;
    double* dx = P.d_vec.p + std::max(P.m, P.n);
    copy_in(P, dy, y, P.n);
    launch_trsv(P, dy, dx, false, nullptr, nullptr, 0, 0, nullptr);
    check_trsv_error(P);
    copy_out(P, x, dx, P.n);
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_rt_solve(rfm_problem* p, const double* y, double* x) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_R, RFM_EINVAL, "no R factor");
    RFM_CHECK(x && y, RFM_EINVAL, "NULL argument");
    double* dy = P.d_vec.p;
    double* dx = P.d_vec.p + std::max(P.m, P.n);
    copy_in(P, dy, y, P.n);
    launch_trsv(P, dy, dx, true, nullptr, nullptr, 0, 0, nullptr);
    check_trsv_error(P);
    copy_out(P, x, dx, P.n);
    RFM_HIP(hipStreamSynchronize(P.stream));
  });
}

rfm_status rfm_stage_lsqr(rfm_problem* p, const double* rhs, double tol, int32_t max_iter, int32_t prec, double* y,
                          int32_t* iters, int32_t* istop) {
  return guarded([&] {
    Problem& P = ready(p);
    RFM_CHECK(P.have_J && P.have_R, RFM_EINVAL, "need a Jacobian and an R factor");
    RFM_CHECK(rhs && y, RFM_EINVAL, "NULL argument");
    RFM_CHECK(tol > 0 && max_iter >= 1, RFM_EINVAL, "bad LSQR tolerance or iteration limit");
    RFM_CHECK(prec == RFM_PREC_F64 || prec == RFM_PREC_F32, RFM_EINVAL, "LSQR precision must be F64 or F32");
    if (prec == RFM_PREC_F32 && !P.have_J32) launch_cast_f32(P);
    double* drhs = P.d_vec.p + 5 * std::max(P.m, P.n);
    copy_in(P, drhs, rhs, P.m);
    DBuf<double> dy;
    dy.resize(P.n);
    int it = 0, is = 0;
    lsqr_run(P, drhs, tol, max_iter, dy.p, &it, &is, prec);
    copy_out(P, y, dy.p, P.n);
    RFM_HIP(hipStreamSynchronize(P.stream));
    if (iters) *iters = it;
    if (istop) *istop = is;
  });
}

static rfm_status guarded_rc(const std::function<rfm_status()>& f) {
  rfm_status rc = RFM_OK;
  rfm_status g = guarded([&] { rc = f(); });
  return g != RFM_OK ? g : rc;
}

rfm_status rfm_solve(rfm_problem* p, const rfm_solve_opts* opts, double* u_inout, rfm_solve_stats* stats) {
  return guarded_rc([&] { return api_solve(ready(p), opts, u_inout, stats); });
}

rfm_status rfm_residual(rfm_problem* p, const double* u, double* F, double* norm) {
  return guarded_rc([&] {
    RFM_CHECK(u != nullptr, RFM_EINVAL, "rfm_residual: u is NULL");
    return api_residual(ready(p), u, F, norm);
  });
}

rfm_status rfm_eval(rfm_problem* p, const double* u, int64_t npts, const double* x, const int32_t* owner,
                    int32_t what, double* out) {
  return guarded_rc([&] {
    RFM_CHECK(u != nullptr, RFM_EINVAL, "rfm_eval: u is NULL");
    return api_eval(ready(p), u, npts, x, owner, what, out);
  });
}

rfm_status rfm_stage_linesearch(rfm_problem* p, const double* u, const double* du, int32_t gs_iters, double* alpha,
                                double* phi) {
  return guarded_rc([&] { return api_linesearch(ready(p), u, du, gs_iters, alpha, phi); });
}

rfm_status rfm_profile_enable(rfm_problem* p, int32_t on) {
  return guarded([&] {
    Problem& P = get(p);
    P.prof.resolve();
    if (on) {
      P.prof.names.clear();
      P.prof.stats.clear();
    }
    P.prof.on = on != 0;
  });
}

int32_t rfm_profile_read(rfm_problem* p, rfm_kernel_stat* out, int32_t max) {
  int32_t count = 0;
  rfm_status rc = guarded([&] {
    Problem& P = get(p);
    RFM_CHECK(max >= 0 && (max == 0 || out), RFM_EINVAL, "rfm_profile_read: bad output");
    RFM_HIP(hipStreamSynchronize(P.stream));
    P.prof.resolve();
    count = (int32_t)P.prof.names.size();
    for (int32_t i = 0; i < count && i < max; ++i) {
      std::memset(&out[i], 0, sizeof(out[i]));
      std::strncpy(out[i].name, P.prof.names[i].c_str(), sizeof(out[i].name) - 1);
      out[i].launches = P.prof.stats[i].launches;
      out[i].seconds = P.prof.stats[i].seconds;
      out[i].flops = P.prof.stats[i].flops;
      out[i].bytes = P.prof.stats[i].bytes;
    }
  });
  return rc == RFM_OK ? count : rc;
}

}  // extern "C"
