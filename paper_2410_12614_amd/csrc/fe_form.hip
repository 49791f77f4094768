// Form preparation (device operand tables), cell-kernel entry point and
// device status readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "fe_internal.h"

namespace fe {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

fe_status check_form(const fe_form_desc *f) {
  if (!f) return FE_EINVAL;
  if (f->cell != FE_TRIANGLE && f->cell != FE_TETRAHEDRON && f->cell != FE_HEXAHEDRON)
    return FE_EINVAL;
  if (f->degree < 1 || f->quad_degree < 0) return FE_EINVAL;
  // hexahedra: Q_1 .. Q_7 (n_phi <= 512), the degrees of the paper's boxed cells
  if (f->cell == FE_HEXAHEDRON && f->degree > FE_MAX_BOX_DEGREE) return FE_EUNSUPPORTED;
  if (f->form != FE_MASS && f->form != FE_STIFFNESS) return FE_EINVAL;
  if (f->has_coeff != 0 && f->has_coeff != 1) return FE_EINVAL;
  if (f->precision < FE_FP64 || f->precision > FE_SPLITFP16_ACC32) return FE_EINVAL;
  if (f->geom_precision < FE_GEOM_FP64 || f->geom_precision > FE_GEOM_AUTO) return FE_EINVAL;
  if (f->degree > FE_MAX_DEGREE || f->quad_degree > FE_MAX_QUAD_DEGREE) return FE_EUNSUPPORTED;
  return FE_OK;
}

void tile_choice(int n_phi, int regmul, int *mt, int *jc) {
  const int m = (n_phi + 15) / 16;
  static const int jc1[12] = {0, 4, 8, 9, 7, 0, 7, 0, 6, 0, 0, 3};
  static const int jc2[12] = {0, 4, 5, 5, 4, 0, 3, 0, 2, 0, 0, 2};
  *mt = m;
  *jc = (m >= 1 && m <= 11) ? (regmul == 1 ? jc1[m] : jc2[m]) : 0;
}

fe_status compute_layout(const fe_form_desc *f, FormLayout *L) {
  fe_status st = check_form(f);
  if (st != FE_OK) return st;
  std::memset(L, 0, sizeof(*L));
  L->d = f->cell == FE_HEXAHEDRON ? 3 : f->cell;
  L->box = f->cell == FE_HEXAHEDRON;
  L->form = f->form;
  L->nd = (f->form == FE_MASS) ? 1 : L->d;
  L->ndt = (f->form == FE_MASS) ? 1 : 3;
  L->n_phi = L->box ? (f->degree + 1) * (f->degree + 1) * (f->degree + 1)
                    : simplex_dim(L->d, f->degree);
  const int m = f->quad_degree / 2 + 1;
  L->n_q = (L->d == 2) ? m * m : m * m * m;
  L->prec = f->precision;
  L->has_coeff = f->has_coeff;
  const bool mfma16 = (f->precision == FE_FP16_ACC32 || f->precision == FE_BF16_ACC32 ||
                       f->precision == FE_SPLITFP16_ACC32);
  L->kstep = mfma16 ? 32 : 4;
  L->kpl = mfma16 ? 8 : 1;
  L->n_q_pad = (L->n_q + L->kstep - 1) / L->kstep * L->kstep;
  L->k_pad = L->ndt * L->n_q_pad;  // derivative slabs s >= nd (triangles) are zero
  L->nks = L->k_pad / L->kstep;
  int jc;
  tile_choice(L->n_phi, 1, &L->mt, &jc);
  // hexahedral forms wider than 8 row tiles run in windows of 8 row tiles,
  // the last one 8 or 6 wide (Q5: 14, Q6: 22, Q7: 32 row tiles)
  if (L->box && L->mt > 8 && L->mt <= 32 && (L->mt % 8 == 0 || L->mt % 8 == 6)) jc = 1;
  if (jc == 0) return FE_EUNSUPPORTED;
  L->elt_bytes = mfma16 ? 2 : (f->precision == FE_FP64 ? 8 : 4);
  L->tab_bytes = (f->precision == FE_FP64) ? 8 : (f->precision == FE_FP16_ACC32 ? 2 : 4);
  L->vtab_bytes = (f->precision == FE_FP16_ACC32 || f->precision == FE_BF16_ACC32) ? 4 : 8;
  size_t off = HEADER_BYTES;
  const size_t afrag = (size_t)L->mt * L->nks * 64 * L->kpl * L->elt_bytes;
  L->off_afrag = off;
  off = align256(off + afrag);
  L->off_afrag_lo = off;
  if (f->precision == FE_SPLITFP16_ACC32) off = align256(off + afrag);
  L->off_wtab = off;
  off = align256(off + (size_t)L->ndt * L->n_phi * L->n_q_pad * L->tab_bytes);
  L->off_vtab = off;
  if (L->has_coeff) off = align256(off + (size_t)L->n_q * L->n_phi * L->vtab_bytes);
  L->off_ptab = off;
  if (L->box) off = align256(off + (size_t)L->n_q * 3 * sizeof(double));
  L->off_wq = off;
  off = align256(off + (size_t)L->n_q_pad * sizeof(double));
  // action tables: FP32 / FP64 forms whose dofs fit the registers of a lane;
  // the K-steps are padded to the counts of the tetrahedral degrees 1..6
  // (the kernels are compiled for those), triangles take a zero third slab
  int act_nks = 0;
  for (int b : {1, 3, 5, 9, 14, 21})
    if (act_nks == 0 && 4 * b >= L->n_phi) act_nks = b;
  if ((f->precision == FE_FP32 || f->precision == FE_FP64) && act_nks > 0 && !L->box) {
    L->act_nt = L->form == FE_STIFFNESS ? 4 : 1;
    L->act_nks = act_nks;
    L->act_mt = (act_nks + 3) / 4;
    L->act_nqt = (L->n_q + 15) / 16;
    L->act_chunk = (size_t)64 * (L->act_nt * L->act_nks + L->act_nt * L->act_mt * 4 + 1);
    L->off_act = off;
    off = align256(off + L->act_chunk * L->act_nqt * L->elt_bytes);
  }
  L->total = off;
  return FE_OK;
}

namespace {

template <class T>
void put(unsigned char *base, size_t off, size_t idx, T v) {
  std::memcpy(base + off + idx * sizeof(T), &v, sizeof(T));
}

void store_elt(int prec, unsigned char *buf, size_t off, size_t lo_off, size_t idx, double x) {
  switch (prec) {
    case FE_FP64: put<double>(buf, off, idx, x); break;
    case FE_FP32: put<float>(buf, off, idx, (float)x); break;
    case FE_FP16_ACC32: put<_Float16>(buf, off, idx, (_Float16)x); break;
    case FE_BF16_ACC32: put<__bf16>(buf, off, idx, (__bf16)x); break;
    case FE_SPLITFP16_ACC32: {
      _Float16 hi = (_Float16)x;
      _Float16 lo = (_Float16)((x - (double)hi) * 2048.0);
      put<_Float16>(buf, off, idx, hi);
      put<_Float16>(buf, lo_off, idx, lo);
      break;
    }
  }
}

}  // namespace
}  // namespace fe

using namespace fe;

extern "C" fe_status fe_form_prepare(const fe_form_desc *f, void *form_buf, size_t *form_bytes,
                                     void *stream) {
  FormLayout L;
  fe_status st = compute_layout(f, &L);
  if (st != FE_OK) return st;
  if (!form_bytes) return FE_EINVAL;
  if (!form_buf) {
    *form_bytes = L.total;
    return FE_OK;
  }
  if (*form_bytes < L.total) return FE_ESIZE;
  int32_t nphi, nq;
  st = fe_tabulate(f->cell, f->degree, f->quad_degree, 1, &nphi, &nq, nullptr, nullptr, nullptr);
  if (st != FE_OK) return st;
  const int d = L.d;
  std::vector<double> pts((size_t)nq * d), w(nq), tab((size_t)(1 + d) * nq * nphi);
  st = fe_tabulate(f->cell, f->degree, f->quad_degree, 1, &nphi, &nq, pts.data(), w.data(),
                   tab.data());
  if (st != FE_OK) return st;
  const size_t slab = (size_t)nq * nphi;
  auto Bop = [&](int s, int q, int i) -> double {
    return (L.form == FE_MASS) ? tab[(size_t)q * nphi + i] : tab[(1 + s) * slab + (size_t)q * nphi + i];
  };
  std::vector<unsigned char> h(L.total, 0);
  FormHeader hdr;
  std::memset(&hdr, 0, sizeof(hdr));
  hdr.magic = FORM_MAGIC;
  hdr.d = d;
  hdr.nd = L.nd;
  hdr.n_phi = nphi;
  hdr.n_q = nq;
  hdr.prec = L.prec;
  hdr.form = L.form;
  hdr.geom = f->geom_precision;
  // B^T fragments.  In the 16-bit modes B is scaled by an exact power of two
  // so that max |B| lies in [2^14, 2^15): small tabulated values then stay
  // normal numbers instead of being flushed by the matrix cores.
  double max_b = 0.0;
  for (int s = 0; s < L.nd; ++s)
    for (int q = 0; q < nq; ++q)
      for (int i = 0; i < nphi; ++i) max_b = std::max(max_b, std::fabs(Bop(s, q, i)));
  double b_scale = 1.0;
  if (L.elt_bytes == 2 && max_b > 0.0) b_scale = std::ldexp(1.0, 14 - std::ilogb(max_b));
  hdr.b_scale = b_scale;
  // fragment of row tile mt, derivative s and quadrature chunk qc at slot
  // frag_slot(mt, s, qc): the fragments one chunk needs are contiguous
  const int nqc = L.n_q_pad / L.kstep;
  for (int qc = 0; qc < nqc; ++qc)
    for (int s = 0; s < L.ndt; ++s)
      for (int mt = 0; mt < L.mt; ++mt)
        for (int lane = 0; lane < 64; ++lane)
          for (int e = 0; e < L.kpl; ++e) {
            const int i = 16 * mt + lane % 16;
            const int q = qc * L.kstep + (lane / 16) * L.kpl + e;
            double v = (i < nphi && q < nq && s < L.nd) ? Bop(s, q, i) * b_scale : 0.0;
            size_t idx = (frag_slot(mt, s, qc, L.mt, L.ndt) * 64 + lane) * L.kpl + e;
            store_elt(L.prec, h.data(), L.off_afrag, L.off_afrag_lo, idx, v);
          }
  // weighted table w_q B_t(q, j), [t][j][n_q_pad]; in FP16 storage (the
  // storage precision that also forms H) scaled by an exact power of two so
  // that its largest entry lies in [2^14, 2^15)
  double max_wb = 0.0;
  for (int t = 0; t < L.nd; ++t)
    for (int j = 0; j < nphi; ++j)
      for (int q = 0; q < nq; ++q) max_wb = std::max(max_wb, std::fabs(w[q] * Bop(t, q, j)));
  double w_scale = 1.0;
  if (L.tab_bytes == 2 && max_wb > 0.0) w_scale = std::ldexp(1.0, 14 - std::ilogb(max_wb));
  hdr.w_scale = w_scale;
  for (int t = 0; t < L.ndt; ++t)
    for (int j = 0; j < nphi; ++j)
      for (int q = 0; q < L.n_q_pad; ++q) {
        double v = 0.0;
        if (q < nq && t < L.nd) v = w[q] * Bop(t, q, j);
        size_t idx = ((size_t)t * nphi + j) * L.n_q_pad + q;
        if (L.tab_bytes == 8) put<double>(h.data(), L.off_wtab, idx, v);
        else if (L.tab_bytes == 2) put<_Float16>(h.data(), L.off_wtab, idx, (_Float16)(v * w_scale));
        else put<float>(h.data(), L.off_wtab, idx, (float)v);
      }
  double leb = 0.0;
  for (int q = 0; q < nq; ++q) {
    double s = 0.0;
    for (int k = 0; k < nphi; ++k) s += std::fabs(tab[(size_t)q * nphi + k]);
    leb = std::max(leb, s);
  }
  if (L.has_coeff)
    for (int q = 0; q < nq; ++q)
      for (int k = 0; k < nphi; ++k) {
        double v = tab[(size_t)q * nphi + k];
        size_t idx = (size_t)q * nphi + k;
        if (L.vtab_bytes == 8) put<double>(h.data(), L.off_vtab, idx, v);
        else put<float>(h.data(), L.off_vtab, idx, (float)v);
      }
  if (L.act_nt > 0) {
    // action tables, chunk per tile of 16 quadrature points (layout in
    // fe_internal.h); the FP64 instruction interleaves its output rows
    auto tabv = [&](int t, int q, int k) -> double {
      if (q >= nq || k >= nphi || t > d) return 0.0;
      return tab[(size_t)t * slab + (size_t)q * nphi + k];
    };
    auto orow = [&](int kb, int r) { return L.prec == FE_FP64 ? kb + 4 * r : 4 * kb + r; };
    const size_t e_off = 0, c_off = (size_t)64 * L.act_nt * L.act_nks,
                 w_off = c_off + (size_t)64 * L.act_nt * L.act_mt * 4;
    for (int qt = 0; qt < L.act_nqt; ++qt) {
      const size_t base = (size_t)qt * L.act_chunk;
      for (int t = 0; t < L.act_nt; ++t)
        for (int ks = 0; ks < L.act_nks; ++ks)
          for (int lane = 0; lane < 64; ++lane) {
            const double v = tabv(t, 16 * qt + lane % 16, 4 * ks + lane / 16);
            const size_t idx = base + e_off + ((size_t)t * L.act_nks + ks) * 64 + lane;
            if (L.prec == FE_FP64) put<double>(h.data(), L.off_act, idx, v);
            else put<float>(h.data(), L.off_act, idx, (float)v);
          }
      for (int t = 0; t < L.act_nt; ++t)
        for (int mt = 0; mt < L.act_mt; ++mt)
          for (int r = 0; r < 4; ++r)
            for (int lane = 0; lane < 64; ++lane) {
              const double v = tabv(t, 16 * qt + orow(lane / 16, r), 16 * mt + lane % 16);
              const size_t idx = base + c_off + (((size_t)t * L.act_mt + mt) * 4 + r) * 64 + lane;
              if (L.prec == FE_FP64) put<double>(h.data(), L.off_act, idx, v);
              else put<float>(h.data(), L.off_act, idx, (float)v);
            }
      for (int j = 0; j < 64; ++j) {
        const int q = 16 * qt + j;
        const double v = (j < 16 && q < nq) ? w[q] : 0.0;
        if (L.prec == FE_FP64) put<double>(h.data(), L.off_act, base + w_off + j, v);
        else put<float>(h.data(), L.off_act, base + w_off + j, (float)v);
      }
    }
  }
  if (L.box)
    for (int q = 0; q < nq; ++q)
      for (int e = 0; e < 3; ++e) put<double>(h.data(), L.off_ptab, (size_t)q * 3 + e, pts[(size_t)q * 3 + e]);
  double max_w = 0.0;
  for (int q = 0; q < nq; ++q) {
    put<double>(h.data(), L.off_wq, q, w[q]);
    max_w = std::max(max_w, std::fabs(w[q]));
  }
  hdr.max_wb = max_wb;
  hdr.max_w = max_w;
  hdr.lebesgue = leb;
  std::memcpy(h.data(), &hdr, sizeof(hdr));
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(form_buf, h.data(), L.total, hipMemcpyHostToDevice, s) != hipSuccess)
    return FE_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return FE_EHIP;
  return FE_OK;
}

namespace fe {
// The fused path needs the weighted table staged in LDS next to the row
// buffers (see fe_fused.h): 8 waves x FUSED_SPAN values + table (+ fragments).
bool fused_eligible(const FormLayout &L) {
  // the tables (fragments included) must sit on chip next to the row
  // buffers of at least 8 waves; otherwise the cell kernels and the row
  // gather are faster
  const FormLayout *one[1] = {&L};
  // hexahedral Poisson forms (a geometry tensor per point) and forms with
  // more than 256 dofs per cell (schedule records hold j in a byte) take the
  // gather
  if (L.box && L.ndt == 3) return false;
  if (L.n_phi > 256) return false;
  return !L.has_coeff && fused_lds(one, 1, 8, true) <= FUSED_LDS_BUDGET;
}

bool cellwise_eligible(const FormLayout &L) {
  if (L.prec != FE_FP16_ACC32 || L.box || L.d != 3) return false;
  if (L.ndt == 3) return L.mt == 6 && L.n_phi % 4 == 0 && L.n_q_pad <= 512;
  // (11 row tiles: rows packed at any n_phi up to 175, the most whose row
  // block, staged up to three floats into the LDS buffer of 16 x 176 floats
  // with the last tile column's overhang, fits it; P8 has 165)
  return !L.has_coeff && (((L.mt == 4 || L.mt == 6 || L.mt == 8) && L.n_phi % 4 == 0) ||
                          (L.mt == 11 && L.n_phi <= 175));
}

fe_status launch_info(const void *kern, int threads, size_t smem, LaunchInfo *out) {
  static std::mutex mu;
  static std::map<std::tuple<const void *, int, int, size_t>, LaunchInfo> info;
  static std::map<std::pair<const void *, int>, size_t> lds_limit;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FE_EHIP;
  std::lock_guard<std::mutex> lock(mu);
  if (smem > 65536) {
    size_t &lim = lds_limit[{kern, dev}];
    if (smem > lim) {
      if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) !=
          hipSuccess)
        return FE_EHIP;
      lim = smem;
    }
  }
  const auto key = std::make_tuple(kern, dev, threads, smem);
  auto it = info.find(key);
  if (it == info.end()) {
    LaunchInfo li;
    if (hipDeviceGetAttribute(&li.ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&li.per_cu, kern, threads, smem) != hipSuccess)
      return FE_EHIP;
    it = info.emplace(key, li).first;
  }
  *out = it->second;
  return FE_OK;
}

fe_status launch_cell(const CellLaunch &a) {
  switch (a.L->prec) {
    case FE_FP64: return launch_cell_fp64(a);
    case FE_FP32: return launch_cell_fp32(a);
    case FE_FP16_ACC32: return launch_cell_fp16(a);
    case FE_BF16_ACC32: return launch_cell_bf16(a);
    case FE_SPLITFP16_ACC32: return launch_cell_split(a);
  }
  return FE_EUNSUPPORTED;
}

namespace {
fe_status cell_kernels(const fe_form_desc *f, const void *form_buf, const fe_mesh_view *m,
                       void *A_local, int tile, void *stream) {
  FormLayout L;
  fe_status st = compute_layout(f, &L);
  if (st != FE_OK) return st;
  if (!form_buf || !m || m->n_cells < 0 || m->n_dofs < 1) return FE_EINVAL;
  if (m->n_cells == 0) return FE_OK;
  if (!m->cell_coords || !A_local) return FE_EINVAL;
  if (f->has_coeff && (!m->coeff || !m->dofmap)) return FE_EINVAL;
  if (m->n_dofs > INT32_MAX) return FE_EOVERFLOW;
  CellLaunch a;
  a.L = &L;
  a.form_buf = (const unsigned char *)form_buf;
  a.status = (int32_t *)form_buf;
  a.n_cells = m->n_cells;
  a.coords = m->cell_coords;
  a.dofmap = m->dofmap;
  a.n_dofs = m->n_dofs;
  a.coeff = f->has_coeff ? m->coeff : nullptr;
  a.A_local = A_local;
  a.stream = stream;
  a.tile = tile;
  if (tile == CELL_TILE_SMALL) return launch_small_fp16(a);
  if (tile == CELL_TILE_WHOLE) {
    // the whole-cell kernel; without a workspace only forms without a
    // coefficient (the coefficient at the points needs one)
    if (f->has_coeff || !cellwise_eligible(L)) return FE_EUNSUPPORTED;
    CellwiseLaunch c;
    c.L = &L;
    c.form_buf = a.form_buf;
    c.status = a.status;
    c.n_cells = a.n_cells;
    c.coords = a.coords;
    c.dofmap = a.dofmap;
    c.n_dofs = a.n_dofs;
    c.coeff = nullptr;
    c.zpt = c.zmax = nullptr;
    c.rec = nullptr;
    c.A_local = (float *)A_local;
    c.stream = stream;
    return launch_cellwise_fp16(c);
  }
  return launch_cell(a);
}

// Block-diagonal CSR pattern of a discontinuous space over degree blocks:
// row r of block b (cell K = r / n_phi_b) holds the n_phi_b dofs of K.
__global__ void k_dg_pattern(int64_t n_rows, int n_phi, int64_t dof_off, int64_t nnz_off,
                             int64_t *row_ptr, int32_t *col_idx) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t start = nnz_off + r * n_phi;
    row_ptr[dof_off + r] = start;
    const int64_t first = dof_off + (r / n_phi) * n_phi;
    for (int j = 0; j < n_phi; ++j) col_idx[start + j] = (int32_t)(first + j);
  }
}

__global__ void k_set_i64(int64_t *x, int64_t v) { *x = v; }
}  // namespace
}  // namespace fe

extern "C" fe_status fe_cell_kernels(const fe_form_desc *f, const void *form_buf,
                                     const fe_mesh_view *m, void *A_local, void *stream) {
  return cell_kernels(f, form_buf, m, A_local, -1, stream);
}

extern "C" fe_status fe_cell_kernels_tile(const fe_form_desc *f, const void *form_buf,
                                          const fe_mesh_view *m, void *A_local, int32_t tile,
                                          void *stream) {
  if (tile < -1 || tile >= CELL_TILES) return FE_EINVAL;
  return cell_kernels(f, form_buf, m, A_local, tile, stream);
}

extern "C" fe_status fe_tune_cell_kernels(const fe_form_desc *f, const void *form_buf,
                                          const fe_mesh_view *m, void *A_local, int32_t reps,
                                          int32_t *best_tile, float *times_ms, void *stream) {
  if (!best_tile || reps < 1) return FE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return FE_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return FE_EHIP;
  }
  fe_status result = FE_EUNSUPPORTED;
  float best = 0.0f;
  *best_tile = -1;
  for (int t = 0; t < CELL_TILES; ++t) {
    if (times_ms) times_ms[t] = -1.0f;
    fe_status st = cell_kernels(f, form_buf, m, A_local, t, stream);  // warm-up
    if (st == FE_EUNSUPPORTED) continue;
    if (st != FE_OK) {
      result = st;
      break;
    }
    if (hipEventRecord(e0, s) != hipSuccess) {
      result = FE_EHIP;
      break;
    }
    for (int r = 0; r < reps && st == FE_OK; ++r) st = cell_kernels(f, form_buf, m, A_local, t, stream);
    float ms = 0.0f;
    if (st != FE_OK || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      result = st != FE_OK ? st : FE_EHIP;
      break;
    }
    ms /= (float)reps;
    if (times_ms) times_ms[t] = ms;
    if (*best_tile < 0 || ms < best) {
      best = ms;
      *best_tile = t;
    }
    result = FE_OK;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return result;
}

extern "C" fe_status fe_dg_pattern(int32_t n_blocks, const int64_t *n_cells, const int32_t *n_phi,
                                   int64_t *row_ptr, int32_t *col_idx, int64_t *nnz,
                                   void *stream) {
  if (n_blocks < 1 || !n_cells || !n_phi || !nnz) return FE_EINVAL;
  int64_t dofs = 0, entries = 0;
  for (int b = 0; b < n_blocks; ++b) {
    if (n_cells[b] < 0 || n_phi[b] < 1 || n_phi[b] > 1024) return FE_EINVAL;
    dofs += n_cells[b] * n_phi[b];
    entries += n_cells[b] * n_phi[b] * n_phi[b];
  }
  if (dofs >= INT32_MAX) return FE_EOVERFLOW;
  *nnz = entries;
  if (!row_ptr || !col_idx) return FE_OK;  // size query
  hipStream_t s = (hipStream_t)stream;
  int64_t dof_off = 0, nnz_off = 0;
  for (int b = 0; b < n_blocks; ++b) {
    const int64_t rows = n_cells[b] * n_phi[b];
    if (rows > 0) {
      const unsigned grid = (unsigned)std::min<int64_t>((rows + 255) / 256, 65536);
      hipLaunchKernelGGL(k_dg_pattern, dim3(grid), dim3(256), 0, s, rows, n_phi[b], dof_off,
                         nnz_off, row_ptr, col_idx);
    }
    dof_off += rows;
    nnz_off += rows * n_phi[b];
  }
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, row_ptr + dof_off, nnz_off);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

extern "C" fe_status fe_get_device_status(const void *buf, void *stream) {
  if (!buf) return FE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int32_t v = 0;
  if (hipMemcpyAsync(&v, buf, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess) return FE_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return FE_EHIP;
  const int32_t zero = 0;
  if (hipMemcpyAsync((void *)buf, &zero, sizeof(zero), hipMemcpyHostToDevice, s) != hipSuccess)
    return FE_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return FE_EHIP;
  if (v & STATUS_BAD_DOF) return FE_EINVAL;
  if (v & STATUS_DEGENERATE) return FE_EDEGENERATE;
  return FE_OK;
}
