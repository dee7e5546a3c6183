// rm_io.cpp -- the file boundary of the outer-region code: readers of the
// inner-region output (H.DAT / H.DATXXX Fortran unformatted files, sizeH.dat
// and sizeBP.dat) and the writer of the collision strengths (OMEGA / OMEGAU).
// Record layouts follow the PSTGF paper, section "Input files" (H.DAT tables,
// sizeH.dat formats) and section "Output files" (OMEGA table).  Host code only.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "rm.h"

namespace {

// A Fortran unformatted sequential file: records framed by 4-byte length
// markers, subrecords (records over 2 GiB) with negative markers, either byte
// order (told apart by the first record's length, which the caller knows).
struct FortranFile {
  FILE *f = nullptr;
  bool swap = false;
  int64_t size = 0;  // file length: no record may claim more than what is left
  std::string err;

  ~FortranFile() { close(); }
  void close() {
    if (f) fclose(f);
    f = nullptr;
  }
  static int32_t bswap(int32_t v) {
    uint32_t u = (uint32_t)v;
    u = (u >> 24) | ((u >> 8) & 0xff00u) | ((u << 8) & 0xff0000u) | (u << 24);
    return (int32_t)u;
  }
  bool open(const char *path) {
    close();
    f = fopen(path, "rb");
    if (!f) {
      err = std::string("cannot open ") + path;
      return false;
    }
    size = (fseek(f, 0, SEEK_END) == 0) ? (int64_t)ftell(f) : -1;
    if (size < 0 || fseek(f, 0, SEEK_SET) != 0) {
      err = std::string("cannot seek in ") + path;
      close();
      return false;
    }
    return true;
  }
  // Sets the byte order from the first record's head marker, which must read
  // as `expect` bytes in one of the two orders.
  bool detect(int32_t expect) {
    int32_t m = 0;
    const long pos = ftell(f);
    if (fread(&m, 4, 1, f) != 1) {
      err = "empty file";
      return false;
    }
    fseek(f, pos, SEEK_SET);
    if (m == expect) swap = false;
    else if (bswap(m) == expect) swap = true;
    else {
      err = "first record has an unexpected length (not an H.DAT target record)";
      return false;
    }
    return true;
  }
  // Reads one logical record; false at end of file (eof set) or on a framing error.
  bool record(std::vector<char> &out, bool &eof) {
    out.clear();
    eof = false;
    for (int part = 0;; ++part) {
      int32_t head = 0, tail = 0;
      if (part == 0 && (int64_t)ftell(f) == size) {  // the end of the file, between records
        eof = true;
        return false;
      }
      if (fread(&head, 4, 1, f) != 1) {  // a partial marker
        err = "truncated record";
        return false;
      }
      if (swap) head = bswap(head);
      const int64_t len = head < 0 ? -(int64_t)head : head;
      if (len + 4 > size - (int64_t)ftell(f)) {  // the payload and its tail marker must fit in the file
        err = "truncated record";
        return false;
      }
      const size_t at = out.size();
      out.resize(at + (size_t)len);
      if (len && fread(out.data() + at, 1, (size_t)len, f) != (size_t)len) {
        err = "truncated record";
        return false;
      }
      if (fread(&tail, 4, 1, f) != 1) {
        err = "truncated record";
        return false;
      }
      if (swap) tail = bswap(tail);
      if ((tail < 0 ? -(int64_t)tail : tail) != len) {
        err = "record markers disagree";
        return false;
      }
      if (head >= 0) return true;
    }
  }
};

// Sequential reader of the values of one record.
struct Fields {
  const std::vector<char> &r;
  bool swap;
  size_t pos = 0;
  bool ok = true;
  Fields(const std::vector<char> &rec, bool sw) : r(rec), swap(sw) {}
  template <typename T>
  T get() {
    T v{};
    if (pos + sizeof(T) > r.size()) {
      ok = false;
      return v;
    }
    std::memcpy(&v, r.data() + pos, sizeof(T));
    pos += sizeof(T);
    if (swap) {
      char *b = reinterpret_cast<char *>(&v);
      for (size_t i = 0; i < sizeof(T) / 2; ++i) std::swap(b[i], b[sizeof(T) - 1 - i]);
    }
    return v;
  }
  template <typename T>
  void get(T *dst, size_t n) {
    for (size_t i = 0; i < n; ++i) dst[i] = get<T>();
  }
};

}  // namespace

struct rm_hdat {
  FortranFile ff;
  std::string err;
  rm_hdat_target tgt{};
  std::vector<double> enat, coeff;
  std::vector<int32_t> lat, isat;
  std::vector<int32_t> nbutd;
  std::vector<std::vector<double>> ebutd, cbutd;
  // current symmetry
  bool have = false;
  rm_hdat_sym sym{};
  std::vector<int32_t> nconat, l2p, target;
  std::vector<double> cf, value, wmat, ethr;
};

namespace {

rm_status fail(rm_hdat *h, const std::string &m) {
  h->err = m.empty() ? h->ff.err : m;
  return RM_E_IO;
}

}  // namespace

extern "C" {

static rm_status hdat_open_impl(const char *path, rm_hdat **out) {
  if (!path || !out) return RM_E_ARG;
  *out = nullptr;
  rm_hdat *h = new (std::nothrow) rm_hdat();
  if (!h) return RM_E_NOMEM;
  *out = h;
  if (!h->ff.open(path)) return fail(h, "");
  // target record 1: NELC, NZ, LRANG2, LAMAX, NAST (INT*4), RA, BSTO (REAL*8)
  if (!h->ff.detect(5 * 4 + 2 * 8)) return fail(h, "");
  std::vector<char> rec;
  bool eof;
  if (!h->ff.record(rec, eof)) return fail(h, eof ? "missing target record 1" : "");
  {
    Fields f(rec, h->ff.swap);
    h->tgt.nelc = f.get<int32_t>();
    h->tgt.nz = f.get<int32_t>();
    h->tgt.lrang2 = f.get<int32_t>();
    h->tgt.lamax = f.get<int32_t>();
    h->tgt.nast = f.get<int32_t>();
    h->tgt.ra = f.get<double>();
    h->tgt.bsto = f.get<double>();
    if (!f.ok || h->tgt.nast < 1 || h->tgt.lrang2 < 0 || h->tgt.lamax < 0 || !(h->tgt.ra > 0))
      return fail(h, "invalid target record 1");
  }
  const int nast = h->tgt.nast, lr = h->tgt.lrang2;
  // each record is read and its length checked against the count the header
  // gives before that many values are allocated, so a damaged count cannot
  // ask for more memory than the file holds
  auto rd = [&](const char *what, int64_t bytes, auto &&fn) -> rm_status {
    if (!h->ff.record(rec, eof)) return fail(h, eof ? std::string("missing target record: ") + what : "");
    if ((int64_t)rec.size() != bytes) return fail(h, std::string("target record of wrong length: ") + what);
    Fields f(rec, h->ff.swap);
    fn(f);
    if (!f.ok || f.pos != rec.size()) return fail(h, std::string("target record of wrong length: ") + what);
    return RM_OK;
  };
  auto fill = [](auto &v, size_t n, Fields &f) {
    v.resize(n);
    f.get(v.data(), n);
  };
  if (rm_status st = rd("ENAT", 8LL * nast, [&](Fields &f) { fill(h->enat, nast, f); })) return st;
  if (rm_status st = rd("LAT", 4LL * nast, [&](Fields &f) { fill(h->lat, nast, f); })) return st;
  if (rm_status st = rd("ISAT", 4LL * nast, [&](Fields &f) { fill(h->isat, nast, f); })) return st;
  if (rm_status st = rd("COEFF", 24LL * lr, [&](Fields &f) { fill(h->coeff, 3 * (size_t)lr, f); })) return st;
  // Buttle correction, three records per L (LRANG2 is bounded by the COEFF record's length)
  h->nbutd.resize(lr);
  h->ebutd.resize(lr);
  h->cbutd.resize(lr);
  for (int l = 0; l < lr; ++l) {
    if (rm_status st = rd("NBUTD", 4, [&](Fields &f) { h->nbutd[l] = f.get<int32_t>(); })) return st;
    if (h->nbutd[l] < 0) return fail(h, "negative NBUTD");
    const int nb = h->nbutd[l];
    if (rm_status st = rd("EBUTD", 8LL * nb, [&](Fields &f) { fill(h->ebutd[l], nb, f); })) return st;
    if (rm_status st = rd("CBUTD", 8LL * nb, [&](Fields &f) { fill(h->cbutd[l], nb, f); })) return st;
  }
  return RM_OK;
}

rm_status rm_hdat_close(rm_hdat *h) {
  delete h;
  return RM_OK;
}

const char *rm_hdat_error(const rm_hdat *h) { return h ? h->err.c_str() : "null handle"; }

rm_status rm_hdat_target_info(const rm_hdat *h, rm_hdat_target *t, double *enat, int32_t *lat, int32_t *isat) {
  if (!h || !t) return RM_E_ARG;
  *t = h->tgt;
  if (enat) std::memcpy(enat, h->enat.data(), sizeof(double) * h->enat.size());
  if (lat) std::memcpy(lat, h->lat.data(), sizeof(int32_t) * h->lat.size());
  if (isat) std::memcpy(isat, h->isat.data(), sizeof(int32_t) * h->isat.size());
  return RM_OK;
}

rm_status rm_hdat_attach(rm_hdat *h, const char *path) {
  if (!h || !path) return RM_E_ARG;
  const bool swap = h->ff.swap;
  if (!h->ff.open(path)) return fail(h, "");
  h->ff.swap = swap;  // the symmetry files come from the same inner-region run
  h->have = false;
  return RM_OK;
}

static rm_status hdat_next_impl(rm_hdat *h, rm_hdat_sym *sym) {
  if (!h || !sym) return RM_E_ARG;
  h->have = false;
  std::vector<char> rec;
  bool eof;
  if (!h->ff.record(rec, eof)) {
    if (eof) {
      h->err = "no more symmetries";
      return RM_E_NOTFOUND;
    }
    return fail(h, "");
  }
  rm_hdat_sym s{};
  {
    Fields f(rec, h->ff.swap);
    s.lrgl2 = f.get<int32_t>();
    s.nspn2 = f.get<int32_t>();
    s.npty2 = f.get<int32_t>();
    s.nchan = f.get<int32_t>();
    s.mnp2 = f.get<int32_t>();
    s.more2 = f.get<int32_t>();
    if (!f.ok || f.pos != rec.size() || s.nchan < 1 || s.nchan > RM_MAX_CHANNELS || s.mnp2 < 1)
      return fail(h, "invalid symmetry record 1");
  }
  const int nast = h->tgt.nast, n = s.nchan, M = s.mnp2, lam = h->tgt.lamax;
  // as for the target records: a record's length is checked against the
  // header's counts before that many values are allocated
  auto rd = [&](const char *what, int64_t bytes, auto &&fn) -> rm_status {
    if (!h->ff.record(rec, eof)) return fail(h, eof ? std::string("missing symmetry record: ") + what : "");
    if ((int64_t)rec.size() != bytes) return fail(h, std::string("symmetry record of wrong length: ") + what);
    Fields f(rec, h->ff.swap);
    fn(f);
    if (!f.ok || f.pos != rec.size()) return fail(h, std::string("symmetry record of wrong length: ") + what);
    return RM_OK;
  };
  auto fill = [](auto &v, size_t cnt, Fields &f) {
    v.resize(cnt);
    f.get(v.data(), cnt);
  };
  const int64_t ncf = (int64_t)lam * n * n, nw = (int64_t)M * n;  // lam < 2^31, n <= RM_MAX_CHANNELS: no overflow
  if (rm_status st = rd("NCONAT", 4LL * nast, [&](Fields &f) { fill(h->nconat, nast, f); })) return st;
  if (rm_status st = rd("L2P", 4LL * n, [&](Fields &f) { fill(h->l2p, n, f); })) return st;
  if (rm_status st = rd("CF", 8 * ncf, [&](Fields &f) { fill(h->cf, (size_t)ncf, f); })) return st;
  if (rm_status st = rd("VALUE", 8LL * M, [&](Fields &f) { fill(h->value, M, f); })) return st;
  if (rm_status st = rd("WMAT", 8 * nw, [&](Fields &f) { fill(h->wmat, (size_t)nw, f); })) return st;
  // channels are ordered by target: the first NCONAT(1) belong to target 1, ...
  long tot = 0;
  for (int t = 0; t < nast; ++t) {
    if (h->nconat[t] < 0) return fail(h, "negative NCONAT");
    tot += h->nconat[t];
  }
  if (tot != n) return fail(h, "NCONAT does not add up to NCHAN");
  h->target.resize(n);
  h->ethr.resize(n);
  for (int t = 0, i = 0; t < nast; ++t)
    for (int c = 0; c < h->nconat[t]; ++c, ++i) {
      h->target[i] = t;
      h->ethr[i] = h->enat[t] - h->enat[0];
    }
  for (int k = 1; k < M; ++k)
    if (!(h->value[k] >= h->value[k - 1])) return fail(h, "VALUE (pole energies) not ascending");
  h->sym = s;
  h->have = true;
  *sym = s;
  return RM_OK;
}

rm_status rm_hdat_arrays(const rm_hdat *h, int32_t *nconat, int32_t *l2p, double *cf, double *value, double *wmat) {
  if (!h || !h->have) return RM_E_ARG;
  if (nconat) std::memcpy(nconat, h->nconat.data(), sizeof(int32_t) * h->nconat.size());
  if (l2p) std::memcpy(l2p, h->l2p.data(), sizeof(int32_t) * h->l2p.size());
  if (cf) std::memcpy(cf, h->cf.data(), sizeof(double) * h->cf.size());
  if (value) std::memcpy(value, h->value.data(), sizeof(double) * h->value.size());
  if (wmat) std::memcpy(wmat, h->wmat.data(), sizeof(double) * h->wmat.size());
  return RM_OK;
}

rm_status rm_hdat_pw_desc(const rm_hdat *h, rm_pw_desc *d) {
  if (!h || !d || !h->have) return RM_E_ARG;
  const rm_hdat_sym &s = h->sym;
  d->nchan = s.nchan;
  d->npole = s.mnp2;
  d->ntarget = h->tgt.nast;
  d->a = h->tgt.ra;
  d->b = h->tgt.bsto;
  d->z = (double)h->tgt.nz - (double)h->tgt.nelc;  // in double: both come from the file
  // statistical weight: (2S+1)(2L+1) in LS coupling, 2J+1 (LRGL2 = 2J) in J coupling
  d->g = s.nspn2 > 0 ? (double)s.nspn2 * (2.0 * s.lrgl2 + 1.0) : (double)s.lrgl2 + 1.0;
  d->e_thr = h->ethr.data();
  d->l = h->l2p.data();
  d->target = h->target.data();
  d->Ek = h->value.data();
  d->w = h->wmat.data();
  return RM_OK;
}

static rm_status sizeh_read_impl(const char *path, int32_t kind, int32_t cap, rm_sizeh_row *rows, int32_t *count) {
  if (!path || !count || cap < 0 || (cap > 0 && !rows) || (kind != 0 && kind != 1)) return RM_E_ARG;
  FILE *f = fopen(path, "r");
  if (!f) return RM_E_IO;
  // fixed columns (1-based, inclusive) of the Fortran formats
  //   sizeH.dat:  8X,I5,10X,I6,8X,I6,3(4X,I3)  NCHAN, NCON, MNP2, S, L, IPI
  //   sizeBP.dat: 3I7,9X,I3,8X,I3              NCHAN, NCON, MNP2, J2, IPI
  static const int colH[6][2] = {{9, 13}, {24, 29}, {38, 43}, {48, 50}, {55, 57}, {62, 64}};
  static const int colB[5][2] = {{1, 7}, {8, 14}, {15, 21}, {31, 33}, {42, 44}};
  char line[1024];
  int32_t n = 0;
  rm_status st = RM_OK;
  while (fgets(line, sizeof line, f)) {
    const size_t len = strcspn(line, "\r\n");
    if (!line[len] && len == sizeof line - 1) {  // longer than any line of these formats
      st = RM_E_IO;
      break;
    }
    line[len] = 0;
    bool blank = true;
    for (size_t i = 0; i < len; ++i) blank &= line[i] == ' ' || line[i] == '\t';
    if (blank) continue;
    auto field = [&](int a, int b, int32_t &v) {
      // Fortran I-format input: blanks are ignored, an all-blank field is 0
      char buf[32];
      int k = 0;
      for (int c = a - 1; c < b && c < (int)len; ++c)
        if (line[c] != ' ') buf[k++] = line[c];
      buf[k] = 0;
      if (!k) {
        v = 0;
        return true;
      }
      char *end;
      const long x = strtol(buf, &end, 10);
      v = (int32_t)x;
      return *end == 0;
    };
    rm_sizeh_row r{};
    bool ok = true;
    if (kind == 0) {
      ok &= field(colH[0][0], colH[0][1], r.nchan) && field(colH[1][0], colH[1][1], r.ncon) &&
            field(colH[2][0], colH[2][1], r.mnp2) && field(colH[3][0], colH[3][1], r.s) &&
            field(colH[4][0], colH[4][1], r.l) && field(colH[5][0], colH[5][1], r.ipi);
    } else {
      r.s = 0;  // J coupling: the L field carries 2J
      ok &= field(colB[0][0], colB[0][1], r.nchan) && field(colB[1][0], colB[1][1], r.ncon) &&
            field(colB[2][0], colB[2][1], r.mnp2) && field(colB[3][0], colB[3][1], r.l) &&
            field(colB[4][0], colB[4][1], r.ipi);
    }
    if (!ok) {  // a field that is not an integer
      st = RM_E_IO;
      break;
    }
    if (n < cap) rows[n] = r;
    ++n;
  }
  fclose(f);
  *count = n;
  return st;
}

static rm_status omega_write_impl(const char *path, int32_t formatted, int32_t nz, int32_t nel, int32_t nlev,
                                  const int32_t *S, const int32_t *L, const double *elev, int32_t ne, const double *E,
                                  const double *omega, int32_t nomwrt, int32_t elastic) {
  if (!path || nlev < 1 || ne < 0 || !S || !L || !elev || (ne > 0 && (!E || !omega))) return RM_E_ARG;
  // transitions of the upper triangle (i < j, or i <= j with elastic ones),
  // row-wise for nomwrt > 0, column-wise for nomwrt < 0; the first |nomwrt|
  std::vector<std::pair<int, int>> tr;
  if (nomwrt >= 0) {
    for (int i = 0; i < nlev; ++i)
      for (int j = elastic ? i : i + 1; j < nlev; ++j) tr.emplace_back(i, j);
  } else {
    for (int j = 0; j < nlev; ++j)
      for (int i = 0; i <= (elastic ? j : j - 1); ++i) tr.emplace_back(i, j);
  }
  const long want = nomwrt >= 0 ? (long)nomwrt : -(long)nomwrt;
  if ((long)tr.size() > want) tr.resize((size_t)want);
  const int32_t nw = nomwrt >= 0 ? (int32_t)tr.size() : -(int32_t)tr.size();
  // energies in z-scaled Rydberg units, E / z^2 (z = NZ - NEL; unscaled for a neutral target)
  const double zz = (double)nz - (double)nel;
  const double z2 = zz > 0 ? zz * zz : 1.0;
  // every buffer is allocated before the file is opened, so nothing between
  // fopen and fclose can throw
  std::vector<int32_t> sl(2 * (size_t)nlev);
  for (int i = 0; i < nlev; ++i) {
    sl[2 * i] = S[i];
    sl[2 * i + 1] = L[i];
  }
  std::vector<double> el(nlev), row(tr.size() + 1);
  for (int i = 0; i < nlev; ++i) el[i] = elev[i] / z2;
  FILE *f = fopen(path, formatted ? "w" : "wb");
  if (!f) return RM_E_IO;
  bool ok = true;
  auto rec = [&](const void *p, size_t bytes) {
    const int32_t m = (int32_t)bytes;
    ok &= fwrite(&m, 4, 1, f) == 1;
    ok &= bytes == 0 || fwrite(p, 1, bytes, f) == bytes;
    ok &= fwrite(&m, 4, 1, f) == 1;
  };
  if (formatted) {
    ok &= fprintf(f, "%d %d\n%d %d %d\n", nz, nel, nlev, ne, nw) > 0;
    for (int i = 0; i < nlev; ++i) ok &= fprintf(f, "%d %d%c", S[i], L[i], i + 1 < nlev ? ' ' : '\n') > 0;
    for (int i = 0; i < nlev; ++i) ok &= fprintf(f, "%.16e%c", el[i], i + 1 < nlev ? ' ' : '\n') > 0;
  } else {
    const int32_t h1[2] = {nz, nel}, h2[3] = {nlev, ne, nw};
    rec(h1, sizeof h1);
    rec(h2, sizeof h2);
    rec(sl.data(), sizeof(int32_t) * sl.size());
    rec(el.data(), sizeof(double) * el.size());
  }
  for (int e = 0; e < ne; ++e) {
    row[0] = E[e] / z2;
    for (size_t t = 0; t < tr.size(); ++t)
      row[t + 1] = omega[((size_t)e * nlev + tr[t].first) * nlev + tr[t].second];
    if (formatted) {
      for (size_t t = 0; t < row.size(); ++t) ok &= fprintf(f, "%.16e%c", row[t], t + 1 < row.size() ? ' ' : '\n') > 0;
    } else {
      rec(row.data(), sizeof(double) * row.size());
    }
  }
  ok &= fclose(f) == 0;
  return ok ? RM_OK : RM_E_IO;
}

// The entry points: a host allocation that fails (a very large but
// consistent file, or a caller's nlev) is reported, never thrown across the
// C ABI.
rm_status rm_hdat_open(const char *path, rm_hdat **out) {
  try {
    return hdat_open_impl(path, out);
  } catch (const std::bad_alloc &) {
    if (out && *out) (*out)->err = "out of host memory";
    return RM_E_NOMEM;
  }
}

rm_status rm_hdat_next(rm_hdat *h, rm_hdat_sym *sym) {
  try {
    return hdat_next_impl(h, sym);
  } catch (const std::bad_alloc &) {
    h->have = false;
    h->err = "out of host memory";
    return RM_E_NOMEM;
  }
}

rm_status rm_sizeh_read(const char *path, int32_t kind, int32_t cap, rm_sizeh_row *rows, int32_t *count) {
  try {
    return sizeh_read_impl(path, kind, cap, rows, count);
  } catch (const std::bad_alloc &) {
    return RM_E_NOMEM;
  }
}

rm_status rm_omega_write(const char *path, int32_t formatted, int32_t nz, int32_t nel, int32_t nlev,
                         const int32_t *S, const int32_t *L, const double *elev, int32_t ne, const double *E,
                         const double *omega, int32_t nomwrt, int32_t elastic) {
  try {
    return omega_write_impl(path, formatted, nz, nel, nlev, S, L, elev, ne, E, omega, nomwrt, elastic);
  } catch (const std::bad_alloc &) {
    return RM_E_NOMEM;
  }
}

}  // extern "C"
