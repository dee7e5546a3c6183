// Drives the library's file readers (rm_io.cpp) over files named on the
// command line, for a build with the address and undefined-behaviour
// sanitizers: every H.DAT file is opened, its target records read, each
// symmetry read and copied out through buffers sized from what the reader
// reports, and its descriptor formed; every sizeH.dat / sizeBP.dat file is read
// with both kinds; the OMEGA writer is run over its edge arguments.  A damaged
// file must end in an error status, never in a read or write outside a buffer
// (the sanitizers abort the run on one).
// Prints one line per file: its name and the statuses seen.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "rm.h"

static void read_hdat(const char *path) {
  rm_hdat *h = nullptr;
  const rm_status so = rm_hdat_open(path, &h);
  std::printf("%s open %d", path, (int)so);
  if (so == RM_OK) {
    rm_hdat_target t;
    if (rm_hdat_target_info(h, &t, nullptr, nullptr, nullptr) == RM_OK && t.nast > 0 && t.nast < (1 << 20)) {
      std::vector<double> enat(t.nast);
      std::vector<int32_t> lat(t.nast), isat(t.nast);
      rm_hdat_target_info(h, &t, enat.data(), lat.data(), isat.data());
      rm_hdat_sym s;
      int nsym = 0;
      rm_status sn;
      while ((sn = rm_hdat_next(h, &s)) == RM_OK) {
        ++nsym;
        const size_t n = (size_t)s.nchan, M = (size_t)s.mnp2, L = (size_t)(t.lamax > 0 ? t.lamax : 0);
        std::vector<int32_t> nconat(t.nast), l2p(n);
        std::vector<double> cf(L * n * n), value(M), wmat(M * n);
        const rm_status sa = rm_hdat_arrays(h, nconat.data(), l2p.data(), L ? cf.data() : nullptr, value.data(),
                                            wmat.data());
        rm_pw_desc d;
        const rm_status sd = rm_hdat_pw_desc(h, &d);
        double sum = 0.0;  // touch every entry the descriptor points at
        if (sd == RM_OK) {
          for (int32_t i = 0; i < d.nchan; ++i) sum += d.e_thr[i] + d.l[i] + d.target[i];
          for (size_t k = 0; k < (size_t)d.npole; ++k) sum += d.Ek[k];
          for (size_t k = 0; k < (size_t)d.npole * (size_t)d.nchan; ++k) sum += d.w[k];
        }
        std::printf(" sym %d arrays %d desc %d%s", nsym, (int)sa, (int)sd, sum == sum ? "" : " nan");
      }
      std::printf(" next %d", (int)sn);
    }
  } else if (h) {
    std::printf(" (%s)", rm_hdat_error(h));
  }
  if (h) rm_hdat_close(h);
  std::printf("\n");
}

static void read_sizeh(const char *path) {
  for (int kind = 0; kind < 2; ++kind) {
    int32_t count = 0;
    rm_sizeh_row rows[4];
    const rm_status s = rm_sizeh_read(path, kind, 4, rows, &count);
    std::printf("%s sizeh kind %d status %d rows %d\n", path, kind, (int)s, (int)count);
  }
}

// The OMEGA writer over its edge arguments (one level, no energies, nomwrt at
// both ends of its range and zero, elastic or not, both formats), each file
// written into dir.
static void write_omegas(const char *dir) {
  const int32_t nomwrts[] = {INT32_MIN, -3, 0, 2, INT32_MAX};
  int k = 0;
  for (int32_t nlev : {1, 2, 5})
    for (int32_t ne : {0, 3})
      for (int32_t nomwrt : nomwrts)
        for (int32_t elastic = 0; elastic < 2; ++elastic)
          for (int32_t formatted = 0; formatted < 2; ++formatted) {
            std::vector<int32_t> S(nlev, 2), L(nlev, 1);
            std::vector<double> elev(nlev, 0.5), E(ne, 1.5), om((size_t)ne * nlev * nlev, 0.25);
            char path[4096];
            std::snprintf(path, sizeof path, "%s/omega_%d", dir, k++);
            const rm_status s = rm_omega_write(path, formatted, 26, 23, nlev, S.data(), L.data(), elev.data(), ne,
                                               ne ? E.data() : nullptr, ne ? om.data() : nullptr, nomwrt, elastic);
            std::printf("%s omega nlev %d ne %d nomwrt %d elastic %d formatted %d status %d\n", path, nlev, ne,
                        nomwrt, elastic, formatted, (int)s);
          }
}

int main(int argc, char **argv) {
  // arguments: "hdat" or "sizeh", then the files of that kind, repeated; or
  // "omega" and a directory to write into
  bool hdat = true;
  for (int i = 1; i < argc; ++i) {
    if (!std::strcmp(argv[i], "hdat")) hdat = true;
    else if (!std::strcmp(argv[i], "sizeh")) hdat = false;
    else if (!std::strcmp(argv[i], "omega") && i + 1 < argc) write_omegas(argv[++i]);
    else if (hdat) read_hdat(argv[i]);
    else read_sizeh(argv[i]);
  }
  return 0;
}
