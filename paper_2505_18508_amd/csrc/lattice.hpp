// Torus geometry shared by the host library and the kernels.
//
// The instance is the toroidal grid of the paper (Section I; Appendix A,
// Fig. 2): each site coupled to its nearest neighbours, periodic in every
// dimension.  Internally a 2-D {rows, cols} torus is the 3-D shape
// {Lz = 1, Ly = rows, Lx = cols} without z edges, so one set of formulas
// serves both.
//
// Colour-split ("checkerboard") order used for on-chip state: site
// (x, y, z) has colour p = (x + y + z) & 1 and, within its colour, index
// h = line * hx + (x >> 1) with line = z * Ly + y and hx = Lx / 2.  The word of
// site (p, h) sits at p * half + h.  All neighbours of a colour-p site are
// colour 1-p sites (even dimensions), on the same line at x +/- 1 or on the
// neighbouring lines at the same x.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

// Exact unsigned 32-bit division by a runtime constant d >= 1
// (Granlund & Montgomery, "Division by invariant integers using
// multiplication", PLDI'94, Fig. 4.1): q = (t + ((n - t) >> s1)) >> s2 with
// t = mulhi(m, n).
struct FastDiv {
  uint32_t d, m, s1, s2;
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while (l < 32 && ((uint64_t)1 << l) < d) ++l;
  FastDiv f;
  f.d = d;
  f.m = (uint32_t)(((((uint64_t)1 << l) - d) << 32) / d + 1);
  f.s1 = l < 1 ? l : 1;
  f.s2 = l > 1 ? l - 1 : 0;
  return f;
}

__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t t = __umulhi(f.m, n);
#else
  const uint32_t t = (uint32_t)(((uint64_t)f.m * n) >> 32);
#endif
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

struct Lattice {
  int32_t ndim;   // 2 or 3
  int32_t Lx, Ly, Lz;
  int32_t hx;     // Lx / 2
  int32_t half;   // n / 2 sites per colour
  int32_t lines;  // Ly * Lz
  int32_t n;      // sites
  FastDiv div_lx, div_ly;
};

inline Lattice make_lattice(int ndim, const int32_t* dims) {
  Lattice L;
  L.ndim = ndim;
  if (ndim == 2) {
    L.Lz = 1;
    L.Ly = dims[0];
    L.Lx = dims[1];
  } else {
    L.Lz = dims[0];
    L.Ly = dims[1];
    L.Lx = dims[2];
  }
  L.hx = L.Lx / 2;
  L.lines = L.Ly * L.Lz;
  L.n = L.Lx * L.lines;
  L.half = L.n / 2;
  L.div_lx = make_fastdiv((uint32_t)L.Lx);
  L.div_ly = make_fastdiv((uint32_t)L.Ly);
  return L;
}

// Direction order of a site's incident edge slots, used for per-site weight
// sign bits: 0 = +x, 1 = -x, 2 = +y, 3 = -y, 4 = +z, 5 = -z.
// Canonical edge of direction d of site i: +axis edges are ndim*i + axis;
// -axis edges are the +axis edge of the -1 neighbour.

// Position of canonical site i in colour-split order.
__host__ __device__ inline void site_to_split(const Lattice& L, uint32_t i, int& p, uint32_t& h) {
  const uint32_t line = fdiv(i, L.div_lx);
  const uint32_t x = i - line * (uint32_t)L.Lx;
  const uint32_t z = fdiv(line, L.div_ly);
  const uint32_t y = line - z * (uint32_t)L.Ly;
  p = (int)((x + y + z) & 1u);
  h = line * (uint32_t)L.hx + (x >> 1);
}

}  // namespace ising
