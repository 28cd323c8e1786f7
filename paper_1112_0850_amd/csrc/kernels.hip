// kernels.hip -- gfx950 kernels of the D3Q19 BGK hot path.
//
// One thread updates one cell (Sec. 6: a single thread computes the update
// of a single lattice node).  The fused kernel follows the paper's
// stream-collide ("pull") ordering: it gathers the 19 post-collision values
// of the previous step from the neighbours x - c_i (Sec. 2 step 3, with
// half-way bounce-back at solid neighbours), computes the moments and the
// equilibrium and relaxes (Sec. 2 steps 1-2, Eq. (1)), adds the Guo forcing
// term, and writes the 19 results to its own cell of the second lattice
// (aligned, coalesced stores).  Populations are structure-of-arrays with x
// contiguous, so each of the 19 gathers of a wavefront is one contiguous
// 64-element run shifted by at most one element.
//
// All population values are offsets g = f - w (rest state = 0), which keeps
// FP32/FP16/BF16 storage free of the f ~ w cancellation.  In offset form,
// with delta_rho = sum g_i, j = sum g_i c_i and j' = j + F/2 = rho u,
//   u = j'/(1 + delta_rho),
//   g^eq_i = w_i [delta_rho + rho (3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u)]
//          = w_i (delta_rho - 3/2 j'.u) + 9/2 w_i (c_i.j')(c_i.u) + 3 w_i (c_i.j'),
//   S_i = (1 - omega/2) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F       (Guo 2002),
//   g*_i = (1 - omega) g_i + omega g^eq_i + S_i.
// The second form of g^eq never rounds rho = 1 + delta_rho (see collide()).
// With the incompressible equilibrium of He & Luo (rho0 = 1) u = j' and the
// same coefficient form holds with t = 0 below.  Walls moving with u_w add
// 6 w_i (c_i.u_w) to each bounced-back population (Ladd 1994, rho0 = 1).
#include "d3q19.h"
#include "kernels.h"

namespace lbm {

Geo make_geo(int nx, int ny, int nz, int xs, uint64_t dir_stride) {
  Geo g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.xs = xs;
  g.plane = uint32_t(dir_stride);
  g.nseg = (nx + 63) / 64;
  g.nrows = ny * nz;
  const int64_t segs = int64_t(g.nseg) * g.nrows;
  g.nblocks = int32_t((segs + 3) / 4);
  g.nb8 = (g.nblocks / 8) * 8;
  g.yb = g.ny;
  return g;
}

template <typename C>
struct Phys {
  C omega;
  C F[3];
  C scale;
  C inv_scale;
  C Kw[Q];     // moving-wall term 6 w_i (c_i.u_w) of a bounced-back population (unscaled)
  int moving;  // moving-wall markers in use
  int incomp;  // incompressible equilibrium
};

// 6 w_i (c_i.u_w): what the half-way bounce-back of direction i gains from a
// wall cell moving with u_w (pull form: the population arriving along c_i).
static double wall_term(int i, const double* uw) {
  return 6.0 * weight<double>(i) *
         (D3Q19::cx[i] * uw[0] + D3Q19::cy[i] * uw[1] + D3Q19::cz[i] * uw[2]);
}

template <typename C>
static Phys<C> to_phys(const PhysParams& p) {
  Phys<C> r;
  r.omega = C(p.omega);
  for (int d = 0; d < 3; ++d) r.F[d] = C(p.F[d]);
  r.scale = C(p.scale);
  r.inv_scale = C(1.0 / p.scale);
  for (int i = 0; i < Q; ++i) r.Kw[i] = C(wall_term(i, p.wall_u));
  r.moving = p.moving ? 1 : 0;
  r.incomp = p.incomp ? 1 : 0;
  return r;
}

// Marker of a solid cell in storage format K: the moving-wall marker for a
// moving-wall cell while moving-wall markers are in use, else the resting one.
template <int K>
__device__ __forceinline__ typename Storage<K>::T solid_marker(uint8_t fl, bool moving) {
  return from_bits<K>((moving && (fl & FLAG_MOVING)) ? Storage<K>::kMoving : Storage<K>::kRest);
}

// ---------------------------------------------------------------------------
// Thread -> cell mapping.
// ---------------------------------------------------------------------------
struct Loc {
  int x, y, z;
  int lblock;  // logical block id after the XCD remap
  bool valid;
};

__device__ __forceinline__ Loc locate(const Geo& g) {
  Loc l;
  const int b = blockIdx.x;
  // Hardware hands block b to XCD b % 8; give XCD k the k-th contiguous
  // eighth of the logical blocks (the tail beyond nb8 maps to itself).
  const int lb = (b < g.nb8) ? ((b & 7) * (g.nb8 >> 3) + (b >> 3)) : b;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int seg = lb * 4 + wave;
  const int row = seg / g.nseg;
  l.x = (seg - row * g.nseg) * 64 + int(threadIdx.x & 63);
  l.z = row / g.ny;
  l.y = row - l.z * g.ny;
  l.lblock = lb;
  l.valid = (row < g.nrows) && (l.x < g.nx);
  return l;
}

// Offsets of the 3x3 neighbouring rows (periodic) and of the x-neighbours.
struct Nbhd {
  uint32_t row[3][3];   // [dz+1][dy+1]: element offset of row (y+dy, z+dz) in one direction array
  uint32_t frow[3][3];  // same row in the unpadded cell numbering (flags, fields)
  uint32_t xn[3];       // [cx+1]: the x of the pull source x - cx
  uint32_t own, fown;
};

__device__ __forceinline__ Nbhd neighbourhood(const Geo& g, const Loc& l) {
  Nbhd n;
  const int ys[3] = {l.y == 0 ? g.ny - 1 : l.y - 1, l.y, l.y + 1 == g.ny ? 0 : l.y + 1};
  const int zs[3] = {l.z == 0 ? g.nz - 1 : l.z - 1, l.z, l.z + 1 == g.nz ? 0 : l.z + 1};
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const uint32_t r = uint32_t(zs[dz] * g.ny + ys[dy]);
      n.row[dz][dy] = r * uint32_t(g.xs);
      n.frow[dz][dy] = r * uint32_t(g.nx);
    }
  n.xn[0] = (l.x + 1 == g.nx) ? 0u : uint32_t(l.x + 1);
  n.xn[1] = uint32_t(l.x);
  n.xn[2] = (l.x == 0) ? uint32_t(g.nx - 1) : uint32_t(l.x - 1);
  n.own = n.row[1][1] + uint32_t(l.x);
  n.fown = n.frow[1][1] + uint32_t(l.x);
  return n;
}

// Offset of the pull source x - c_i of direction i (compile-time i).
__device__ __forceinline__ uint32_t src_off(const Nbhd& n, int i) {
  return n.row[1 - D3Q19::cz[i]][1 - D3Q19::cy[i]] + n.xn[D3Q19::cx[i] + 1];
}
__device__ __forceinline__ uint32_t src_foff(const Nbhd& n, int i) {
  return n.frow[1 - D3Q19::cz[i]][1 - D3Q19::cy[i]] + n.xn[D3Q19::cx[i] + 1];
}

// The pull source of direction i split into its wave-uniform row offset and
// its per-lane x (the step kernel's waves each own part of one row).
__device__ __forceinline__ uint32_t src_row(const Nbhd& n, int i) {
  return n.row[1 - D3Q19::cz[i]][1 - D3Q19::cy[i]];
}
__device__ __forceinline__ uint32_t src_x(const Nbhd& n, int i) { return n.xn[D3Q19::cx[i] + 1]; }

// Element (i, row + x) with the row offset folded into the wave-uniform base,
// so that each load is a scalar base plus one of three per-lane x offsets
// (x - 1, x, x + 1) and needs no per-load vector address arithmetic.
template <typename T>
__device__ __forceinline__ T* elem_rx(T* grid, size_t plane_bytes, int i, uint32_t row, uint32_t x) {
  char* b = reinterpret_cast<char*>(grid) + size_t(i) * plane_bytes + size_t(row) * sizeof(T);
  return reinterpret_cast<T*>(b + x * uint32_t(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const T* elem_rx(const T* grid, size_t plane_bytes, int i, uint32_t row,
                                            uint32_t x) {
  const char* b = reinterpret_cast<const char*>(grid) + size_t(i) * plane_bytes + size_t(row) * sizeof(T);
  return reinterpret_cast<const T*>(b + x * uint32_t(sizeof(T)));
}

// Population element (i, off): a wave-uniform base of direction array i plus
// a 32-bit per-lane byte offset (one direction array is < 4 GiB), which maps
// onto the scalar-base + 32-bit-offset form of global loads and stores and
// keeps 64-bit address arithmetic out of the per-lane registers.
template <typename T>
__device__ __forceinline__ T* elem(T* grid, size_t plane_bytes, int i, uint32_t off) {
  char* b = reinterpret_cast<char*>(grid) + size_t(i) * plane_bytes;
  return reinterpret_cast<T*>(b + off * uint32_t(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const T* elem(const T* grid, size_t plane_bytes, int i, uint32_t off) {
  const char* b = reinterpret_cast<const char*>(grid) + size_t(i) * plane_bytes;
  return reinterpret_cast<const T*>(b + off * uint32_t(sizeof(T)));
}

// c_i . (x, y, z) without multiplications by the constant components (the
// -0.0 start folds away exactly under IEEE rules).
template <typename C>
__device__ __forceinline__ C cdot(int i, C x, C y, C z) {
  C r = C(-0.0);
  r = D3Q19::cx[i] > 0 ? r + x : (D3Q19::cx[i] < 0 ? r - x : r);
  r = D3Q19::cy[i] > 0 ? r + y : (D3Q19::cy[i] < 0 ? r - y : r);
  r = D3Q19::cz[i] > 0 ? r + z : (D3Q19::cz[i] < 0 ? r - z : r);
  return r;
}

// delta_rho = sum of the offsets, summed over opposite pairs first.  An
// offset is dominated by its first-order part w_i 3 c_i.u, which cancels in
// g_i + g_opp(i) (exactly when the two have opposite signs and are within a
// factor of two of each other), so the partial sums stay at the scale of
// delta_rho instead of that of the offsets.
template <typename C>
__device__ __forceinline__ C delta_rho(const C* f) {
  const C s1 = f[1] + f[2], s3 = f[3] + f[4], s5 = f[5] + f[6], s7 = f[7] + f[8],
          s9 = f[9] + f[10], s11 = f[11] + f[12], s13 = f[13] + f[14], s15 = f[15] + f[16],
          s17 = f[17] + f[18];
  return f[0] + ((((s1 + s3) + (s5 + s7)) + ((s9 + s11) + (s13 + s15))) + s17);
}

// Moments of an offset population set: delta_rho and j.
template <typename C>
__device__ __forceinline__ void moments(const C* f, C& drho, C& jx, C& jy, C& jz) {
  drho = delta_rho(f);
  jx = ((f[1] - f[2]) + (f[7] - f[8])) + ((f[9] - f[10]) + (f[11] - f[12])) + (f[13] - f[14]);
  jy = ((f[3] - f[4]) + (f[7] - f[8])) + ((f[10] - f[9]) + (f[15] - f[16])) + (f[17] - f[18]);
  jz = ((f[5] - f[6]) + (f[11] - f[12])) + ((f[14] - f[13]) + (f[15] - f[16])) + (f[18] - f[17]);
}

// u from j' = rho u and delta_rho without rounding rho = 1 + delta_rho:
// u = j' / (1 + drho) = j' - j' t,  t = drho / (1 + drho).  (Near rho = 1 a
// rounded rho carries an error that is a smooth function of the field and
// accumulates coherently; j' - j' t is accurate to the rounding of u.)
template <typename C>
__device__ __forceinline__ C inv_rho_factor(C drho) {
  return drho / (C(1) + drho);
}

// t = drho / (S + drho) for the step kernel.  FP32 uses the hardware
// reciprocal (1 ulp): t ~ drho is a small correction, so its relative error
// reaches u only at the level of drho * 2^-23.
__device__ __forceinline__ float step_t_factor(float drho, float S) {
  return drho * __builtin_amdgcn_rcpf(S + drho);
}
__device__ __forceinline__ double step_t_factor(double drho, double S) {
  return drho / (S + drho);
}

// Uniform constants of the fused step, computed once on the host in the
// compute precision.  Populations are handled in storage units g' = S g
// (S = 2^s for FP16 storage, 1 otherwise); every term below is linear in g'
// except u, which is formed unscaled, so the result equals the unscaled
// computation scaled by the exact power of two S.  Classes: 0 rest,
// 1 axis, 2 diagonal; pairs p = 0..8 are directions (2p+1, 2p+2) = (c, -c).
template <typename C>
struct StepK {
  C omega, om1;  // omega = 1/tau, 1 - omega
  C oW[3];       // omega W                 (equilibrium, delta_rho - 3/2 j.u part)
  C oc[3];       // omega c (exact)         (equilibrium, (c.j)(c.u) part)
  C a[3];        // a                       (equilibrium, c.j part; multiplied by omega)
  C S, invS;     // storage scale and its inverse
  C Fh[3];       // S F / 2                 (j' = j + F/2)
  C F[3];        // F                       (u.F)
  C K3W[3];      // 3 (1 - omega/2) W S     (Guo, -3 W u.F part)
  C Kq[9];       // (1 - omega/2) q (c.F) S (Guo, 9 W (c.u)(c.F) part)
  C Ka[9];       // (1 - omega/2) a (c.F) S (Guo, 3 W c.F part)
  C Kw[Q];       // 6 w_i (c_i.u_w) S      (moving-wall bounce-back term)
  int moving;    // moving-wall markers in use (marker choice of WALLS = 3)
};

// Fused multiply-add.  The product remainder fma(a, b, -fl(ab)) is exact in
// round-to-nearest binary floating point (Ogita, Rump & Oishi, SIAM J. Sci.
// Comput. 26, 2005).
template <typename C>
__device__ __forceinline__ C fmac(C a, C b, C c);
template <>
__device__ __forceinline__ float fmac<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fmac<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// BGK relaxation towards the Qian equilibrium with Guo forcing, in place, in
// offset form with rho never formed (j' = j + F/2 = rho u):
//   g^eq_i = W_i (drho - 3/2 j'.u) + c_i (c_i.j')(c_i.u) +- a_i (c_i.j')
//   S_i    = (1 - omega/2) [q_i (c_i.u)(c_i.F) - 3 W_i u.F +- a_i (c_i.F)]
//   g*_i   = (1 - omega) g_i + omega g^eq_i + S_i.
// The momentum-carrying term is omega * (a_i c_i.j') with the conservation-
// exact a_i, so the collision keeps sum g* c = j + F without a rounding bias
// from the constants.  `fon` is 1 (forced cell) or 0 (no-force cell).  INC:
// the incompressible equilibrium, u = j' (rho0 = 1).
//
// EXACT (FP32 arithmetic on FP32 storage): j' and the momentum-carrying term
// are carried as unevaluated sums hi + lo.  An error made in j' returns as
// omega times that error in the momentum of every step, and it is a smooth
// function of the smooth momentum field, so plain FP32 rounding of j' and of
// omega a_i (c_i.j') recurs coherently from step to step and grows linearly
// in time (8.7e-6 relative in u after 1000 steps of the porous 128^3 crop
// against 2.4e-7 with the compensation; rounding of the stores alone, FP64
// arithmetic, gives 7e-8).  j' and, for the diagonal directions, c_i.j' are
// summed in FP64 -- a difference of two FP32 populations is exact there
// unless their magnitudes differ by more than 2^29, and the sums carry 53
// bits -- and split into an FP32 head and the FP32 rounding of the exact
// remainder (FP64 additions and conversions issue at the FP32 rate on this
// GPU, so this costs fewer instructions than compensated FP32 sums).  The
// high part of the momentum term enters the fused multiply-add with
// (1 - omega) g_i, whose rounding depends on the population's own low bits;
// the low parts go in with the second-order terms.
template <typename C, bool FORCE, bool SCALED, bool INC, bool EXACT>
__device__ __forceinline__ void collide(C* f, const StepK<C>& k, C fon) {
  const C drho = delta_rho(f);
  C jx, jy, jz, lx = C(0), ly = C(0), lz = C(0);
  double Jx = 0, Jy = 0, Jz = 0;
  if (EXACT) {
    // j' in FP64, then head + tail: the FP32 rounding of J and the FP32
    // rounding of the exact remainder J - head.
    double d[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) d[p] = double(f[2 * p + 1]) - double(f[2 * p + 2]);
    Jx = (((d[0] + d[3]) + (d[4] + d[5])) + d[6]);
    Jy = (((d[1] + d[3]) - (d[4] - d[7])) + d[8]);
    Jz = (((d[2] + d[5]) - (d[6] - d[7])) - d[8]);
    if (FORCE) {
      Jx += double(fon * k.Fh[0]);
      Jy += double(fon * k.Fh[1]);
      Jz += double(fon * k.Fh[2]);
    }
    jx = C(Jx);
    jy = C(Jy);
    jz = C(Jz);
    lx = C(Jx - double(jx));
    ly = C(Jy - double(jy));
    lz = C(Jz - double(jz));
  } else {
    const C d1 = f[1] - f[2], d3 = f[3] - f[4], d5 = f[5] - f[6], d7 = f[7] - f[8],
            d9 = f[9] - f[10], d11 = f[11] - f[12], d13 = f[13] - f[14], d15 = f[15] - f[16],
            d17 = f[17] - f[18];
    jx = ((d1 + d7) + (d9 + d11)) + d13;
    jy = ((d3 + d7) - (d9 - d15)) + d17;
    jz = ((d5 + d11) - (d13 - d15)) - d17;
    if (FORCE) {
      jx += fon * k.Fh[0];
      jy += fon * k.Fh[1];
      jz += fon * k.Fh[2];
    }
  }
  C ux = jx, uy = jy, uz = jz;
  if (!INC) {
    const C t = step_t_factor(drho, SCALED ? k.S : C(1));
    ux = jx - jx * t;
    uy = jy - jy * t;
    uz = jz - jz * t;
  }
  if (SCALED) {
    ux *= k.invS;
    uy *= k.invS;
    uz *= k.invS;
  }
  const C base = drho - C(1.5) * (jx * ux + jy * uy + jz * uz);
  C uF = C(0);
  if (FORCE) uF = fon * (ux * k.F[0] + uy * k.F[1] + uz * k.F[2]);
  C oWb[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) oWb[c] = FORCE ? k.oW[c] * base - k.K3W[c] * uF : k.oW[c] * base;
  f[0] = k.om1 * f[0] + oWb[0];
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    const int i = 2 * p + 1, c = speed_class(i);
    const C eu = cdot<C>(i, ux, uy, uz);
    if (EXACT) {
      C ej, el;
      if (D3Q19::cx[i] != 0 && D3Q19::cy[i] != 0) {
        const double J = (D3Q19::cx[i] > 0 ? Jx : -Jx) + (D3Q19::cy[i] > 0 ? Jy : -Jy);
        ej = C(J);
        el = C(J - double(ej));
      } else if (D3Q19::cx[i] != 0 && D3Q19::cz[i] != 0) {
        const double J = (D3Q19::cx[i] > 0 ? Jx : -Jx) + (D3Q19::cz[i] > 0 ? Jz : -Jz);
        ej = C(J);
        el = C(J - double(ej));
      } else if (D3Q19::cy[i] != 0 && D3Q19::cz[i] != 0) {
        const double J = (D3Q19::cy[i] > 0 ? Jy : -Jy) + (D3Q19::cz[i] > 0 ? Jz : -Jz);
        ej = C(J);
        el = C(J - double(ej));
      } else {
        ej = cdot<C>(i, jx, jy, jz);
        el = cdot<C>(i, lx, ly, lz);
      }
      C sym = k.oc[c] * (ej * eu) + oWb[c];
      // omega a ej = hi + lo: two rounded products and their exact remainders
      const C p1 = k.a[c] * ej;
      const C hi = k.omega * p1;
      C lo = fmac(k.omega, fmac(k.a[c], ej, -p1), fmac(k.omega, p1, -hi));
      lo += k.omega * (k.a[c] * el);
      if (FORCE) {
        sym += k.Kq[p] * (fon * eu);
        lo += fon * k.Ka[p];
      }
      const C lp = sym + lo, lm = sym - lo;
      f[i] = fmac(k.om1, f[i], hi) + lp;
      f[i + 1] = fmac(k.om1, f[i + 1], -hi) + lm;
    } else {
      const C ej = cdot<C>(i, jx, jy, jz);
      C sym = k.oc[c] * (ej * eu) + oWb[c];
      C anti = k.omega * (k.a[c] * ej);
      if (FORCE) {
        sym += k.Kq[p] * (fon * eu);
        anti += fon * k.Ka[p];
      }
      f[i] = k.om1 * f[i] + (sym + anti);
      f[i + 1] = k.om1 * f[i + 1] + (sym - anti);
    }
  }
}

// ---------------------------------------------------------------------------
// Fused stream-collide step.
//
// Half-way bounce-back through solid markers: every slot of a solid cell
// holds a quiet NaN, rewritten by the solid cell's own lane each step.  Each
// lane pulls x - c_i for all i unconditionally; a pull that lands on a solid
// cell returns the marker, and only then does the lane load the half-way
// bounce-back value f*_opp(i)(x) from its own cell.  So no population load
// waits for geometry, and every lane -- fluid or solid -- stores all 19 of
// its own slots, which keeps every store instruction a full, coalesced line
// (partially written lines cost far more HBM time than their bytes).  The
// flags are read only for the solid test and the per-cell force switch.
//
// WALLS: 0 = no solid cells, 1 = solid cells at rest, 2 = moving walls as
// well.  In the last case a moving-wall cell's marker is +infinity instead
// of NaN, and a bounced-back value whose pull returned infinity gains the
// wall term 6 w_i (c_i.u_w) -- the moving wall costs nothing away from it.
// WALLS = 3 is the paper's split design (non-fluid cells treated in a
// separate kernel, Sec. 7): k_obstacle has already written the bounce-back
// values into the solid cells' slots of src, so the step pulls with no
// marker test at all; flags still give the solid and no-force bits.
// WALLS = 4 is the pull-copy probe: the same loads and stores with neither
// geometry nor collision, f_i(x) <- f_i(x - c_i) on a periodic box -- the
// speed this memory pattern itself allows.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void stream_store(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// Pins a collision result as a rounded FP32 register value before its FP16
// store conversion.  Without it the compiler may fold the last fused
// multiply-add and the conversion into one mixed-precision instruction that
// rounds once, straight to FP16 -- in some kernel variants and not in
// others, so that variants differ in the last bit; with it every FP16 store
// is the FP32 result rounded to nearest even, as in the other storages.
__device__ __forceinline__ float fp32_result(float v) {
  asm volatile("" : "+v"(v));
  return v;
}

// A pulled element is a solid marker when its raw bits are one of the two
// marker patterns (WALLS = 2) or the resting one (WALLS = 1); any other
// value -- a NaN or infinity that arose in a fluid cell included -- is data.
template <int K, int WALLS>
__device__ __forceinline__ bool is_marker(typename Storage<K>::U r) {
  if (WALLS == 2) return (r | 1u) == Storage<K>::kMoving;  // kMoving = kRest | 1
  return r == Storage<K>::kRest;
}

// Cells per lane of the step kernel: a wave owns a run of 64*M cells of one
// row and each lane updates the cells x0 + 64 m, m < M.  More cells
// per lane put more bytes in flight per wave, which is what the 16-bit
// storages need to cover memory latency at the occupancy limit.
template <int K>
struct StepCells {
  static constexpr int M = (K == ST_F16 || K == ST_BF16) ? 4 : 1;
};

template <int K, int WALLS, bool FORCE, bool INC, int M>
__global__ __launch_bounds__(kBlock) void k_step(const typename Storage<K>::T* __restrict__ src,
                                                 typename Storage<K>::T* __restrict__ dst,
                                                 const uint8_t* __restrict__ flags, Geo g,
                                                 StepK<typename Storage<K>::C> k) {
  using C = typename Storage<K>::C;
  using T = typename Storage<K>::T;
  constexpr bool SCALED = (K == ST_F16);
  constexpr bool SOLIDS = WALLS >= 1 && WALLS <= 3;
  constexpr bool MARKERS = WALLS == 1 || WALLS == 2;
  constexpr bool COPY = WALLS == 4;
  // g describes 64*M-cell segments (step_geo); same block remap as locate().
  const int b = blockIdx.x;
  const int lb = (b < g.nb8) ? ((b & 7) * (g.nb8 >> 3) + (b >> 3)) : b;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int seg = lb * 4 + wave;
  const int row = seg / g.nseg;
  if (row >= g.nrows) return;
  // Rows are visited in bands of yb consecutive y; inside a band y runs
  // fastest, then z.  The rows y - 1 and y + 1 of a row are then processed
  // by neighbouring waves and the rows z - 1 and z + 1 yb rows (a few dozen
  // blocks) away, so a bounce-back reload of f*_opp(i)(x) finds in L2 the
  // line that the solid neighbour's lane pulled (or brings it in for that
  // lane).
  Loc l;
  {
    const int per_band = g.nz * g.yb;
    const int band = row / per_band;
    const int y0 = band * g.yb;
    const int h = min(g.yb, g.ny - y0);
    const int idx = row - band * per_band;
    l.z = idx / h;
    l.y = y0 + (idx - l.z * h);
  }
  const int x0 = (seg - row * g.nseg) * 64 * M + int(threadIdx.x & 63);
  Nbhd n[M];
  bool valid[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int x = x0 + 64 * m;
    valid[m] = x < g.nx;
    l.x = valid[m] ? x : g.nx - 1;  // past the row end: load in bounds, store nothing
    n[m] = neighbourhood(g, l);
  }
  if (!valid[0]) return;
  uint8_t fl[M];
#pragma unroll
  for (int m = 0; m < M; ++m) fl[m] = SOLIDS ? flags[n[m].fown] : uint8_t(0);
  const size_t pb = size_t(g.plane) * sizeof(T);
  C f[M][Q];
  bool mark[M][Q];  // the pull returned a solid marker (raw-bit test at the load)
  bool mov[M][Q];   // ... the moving-wall marker
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T v = *elem_rx(src, pb, i, src_row(n[m], i), src_x(n[m], i));
      mark[m][i] = MARKERS && i != 0 && is_marker<K, WALLS>(raw_bits<K>(v));
      mov[m][i] = WALLS == 2 && i != 0 && raw_bits<K>(v) == Storage<K>::kMoving;
      f[m][i] = C(v);
    }
  bool solid[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    solid[m] = SOLIDS && (fl[m] & FLAG_SOLID);
    if (MARKERS) {
#pragma unroll
      for (int i = 1; i < Q; ++i)
        if (mark[m][i] && !solid[m]) {
          C b = C(*elem_rx(src, pb, D3Q19::opp[i], n[m].row[1][1], n[m].xn[1]));
          if (WALLS == 2 && mov[m][i]) b += k.Kw[i];
          f[m][i] = b;
        }
    }
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    // Solid lanes run the collision on their (meaningless) pulls and discard it.
    if (COPY) {
    } else if (FORCE && SOLIDS) {
      collide<C, FORCE, SCALED, INC, K == ST_F32>(f[m], k, (fl[m] & FLAG_NOFORCE) ? C(0) : C(1));
    } else {
      collide<C, FORCE, SCALED, INC, K == ST_F32>(f[m], k, C(1));
    }
    const T marker = solid_marker<K>(fl[m], WALLS == 2 || (WALLS == 3 && k.moving));
    if (valid[m]) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        C out = f[m][i];
        if constexpr (K == ST_F16) out = fp32_result(out);
        stream_store(elem_rx(dst, pb, i, n[m].row[1][1], n[m].xn[1]), solid[m] ? marker : T(out));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Two fused steps per pass (temporal blocking over z): f*(t) -> f*(t+2).
//
// A block owns an output tile of 64 x TY cells in (x, y) and walks a chunk
// of z planes.  Step 1 computes the intermediate level f*(t+1) on the tile
// and its one-cell halo ((64 + 2) x (TY + 2) cells) of plane p, pulling from
// src exactly as the single-step kernel does; step 2 computes f*(t+2) on the
// tile at plane p - 1 from the intermediate level, which never leaves the
// chip.  The 16 populations that move in x or y go through a ring of LDS
// plane-arrays over the halo-extended tile, each value stored at the cell
// that pulls it (A_i[x + c_i] = f*_i(x)): a step-2 read of direction i is
// A_i at the cell's own index.  The own cell's intermediate values, which a
// step-2 bounce-back needs, are the thread's own step-1 results of the
// previous plane and stay in its registers (an LDS read there would wait
// behind the marker test of the pulled value); so do the three populations
// that do not move in x or y (0 and the pure-z pair).  The ring holds as
// many planes of a direction as are live: step 2 at plane p - 1 reads
// direction i at plane p - 1 - c_z, so c_z = +1 is read two planes after it
// was written (3 slots), c_z = 0 one plane after (2 slots) and c_z = -1 in
// the same iteration (1 slot); two barriers per plane separate writes from
// reads.  The next plane's 19 pulls are issued before the first barrier,
// so their latency hides behind step 2.  Both steps run the single-step
// kernel's pull, bounce-back (the marker test, or the link mask at resting
// walls: WALLS = 4 below), collision and rounding, and the intermediate
// values are rounded to the storage type, so a pass equals two single steps
// bit for bit.  Threads: TY + 2 waves, one per extended row (lane = x), plus
// one wave for the 2 (TY + 2) halo cells left and right of the tile.  HBM
// traffic per pass: one read of f*(t) (plus the halo lines that miss in L2)
// and one write of f*(t+2) -- about half of two single steps.
// ---------------------------------------------------------------------------
constexpr int kTB2Arrays = 32;  // LDS plane-arrays of [TY + 2][66]
// link-mask bits besides the 18 links (bit i: the pull along c_i is blocked)
constexpr uint32_t kLinkSolid = 1u << 19;
constexpr uint32_t kLinkNoforce = 1u << 20;
// All ones when bit i of m is set, else 0 (one sign-extending bit extract).
__device__ __forceinline__ uint32_t link_sel(uint32_t m, int i) {
  return uint32_t(__builtin_amdgcn_sbfe(int32_t(m), i, 1));
}
// sel ? a : b for sel all ones or 0: one bitfield select per dword (written
// as an instruction: the compiler turns the bit operations back into a
// compare and a conditional move, two instructions more).
__device__ __forceinline__ uint32_t bfi32(uint32_t sel, uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(sel), "v"(a), "v"(b));
  return r;
}
template <typename U>
__device__ __forceinline__ U pick(uint32_t sel, U a, U b) {
  if constexpr (sizeof(U) == 8) {
    const uint32_t lo = bfi32(sel, uint32_t(a), uint32_t(b));
    const uint32_t hi = bfi32(sel, uint32_t(a >> 32), uint32_t(b >> 32));
    return (U(hi) << 32) | U(lo);
  } else {
    return U(bfi32(sel, uint32_t(a), uint32_t(b)));
  }
}
constexpr int kTB2Chunk = 128;     // longest z chunk (planes per block)
constexpr int kTB2MinChunk = 16;   // shortest z chunk
constexpr int kTB2MinBlocks = 1280;  // five blocks per CU on 256 CUs

// Tile rows per block: 13 (16 waves, 1024 threads, one block per CU: the
// FP32 ring takes 127 KB of LDS) for 4- and 2-byte storage, which fit 128
// VGPRs without spills; measured at 512^3, 13 rows beat 12, 8, 6 and 5.
// FP64 storage takes 5 (118 KB of LDS; 6 rows cap the 9 waves at 168
// VGPRs, spill and ran 0.7% slower), and F32X (FP64 arithmetic) 8, whose 11
// waves may use 168 VGPRs.
template <int K>
__host__ __device__ constexpr int tb2_rows() {
  return K == ST_F64 ? 5 : (K == ST_F32X ? 8 : 13);
}
__host__ __device__ constexpr int tb2_nslot(int i) {
  return D3Q19::cz[i] > 0 ? 3 : (D3Q19::cz[i] == 0 ? 2 : 1);
}
// first plane-array of direction i (the 16 directions with c_x or c_y != 0)
__host__ __device__ constexpr int tb2_base(int i) {
  int b = 0;
  for (int j = 1; j < i; ++j)
    if (D3Q19::cx[j] != 0 || D3Q19::cy[j] != 0) b += tb2_nslot(j);
  return b;
}
static_assert(tb2_base(Q) == kTB2Arrays, "ring plane-arrays");

__device__ __forceinline__ int wrap_mod(int v, int n) {
  const int r = v % n;
  return r < 0 ? r + n : r;
}

// An opaque copy of a wave-uniform 64-bit value: an empty asm statement on a
// scalar register pair, kept in place.  The two-step kernel walks the 19
// direction arrays with a running base address renewed on every plane
// through such copies; left to itself the compiler hoists all 19 source and
// 19 destination bases out of the plane loop, they overflow the scalar
// register file, and every use reloads them from spill lanes with vector
// instructions.
__device__ __forceinline__ uint64_t uniform_opaque(uint64_t v) {
  asm volatile("" : "+s"(v));
  return v;
}
// An opaque copy of a per-lane 32-bit value: an LDS ring address is one such
// base per plane phase plus a compile-time offset, which the LDS instruction
// takes as its immediate.
__device__ __forceinline__ uint32_t lane_opaque(uint32_t v) {
  asm("" : "+v"(v));
  return v;
}
// The same for a value used in several conditional blocks: a fresh copy in
// each block keeps the compiler from sharing one 64-bit widened offset
// between the blocks, which would rule out the scalar-base load form.
__device__ __forceinline__ uint32_t lane_fresh(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}
// Element at `base` (a wave-uniform global address) + `off` bytes (per
// lane): the scalar-base + 32-bit-offset form of global loads and stores
// (the pointer is made in the global address space, else the compiler can
// only emit flat accesses with 64-bit per-lane addresses).
template <typename T>
__device__ __forceinline__ T load_at(uint64_t base, uint32_t off) {
  return *reinterpret_cast<const __attribute__((address_space(1))) T*>(base + off);
}
template <typename T>
__device__ __forceinline__ void store_nt_at(uint64_t base, uint32_t off, T v) {
  __builtin_nontemporal_store(v, reinterpret_cast<__attribute__((address_space(1))) T*>(base + off));
}

// MID: the intermediate level f*(t+1) is stored as well, into `mid` (each
// cell by the block whose tile and chunk own it), for callers that need every
// state -- the adjoint's recomputation between checkpoints.
//
// WALLS = 4 here (resting walls, with the link mask; in the single-step
// kernel 4 is the pull-copy probe): the solid neighbours of a
// cell are known from its mask before its pulls are issued, so each pull
// reads the population it needs -- the neighbour's f*_i, or for a blocked
// link the own cell's f*_opp(i) -- in one load, with no marker test and no
// dependent reload; step 2 takes the own cell's value for a blocked link by
// its mask bit.  The same values reach the collision as with the markers,
// so the results are the same bits.  The mask of a plane is loaded two
// planes ahead.
template <int K, int WALLS, bool FORCE, bool INC, bool MID>
__global__ __launch_bounds__(64 * (tb2_rows<K>() + 3)) void k_step2(
    const typename Storage<K>::T* __restrict__ src, typename Storage<K>::T* __restrict__ mid,
    typename Storage<K>::T* __restrict__ dst, const uint8_t* __restrict__ flags,
    const uint32_t* __restrict__ lmask, Geo2 g, StepK<typename Storage<K>::C> k) {
  using C = typename Storage<K>::C;
  using T = typename Storage<K>::T;
  constexpr int TY = tb2_rows<K>(), TX = 64, EX = TX + 2, EY = TY + 2;
  constexpr uint32_t SZ = sizeof(T);
  constexpr uint32_t PLB = uint32_t(EY * EX) * SZ;  // bytes of one LDS plane-array
  constexpr bool SOLIDS = WALLS >= 1;
  constexpr bool LINKS = WALLS == 4;
  constexpr bool MARKERS = SOLIDS && !LINKS;
  static_assert(sizeof(T) * kTB2Arrays * EY * EX <= 160 * 1024, "ring exceeds the LDS of a CU");
  __shared__ T ring[kTB2Arrays * EY * EX];
  // block -> tile: x tiles fastest, then y tiles, then z chunks; XCD k gets
  // the k-th contiguous eighth of that order
  const int b = blockIdx.x;
  const int lb = (b < g.nb8) ? ((b & 7) * (g.nb8 >> 3) + (b >> 3)) : b;
  const int x0 = (lb % g.ntx) * TX;
  const int y0 = ((lb / g.ntx) % g.nty) * TY;
  const int z0 = (lb / (g.ntx * g.nty)) * g.zc;
  const int zend = min(z0 + g.zc, g.nz);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = int(threadIdx.x & 63);
  // this thread's step-1 cell (ex, ey), tile coordinates; ex in [-1, 64], ey in [-1, TY]
  int ex = lane, ey = wave - 1;
  if (wave == TY + 2) {  // the halo columns x0 - 1 and x0 + 64 of every extended row
    ey = lane < 2 * EY ? (lane >> 1) - 1 : TY;  // lanes past the halo repeat a halo cell
    ex = (lane & 1) ? TX : -1;
  }
  const int gx = wrap_mod(x0 + ex, g.nx), gy = wrap_mod(y0 + ey, g.ny);
  const bool interior = wave >= 1 && wave <= TY;  // also computes step 2 at (ex, ey)
  const bool out_ok = interior && x0 + ex < g.nx && y0 + ey < g.ny;
  // Byte offsets inside one direction array (< 4 GiB, checked on the host):
  // pull columns x - c_x and rows y - c_y at index c + 1 ({x + 1, x, x - 1}),
  // periodic, and the stride of one z plane.
  const uint32_t rowb = uint32_t(g.xs) * SZ;
  const uint32_t xb_[3] = {uint32_t(gx + 1 == g.nx ? 0 : gx + 1) * SZ, uint32_t(gx) * SZ,
                           uint32_t(gx == 0 ? g.nx - 1 : gx - 1) * SZ};
  const uint32_t yb_[3] = {uint32_t(gy + 1 == g.ny ? 0 : gy + 1) * rowb, uint32_t(gy) * rowb,
                           uint32_t(gy == 0 ? g.ny - 1 : gy - 1) * rowb};
  const uint32_t zstride = uint32_t(g.ny) * rowb;
  const uint32_t own_yx = yb_[1] + xb_[1];
  const uint32_t fl_yx = uint32_t(gy) * uint32_t(g.nx) + uint32_t(gx);
  const uint32_t fl_z = uint32_t(g.ny) * uint32_t(g.nx);
  const uint64_t src_u = reinterpret_cast<uint64_t>(src), dst_u = reinterpret_cast<uint64_t>(dst);
  const uint64_t pb = uint64_t(g.plane) * SZ;  // bytes from one direction array to the next
  // LDS ring: this lane's cell of the extended tile in plane-array 0; the
  // element of direction i in its array for plane phase m, (dy, dx) cells
  // away, sits at lane_b + m PLB + [tb2_base(i) PLB + (dy EX + dx) SZ], the
  // bracket a compile-time constant.
  const uint32_t lane_b = uint32_t((ey + 1) * EX + ex + 1) * SZ;
  auto ring_at = [&](uint32_t base, int i, int dy, int dx) -> T& {
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(ring) + base +
                                 (uint32_t(tb2_base(i)) * PLB + uint32_t((dy * EX + dx) * int(SZ))));
  };
  auto phase_base = [&](int p, int ns) { return lane_opaque(lane_b + uint32_t(wrap_mod(p, ns)) * PLB); };
  // the next plane's pulls and flag byte, issued one iteration ahead
  T nv[Q];
  uint8_t nfl = 0;
  // LINKS: the masks of planes p (m0, its pulls in flight), p + 1 (m1) and
  // p + 2 (m2, loading)
  uint32_t m0 = 0, m1 = 0, m2 = 0;
  auto mask_at = [&](int p) { return lmask[uint32_t(wrap_mod(p, g.nz)) * fl_z + fl_yx]; };
  auto issue = [&](int p) {
    const int pz = wrap_mod(p, g.nz);
    const uint32_t zb_[3] = {uint32_t(pz + 1 == g.nz ? 0 : pz + 1) * zstride, uint32_t(pz) * zstride,
                             uint32_t(pz == 0 ? g.nz - 1 : pz - 1) * zstride};
    uint64_t base = uniform_opaque(src_u);
    if constexpr (LINKS) {
      // pairs (i, i + 1) = (c, -c) from the base of array i: a blocked i
      // reads f*_{i+1} of the own cell (pb further), a blocked i + 1 reads
      // f*_i of the own cell (offsets < 4 GiB: two arrays of at most 2 GiB,
      // checked on the host)
      const uint32_t m = m1;
      const uint32_t own = zb_[1] + own_yx, pb32 = uint32_t(pb);
      nv[0] = load_at<T>(base, own);
      base = uniform_opaque(base + pb);
#pragma unroll
      for (int i = 1; i < Q; i += 2) {
        const uint32_t ni = zb_[1 + D3Q19::cz[i]] + yb_[1 + D3Q19::cy[i]] + xb_[1 + D3Q19::cx[i]];
        const uint32_t nj =
            zb_[1 + D3Q19::cz[i + 1]] + yb_[1 + D3Q19::cy[i + 1]] + xb_[1 + D3Q19::cx[i + 1]];
        nv[i] = load_at<T>(base, pick(link_sel(m, i), pb32 + own, ni));
        nv[i + 1] = load_at<T>(base, pick(link_sel(m, i + 1), own, pb32 + nj));
        if (i + 2 < Q) base = uniform_opaque(base + 2 * pb);
      }
      m2 = mask_at(p + 1);
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        nv[i] = load_at<T>(base, zb_[1 + D3Q19::cz[i]] + yb_[1 + D3Q19::cy[i]] +
                                     xb_[1 + D3Q19::cx[i]]);
        if (i + 1 < Q) base = uniform_opaque(base + pb);
      }
      nfl = SOLIDS ? flags[uint32_t(pz) * fl_z + fl_yx] : uint8_t(0);
    }
  };
  // own column's step-1 results: planes p - 1 (prev) and p - 2 (pp5)
  T prevv[Q], pp5 = T(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) prevv[i] = T(0);
  uint8_t fl_prev = 0;
  uint32_t m_prev = 0;
  if constexpr (LINKS) m1 = mask_at(z0 - 1);
  issue(z0 - 1);
  for (int p = z0 - 1; p <= zend; ++p) {
    // ---- step 1 at (gx, gy, p): the single-step kernel's update ----
    const uint32_t ownb = uint32_t(wrap_mod(p, g.nz)) * zstride + own_yx;
    if constexpr (LINKS) {
      m0 = m1;
      m1 = m2;
    }
    const uint8_t fl = LINKS ? uint8_t((m0 & kLinkSolid ? FLAG_SOLID : 0) |
                                       (m0 & kLinkNoforce ? FLAG_NOFORCE : 0))
                             : nfl;
    const bool solid = SOLIDS && (fl & FLAG_SOLID);
    C f[Q];
    bool mark[Q], mov[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      mark[i] = MARKERS && i != 0 && is_marker<K, WALLS>(raw_bits<K>(nv[i]));
      mov[i] = WALLS == 2 && i != 0 && raw_bits<K>(nv[i]) == Storage<K>::kMoving;
      f[i] = C(nv[i]);
    }
    if (MARKERS) {
      // pairs (i, i + 1) = (c, -c): each bounces back the other's slot of the own cell
      uint64_t base = uniform_opaque(src_u + pb);
#pragma unroll
      for (int i = 1; i < Q; i += 2) {
        const uint64_t bo = base + pb;
        if (mark[i] && !solid) {
          C bb = C(load_at<T>(bo, lane_fresh(ownb)));
          if (WALLS == 2 && mov[i]) bb += k.Kw[i];
          f[i] = bb;
        }
        if (mark[i + 1] && !solid) {
          C bb = C(load_at<T>(base, lane_fresh(ownb)));
          if (WALLS == 2 && mov[i + 1]) bb += k.Kw[i + 1];
          f[i + 1] = bb;
        }
        if (i + 2 < Q) base = uniform_opaque(bo + pb);
      }
    }
    if (FORCE && SOLIDS)
      collide<C, FORCE, K == ST_F16, INC, K == ST_F32>(f, k, (fl & FLAG_NOFORCE) ? C(0) : C(1));
    else
      collide<C, FORCE, K == ST_F16, INC, K == ST_F32>(f, k, C(1));
    const T marker = solid_marker<K>(fl, WALLS == 2);
    const uint32_t w1 = lane_opaque(lane_b), w2 = phase_base(p, 2), w3 = phase_base(p, 3);
    T cur[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      C o = f[i];
      if constexpr (K == ST_F16) o = fp32_result(o);
      const T v = solid ? marker : T(o);
      cur[i] = v;
      if (i != 0 && i != 5 && i != 6) {
        const int tx = ex + D3Q19::cx[i], ty = ey + D3Q19::cy[i];
        if (tx >= -1 && tx <= TX && ty >= -1 && ty <= TY)
          ring_at(tb2_nslot(i) == 3 ? w3 : (tb2_nslot(i) == 2 ? w2 : w1), i, D3Q19::cy[i],
                  D3Q19::cx[i]) = v;
      }
    }
    if constexpr (MID) {
      if (out_ok && p >= z0 && p < zend) {
        uint64_t base = uniform_opaque(reinterpret_cast<uint64_t>(mid));
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          store_nt_at<T>(base, ownb, cur[i]);
          if (i + 1 < Q) base = uniform_opaque(base + pb);
        }
      }
    }
    if (p < zend) issue(p + 1);
    __syncthreads();
    // ---- step 2 at (gx, gy, q = p - 1) from the intermediate level ----
    const int q = p - 1;
    if (interior && q >= z0) {
      const uint32_t qownb = uint32_t(wrap_mod(q, g.nz)) * zstride + own_yx;
      const bool solid2 = SOLIDS && (fl_prev & FLAG_SOLID);
      const uint32_t m_step2 = solid2 ? 0u : m_prev;  // LINKS: the links step 2 bounces back
      // plane q - c_z of direction i: p - 2 (c_z = +1, 3 slots), p - 1, p
      const uint32_t r3 = phase_base(p - 2, 3), r2 = phase_base(q, 2);
      C h[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        T w;
        if (i == 0) w = prevv[0];
        else if (i == 5) w = pp5;
        else if (i == 6) w = cur[6];
        else w = ring_at(D3Q19::cz[i] > 0 ? r3 : (D3Q19::cz[i] == 0 ? r2 : w1), i, 0, 0);
        h[i] = C(w);
        if (MARKERS && i != 0 && is_marker<K, WALLS>(raw_bits<K>(w)) && !solid2) {
          // half-way bounce-back: the own cell's opposite population at plane q
          C bb = C(prevv[D3Q19::opp[i]]);  // this thread's own step-1 output at plane q
          if (WALLS == 2 && raw_bits<K>(w) == Storage<K>::kMoving) bb += k.Kw[i];
          h[i] = bb;
        }
        if (LINKS && i != 0)  // blocked link: the own cell's opposite population at plane q
          h[i] = C(from_bits<K>(pick<typename Storage<K>::U>(
              link_sel(m_step2, i), raw_bits<K>(prevv[D3Q19::opp[i]]), raw_bits<K>(w))));
      }
      if (FORCE && SOLIDS)
        collide<C, FORCE, K == ST_F16, INC, K == ST_F32>(h, k, (fl_prev & FLAG_NOFORCE) ? C(0) : C(1));
      else
        collide<C, FORCE, K == ST_F16, INC, K == ST_F32>(h, k, C(1));
      const T marker2 = solid_marker<K>(fl_prev, WALLS == 2);
      if (out_ok) {
        uint64_t base = uniform_opaque(dst_u);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          C o = h[i];
          if constexpr (K == ST_F16) o = fp32_result(o);
          store_nt_at<T>(base, qownb, solid2 ? marker2 : T(o));
          if (i + 1 < Q) base = uniform_opaque(base + pb);
        }
      }
    }
    __syncthreads();
    pp5 = prevv[5];
#pragma unroll
    for (int i = 0; i < Q; ++i) prevv[i] = cur[i];
    fl_prev = fl;
    m_prev = m0;
  }
}

// The link mask of every cell for the two-step kernel's resting walls: bit i
// (1..18) set when the pull along c_i is blocked (x - c_i solid, periodic),
// plus the cell's own SOLID and NOFORCE flags.
__global__ __launch_bounds__(kBlock) void k_link_mask(const uint8_t* __restrict__ flags,
                                                      uint32_t* __restrict__ mask, Geo g) {
  const size_t n = size_t(g.nx) * g.ny * g.nz;
  const size_t idx = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (idx >= n) return;
  const int x = int(idx % uint32_t(g.nx));
  const size_t r = idx / uint32_t(g.nx);
  const int y = int(r % uint32_t(g.ny)), z = int(r / uint32_t(g.ny));
  const uint8_t fl = flags[idx];
  uint32_t m = (fl & FLAG_SOLID ? kLinkSolid : 0u) | (fl & FLAG_NOFORCE ? kLinkNoforce : 0u);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int xs = wrap_mod(x - D3Q19::cx[i], g.nx), ys = wrap_mod(y - D3Q19::cy[i], g.ny),
              zs = wrap_mod(z - D3Q19::cz[i], g.nz);
    if (flags[(size_t(zs) * g.ny + ys) * g.nx + xs] & FLAG_SOLID) m |= 1u << i;
  }
  mask[idx] = m;
}

// The separate obstacle kernel of the split design (WALLS = 3 steps): every
// solid cell s writes, into its slot i, the value the fluid neighbour
// x = s + c_i will pull along c_i: f*_opp(i)(x), plus the moving-wall term
// for a moving wall.  Each written slot has exactly one writer and no
// written slot is read by this kernel, so it runs in place on the source
// grid of the following step.
template <int K>
__global__ __launch_bounds__(kBlock) void k_obstacle(typename Storage<K>::T* __restrict__ grid,
                                                     const uint8_t* __restrict__ flags, Geo g,
                                                     Phys<typename Storage<K>::C> ph) {
  using T = typename Storage<K>::T;
  using C = typename Storage<K>::C;
  const Loc l = locate(g);
  if (!l.valid) return;
  const Nbhd n = neighbourhood(g, l);
  const uint8_t fl = flags[n.fown];
  if (!(fl & FLAG_SOLID)) return;
  const bool mv = ph.moving && (fl & FLAG_MOVING);
  const size_t pb = size_t(g.plane) * sizeof(T);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int o = D3Q19::opp[i];
    // s - c_o = s + c_i is the fluid neighbour that pulls slot i of s
    if (flags[src_foff(n, o)] & FLAG_SOLID) continue;
    C v = C(*elem(grid, pb, o, src_off(n, o)));
    if (mv) v += ph.Kw[i] * ph.scale;
    *elem(grid, pb, i, n.own) = T(v);
  }
}

// Writes the solid marker into every slot of the solid cells of a grid.
template <int K>
__global__ __launch_bounds__(kBlock) void k_mark_solids(typename Storage<K>::T* __restrict__ grid,
                                                        const uint8_t* __restrict__ flags, Geo g,
                                                        int moving) {
  using T = typename Storage<K>::T;
  const Loc l = locate(g);
  if (!l.valid) return;
  const Nbhd n = neighbourhood(g, l);
  const uint8_t fl = flags[n.fown];
  if (!(fl & FLAG_SOLID)) return;
  const size_t pb = size_t(g.plane) * sizeof(T);
  const T marker = solid_marker<K>(fl, moving != 0);
#pragma unroll
  for (int i = 0; i < Q; ++i) *elem(grid, pb, i, n.own) = marker;
}

// ---------------------------------------------------------------------------
// Initial state f*(0) = f^eq(rho0, u0), written as offsets.
// ---------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(kBlock) void k_init(typename Storage<K>::T* __restrict__ grid,
                                                 const uint8_t* __restrict__ flags,
                                                 const float* __restrict__ rho0,
                                                 const float* __restrict__ u0, Geo g,
                                                 Phys<typename Storage<K>::C> ph) {
  using C = typename Storage<K>::C;
  using T = typename Storage<K>::T;
  const Loc l = locate(g);
  if (!l.valid) return;
  const Nbhd n = neighbourhood(g, l);
  const uint32_t c = n.fown;
  const size_t pb = size_t(g.plane) * sizeof(T);
  if (flags && (flags[c] & FLAG_SOLID)) {  // solid marker
    const T marker = solid_marker<K>(flags[c], ph.moving != 0);
#pragma unroll
    for (int i = 0; i < Q; ++i) *elem(grid, pb, i, n.own) = marker;
    return;
  }
  const size_t ncell = size_t(g.nx) * g.ny * g.nz;
  const C rho = rho0 ? C(rho0[c]) : C(1);
  C ux = C(0), uy = C(0), uz = C(0);
  if (u0) {
    ux = C(u0[c]);
    uy = C(u0[ncell + c]);
    uz = C(u0[2 * ncell + c]);
  }
  // f^eq(rho0, u0) - w in the collision's coefficient form, j' = rho0 u0
  // (j' = u0 for the incompressible equilibrium).
  const C drho = rho - C(1);
  const C jx = ph.incomp ? ux : rho * ux, jy = ph.incomp ? uy : rho * uy,
          jz = ph.incomp ? uz : rho * uz;
  const C base = drho - C(1.5) * (jx * ux + jy * uy + jz * uz);
  C f[Q];
  f[0] = coef_W<C>(0) * base;
#pragma unroll
  for (int k = 1; k < Q; k += 2) {
    const C ej = cdot<C>(k, jx, jy, jz);
    const C eu = cdot<C>(k, ux, uy, uz);
    const C sym = coef_W<C>(k) * base + coef_c<C>(k) * ej * eu;
    const C anti = coef_a<C>(k) * ej;
    f[k] = sym + anti;
    f[k + 1] = sym - anti;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) *elem(grid, pb, i, n.own) = Storage<K>::store(f[i], ph.scale);
}

// ---------------------------------------------------------------------------
// Macroscopic fields from the stored post-collision state:
// rho = 1 + sum g*_i, rho u = sum g*_i c_i - F/2 (rho0 u, rho0 = 1, for the
// incompressible equilibrium).
// ---------------------------------------------------------------------------
template <int K, typename O>
__global__ __launch_bounds__(kBlock) void k_macro(const typename Storage<K>::T* __restrict__ grid,
                                                  const uint8_t* __restrict__ flags,
                                                  O* __restrict__ rho_out, O* __restrict__ u_out,
                                                  Geo g, O Fx, O Fy, O Fz, O inv_scale, int incomp) {
  const Loc l = locate(g);
  if (!l.valid) return;
  const uint32_t c = uint32_t((l.z * g.ny + l.y) * g.nx + l.x);
  const size_t ncell = size_t(g.nx) * g.ny * g.nz;
  const uint32_t own = uint32_t(l.z * g.ny + l.y) * uint32_t(g.xs) + uint32_t(l.x);
  const uint8_t fl = flags ? flags[c] : uint8_t(0);
  O r = O(0), ux = O(0), uy = O(0), uz = O(0);
  if (!(fl & FLAG_SOLID)) {
    O f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
      f[i] = O(Storage<K>::load(grid[size_t(i) * g.plane + own],
                                typename Storage<K>::C(inv_scale)));
    O drho, jx, jy, jz;
    moments(f, drho, jx, jy, jz);
    if (fl & FLAG_NOFORCE) Fx = Fy = Fz = O(0);
    r = O(1) + drho;
    const O mx = jx - O(0.5) * Fx, my = jy - O(0.5) * Fy, mz = jz - O(0.5) * Fz;
    ux = mx;
    uy = my;
    uz = mz;
    if (!incomp) {
      const O t = inv_rho_factor(drho);
      ux = mx - mx * t;
      uy = my - my * t;
      uz = mz - mz * t;
    }
  }
  if (rho_out) rho_out[c] = r;
  if (u_out) {
    u_out[c] = ux;
    u_out[ncell + c] = uy;
    u_out[2 * ncell + c] = uz;
  }
}

// ---------------------------------------------------------------------------
// FP64 reductions: per-block partials (fixed cell -> thread assignment and a
// fixed LDS tree), then one block sums the partials in a fixed order.
// ---------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ void block_sum(double (&v)[NC], double* sh) {
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NC; ++k) sh[k * kBlock + t] = v[k];
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    __syncthreads();
    if (t < s) {
#pragma unroll
      for (int k = 0; k < NC; ++k) sh[k * kBlock + t] += sh[k * kBlock + t + s];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NC; ++k) v[k] = sh[k * kBlock];
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_reduce_partials(const typename Storage<K>::T* __restrict__ grid,
                                                            const uint8_t* __restrict__ flags, Geo g,
                                                            double Fx, double Fy, double Fz,
                                                            double inv_scale, int incomp,
                                                            double* __restrict__ out) {
  __shared__ double sh[5 * kBlock];
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t ncell = int64_t(g.nx) * g.ny * g.nz;
  for (int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x; c < ncell;
       c += int64_t(gridDim.x) * kBlock) {
    const uint8_t fl = flags ? flags[c] : uint8_t(0);
    if (fl & FLAG_SOLID) continue;
    const int64_t row = c / g.nx;
    const uint32_t own = uint32_t(row * g.xs + (c - row * g.nx));
    double f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
      f[i] = double(Storage<K>::load(grid[size_t(i) * g.plane + own],
                                     typename Storage<K>::C(inv_scale)));
    double drho, jx, jy, jz;
    moments(f, drho, jx, jy, jz);
    const double h = (fl & FLAG_NOFORCE) ? 0.0 : 0.5;
    const double rho = 1.0 + drho;
    const double px = jx - h * Fx, py = jy - h * Fy, pz = jz - h * Fz;
    acc[0] += rho;
    acc[1] += px;
    acc[2] += py;
    acc[3] += pz;
    acc[4] += 0.5 * (px * px + py * py + pz * pz) / (incomp ? 1.0 : rho);
  }
  block_sum<5>(acc, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) out[blockIdx.x * 5 + k] = acc[k];
}

// Sums nparts partial records of NC doubles each, in a fixed order.
template <int NC>
__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* __restrict__ parts, int nparts,
                                                         double* __restrict__ out) {
  __shared__ double sh[NC * kBlock];
  double acc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = 0.0;
  for (int p = threadIdx.x; p < nparts; p += kBlock)
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] += parts[size_t(p) * NC + k];
  block_sum<NC>(acc, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < NC; ++k) out[k] = acc[k];
}

// ---------------------------------------------------------------------------
// Discrete adjoint (FP32 storage).  With lambda = dL/d f* at a fluid cell and
// the weighted moments of lambda
//   L0 = sum w_i lam_i,  L1 = sum w_i lam_i c_i,  L2 = sum w_i lam_i c_i c_i^T,
// the transposed collision Jacobian is rank-structured:
//   a  = omega (L0 + 3 L1.u + 9/2 u.L2 u - 3/2 u.u L0)
//   b  = omega rho (3 L1 + 9 L2 u - 3 u L0) + (1 - omega/2)(9 L2 F - 3 F L0)
//   mu_j = (1 - omega) lam_j + a + b . (c_j - u) / rho
//   dL/dF += (1 - omega/2)(3 L1 - 3 u L0 + 9 L2 u) + b / (2 rho)
// With the incompressible equilibrium (u = j', d f^eq_i / d rho = w_i) the
// same holds with a = omega L0, rho -> 1 in b and in b/(2 rho), and
// mu_j = (1 - omega) lam_j + a + b . c_j.  A moving wall adds a constant to
// the streaming, which enters the recomputed state only.
// ---------------------------------------------------------------------------
struct LamMoments {
  float L0, L1x, L1y, L1z, Lxx, Lyy, Lzz, Lxy, Lxz, Lyz;
};

__device__ __forceinline__ LamMoments lam_moments(const float* lam) {
  LamMoments m;
  m.L0 = m.L1x = m.L1y = m.L1z = -0.0f;
  m.Lxx = m.Lyy = m.Lzz = m.Lxy = m.Lxz = m.Lyz = -0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float wl = weight<float>(i) * lam[i];
    const int cx = D3Q19::cx[i], cy = D3Q19::cy[i], cz = D3Q19::cz[i];
    m.L0 += wl;
    if (cx) m.L1x += cx > 0 ? wl : -wl;
    if (cy) m.L1y += cy > 0 ? wl : -wl;
    if (cz) m.L1z += cz > 0 ? wl : -wl;
    if (cx) m.Lxx += wl;
    if (cy) m.Lyy += wl;
    if (cz) m.Lzz += wl;
    if (cx * cy) m.Lxy += cx * cy > 0 ? wl : -wl;
    if (cx * cz) m.Lxz += cx * cz > 0 ? wl : -wl;
    if (cy * cz) m.Lyz += cy * cz > 0 ? wl : -wl;
  }
  return m;
}

// The adjoint carries nu^n = dL/df(n), the adjoint of the pre-collision state
// f(n) = P f*(n-1) (P: the pull with half-way bounce-back).  With
// lambda^n = dL/df*(n) = P^T nu^{n+1}, one reverse step in pull form is
//   lambda^n_i(x) = nu^{n+1}_i(x + c_i), or nu^{n+1}_{opp i}(x) if x + c_i is
//                   solid (P^T as a gather along +c_i),
//   f(n) = P f*(n-1) (the forward pull, gathered along -c_i),
//   nu^n = J(f(n))^T lambda^n,  dL/dF += JF(f(n))^T lambda^n,
// and nu^n is stored at x: 19 gathers of nu, 19 of f* and 19 aligned stores
// per cell (228 B in FP32).  The seed forms lambda^T locally from dL/drho_T
// and dL/du_T (the moments of f(T) equal those read from f*(T)) and applies
// the same transposed collision; the initial step gathers lambda^0 = P^T nu^1.
// The solid cells of a nu grid hold the resting marker, written by the
// solid lanes, so both gathers test markers as the forward pull does.
template <bool SOLIDS, bool MOVING, bool SEED>
__global__ __launch_bounds__(kBlock) void k_adj(const float* __restrict__ fprev,
                                                const float* __restrict__ nu1,
                                                float* __restrict__ nu0,
                                                const uint8_t* __restrict__ flags,
                                                const float* __restrict__ gr,
                                                const float* __restrict__ gu,
                                                double* __restrict__ partials, Geo g,
                                                Phys<float> ph) {
  using U = Storage<ST_F32>::U;
  __shared__ double sh[3 * kBlock];
  double d[3] = {0.0, 0.0, 0.0};
  // the step kernel's cell order: 64-cell segments, y-banded rows, XCD remap
  const int b = blockIdx.x;
  const int lb = (b < g.nb8) ? ((b & 7) * (g.nb8 >> 3) + (b >> 3)) : b;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int seg = lb * 4 + wave;
  const int row = seg / g.nseg;
  Loc l;
  l.x = (seg - row * g.nseg) * 64 + int(threadIdx.x & 63);
  {
    const int rr = row < g.nrows ? row : 0;
    const int per_band = g.nz * g.yb;
    const int band = rr / per_band;
    const int y0 = band * g.yb;
    const int h = min(g.yb, g.ny - y0);
    const int idx = rr - band * per_band;
    l.z = idx / h;
    l.y = y0 + (idx - l.z * h);
  }
  l.valid = row < g.nrows && l.x < g.nx;
  if (l.valid) {
    const Nbhd n = neighbourhood(g, l);
    const uint8_t fl = SOLIDS ? flags[n.fown] : uint8_t(0);
    const bool solid = SOLIDS && (fl & FLAG_SOLID);
    const size_t pb = size_t(g.plane) * sizeof(float);
    // f(n) = P f*(n-1), exactly as the forward pull
    float f[Q];
    bool mk[Q], mv[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float v = *elem_rx(fprev, pb, i, src_row(n, i), src_x(n, i));
      const U r = raw_bits<ST_F32>(v);
      mk[i] = SOLIDS && i != 0 && (MOVING ? (r | 1u) == Storage<ST_F32>::kMoving
                                         : r == Storage<ST_F32>::kRest);
      mv[i] = MOVING && i != 0 && r == Storage<ST_F32>::kMoving;
      f[i] = v;
    }
    if (SOLIDS) {
#pragma unroll
      for (int i = 1; i < Q; ++i)
        if (mk[i] && !solid) {
          float v = *elem_rx(fprev, pb, D3Q19::opp[i], n.row[1][1], n.xn[1]);
          if (MOVING && mv[i]) v += ph.Kw[i];
          f[i] = v;
        }
    }
    float lam[Q];
    if (!SEED) {
      // lambda^n = P^T nu^{n+1}: pull along +c_i.  Each nu value is gathered
      // by one cell only, so the loads are non-temporal (1.8% faster at
      // 256^3 than cached loads, which evict the f* lines the neighbours
      // share).
      bool mb[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const float v = __builtin_nontemporal_load(
            elem_rx(nu1, pb, i, n.row[1 + D3Q19::cz[i]][1 + D3Q19::cy[i]], n.xn[1 - D3Q19::cx[i]]));
        mb[i] = SOLIDS && i != 0 && raw_bits<ST_F32>(v) == Storage<ST_F32>::kRest;
        lam[i] = v;
      }
      if (SOLIDS) {
#pragma unroll
        for (int i = 1; i < Q; ++i)
          if (mb[i] && !solid) lam[i] = *elem_rx(nu1, pb, D3Q19::opp[i], n.row[1][1], n.xn[1]);
      }
    }
    const bool forced = !(fl & FLAG_NOFORCE);
    const float Fx = forced ? ph.F[0] : 0.0f, Fy = forced ? ph.F[1] : 0.0f,
                Fz = forced ? ph.F[2] : 0.0f;
    float drho, jx, jy, jz;
    moments(f, drho, jx, jy, jz);
    const bool inc = ph.incomp != 0;
    const float rho = inc ? 1.0f : 1.0f + drho;  // the density dividing j' in u
    const float inv_rho = inc ? 1.0f : 1.0f / rho;
    const float ux = (jx + 0.5f * Fx) * inv_rho, uy = (jy + 0.5f * Fy) * inv_rho,
                uz = (jz + 0.5f * Fz) * inv_rho;
    if (SEED) {
      // lambda^T_i = dL/drho + dL/du . (c_i - u)/rho  (dL/du . c_i when incompressible);
      // u = (j + F/2)/rho of f(T) equals the velocity read from f*(T)
      const float G = gr ? gr[n.fown] : 0.0f;
      float hx = 0.0f, hy = 0.0f, hz = 0.0f;
      if (gu) {
        const size_t ncell = size_t(g.nx) * g.ny * g.nz;
        hx = gu[n.fown] * inv_rho;
        hy = gu[ncell + n.fown] * inv_rho;
        hz = gu[2 * ncell + n.fown] * inv_rho;
      }
      const float base = inc ? G : G - (hx * ux + hy * uy + hz * uz);
#pragma unroll
      for (int i = 0; i < Q; ++i) lam[i] = base + cdot<float>(i, hx, hy, hz);
      if (forced && !solid) {
        d[0] = -double(hx) / 2.0;
        d[1] = -double(hy) / 2.0;
        d[2] = -double(hz) / 2.0;
      }
    }
    const float om = ph.omega, om1 = 1.0f - om, fpre = 1.0f - 0.5f * om;
    const LamMoments m = lam_moments(lam);
    const float Lux = m.Lxx * ux + m.Lxy * uy + m.Lxz * uz;
    const float Luy = m.Lxy * ux + m.Lyy * uy + m.Lyz * uz;
    const float Luz = m.Lxz * ux + m.Lyz * uy + m.Lzz * uz;
    const float LFx = m.Lxx * Fx + m.Lxy * Fy + m.Lxz * Fz;
    const float LFy = m.Lxy * Fx + m.Lyy * Fy + m.Lyz * Fz;
    const float LFz = m.Lxz * Fx + m.Lyz * Fy + m.Lzz * Fz;
    const float uu = ux * ux + uy * uy + uz * uz;
    const float a = inc ? om * m.L0
                        : om * (m.L0 + 3.0f * (m.L1x * ux + m.L1y * uy + m.L1z * uz) +
                                4.5f * (ux * Lux + uy * Luy + uz * Luz) - 1.5f * uu * m.L0);
    const float orho = om * rho;
    const float bx = orho * (3.0f * m.L1x + 9.0f * Lux - 3.0f * ux * m.L0) +
                     fpre * (9.0f * LFx - 3.0f * Fx * m.L0);
    const float by = orho * (3.0f * m.L1y + 9.0f * Luy - 3.0f * uy * m.L0) +
                     fpre * (9.0f * LFy - 3.0f * Fy * m.L0);
    const float bz = orho * (3.0f * m.L1z + 9.0f * Luz - 3.0f * uz * m.L0) +
                     fpre * (9.0f * LFz - 3.0f * Fz * m.L0);
    const float bhx = bx * inv_rho, bhy = by * inv_rho, bhz = bz * inv_rho;
    const float a0 = inc ? a : a - (bhx * ux + bhy * uy + bhz * uz);
    const float marker = from_bits<ST_F32>(Storage<ST_F32>::kRest);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float mu = om1 * lam[i] + a0 + cdot<float>(i, bhx, bhy, bhz);
      stream_store(elem_rx(nu0, pb, i, n.row[1][1], n.xn[1]), solid ? marker : mu);
    }
    if (forced && !solid) {
      d[0] += double(fpre * (3.0f * m.L1x - 3.0f * ux * m.L0 + 9.0f * Lux) + 0.5f * bhx);
      d[1] += double(fpre * (3.0f * m.L1y - 3.0f * uy * m.L0 + 9.0f * Luy) + 0.5f * bhy);
      d[2] += double(fpre * (3.0f * m.L1z - 3.0f * uz * m.L0 + 9.0f * Luz) + 0.5f * bhz);
    }
  }
  block_sum<3>(d, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) {
      if (SEED) partials[size_t(lb) * 3 + k] = d[k];
      else partials[size_t(lb) * 3 + k] += d[k];
    }
}

// dL/du0 = sum_i lam0_i w_i rho0 (3 c_i + 9 (c_i.u0) c_i - 3 u0) = rho0 (3 L1 + 9 L2 u0 - 3 u0 L0),
// with lambda^0 = P^T nu^1 gathered along +c_i (rho0 -> 1 in the prefactor for
// the incompressible equilibrium).
template <bool SOLIDS>
__global__ __launch_bounds__(kBlock) void k_adj_init(const float* __restrict__ nu1,
                                                     const uint8_t* __restrict__ flags,
                                                     const float* __restrict__ rho0,
                                                     const float* __restrict__ u0,
                                                     float* __restrict__ du0, Geo g, int incomp) {
  const Loc l = locate(g);
  if (!l.valid) return;
  const Nbhd n = neighbourhood(g, l);
  const uint32_t c = n.fown;
  const size_t ncell = size_t(g.nx) * g.ny * g.nz;
  float rx = 0.0f, ry = 0.0f, rz = 0.0f;
  if (!(SOLIDS && (flags[c] & FLAG_SOLID))) {
    const size_t pb = size_t(g.plane) * sizeof(float);
    float lam[Q];
    bool mb[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float v = *elem_rx(nu1, pb, i, n.row[1 + D3Q19::cz[i]][1 + D3Q19::cy[i]],
                               n.xn[1 - D3Q19::cx[i]]);
      mb[i] = SOLIDS && i != 0 && raw_bits<ST_F32>(v) == Storage<ST_F32>::kRest;
      lam[i] = v;
    }
    if (SOLIDS) {
#pragma unroll
      for (int i = 1; i < Q; ++i)
        if (mb[i]) lam[i] = *elem_rx(nu1, pb, D3Q19::opp[i], n.row[1][1], n.xn[1]);
    }
    const LamMoments m = lam_moments(lam);
    const float rho = (rho0 && !incomp) ? rho0[c] : 1.0f;
    float ux = 0.0f, uy = 0.0f, uz = 0.0f;
    if (u0) {
      ux = u0[c];
      uy = u0[ncell + c];
      uz = u0[2 * ncell + c];
    }
    const float Lux = m.Lxx * ux + m.Lxy * uy + m.Lxz * uz;
    const float Luy = m.Lxy * ux + m.Lyy * uy + m.Lyz * uz;
    const float Luz = m.Lxz * ux + m.Lyz * uy + m.Lzz * uz;
    rx = rho * (3.0f * m.L1x + 9.0f * Lux - 3.0f * ux * m.L0);
    ry = rho * (3.0f * m.L1y + 9.0f * Luy - 3.0f * uy * m.L0);
    rz = rho * (3.0f * m.L1z + 9.0f * Luz - 3.0f * uz * m.L0);
  }
  du0[c] = rx;
  du0[ncell + c] = ry;
  du0[2 * ncell + c] = rz;
}

// ---------------------------------------------------------------------------
// Utility kernels.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_fill_zero(uint4* __restrict__ p, size_t n16) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n16; i += size_t(gridDim.x) * kBlock)
    p[i] = z;
}

__global__ __launch_bounds__(kBlock) void k_fill_zero_bytes(uint8_t* __restrict__ p, size_t n) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = 0;
}

// STREAM copy c = a: one 16-byte element per thread (more waves in flight
// measured faster than several elements per thread).
__global__ __launch_bounds__(kBlock) void k_copy(uint4* __restrict__ c, const uint4* __restrict__ a,
                                                 size_t n16) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n16) c[i] = a[i];
}

// The copy's variants for the attainable-bandwidth sweep: V 16-byte elements
// per thread per pass (a wave moves V consecutive 1 KiB runs), optionally
// with non-temporal loads and stores, over a grid of `blocks` blocks that
// strides through the array (blocks large enough for one pass = no stride).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int V, bool NT>
__global__ __launch_bounds__(kBlock) void k_copy_v(u32x4* __restrict__ c, const u32x4* __restrict__ a,
                                                   size_t n16) {
  const size_t stride = size_t(gridDim.x) * kBlock * V;
  for (size_t base = size_t(blockIdx.x) * kBlock * V + threadIdx.x; base < n16; base += stride) {
    u32x4 v[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const size_t i = base + size_t(k) * kBlock;
      if (i < n16) v[k] = NT ? __builtin_nontemporal_load(a + i) : a[i];
    }
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const size_t i = base + size_t(k) * kBlock;
      if (i < n16) {
        if (NT) __builtin_nontemporal_store(v[k], c + i);
        else c[i] = v[k];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (n16) {
    size_t blocks = (n16 + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_zero, dim3(unsigned(blocks)), dim3(kBlock), 0, s,
                       reinterpret_cast<uint4*>(p), n16);
  }
  const size_t tail = bytes - n16 * 16;
  if (tail)
    hipLaunchKernelGGL(k_fill_zero_bytes, dim3(1), dim3(kBlock), 0, s,
                       reinterpret_cast<uint8_t*>(p) + n16 * 16, tail);
  return hipGetLastError();
}

template <int K>
static void init_t(const Geo& g, const PhysParams& ph, void* grid, const uint8_t* flags,
                   const float* rho0, const float* u0, hipStream_t s) {
  using S = Storage<K>;
  hipLaunchKernelGGL(k_init<K>, dim3(g.nblocks), dim3(kBlock), 0, s,
                     reinterpret_cast<typename S::T*>(grid), flags, rho0, u0, g,
                     to_phys<typename S::C>(ph));
}

hipError_t launch_init(int storage, const Geo& g, const PhysParams& ph, void* grid,
                       const uint8_t* flags, const float* rho0, const float* u0, hipStream_t s) {
  switch (storage) {
    case ST_F32: init_t<ST_F32>(g, ph, grid, flags, rho0, u0, s); break;
    case ST_F16: init_t<ST_F16>(g, ph, grid, flags, rho0, u0, s); break;
    case ST_BF16: init_t<ST_BF16>(g, ph, grid, flags, rho0, u0, s); break;
    case ST_F64: init_t<ST_F64>(g, ph, grid, flags, rho0, u0, s); break;
    case ST_F32X: init_t<ST_F32X>(g, ph, grid, flags, rho0, u0, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int K>
static void mark_t(const Geo& g, bool moving, void* grid, const uint8_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_mark_solids<K>, dim3(g.nblocks), dim3(kBlock), 0, s,
                     reinterpret_cast<typename Storage<K>::T*>(grid), flags, g, moving ? 1 : 0);
}

hipError_t launch_mark_solids(int storage, const Geo& g, const PhysParams& ph, void* grid,
                              const uint8_t* flags, hipStream_t s) {
  const bool mv = ph.moving;
  switch (storage) {
    case ST_F32: mark_t<ST_F32>(g, mv, grid, flags, s); break;
    case ST_F16: mark_t<ST_F16>(g, mv, grid, flags, s); break;
    case ST_BF16: mark_t<ST_BF16>(g, mv, grid, flags, s); break;
    case ST_F64: mark_t<ST_F64>(g, mv, grid, flags, s); break;
    case ST_F32X: mark_t<ST_F32X>(g, mv, grid, flags, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Host-side construction of the uniform step constants (see StepK).
template <typename C>
static StepK<C> make_stepk(const PhysParams& p) {
  StepK<C> k;
  const double om = p.omega, fpre = 1.0 - 0.5 * om, S = p.scale;
  k.omega = C(om);
  k.om1 = C(1) - k.omega;
  const int rep[3] = {0, 1, 7};  // a direction of each speed class
  for (int c = 0; c < 3; ++c) {
    const int i = rep[c];
    k.oW[c] = C(om * weight<double>(i));
    k.oc[c] = c ? k.omega * coef_c<C>(i) : C(0);  // exact: c is 1/4 or 1/8
    k.a[c] = c ? coef_a<C>(i) : C(0);
    k.K3W[c] = C(3.0 * fpre * weight<double>(i) * S);
  }
  k.S = C(S);
  k.invS = C(1.0 / S);
  for (int d = 0; d < 3; ++d) {
    k.Fh[d] = C(0.5 * S * p.F[d]);
    k.F[d] = C(p.F[d]);
  }
  for (int q = 0; q < 9; ++q) {
    const int i = 2 * q + 1;
    const double cF = D3Q19::cx[i] * p.F[0] + D3Q19::cy[i] * p.F[1] + D3Q19::cz[i] * p.F[2];
    k.Kq[q] = C(fpre * 9.0 * weight<double>(i) * cF * S);
    k.Ka[q] = C(fpre * 3.0 * weight<double>(i) * cF * S);
  }
  for (int i = 0; i < Q; ++i) k.Kw[i] = C(wall_term(i, p.wall_u) * S);
  k.moving = p.moving ? 1 : 0;
  return k;
}

// Rows per y-band of the step kernel's visiting order (see k_step), by
// cells per lane: kernel traces at 512^3 put the 4-cell kernels' best at 16
// rows (6% faster than plain (z, y) order) and the 1-cell kernels' at 32.
constexpr int band_rows(int M) { return M >= 4 ? 16 : 32; }

// Geometry of 64*M-cell segments for the step kernel.
static Geo step_geo(const Geo& g, int M) {
  Geo h = g;
  h.yb = band_rows(M) < g.ny ? band_rows(M) : g.ny;
  h.nseg = (g.nx + 64 * M - 1) / (64 * M);
  const int64_t segs = int64_t(h.nseg) * g.nrows;
  h.nblocks = int32_t((segs + 3) / 4);
  h.nb8 = (h.nblocks / 8) * 8;
  return h;
}

template <int K, int WALLS, bool FORCE, bool INC>
static void step_t(const Geo& g, const PhysParams& ph, const void* src, void* dst,
                   const uint8_t* flags, hipStream_t s) {
  using S = Storage<K>;
  constexpr int M = StepCells<K>::M;
  const Geo h = step_geo(g, M);
  hipLaunchKernelGGL((k_step<K, WALLS, FORCE, INC, M>), dim3(h.nblocks), dim3(kBlock), 0, s,
                     reinterpret_cast<const typename S::T*>(src),
                     reinterpret_cast<typename S::T*>(dst), flags, h,
                     make_stepk<typename S::C>(ph));
}

template <int K, int WALLS, bool INC>
static void step_f(bool force, const Geo& g, const PhysParams& ph, const void* src, void* dst,
                   const uint8_t* flags, hipStream_t s) {
  if (force) step_t<K, WALLS, true, INC>(g, ph, src, dst, flags, s);
  else step_t<K, WALLS, false, INC>(g, ph, src, dst, flags, s);
}

template <int K, bool INC>
static void step_w(bool solids, bool force, const Geo& g, const PhysParams& ph, const void* src,
                   void* dst, const uint8_t* flags, hipStream_t s) {
  if (!solids) step_f<K, 0, INC>(force, g, ph, src, dst, flags, s);
  else if (ph.split) step_f<K, 3, INC>(force, g, ph, src, dst, flags, s);
  else if (!ph.moving) step_f<K, 1, INC>(force, g, ph, src, dst, flags, s);
  else step_f<K, 2, INC>(force, g, ph, src, dst, flags, s);
}

template <int K>
static void step_k(bool solids, bool force, const Geo& g, const PhysParams& ph, const void* src,
                   void* dst, const uint8_t* flags, hipStream_t s) {
  if (ph.incomp) step_w<K, true>(solids, force, g, ph, src, dst, flags, s);
  else step_w<K, false>(solids, force, g, ph, src, dst, flags, s);
}

hipError_t launch_step(int storage, bool solids, bool force, const Geo& g, const PhysParams& ph,
                       const void* src, void* dst, const uint8_t* flags, hipStream_t s) {
  switch (storage) {
    case ST_F32: step_k<ST_F32>(solids, force, g, ph, src, dst, flags, s); break;
    case ST_F16: step_k<ST_F16>(solids, force, g, ph, src, dst, flags, s); break;
    case ST_BF16: step_k<ST_BF16>(solids, force, g, ph, src, dst, flags, s); break;
    case ST_F64: step_k<ST_F64>(solids, force, g, ph, src, dst, flags, s); break;
    case ST_F32X: step_k<ST_F32X>(solids, force, g, ph, src, dst, flags, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Geometry of the two-step kernel's launch.
static Geo2 make_geo2(const Geo& g, int rows) {
  Geo2 h;
  h.nx = g.nx;
  h.ny = g.ny;
  h.nz = g.nz;
  h.xs = g.xs;
  h.plane = g.plane;
  h.ntx = (g.nx + 63) / 64;
  h.nty = (g.ny + rows - 1) / rows;
  // The longest z chunk (128, 64, 32, 16 planes) that still gives at least
  // kTB2MinBlocks blocks, else 16: a chunk recomputes two planes of step 1,
  // and fewer blocks than five per CU leave CUs idle (measured on periodic
  // cubes: 256^3 runs 45.0k MLUPS FP32 with 128-plane chunks, 160 blocks,
  // and 56.9k with 16-plane chunks, 1280 blocks; 512^3 runs best with 128).
  h.zc = g.nz < kTB2Chunk ? g.nz : kTB2Chunk;
  while (h.zc > kTB2MinChunk &&
         int64_t(h.ntx) * h.nty * ((g.nz + h.zc - 1) / h.zc) < kTB2MinBlocks)
    h.zc = h.zc / 2 > kTB2MinChunk ? h.zc / 2 : kTB2MinChunk;
  const int nzc = (g.nz + h.zc - 1) / h.zc;
  h.nblocks = h.ntx * h.nty * nzc;
  h.nb8 = (h.nblocks / 8) * 8;
  return h;
}

template <int K, int WALLS, bool FORCE, bool INC, bool MID = false>
static void step2_t(const Geo& g, const PhysParams& ph, const void* src, void* dst,
                    const uint8_t* flags, const uint32_t* lmask, hipStream_t s,
                    void* mid = nullptr) {
  using S = Storage<K>;
  constexpr int rows = tb2_rows<K>();
  const Geo2 h = make_geo2(g, rows);
  hipLaunchKernelGGL((k_step2<K, WALLS, FORCE, INC, MID>), dim3(h.nblocks), dim3(64 * (rows + 3)),
                     0, s, reinterpret_cast<const typename S::T*>(src),
                     reinterpret_cast<typename S::T*>(mid), reinterpret_cast<typename S::T*>(dst),
                     flags, lmask, h, make_stepk<typename S::C>(ph));
}

template <int K, int WALLS, bool INC>
static void step2_f(bool force, const Geo& g, const PhysParams& ph, const void* src, void* dst,
                    const uint8_t* flags, const uint32_t* lmask, hipStream_t s) {
  if (force) step2_t<K, WALLS, true, INC>(g, ph, src, dst, flags, lmask, s);
  else step2_t<K, WALLS, false, INC>(g, ph, src, dst, flags, lmask, s);
}

// walls: none (0), resting with markers (1) or with the link mask (4), moving (2)
template <int K, bool INC>
static void step2_w(bool solids, bool force, const Geo& g, const PhysParams& ph, const void* src,
                    void* dst, const uint8_t* flags, const uint32_t* lmask, hipStream_t s) {
  if (!solids) step2_f<K, 0, INC>(force, g, ph, src, dst, flags, lmask, s);
  else if (!ph.moving && lmask) step2_f<K, 4, INC>(force, g, ph, src, dst, flags, lmask, s);
  else if (!ph.moving) step2_f<K, 1, INC>(force, g, ph, src, dst, flags, lmask, s);
  else step2_f<K, 2, INC>(force, g, ph, src, dst, flags, lmask, s);
}

template <int K>
static void step2_k(bool solids, bool force, const Geo& g, const PhysParams& ph, const void* src,
                    void* dst, const uint8_t* flags, const uint32_t* lmask, hipStream_t s) {
  if (ph.incomp) step2_w<K, true>(solids, force, g, ph, src, dst, flags, lmask, s);
  else step2_w<K, false>(solids, force, g, ph, src, dst, flags, lmask, s);
}

int step2_blocks(int storage, const Geo& g) {
  switch (storage) {
    case ST_F32: return make_geo2(g, tb2_rows<ST_F32>()).nblocks;
    case ST_F16: return make_geo2(g, tb2_rows<ST_F16>()).nblocks;
    case ST_BF16: return make_geo2(g, tb2_rows<ST_BF16>()).nblocks;
    case ST_F64: return make_geo2(g, tb2_rows<ST_F64>()).nblocks;
    case ST_F32X: return make_geo2(g, tb2_rows<ST_F32X>()).nblocks;
    default: return 0;
  }
}

hipError_t launch_step2(int storage, bool solids, bool force, const Geo& g, const PhysParams& ph,
                        const void* src, void* dst, const uint8_t* flags, const uint32_t* lmask,
                        hipStream_t s) {
  switch (storage) {
    case ST_F32: step2_k<ST_F32>(solids, force, g, ph, src, dst, flags, lmask, s); break;
    case ST_F16: step2_k<ST_F16>(solids, force, g, ph, src, dst, flags, lmask, s); break;
    case ST_BF16: step2_k<ST_BF16>(solids, force, g, ph, src, dst, flags, lmask, s); break;
    case ST_F64: step2_k<ST_F64>(solids, force, g, ph, src, dst, flags, lmask, s); break;
    case ST_F32X: step2_k<ST_F32X>(solids, force, g, ph, src, dst, flags, lmask, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Two fused steps that also store the intermediate level (FP32 storage, the
// adjoint's storage): src = f*(t) -> mid = f*(t+1), dst = f*(t+2).
template <int WALLS, bool INC>
static void step2_mid_f(bool force, const Geo& g, const PhysParams& ph, const void* src, void* mid,
                        void* dst, const uint8_t* flags, const uint32_t* lmask, hipStream_t s) {
  if (force) step2_t<ST_F32, WALLS, true, INC, true>(g, ph, src, dst, flags, lmask, s, mid);
  else step2_t<ST_F32, WALLS, false, INC, true>(g, ph, src, dst, flags, lmask, s, mid);
}

template <bool INC>
static void step2_mid_w(bool solids, bool force, const Geo& g, const PhysParams& ph,
                        const void* src, void* mid, void* dst, const uint8_t* flags,
                        const uint32_t* lmask, hipStream_t s) {
  if (!solids) step2_mid_f<0, INC>(force, g, ph, src, mid, dst, flags, lmask, s);
  else if (!ph.moving && lmask) step2_mid_f<4, INC>(force, g, ph, src, mid, dst, flags, lmask, s);
  else if (!ph.moving) step2_mid_f<1, INC>(force, g, ph, src, mid, dst, flags, lmask, s);
  else step2_mid_f<2, INC>(force, g, ph, src, mid, dst, flags, lmask, s);
}

hipError_t launch_step2_mid(int storage, bool solids, bool force, const Geo& g,
                            const PhysParams& ph, const void* src, void* mid, void* dst,
                            const uint8_t* flags, const uint32_t* lmask, hipStream_t s) {
  if (storage != ST_F32) return hipErrorInvalidValue;
  if (ph.incomp) step2_mid_w<true>(solids, force, g, ph, src, mid, dst, flags, lmask, s);
  else step2_mid_w<false>(solids, force, g, ph, src, mid, dst, flags, lmask, s);
  return hipGetLastError();
}

hipError_t launch_link_mask(const Geo& g, const uint8_t* flags, uint32_t* mask, hipStream_t s) {
  const size_t n = size_t(g.nx) * g.ny * g.nz;
  hipLaunchKernelGGL(k_link_mask, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     flags, mask, g);
  return hipGetLastError();
}

template <int K>
static void pull_t(const Geo& g, const void* src, void* dst, hipStream_t s) {
  using S = Storage<K>;
  constexpr int M = StepCells<K>::M;
  const Geo h = step_geo(g, M);
  hipLaunchKernelGGL((k_step<K, 4, false, false, M>), dim3(h.nblocks), dim3(kBlock), 0, s,
                     reinterpret_cast<const typename S::T*>(src),
                     reinterpret_cast<typename S::T*>(dst), nullptr, h, StepK<typename S::C>{});
}

hipError_t launch_pull_copy(int storage, const Geo& g, const void* src, void* dst, hipStream_t s) {
  switch (storage) {
    case ST_F32: pull_t<ST_F32>(g, src, dst, s); break;
    case ST_F16: pull_t<ST_F16>(g, src, dst, s); break;
    case ST_BF16: pull_t<ST_BF16>(g, src, dst, s); break;
    case ST_F64: pull_t<ST_F64>(g, src, dst, s); break;
    case ST_F32X: pull_t<ST_F32X>(g, src, dst, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int K>
static void obstacle_t(const Geo& g, const PhysParams& ph, void* grid, const uint8_t* flags,
                       hipStream_t s) {
  using S = Storage<K>;
  hipLaunchKernelGGL(k_obstacle<K>, dim3(g.nblocks), dim3(kBlock), 0, s,
                     reinterpret_cast<typename S::T*>(grid), flags, g,
                     to_phys<typename S::C>(ph));
}

hipError_t launch_obstacle(int storage, const Geo& g, const PhysParams& ph, void* grid,
                           const uint8_t* flags, hipStream_t s) {
  switch (storage) {
    case ST_F32: obstacle_t<ST_F32>(g, ph, grid, flags, s); break;
    case ST_F16: obstacle_t<ST_F16>(g, ph, grid, flags, s); break;
    case ST_BF16: obstacle_t<ST_BF16>(g, ph, grid, flags, s); break;
    case ST_F64: obstacle_t<ST_F64>(g, ph, grid, flags, s); break;
    case ST_F32X: obstacle_t<ST_F32X>(g, ph, grid, flags, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int K, typename O>
static void macro_t(const Geo& g, const PhysParams& ph, const void* grid, const uint8_t* flags,
                    void* rho, void* u, hipStream_t s) {
  hipLaunchKernelGGL((k_macro<K, O>), dim3(g.nblocks), dim3(kBlock), 0, s,
                     reinterpret_cast<const typename Storage<K>::T*>(grid), flags,
                     reinterpret_cast<O*>(rho), reinterpret_cast<O*>(u), g, O(ph.F[0]),
                     O(ph.F[1]), O(ph.F[2]), O(1.0 / ph.scale), ph.incomp ? 1 : 0);
}

template <typename O>
static hipError_t macro_o(int storage, const Geo& g, const PhysParams& ph, const void* grid,
                          const uint8_t* flags, void* rho, void* u, hipStream_t s) {
  switch (storage) {
    case ST_F32: macro_t<ST_F32, O>(g, ph, grid, flags, rho, u, s); break;
    case ST_F16: macro_t<ST_F16, O>(g, ph, grid, flags, rho, u, s); break;
    case ST_BF16: macro_t<ST_BF16, O>(g, ph, grid, flags, rho, u, s); break;
    case ST_F64: macro_t<ST_F64, O>(g, ph, grid, flags, rho, u, s); break;
    case ST_F32X: macro_t<ST_F32X, O>(g, ph, grid, flags, rho, u, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_macro(int storage, bool out_f64, const Geo& g, const PhysParams& ph,
                        const void* grid, const uint8_t* flags, void* rho, void* u, hipStream_t s) {
  return out_f64 ? macro_o<double>(storage, g, ph, grid, flags, rho, u, s)
                 : macro_o<float>(storage, g, ph, grid, flags, rho, u, s);
}

template <int K>
static void reduce_t(const Geo& g, const PhysParams& ph, const void* grid, const uint8_t* flags,
                     double* scratch, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partials<K>, dim3(kReduceBlocks), dim3(kBlock), 0, s,
                     reinterpret_cast<const typename Storage<K>::T*>(grid), flags, g, ph.F[0],
                     ph.F[1], ph.F[2], 1.0 / ph.scale, ph.incomp ? 1 : 0, scratch);
}

hipError_t launch_reduce(int storage, const Geo& g, const PhysParams& ph, const void* grid,
                         const uint8_t* flags, double* scratch, double* out5, hipStream_t s) {
  switch (storage) {
    case ST_F32: reduce_t<ST_F32>(g, ph, grid, flags, scratch, s); break;
    case ST_F16: reduce_t<ST_F16>(g, ph, grid, flags, scratch, s); break;
    case ST_BF16: reduce_t<ST_BF16>(g, ph, grid, flags, scratch, s); break;
    case ST_F64: reduce_t<ST_F64>(g, ph, grid, flags, scratch, s); break;
    case ST_F32X: reduce_t<ST_F32X>(g, ph, grid, flags, scratch, s); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_partials<5>, dim3(1), dim3(kBlock), 0, s, scratch, kReduceBlocks, out5);
  return hipGetLastError();
}

template <bool SEED>
static void adj_t(bool solids, const Geo& g, const PhysParams& ph, const float* fprev,
                  const float* nu1, float* nu0, const uint8_t* flags, const float* gr,
                  const float* gu, double* partials, hipStream_t s) {
  const Geo h = step_geo(g, 1);
  const Phys<float> p = to_phys<float>(ph);
  if (!solids)
    hipLaunchKernelGGL((k_adj<false, false, SEED>), dim3(h.nblocks), dim3(kBlock), 0, s, fprev, nu1,
                       nu0, flags, gr, gu, partials, h, p);
  else if (!ph.moving)
    hipLaunchKernelGGL((k_adj<true, false, SEED>), dim3(h.nblocks), dim3(kBlock), 0, s, fprev, nu1,
                       nu0, flags, gr, gu, partials, h, p);
  else
    hipLaunchKernelGGL((k_adj<true, true, SEED>), dim3(h.nblocks), dim3(kBlock), 0, s, fprev, nu1,
                       nu0, flags, gr, gu, partials, h, p);
}

hipError_t launch_adj_seed(bool solids, const Geo& g, const PhysParams& ph, const float* fprev,
                           const uint8_t* flags, const float* dL_drho, const float* dL_du,
                           float* nu_T, double* partials, hipStream_t s) {
  adj_t<true>(solids, g, ph, fprev, nullptr, nu_T, flags, dL_drho, dL_du, partials, s);
  return hipGetLastError();
}

hipError_t launch_adj_step(bool solids, const Geo& g, const PhysParams& ph, const float* fprev,
                           const uint8_t* flags, const float* nu_np1, float* nu_n,
                           double* partials, hipStream_t s) {
  adj_t<false>(solids, g, ph, fprev, nu_np1, nu_n, flags, nullptr, nullptr, partials, s);
  return hipGetLastError();
}

hipError_t launch_adj_init(bool solids, const Geo& g, const PhysParams& ph, const uint8_t* flags,
                           const float* nu1, const float* rho0, const float* u0, float* dL_du0,
                           hipStream_t s) {
  if (solids)
    hipLaunchKernelGGL(k_adj_init<true>, dim3(g.nblocks), dim3(kBlock), 0, s, nu1, flags, rho0, u0,
                       dL_du0, g, ph.incomp ? 1 : 0);
  else
    hipLaunchKernelGGL(k_adj_init<false>, dim3(g.nblocks), dim3(kBlock), 0, s, nu1, flags, rho0, u0,
                       dL_du0, g, ph.incomp ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_adj_finish(const Geo& g, const double* partials, double* out3, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials<3>, dim3(1), dim3(kBlock), 0, s, partials, g.nblocks, out3);
  return hipGetLastError();
}

hipError_t launch_copy(void* c, const void* a, size_t n16, hipStream_t s) {
  const size_t blocks = (n16 + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_copy, dim3(unsigned(blocks)), dim3(kBlock), 0, s,
                     reinterpret_cast<uint4*>(c), reinterpret_cast<const uint4*>(a), n16);
  return hipGetLastError();
}

template <int V, bool NT>
static void copy_v(void* c, const void* a, size_t n16, size_t blocks, hipStream_t s) {
  const size_t full = (n16 + size_t(kBlock) * V - 1) / (size_t(kBlock) * V);
  const size_t b = (blocks == 0 || blocks > full) ? full : blocks;
  hipLaunchKernelGGL((k_copy_v<V, NT>), dim3(unsigned(b)), dim3(kBlock), 0, s,
                     reinterpret_cast<u32x4*>(c), reinterpret_cast<const u32x4*>(a), n16);
}

hipError_t launch_copy_variant(void* c, const void* a, size_t n16, int vec, bool nt, size_t blocks,
                               hipStream_t s) {
  switch (vec * 2 + (nt ? 1 : 0)) {
    case 2: copy_v<1, false>(c, a, n16, blocks, s); break;
    case 3: copy_v<1, true>(c, a, n16, blocks, s); break;
    case 4: copy_v<2, false>(c, a, n16, blocks, s); break;
    case 5: copy_v<2, true>(c, a, n16, blocks, s); break;
    case 8: copy_v<4, false>(c, a, n16, blocks, s); break;
    case 9: copy_v<4, true>(c, a, n16, blocks, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lbm
