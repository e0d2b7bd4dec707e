// Host-side construction of the planewave basis and operator tables
// (dks_init_basis) and the C-ABI entry points that need no kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <new>
#include <stdexcept>

#include "dks_internal.h"
#include "fft_split.h"

namespace dks {

static thread_local std::string g_err;
void set_error(const std::string &m) { g_err = m; }
const char *get_error() { return g_err.c_str(); }

dks_status status_of_current_exception(std::string &msg) {
  try {
    throw;
  } catch (const Error &e) {
    msg = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    msg = "host allocation failed";
    return DKS_ENOMEM;
  } catch (const std::exception &e) {
    msg = std::string("internal error: ") + e.what();
    return DKS_EINTERNAL;
  } catch (...) {
    msg = "internal error: unknown exception";
    return DKS_EINTERNAL;
  }
}

void upload(DevBuf &b, const void *host, size_t bytes) {
  b.ensure(bytes);
  if (bytes) DKS_HIP(hipMemcpy(b.p, host, bytes, hipMemcpyHostToDevice));
}

FftPlan make_plan(int n) {
  FftPlan p{};
  p.n = n;
  p.npass = 0;
  int m = n;
  const int pref[6] = {8, 6, 5, 4, 3, 2};
  while (m > 1) {
    bool found = false;
    for (int r : pref) {
      if (m % r == 0) {
        DKS_REQUIRE(p.npass < kMaxPass, DKS_EINVAL, "FFT length has too many factors");
        p.radix[p.npass++] = r;
        m /= r;
        found = true;
        break;
      }
    }
    DKS_REQUIRE(found, DKS_EINVAL, "FFT grid size " + std::to_string(n) + " is not a product of 2, 3, 5");
  }
  return p;
}

typedef std::complex<double> zc;

// complex solid harmonic |q|^l Y_lm(q^), Condon-Shortley phase, l <= 3
static zc solid_harmonic(int l, int m, double x, double y, double z) {
  const double pi = M_PI;
  const zc xp(x, y), xm(x, -y);
  const double r2 = x * x + y * y + z * z;
  // S_{l,-m} = (-1)^m conj(S_{l,m})
  if (m < 0) {
    zc v = std::conj(solid_harmonic(l, -m, x, y, z));
    return (m % 2 == 0) ? v : -v;
  }
  switch (l) {
    case 0: return zc(0.5 / std::sqrt(pi), 0.0);
    case 1:
      if (m == 0) return zc(std::sqrt(3.0 / (4 * pi)) * z, 0.0);
      return -std::sqrt(3.0 / (8 * pi)) * xp;
    case 2:
      if (m == 0) return zc(std::sqrt(5.0 / (16 * pi)) * (3 * z * z - r2), 0.0);
      if (m == 1) return -std::sqrt(15.0 / (8 * pi)) * z * xp;
      return std::sqrt(15.0 / (32 * pi)) * xp * xp;
    case 3:
      if (m == 0) return zc(std::sqrt(7.0 / (16 * pi)) * z * (5 * z * z - 3 * r2), 0.0);
      if (m == 1) return -std::sqrt(21.0 / (64 * pi)) * (5 * z * z - r2) * xp;
      if (m == 2) return std::sqrt(105.0 / (32 * pi)) * z * xp * xp;
      return -std::sqrt(35.0 / (64 * pi)) * xp * xp * xp;
  }
  return zc(0, 0);
}

// W = D+ (x) P+ + D- (x) P- on index ((i (2l+1) + m + l) * 2 + s), with
// P+- the projectors on j = l +- 1/2 built from L.S = Lz Sz + (L+ S- + L- S+)/2.
static std::vector<zc> coupling(int l, int nrad, const double *dp, const double *dm) {
  const int d = 2 * l + 1, ds = 2 * d;
  std::vector<zc> ls(ds * ds, 0.0);
  for (int a = 0; a < d; ++a) {
    const int m = a - l;
    // Lz Sz
    ls[(a * 2 + 0) * ds + a * 2 + 0] += 0.5 * m;
    ls[(a * 2 + 1) * ds + a * 2 + 1] += -0.5 * m;
    // (L+ S-)/2 maps |m, up> to sqrt(l(l+1) - m(m+1))/2 |m+1, dn>
    if (m < l) {
      const double c = std::sqrt((double)l * (l + 1) - (double)m * (m + 1));
      ls[((a + 1) * 2 + 1) * ds + a * 2 + 0] += 0.5 * c;   // row (m+1, dn), column (m, up)
      // Hermitian partner (L- S+)/2: row (m, up), column (m+1, dn)
      ls[(a * 2 + 0) * ds + (a + 1) * 2 + 1] += 0.5 * c;
    }
  }
  std::vector<zc> pp(ds * ds), pm(ds * ds);
  for (int i = 0; i < ds; ++i)
    for (int j = 0; j < ds; ++j) {
      double id = (i == j) ? 1.0 : 0.0;
      pp[i * ds + j] = ((double)(l + 1) * id + 2.0 * ls[i * ds + j]) / (double)(2 * l + 1);
      pm[i * ds + j] = ((double)l * id - 2.0 * ls[i * ds + j]) / (double)(2 * l + 1);
    }
  const int nd = nrad * ds;
  std::vector<zc> w(nd * nd, 0.0);
  for (int i = 0; i < nrad; ++i)
    for (int ip = 0; ip < nrad; ++ip)
      for (int a = 0; a < ds; ++a)
        for (int b = 0; b < ds; ++b)
          w[(i * ds + a) * nd + ip * ds + b] = dp[i * nrad + ip] * pp[a * ds + b] + dm[i * nrad + ip] * pm[a * ds + b];
  return w;
}

static bool smooth235(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

void init_kernel_attributes();

}  // namespace dks

using namespace dks;

void free_scf_work(dks_basis *b);

dks_basis::~dks_basis() {
  free_scf_work(this);
  for (auto *s : sys) delete s;
  for (auto *p : pot) delete p;
}

extern "C" {

const char *dks_last_error(void) { return get_error(); }

int dks_num_systems(const dks_basis *b) { return b ? (int)b->sys.size() : 0; }

dks_status dks_init_basis(const dks_system_desc *descs, int ndesc, int device, dks_basis **out) {
  if (out) *out = nullptr;
  dks_basis *B = nullptr;
  try {
    DKS_REQUIRE(descs && out && ndesc > 0, DKS_EINVAL, "null argument or ndesc <= 0");
    int ndev = 0;
    DKS_HIP(hipGetDeviceCount(&ndev));
    DKS_REQUIRE(device >= 0 && device < ndev, DKS_EINVAL, "device index out of range");
    DKS_HIP(hipSetDevice(device));
    init_kernel_attributes();
    noalloc_scratch_setup(device);
    B = new dks_basis();
    B->device = device;
    for (int di = 0; di < ndesc; ++di) {
      const dks_system_desc &D = descs[di];
      DKS_REQUIRE(D.nk >= 1 && D.kpts, DKS_EINVAL, "nk < 1 or kpts null");
      DKS_REQUIRE(D.ecut > 0 && D.c > 0, DKS_EINVAL, "ecut and c must be positive");
      DKS_REQUIRE(D.v_loc, DKS_EINVAL, "v_loc is null");
      DKS_REQUIRE(D.natom >= 0 && (D.natom == 0 || D.tau), DKS_EINVAL, "bad atoms");
      DKS_REQUIRE(D.nproj_groups >= 0 && (D.nproj_groups == 0 || D.proj), DKS_EINVAL, "bad projectors");
      for (int d = 0; d < 3; ++d)
        DKS_REQUIRE(smooth235(D.grid[d]) && D.grid[d] <= 512, DKS_EINVAL,
                    "grid sizes must be products of 2, 3, 5 and <= 512");
      DKS_REQUIRE((size_t)D.grid[0] * (D.grid[1] + 1) * sizeof(double2) +
                          sizeof(int) * (size_t)((D.grid[0] + 3) & ~3) <= 163840 &&
                      (size_t)D.grid[0] * D.grid[1] <= 16 * 1024,
                  DKS_EINVAL, "N1 x N2 plane does not fit the 160 KB LDS in FP64");
      // lattice and reciprocal lattice
      const double *A = D.lattice;
      double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                   A[2] * (A[3] * A[7] - A[4] * A[6]);
      DKS_REQUIRE(std::fabs(det) > 1e-12, DKS_EINVAL, "singular lattice");
      // inverse of A (rows a_i): Ainv; reciprocal rows b_j = 2 pi * column j of Ainv
      double inv[9];
      inv[0] = (A[4] * A[8] - A[5] * A[7]) / det;
      inv[1] = (A[2] * A[7] - A[1] * A[8]) / det;
      inv[2] = (A[1] * A[5] - A[2] * A[4]) / det;
      inv[3] = (A[5] * A[6] - A[3] * A[8]) / det;
      inv[4] = (A[0] * A[8] - A[2] * A[6]) / det;
      inv[5] = (A[2] * A[3] - A[0] * A[5]) / det;
      inv[6] = (A[3] * A[7] - A[4] * A[6]) / det;
      inv[7] = (A[1] * A[6] - A[0] * A[7]) / det;
      inv[8] = (A[0] * A[4] - A[1] * A[3]) / det;
      double Bv[9];   // row j = b_j
      for (int j = 0; j < 3; ++j)
        for (int c = 0; c < 3; ++c) Bv[j * 3 + c] = 2.0 * M_PI * inv[c * 3 + j];

      // shared potential
      Potential *P = new Potential();
      B->pot.push_back(P);
      const int n1 = D.grid[0], n2 = D.grid[1], n3 = D.grid[2];
      const size_t ng = (size_t)n1 * n2 * n3;
      for (int d = 0; d < 3; ++d) P->grid[d] = D.grid[d];
      {
        // plane layout [p3][p1][p2] in the real-space order the transforms
        // leave behind: position p of axis d holds natural index nat[d][p]
        // (the plane kernels take the two-step transforms only when both plane
        // axes have a compiled split, else the natural-order radix transforms)
        std::vector<int> nat[3];
        int A0 = 1, B0 = 1;
        const bool plane_fast = fft2::split_plane(D.grid[0], &A0, &B0) && fft2::split_plane(D.grid[1], &A0, &B0);
        for (int d = 0; d < 3; ++d) {
          const int n = D.grid[d];
          nat[d].resize(n);
          int A = 1, Bq = n;
          bool fast = (d == 2) ? fft2::split_z(n, &A, &Bq) : (plane_fast && fft2::split_plane(n, &A, &Bq));
          for (int p = 0; p < n; ++p) nat[d][p] = fast ? fft2::scrambled_to_natural(p, A, Bq) : p;
        }
        std::vector<double> v64(ng);
        std::vector<float> v32(ng);
        double vmin = 1e300, vmax = -1e300, vs = 0;
        for (size_t e = 0; e < ng; ++e) {
          double v = D.v_loc[e];
          DKS_REQUIRE(std::isfinite(v), DKS_EINVAL, "v_loc has a non-finite value");
          vmin = std::min(vmin, v);
          vmax = std::max(vmax, v);
          vs += v;
        }
        for (int p3 = 0; p3 < n3; ++p3)
          for (int p1 = 0; p1 < n1; ++p1)
            for (int p2 = 0; p2 < n2; ++p2) {
              double v = D.v_loc[((size_t)nat[0][p1] * n2 + nat[1][p2]) * n3 + nat[2][p3]];
              size_t o = ((size_t)p3 * n1 + p1) * n2 + p2;
              v64[o] = v;
              v32[o] = (float)v;
            }
        P->vmin = vmin;
        P->vmax = vmax;
        P->vmean = vs / (double)ng;
        upload(P->d_v64, v64.data(), sizeof(double) * ng);
        upload(P->d_v32, v32.data(), sizeof(float) * ng);
        for (int d = 0; d < 3; ++d) upload(P->d_nat[d], nat[d].data(), sizeof(int) * nat[d].size());
        for (int d = 0; d < 3; ++d) {
          const int n = D.grid[d];
          std::vector<double2> t64(n);
          std::vector<float2> t32(n);
          for (int t = 0; t < n; ++t) {
            long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)t / (long double)n;
            t64[t] = make_double2((double)cosl(ang), (double)sinl(ang));
            t32[t] = make_float2((float)cosl(ang), (float)sinl(ang));
          }
          upload(P->d_tw64[d], t64.data(), sizeof(double2) * n);
          upload(P->d_tw32[d], t32.data(), sizeof(float2) * n);
        }
      }

      for (int ki = 0; ki < D.nk; ++ki) {
        System *S = new System();
        B->sys.push_back(S);
        S->vsrc = (int)B->pot.size() - 1;
        std::memcpy(S->lattice, A, sizeof(S->lattice));
        for (int c = 0; c < 3; ++c) S->kpt[c] = D.kpts[ki * 3 + c];
        S->ecut = D.ecut;
        S->c = D.c;
        for (int d = 0; d < 3; ++d) S->grid[d] = D.grid[d];
        S->ng = (int)ng;
        const double *k = S->kpt;
        double knorm = std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
        double qmax = std::sqrt(2.0 * D.ecut) + knorm;
        int nb[3];
        for (int d = 0; d < 3; ++d) {
          double len = std::sqrt(A[d * 3] * A[d * 3] + A[d * 3 + 1] * A[d * 3 + 1] + A[d * 3 + 2] * A[d * 3 + 2]);
          nb[d] = (int)std::floor(qmax * len / (2.0 * M_PI)) + 1;
        }
        // sphere, ordered by (n1, n2) then n3
        int maxabs[3] = {0, 0, 0};
        for (int a = -nb[0]; a <= nb[0]; ++a)
          for (int b = -nb[1]; b <= nb[1]; ++b) {
            int start = -1, len = 0;
            for (int c = -nb[2]; c <= nb[2]; ++c) {
              double q[3];
              for (int x = 0; x < 3; ++x) q[x] = k[x] + a * Bv[x] + b * Bv[3 + x] + c * Bv[6 + x];
              double e = 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
              if (e <= D.ecut) {
                if (len == 0) start = c;
                DKS_REQUIRE(c == start + len, DKS_EINVAL, "sphere column is not contiguous");
                ++len;
                S->miller.push_back(a);
                S->miller.push_back(b);
                S->miller.push_back(c);
                for (int x = 0; x < 3; ++x) S->q.push_back(q[x]);
                S->qmax2 = std::max(S->qmax2, 2.0 * e);
                maxabs[0] = std::max(maxabs[0], std::abs(a));
                maxabs[1] = std::max(maxabs[1], std::abs(b));
                maxabs[2] = std::max(maxabs[2], std::abs(c));
              }
            }
            if (len > 0) {
              S->col_off.push_back((int)(S->miller.size() / 3) - len);
              S->col_info.push_back(make_int4(((a % n1) + n1) % n1, ((b % n2) + n2) % n2, start, len));
            }
          }
        S->N = (int)(S->miller.size() / 3);
        DKS_REQUIRE(S->N > 0, DKS_EINVAL, "empty planewave sphere");
        S->ncol = (int)S->col_info.size();
        S->col_off.push_back(S->N);
        for (int d = 0; d < 3; ++d)
          DKS_REQUIRE(D.grid[d] > 2 * maxabs[d], DKS_EINVAL,
                      "FFT grid too small for the planewave sphere (need N > 2 max|n|)");
        // per-G column and z slot
        std::vector<int2> gmap(S->N);
        for (int c = 0; c < S->ncol; ++c) {
          int4 ci = S->col_info[c];
          for (int i = 0; i < ci.w; ++i) {
            int n3v = ci.z + i;
            gmap[S->col_off[c] + i] = make_int2(c, ((n3v % n3) + n3) % n3);
          }
        }
        // distinct n1 slots
        {
          std::vector<int> r;
          for (auto &ci : S->col_info) r.push_back(ci.x);
          std::sort(r.begin(), r.end());
          r.erase(std::unique(r.begin(), r.end()), r.end());
          S->rows = r;
          S->nrows = (int)r.size();
        }
        // per sphere row r and n2 slot p: the column there, or -1; and which n1
        // slots are sphere rows (the plane kernel's direct form reads these)
        {
          std::vector<int> slot(n1, -1), ctab((size_t)S->nrows * n2, -1), flag(n1, 0);
          for (int r = 0; r < S->nrows; ++r) {
            slot[S->rows[r]] = r;
            flag[S->rows[r]] = 1;
          }
          for (int c = 0; c < S->ncol; ++c) {
            const int4 ci = S->col_info[c];
            ctab[(size_t)slot[ci.x] * n2 + ci.y] = c;
          }
          upload(S->d_ctab, ctab.data(), sizeof(int) * ctab.size());
          upload(S->d_rowflag, flag.data(), sizeof(int) * flag.size());
        }
        upload(S->d_col_off, S->col_off.data(), sizeof(int) * S->col_off.size());
        upload(S->d_col_info, S->col_info.data(), sizeof(int4) * S->col_info.size());
        upload(S->d_rows, S->rows.data(), sizeof(int) * S->rows.size());
        upload(S->d_gmap, gmap.data(), sizeof(int2) * gmap.size());
        {
          const int N = S->N;
          std::vector<double> q64(3 * (size_t)N);
          std::vector<float> q32(3 * (size_t)N);
          for (int g = 0; g < N; ++g)
            for (int x = 0; x < 3; ++x) {
              q64[(size_t)x * N + g] = S->q[3 * (size_t)g + x];
              q32[(size_t)x * N + g] = (float)S->q[3 * (size_t)g + x];
            }
          upload(S->d_q64, q64.data(), sizeof(double) * q64.size());
          upload(S->d_q32, q32.data(), sizeof(float) * q32.size());
        }
        // projectors
        {
          const int N = S->N;
          std::vector<zc> Bm;
          std::vector<zc> Wall;
          std::vector<int4> winfo;
          int p0 = 0;
          for (int gi = 0; gi < D.nproj_groups; ++gi) {
            const dks_proj_group &g = D.proj[gi];
            DKS_REQUIRE(g.atom >= 0 && g.atom < D.natom, DKS_EINVAL, "projector atom index out of range");
            DKS_REQUIRE(g.l >= 0 && g.l <= 3 && g.n_rad >= 1 && g.n_rad <= 3 && g.r_l > 0,
                        DKS_EINVAL, "projector l, n_rad or r_l out of range");
            DKS_REQUIRE(g.d_plus && g.d_minus, DKS_EINVAL, "projector couplings are null");
            const int d = 2 * g.l + 1, dim = g.n_rad * d;
            const double *tau = D.tau + 3 * g.atom;
            std::vector<zc> vals((size_t)dim * N);
            for (int i = 0; i < g.n_rad; ++i) {
              double ss = 0;
              for (int m = -g.l; m <= g.l; ++m) {
                for (int gg = 0; gg < N; ++gg) {
                  const double *q = &S->q[3 * (size_t)gg];
                  double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
                  double x = q2 * g.r_l * g.r_l;
                  double radial = std::pow(x, i) * std::exp(-0.5 * x);
                  double ph = -(q[0] * tau[0] + q[1] * tau[1] + q[2] * tau[2]);
                  zc v = solid_harmonic(g.l, m, q[0], q[1], q[2]) * radial * zc(std::cos(ph), std::sin(ph));
                  vals[(size_t)(i * d + m + g.l) * N + gg] = v;
                  ss += std::norm(v);
                }
              }
              double f = 1.0 / std::sqrt(ss / d);
              for (int m = 0; m < d; ++m)
                for (int gg = 0; gg < N; ++gg) vals[(size_t)(i * d + m) * N + gg] *= f;
            }
            Bm.insert(Bm.end(), vals.begin(), vals.end());
            std::vector<zc> w = coupling(g.l, g.n_rad, g.d_plus, g.d_minus);
            ProjGroupHost ph{g.atom, g.l, g.n_rad, p0, dim, (int)Wall.size()};
            S->groups.push_back(ph);
            winfo.push_back(make_int4(p0, dim, (int)Wall.size(), 0));
            Wall.insert(Wall.end(), w.begin(), w.end());
            // ||W|| <= ||D+||_F + ||D-||_F; each of the dim unit projectors adds at most that
            double fp = 0, fm = 0;
            for (int e = 0; e < g.n_rad * g.n_rad; ++e) {
              fp += g.d_plus[e] * g.d_plus[e];
              fm += g.d_minus[e] * g.d_minus[e];
            }
            S->nl_bound += (std::sqrt(fp) + std::sqrt(fm)) * dim;
            p0 += dim;
          }
          S->nproj = p0;
          S->wtotal = (int)Wall.size();
          if (p0 > 0) {
            std::vector<double2> b64(Bm.size());
            std::vector<float2> b32(Bm.size());
            for (size_t e = 0; e < Bm.size(); ++e) {
              b64[e] = make_double2(Bm[e].real(), Bm[e].imag());
              b32[e] = make_float2((float)Bm[e].real(), (float)Bm[e].imag());
            }
            upload(S->d_B64, b64.data(), sizeof(double2) * b64.size());
            upload(S->d_B32, b32.data(), sizeof(float2) * b32.size());
            std::vector<double2> w64(Wall.size());
            for (size_t e = 0; e < Wall.size(); ++e) w64[e] = make_double2(Wall[e].real(), Wall[e].imag());
            upload(S->d_W64, w64.data(), sizeof(double2) * w64.size());
            upload(S->d_Winfo, winfo.data(), sizeof(int4) * winfo.size());
          }
        }
        for (int d = 0; d < 3; ++d) S->plan[d] = make_plan(D.grid[d]);
        upload(S->d_plan, S->plan, sizeof(S->plan));
        S->tile_z = std::max(1, std::min(32, 4096 / n3));
      }
    }
    *out = B;
    return DKS_OK;
  } catch (...) {
    std::string msg;
    const dks_status rc = status_of_current_exception(msg);
    set_error(msg);
    delete B;
    return rc;
  }
}

dks_status dks_basis_info(const dks_basis *b, int sys, int *npw, int *grid3, int *miller) {
  if (!b || sys < 0 || sys >= (int)b->sys.size()) {
    set_error("bad basis or system index");
    return DKS_EINVAL;
  }
  const System &s = *b->sys[sys];
  if (npw) *npw = s.N;
  if (grid3)
    for (int d = 0; d < 3; ++d) grid3[d] = s.grid[d];
  if (miller) std::memcpy(miller, s.miller.data(), sizeof(int) * s.miller.size());
  return DKS_OK;
}

dks_status dks_filter_constants(const dks_basis *b, int sys, double *C, double *Omega) {
  if (!b || sys < 0 || sys >= (int)b->sys.size() || !C || !Omega) {
    set_error("bad argument");
    return DKS_EINVAL;
  }
  const System &s = *b->sys[sys];
  const Potential &p = *b->pot[s.vsrc];
  const double c = s.c, c2 = c * c;
  // top of the free positive band (shifted), cancellation-free
  const double ekin = c2 * s.qmax2 / (std::sqrt(c2 * c2 + c2 * s.qmax2) + c2);
  *C = -2.0 * c2 - 0.5 * ekin + p.vmean;
  *Omega = (ekin + p.vmax + s.nl_bound) - *C;
  return DKS_OK;
}

void dks_free_basis(dks_basis *b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  extern void dks_free_solver(dks_basis *);
  dks_free_solver(b);
  delete b;
}

}  // extern "C"
