// Host-side mesh, decomposition and numbering (runs once per problem).
//
// Builds the structured right-triangle mesh of the unit square (Section 4.1
// uses uniform triangulations), the nsub_x x nsub_y subdomain grid, the local
// DOF order of every subdomain, the signed Boolean jump rows that glue the
// torn fields (Section 3.1: H_P, H_E of eq. (linalg-system) become the signed
// entries of one row per glued DOF pair), the weights of D = (B B^T)^{-1} for
// the preconditioner, the element DOF tables for the assembly kernels and the
// rigid modes of floating subdomains for the coarse space.
#include <algorithm>
#include <functional>
#include <cmath>
#include <map>
#include <numeric>
#include <tuple>
#include <unordered_map>

#include "feti_internal.h"

namespace feti {

namespace {

bool on_sides(int i, int j, int nmax, uint32_t mask) {
  return ((mask & 1u) && i == 0) || ((mask & 2u) && i == nmax) || ((mask & 4u) && j == 0) ||
         ((mask & 8u) && j == nmax);
}

bool cell_poro(int layout, int i, int j, int n) {
  const double xc = (i + 0.5) / n, yc = (j + 0.5) / n;
  switch (layout) {
    case FETI_XSPLIT: return xc < 0.5;
    case FETI_YSPLIT: return yc < 0.5;
    default: return xc > 0.25 && xc < 0.75 && yc > 0.25 && yc < 0.75;
  }
}

int field_order(int kind) {
  switch (kind) {
    case K_UX: case K_UY: case K_UZ: return 0;
    case K_ETA: return 1;
    case K_XIP: case K_XIE: return 2;
    default: return 3;
  }
}

// inverse of a small symmetric positive definite matrix (size <= 3) by Gauss-Jordan
void small_inverse(int n, double* a) {
  double b[9];
  for (int i = 0; i < n * n; ++i) b[i] = 0.0;
  for (int i = 0; i < n; ++i) b[i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    const double piv = a[k * n + k];
    for (int j = 0; j < n; ++j) { a[k * n + j] /= piv; b[k * n + j] /= piv; }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = a[i * n + k];
      for (int j = 0; j < n; ++j) { a[i * n + j] -= f * a[k * n + j]; b[i * n + j] -= f * b[k * n + j]; }
    }
  }
  for (int i = 0; i < n * n; ++i) a[i] = b[i];
}

}  // namespace

// Everything between the subdomains' DOF codes and the element tables, the same in 2D and
// 3D: categories and local orders, offsets, the positions of the codes, the jump rows
// with their D = (B B^T)^{-1} weights, the gather maps of the interface space and the
// primal tables of the dual-primal coupling.
std::string finish_interface(MeshHost& m, std::unordered_map<int32_t, std::vector<int32_t>>& owners,
                             const std::vector<bool>& has_dir, bool dp,
                             const std::function<bool(int32_t)>& is_primal,
                             const std::function<void(const SubHost&, int32_t&, int32_t&, int32_t&)>& fixed_codes,
                             const std::function<bool(const std::vector<int32_t>&)>& rigid_ok,
                             std::vector<std::unordered_map<int32_t, int32_t>>& pos) {
  const int nsub = (int)m.subs.size();
  // categories and local order
  for (SubHost& s : m.subs) {
    // under the dual-primal coupling the primal corners hold every subdomain
    s.floating = !dp && !has_dir[s.sid];
    int32_t fixA = -1, fixB = -1, fixC = -1;
    if (s.floating) fixed_codes(s, fixA, fixB, fixC);
    struct Key { int cat, fo, node, comp; int32_t code; };
    std::vector<Key> keys;
    keys.reserve(s.codes.size());
    for (int32_t c : s.codes) {
      const int node = c / 8, kind = c % 8;
      const bool shared = owners[c].size() > 1;
      int cat;
      if (c == fixA || c == fixB || c == fixC) cat = C_FIX;
      else if (dp) cat = shared ? (is_primal(c) ? C_BP : C_BU) : ((kind <= K_ETA || kind == K_UZ) ? C_IU : C_IP);
      else if (kind <= K_ETA || kind == K_UZ) cat = shared ? C_BU : C_IU;
      else cat = shared ? C_BP : C_IP;
      keys.push_back({cat, field_order(kind), node, kind == K_UY ? 1 : (kind == K_UZ ? 2 : 0), c});
    }
    std::sort(keys.begin(), keys.end(), [](const Key& x, const Key& y) {
      return std::tie(x.cat, x.fo, x.node, x.comp) < std::tie(y.cat, y.fo, y.node, y.comp);
    });
    s.codes.clear();
    s.cats.clear();
    for (const Key& k : keys) { s.codes.push_back(k.code); s.cats.push_back((int8_t)k.cat); }
    s.ns = (int)s.codes.size();
    s.nI = 0; s.nb = 0; s.nfix = 0;
    for (int8_t c : s.cats) {
      if (c < C_BU) ++s.nI; else ++s.nb;
      if (c == C_FIX) ++s.nfix;
    }
    if (s.floating && s.nfix != 3) return "floating subdomain without its three fixed DOFs";
    if (dp && !has_dir[s.sid]) {
      // primal displacement nodes that remove the rigid-body modes: two distinct ones in
      // 2D, three not on one line in 3D
      std::vector<int32_t> un;
      for (size_t i = 0; i < s.codes.size(); ++i) {
        const int k = s.codes[i] % 8;
        if (s.cats[i] == C_BP && (k == K_UX || k == K_UY || k == K_UZ)) un.push_back(s.codes[i] / 8);
      }
      std::sort(un.begin(), un.end());
      un.erase(std::unique(un.begin(), un.end()), un.end());
      if (!rigid_ok(un)) return "a subdomain without Dirichlet data has too few primal corners";
    }
  }
  // offsets
  int64_t off = 0, boff = 0;
  for (SubHost& s : m.subs) {
    s.off = off; s.boff = boff;
    off += s.ns; boff += s.nb;
    m.max_ns = std::max(m.max_ns, s.ns);
    m.max_nb = std::max(m.max_nb, s.nb);
  }
  m.sum_ns = off;
  m.sum_nb = boff;
  // position of each code in each subdomain
  pos.assign(nsub, {});
  for (SubHost& s : m.subs) {
    pos[s.sid].reserve(s.codes.size() * 2);
    for (int i = 0; i < s.ns; ++i) pos[s.sid][s.codes[i]] = i;
  }
  // jump rows sorted by (kind, node, pair index)
  std::vector<int32_t> shared_codes;
  for (auto& kv : owners)
    if (kv.second.size() > 1 && !(dp && is_primal(kv.first))) shared_codes.push_back(kv.first);
  std::sort(shared_codes.begin(), shared_codes.end(), [](int32_t x, int32_t y) {
    return std::make_pair(x % 8, x / 8) < std::make_pair(y % 8, y / 8);
  });
  for (int32_t c : shared_codes) {
    std::vector<int32_t> S = owners[c];
    std::sort(S.begin(), S.end());
    const int gstart = (int)m.rows.size();
    const int gsize = (int)S.size() - 1;
    for (size_t k = 0; k + 1 < S.size(); ++k) {
      JumpRow jr{};
      jr.sub[0] = S[k]; jr.sub[1] = S[k + 1];
      jr.loc[0] = pos[S[k]][c]; jr.loc[1] = pos[S[k + 1]][c];
      jr.sign[0] = 1; jr.sign[1] = -1;
      if (m.subs[S[k]].poro != m.subs[S[k + 1]].poro && !m.subs[S[k]].poro) {
        jr.sign[0] = -1; jr.sign[1] = 1;
      }
      jr.code = c;
      jr.mult = (int32_t)S.size();
      jr.kind = c % 8;
      m.rows.push_back(jr);
      m.grp_start.push_back(gstart);
      m.grp_size.push_back(gsize);
    }
    if (gsize > 3) return "a node shared by more than four subdomains";
    // D block = (B_g B_g^T)^{-1} over this group's rows
    double bbt[9] = {0};
    for (int a = 0; a < gsize; ++a)
      for (int b = 0; b < gsize; ++b) {
        double v = 0.0;
        const JumpRow& ra = m.rows[gstart + a];
        const JumpRow& rb = m.rows[gstart + b];
        for (int ea = 0; ea < 2; ++ea)
          for (int eb = 0; eb < 2; ++eb)
            if (ra.sub[ea] == rb.sub[eb]) v += (double)ra.sign[ea] * rb.sign[eb];
        bbt[a * gsize + b] = v;
      }
    small_inverse(gsize, bbt);
    for (int a = 0; a < gsize; ++a)
      for (int b = 0; b < 3; ++b) m.dwt.push_back(b < gsize ? bbt[a * gsize + b] : 0.0);
  }
  m.n_lambda = (int64_t)m.rows.size();
  // gather lists and jump maps in the concatenated interface space
  m.bg_row.assign(2 * m.sum_nb, -1);
  m.bg_sign.assign(2 * m.sum_nb, 0.0);
  m.bd_row.assign(3 * m.sum_nb, -1);
  m.bd_wt.assign(3 * m.sum_nb, 0.0);
  m.jr_b.assign(2 * m.n_lambda, -1);
  m.jr_sign.assign(2 * m.n_lambda, 0.0);
  for (int64_t j = 0; j < m.n_lambda; ++j) {
    const JumpRow& jr = m.rows[j];
    for (int e = 0; e < 2; ++e) {
      const SubHost& s = m.subs[jr.sub[e]];
      const int bl = jr.loc[e] - s.nI;
      if (bl < 0) return "jump row on an interior DOF";
      const int64_t gb = s.boff + bl;
      m.jr_b[2 * j + e] = (int32_t)gb;
      m.jr_sign[2 * j + e] = jr.sign[e];
      int slot = m.bg_row[2 * gb] < 0 ? 0 : 1;
      if (m.bg_row[2 * gb + slot] >= 0) return "interface DOF in more than two jump rows";
      m.bg_row[2 * gb + slot] = (int32_t)j;
      m.bg_sign[2 * gb + slot] = jr.sign[e];
    }
  }
  // scaled gather: (B^T D)[b, k] = sum_j B[j, b] D[j, k] over the group of b's DOF
  for (int64_t gb = 0; gb < m.sum_nb; ++gb) {
    if (m.bg_row[2 * gb] < 0) continue;
    const int j0 = m.bg_row[2 * gb];
    const int gs = m.grp_start[j0], gz = m.grp_size[j0];
    for (int k = 0; k < gz; ++k) {
      double v = 0.0;
      for (int slot = 0; slot < 2; ++slot) {
        const int j = m.bg_row[2 * gb + slot];
        if (j < 0) continue;
        v += m.bg_sign[2 * gb + slot] * m.dwt[3 * j + k];
      }
      m.bd_row[3 * gb + k] = gs + k;
      m.bd_wt[3 * gb + k] = v;
    }
  }
  // dual-primal coupling: the global primal order (field order, node, kind), so that the
  // U-type corners (u, eta) precede xi and p; per interface DOF its primal index, per
  // primal DOF its owners' interface indices (increasing subdomain)
  m.bpi.assign(m.sum_nb, -1);
  if (dp) {
    for (auto& kv : owners)
      if (kv.second.size() > 1 && is_primal(kv.first)) m.pi_code.push_back(kv.first);
    std::sort(m.pi_code.begin(), m.pi_code.end(), [](int32_t x, int32_t y) {
      return std::make_tuple(field_order(x % 8), x / 8, x % 8) < std::make_tuple(field_order(y % 8), y / 8, y % 8);
    });
    m.n_pi = (int)m.pi_code.size();
    m.n_pi_u = 0;
    for (int32_t c : m.pi_code)
      if (c % 8 <= K_ETA || c % 8 == K_UZ) ++m.n_pi_u;
    m.pi_own.assign(PI_OWNERS * (size_t)m.n_pi, -1);
    for (int k = 0; k < m.n_pi; ++k) {
      std::vector<int32_t> S = owners[m.pi_code[k]];
      std::sort(S.begin(), S.end());
      if (S.size() > (size_t)PI_OWNERS) return "a primal DOF shared by more than eight subdomains";
      for (size_t e = 0; e < S.size(); ++e) {
        const SubHost& sh = m.subs[S[e]];
        const int bl = pos[S[e]][m.pi_code[k]] - sh.nI;
        if (bl < 0) return "primal DOF in the interior";
        const int64_t gb = sh.boff + bl;
        m.pi_own[PI_OWNERS * (size_t)k + e] = (int32_t)gb;
        m.bpi[gb] = k;
      }
    }
  }
  return "";
}

// DOF -> (element, row) adjacency of the element tables
void build_adjacency(MeshHost& m) {
  // DOF -> (element, row) adjacency, elements in increasing order
  const int64_t nel = (int64_t)m.el_sub.size();
  std::vector<int32_t> cnt(m.sum_ns + 1, 0);
  for (int64_t e = 0; e < nel; ++e) {
    const SubHost& s = m.subs[m.el_sub[e]];
    for (int a = 0; a < m.edof; ++a) {
      const int li = m.el_ldof[e * m.edof + a];
      if (li >= 0) ++cnt[s.off + li + 1];
    }
  }
  m.adj_ptr.assign(m.sum_ns + 1, 0);
  for (int64_t i = 0; i < m.sum_ns; ++i) m.adj_ptr[i + 1] = m.adj_ptr[i] + cnt[i + 1];
  m.adj.assign(m.adj_ptr[m.sum_ns], 0);
  std::vector<int32_t> fill(m.adj_ptr.begin(), m.adj_ptr.end() - 1);
  for (int64_t e = 0; e < nel; ++e) {
    const SubHost& s = m.subs[m.el_sub[e]];
    for (int a = 0; a < m.edof; ++a) {
      const int li = m.el_ldof[e * m.edof + a];
      if (li >= 0) m.adj[fill[s.off + li]++] = (int32_t)(e * m.edof + a);
    }
  }
}

// d = 3: the unit cube in Kuhn tetrahedra (see feti.h), dual-primal coupling only.
std::string build_mesh3d(const feti_mesh_desc& d, MeshHost& m) {
  const int n = d.ncell;
  if (n < 2 || (d.order_u != 1 && d.order_u != 2) || d.nsub_x < 1 || d.nsub_y < 1 || d.nsub_z < 1 ||
      d.nsub_x > n || d.nsub_y > n || d.nsub_z > n)
    return "invalid mesh description";
  if (d.layout != FETI_XSPLIT || d.coupling != FETI_COUPLING_PRIMAL || d.scheme != FETI_SCHEME_COUPLED)
    return "3D takes the x-split layout, the dual-primal coupling and the coupled scheme";
  if (d.cut_x || d.cut_y) return "3D takes the even cuts";
  m = MeshHost();
  m.desc = d;
  m.dim = 3;
  m.ratio = d.order_u == 2 ? 2 : 1;
  const int r = m.ratio;
  const int nu = r * n;
  m.mu = nu + 1;
  m.n1 = n + 1;
  m.n_u_lat = (int64_t)m.mu * m.mu * m.mu;
  m.n_p1_lat = (int64_t)m.n1 * m.n1 * m.n1;
  const int ns3[3] = {d.nsub_x, d.nsub_y, d.nsub_z};
  std::vector<int> cut[3];
  std::vector<uint8_t> oncut[3];
  for (int a = 0; a < 3; ++a) {
    cut[a].resize(ns3[a] + 1);
    oncut[a].assign(n + 1, 0);
    for (int q = 0; q <= ns3[a]; ++q) {
      cut[a][q] = (int)((int64_t)q * n / ns3[a]);
      oncut[a][cut[a][q]] = 1;
    }
  }
  if (n % 2 || !oncut[0][n / 2]) return "a subdomain straddles the interface x = 1/2";
  const int nsub = d.nsub_x * d.nsub_y * d.nsub_z;
  m.subs.resize(nsub);
  auto on_faces = [](int I, int J, int K, int nmax, uint32_t mask) {
    return ((mask & 1u) && I == 0) || ((mask & 2u) && I == nmax) || ((mask & 4u) && J == 0) ||
           ((mask & 8u) && J == nmax) || ((mask & 16u) && K == 0) || ((mask & 32u) && K == nmax);
  };
  const int64_t mu = m.mu, n1 = m.n1;
  std::unordered_map<int32_t, std::vector<int32_t>> owners;
  owners.reserve((size_t)nsub * 256);
  std::vector<bool> has_dir(nsub, false);
  for (int c = 0; c < d.nsub_z; ++c)
    for (int b = 0; b < d.nsub_y; ++b)
      for (int a = 0; a < d.nsub_x; ++a) {
        const int sid = (c * d.nsub_y + b) * d.nsub_x + a;
        SubHost& s = m.subs[sid];
        s.sid = sid;
        s.i0 = cut[0][a]; s.i1 = cut[0][a + 1];
        s.j0 = cut[1][b]; s.j1 = cut[1][b + 1];
        s.k0 = cut[2][c]; s.k1 = cut[2][c + 1];
        s.poro = 2 * s.i1 <= n;
        for (int K = r * s.k0; K <= r * s.k1; ++K)
          for (int J = r * s.j0; J <= r * s.j1; ++J)
            for (int I = r * s.i0; I <= r * s.i1; ++I) {
              if (on_faces(I, J, K, nu, d.dirichlet_u)) { has_dir[sid] = true; continue; }
              const int32_t node = (int32_t)((K * mu + J) * mu + I);
              s.codes.push_back(8 * node + K_UX);
              s.codes.push_back(8 * node + K_UY);
              s.codes.push_back(8 * node + K_UZ);
            }
        for (int k = s.k0; k <= s.k1; ++k)
          for (int j = s.j0; j <= s.j1; ++j)
            for (int i = s.i0; i <= s.i1; ++i) {
              const int32_t node = (int32_t)((k * n1 + j) * n1 + i);
              if (s.poro) {
                s.codes.push_back(8 * node + K_ETA);
                s.codes.push_back(8 * node + K_XIP);
                if (!on_faces(i, j, k, n, d.dirichlet_p)) s.codes.push_back(8 * node + K_P);
              } else {
                s.codes.push_back(8 * node + K_XIE);
              }
            }
        for (int32_t cd : s.codes) owners[cd].push_back(sid);
      }
  auto is_primal = [&](int32_t cd) -> bool {
    const int64_t node = cd / 8;
    const int kind = cd % 8;
    if (kind == K_XIP || kind == K_P || kind == K_XIE) return true;
    if (kind == K_ETA) return oncut[0][node % n1] && oncut[1][(node / n1) % n1] && oncut[2][node / (n1 * n1)];
    const int64_t I = node % mu, J = (node / mu) % mu, K = node / (mu * mu);
    return I % r == 0 && J % r == 0 && K % r == 0 && oncut[0][I / r] && oncut[1][J / r] && oncut[2][K / r];
  };
  auto no_fix = [](const SubHost&, int32_t&, int32_t&, int32_t&) {};
  auto rigid_ok = [&](const std::vector<int32_t>& un) {
    // three primal displacement nodes not on one line
    if (un.size() < 3) return false;
    auto xyz = [&](int32_t node, double* x) {
      x[0] = (double)(node % mu); x[1] = (double)((node / mu) % mu); x[2] = (double)(node / (mu * mu));
    };
    double p0[3], p1[3], p2[3];
    xyz(un[0], p0);
    xyz(un[1], p1);
    const double u[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    for (size_t q = 2; q < un.size(); ++q) {
      xyz(un[q], p2);
      const double v[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
      const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
      if (cx * cx + cy * cy + cz * cz > 0.0) return true;
    }
    return false;
  };
  std::vector<std::unordered_map<int32_t, int32_t>> pos;
  {
    const std::string err = finish_interface(m, owners, has_dir, true, is_primal, no_fix, rigid_ok, pos);
    if (!err.empty()) return err;
  }
  // no floating subdomain, no coarse space
  m.sub_float.assign(nsub, -1);
  m.rb.assign(3 * m.sum_nb, 0.0);
  m.rfull.assign(3 * m.sum_ns, 0.0);
  m.n_float = 0;
  // element tables: cube (i, j, k) -> cell (k n + j) n + i, six tetrahedra per cube
  const int nloc = d.order_u == 2 ? 10 : 4;
  m.edof = 3 * nloc + 12;
  m.sub_el_off.assign(nsub + 1, 0);
  const int EP[6] = {0, 0, 0, 1, 1, 2}, EQ[6] = {1, 2, 3, 2, 3, 3};
  for (SubHost& s : m.subs) {
    const auto& P = pos[s.sid];
    for (int k = s.k0; k < s.k1; ++k)
      for (int j = s.j0; j < s.j1; ++j)
        for (int i = s.i0; i < s.i1; ++i)
          for (int t = 0; t < 6; ++t) {
            const int a = t / 2, rr = t % 2;
            const int b = a == 0 ? 1 + rr : (a == 1 ? 2 * rr : rr);
            int V[4][3] = {{i, j, k}, {i, j, k}, {i, j, k}, {i + 1, j + 1, k + 1}};
            V[1][a] += 1;
            V[2][a] += 1;
            V[2][b] += 1;
            int64_t un[10];
            for (int v = 0; v < 4; ++v) un[v] = ((int64_t)r * V[v][2] * mu + r * V[v][1]) * mu + r * V[v][0];
            if (nloc == 10)
              for (int e = 0; e < 6; ++e) {
                int U[3];
                for (int q = 0; q < 3; ++q) U[q] = (r * V[EP[e]][q] + r * V[EQ[e]][q]) / 2;
                un[4 + e] = ((int64_t)U[2] * mu + U[1]) * mu + U[0];
              }
            m.el_sub.push_back(s.sid);
            m.el_cell.push_back((k * n + j) * n + i);
            m.el_type.push_back(t);
            std::vector<int32_t> codes(m.edof, -1);
            for (int q = 0; q < nloc; ++q) {
              codes[3 * q] = (int32_t)(8 * un[q] + K_UX);
              codes[3 * q + 1] = (int32_t)(8 * un[q] + K_UY);
              codes[3 * q + 2] = (int32_t)(8 * un[q] + K_UZ);
            }
            for (int v = 0; v < 4; ++v) {
              const int32_t node = (int32_t)((V[v][2] * n1 + V[v][1]) * n1 + V[v][0]);
              if (s.poro) {
                codes[3 * nloc + v] = 8 * node + K_XIP;
                codes[3 * nloc + 4 + v] = 8 * node + K_ETA;
                codes[3 * nloc + 8 + v] = 8 * node + K_P;
              } else {
                codes[3 * nloc + v] = 8 * node + K_XIE;
              }
            }
            for (int q = 0; q < m.edof; ++q) {
              int32_t li = -1;
              if (codes[q] >= 0) {
                auto it = P.find(codes[q]);
                if (it != P.end()) li = it->second;
              }
              m.el_ldof.push_back(li);
              m.el_code.push_back(codes[q]);
            }
          }
    m.sub_el_off[s.sid + 1] = (int32_t)m.el_sub.size();
  }
  build_adjacency(m);
  build_deflation(m);
  return "";
}

// Normal-flux vectors of the dual-primal coupling.  For a pair of subdomains A < B that
// share a face (2D: an edge) the vector q has the entries that make q^T B u the integral
// over the face of the jump u_A . n - u_B . n (with the sign of the pair's rows) for the
// finite element u: every non-primal face node whose normal displacement component is a
// dual DOF contributes the face integral of its basis function, on the row between A and
// B, or, at a node with four owners (a 3D grid edge, multipliers chained in increasing
// subdomain order), on each chain row between A and B (the jump u_A - u_B is their sum).
// Face integrals per node are summed over the face's element sides (2D: segments, h/6 at
// the ends and 2h/3 at the midpoint for P2, h/2 at each end for P1) or triangles (3D:
// each cube face split along the diagonal from its low to its high corner; P2: 0 at the
// vertices and |t|/3 at the edge midpoints, P1: |t|/3 at the vertices), in units of the
// element size.  A row takes part in at most two vectors.
void build_deflation(MeshHost& m) {
  m.n_defl = 0;
  m.defl_col.assign(2 * m.n_lambda, -1);
  m.defl_w.assign(2 * m.n_lambda, 0.0);
  m.defl_ptr.assign(1, 0);
  m.defl_rows.clear();
  m.defl_rw.clear();
  const feti_mesh_desc& d = m.desc;
  const bool d3 = m.dim == 3;
  const int nsx = d.nsub_x, nsy = d.nsub_y;
  const int r = m.ratio;
  const int64_t mu = m.mu;
  auto grid = [&](int sid, int* g) {
    g[0] = sid % nsx;
    g[1] = d3 ? (sid / nsx) % nsy : sid / nsx;
    g[2] = d3 ? sid / (nsx * nsy) : 0;
  };
  // first row of every multiplier code (its chain rows follow in pair order)
  std::unordered_map<int32_t, int64_t> first_row;
  for (int64_t j = 0; j < m.n_lambda; ++j) first_row.emplace(m.rows[j].code, j);
  // the face pairs, in the order of their first normal-component row
  std::map<std::pair<int, int>, int> col_of;
  std::vector<std::pair<int, int>> pairs;
  std::vector<int> axis_of;
  for (int64_t j = 0; j < m.n_lambda; ++j) {
    const JumpRow& jr = m.rows[j];
    const int comp = jr.kind == K_UX ? 0 : jr.kind == K_UY ? 1 : jr.kind == K_UZ ? 2 : -1;
    if (comp < 0) continue;
    int g1[3], g2[3];
    grid(jr.sub[0], g1);
    grid(jr.sub[1], g2);
    int ndiff = 0, axis = -1;
    for (int q = 0; q < 3; ++q)
      if (g1[q] != g2[q]) { ++ndiff; axis = q; }
    if (ndiff != 1 || comp != axis) continue;
    const std::pair<int, int> key(std::min(jr.sub[0], jr.sub[1]), std::max(jr.sub[0], jr.sub[1]));
    if (col_of.emplace(key, (int)pairs.size()).second) {
      pairs.push_back(key);
      axis_of.push_back(axis);
    }
  }
  m.n_defl = (int)pairs.size();
  std::vector<std::vector<std::pair<int32_t, double>>> entries(m.n_defl);
  for (int c = 0; c < m.n_defl; ++c) {
    const int sA = pairs[c].first, sB = pairs[c].second, axis = axis_of[c];
    const int kind = axis == 0 ? K_UX : axis == 1 ? K_UY : K_UZ;
    const SubHost& A = m.subs[sA];
    const SubHost& Bs = m.subs[sB];
    const int lo[3] = {r * std::max(A.i0, Bs.i0), r * std::max(A.j0, Bs.j0), r * std::max(A.k0, Bs.k0)};
    const int hi[3] = {r * std::min(A.i1, Bs.i1), r * std::min(A.j1, Bs.j1), r * std::min(A.k1, Bs.k1)};
    std::map<int64_t, double> wm;  // node -> face integral (ordered: a fixed entry order)
    auto node_id = [&](const int* x) { return ((int64_t)x[2] * mu + x[1]) * mu + x[0]; };
    if (!d3) {
      const int t = 1 - axis;
      for (int e = lo[t]; e < hi[t]; e += r) {
        int x0[3] = {lo[0], lo[1], 0}, x1[3] = {lo[0], lo[1], 0};
        x0[t] = e;
        x1[t] = e + r;
        if (r == 2) {
          int xm[3] = {lo[0], lo[1], 0};
          xm[t] = e + 1;
          wm[node_id(x0)] += 1.0 / 6.0;
          wm[node_id(x1)] += 1.0 / 6.0;
          wm[node_id(xm)] += 2.0 / 3.0;
        } else {
          wm[node_id(x0)] += 0.5;
          wm[node_id(x1)] += 0.5;
        }
      }
    } else {
      const int p = axis == 0 ? 1 : 0, q = axis == 2 ? 1 : 2;  // in-plane directions
      const int tri[2][3][2] = {{{0, 0}, {1, 0}, {1, 1}}, {{0, 0}, {0, 1}, {1, 1}}};
      for (int a = lo[p]; a < hi[p]; a += r)
        for (int b = lo[q]; b < hi[q]; b += r)
          for (int t = 0; t < 2; ++t)
            for (int v = 0; v < 3; ++v) {
              int x[3] = {lo[0], lo[1], lo[2]};
              if (r == 1) {
                x[p] = a + tri[t][v][0];
                x[q] = b + tri[t][v][1];
              } else {  // the midpoint of the triangle's edge (v, v + 1)
                const int w2 = (v + 1) % 3;
                x[p] = a + tri[t][v][0] + tri[t][w2][0];
                x[q] = b + tri[t][v][1] + tri[t][w2][1];
              }
              wm[node_id(x)] += 1.0 / 3.0;
            }
    }
    for (const auto& kv : wm) {
      const int32_t code = (int32_t)(8 * kv.first + kind);
      const auto it = first_row.find(code);
      if (it == first_row.end()) continue;  // primal, Dirichlet or not shared
      const int64_t j0 = it->second;
      // the chain: owners S[0] < S[1] < ..., row j0 + k between S[k] and S[k + 1]
      std::vector<int> S{m.rows[j0].sub[0]};
      for (int64_t j = j0; j < m.n_lambda && m.rows[j].code == code; ++j) S.push_back(m.rows[j].sub[1]);
      const int ia = (int)(std::find(S.begin(), S.end(), sA) - S.begin());
      const int ib = (int)(std::find(S.begin(), S.end(), sB) - S.begin());
      if (ia >= (int)S.size() || ib >= (int)S.size()) continue;
      // orientation: the sign that the pair's own rows put on A (a P-E pair puts +1 on P)
      const double sigA = (m.subs[sA].poro != m.subs[sB].poro && !m.subs[sA].poro) ? -1.0 : 1.0;
      for (int k = ia; k < ib; ++k) {
        const int64_t jk = j0 + k;
        const double sgk = m.rows[jk].sign[0];  // sign on S[k]: row = sgk (u_S[k] - u_S[k+1])
        entries[c].push_back({(int32_t)jk, kv.second * sigA / sgk});
      }
    }
  }
  m.defl_ptr.assign(m.n_defl + 1, 0);
  for (int c = 0; c < m.n_defl; ++c) {
    m.defl_ptr[c + 1] = m.defl_ptr[c] + (int32_t)entries[c].size();
    for (const auto& e : entries[c]) {
      m.defl_rows.push_back(e.first);
      m.defl_rw.push_back(e.second);
      const int64_t j = e.first;
      const int slot = m.defl_col[2 * j] < 0 ? 0 : 1;
      m.defl_col[2 * j + slot] = c;
      m.defl_w[2 * j + slot] = e.second;
    }
  }
}

std::string build_mesh(const feti_mesh_desc& d, MeshHost& m) {
  if (d.dim == 3) return build_mesh3d(d, m);
  if (d.dim != 0 && d.dim != 2) return "dimension must be 2 or 3";
  const int n = d.ncell;
  if (n < 1 || (d.order_u != 1 && d.order_u != 2) || d.nsub_x < 1 || d.nsub_y < 1 ||
      d.nsub_x > n || d.nsub_y > n || d.layout < 0 || d.layout > 2)
    return "invalid mesh description";
  if (d.scheme != FETI_SCHEME_COUPLED && d.scheme != FETI_SCHEME_DECOUPLED) return "unknown time scheme";
  if (d.coupling != FETI_COUPLING_DUAL && d.coupling != FETI_COUPLING_PRIMAL) return "unknown coupling";
  const bool decoupled = d.scheme == FETI_SCHEME_DECOUPLED;
  const bool dp = d.coupling == FETI_COUPLING_PRIMAL;
  m = MeshHost();
  m.desc = d;
  m.ratio = d.order_u == 2 ? 2 : 1;
  const int r = m.ratio;
  const int nu = r * n;  // last displacement lattice index
  m.mu = nu + 1;
  m.n1 = n + 1;
  m.n_u_lat = (int64_t)m.mu * m.mu;
  m.n_p1_lat = (int64_t)m.n1 * m.n1;
  std::vector<int> cx(d.nsub_x + 1), cy(d.nsub_y + 1);
  for (int a = 0; a <= d.nsub_x; ++a) cx[a] = d.cut_x ? d.cut_x[a] : (int)((int64_t)a * n / d.nsub_x);
  for (int b = 0; b <= d.nsub_y; ++b) cy[b] = d.cut_y ? d.cut_y[b] : (int)((int64_t)b * n / d.nsub_y);
  if (cx[0] != 0 || cx[d.nsub_x] != n || cy[0] != 0 || cy[d.nsub_y] != n) return "cuts must run from 0 to ncell";
  for (int a = 0; a < d.nsub_x; ++a)
    if (cx[a + 1] <= cx[a]) return "cuts must increase strictly";
  for (int b = 0; b < d.nsub_y; ++b)
    if (cy[b + 1] <= cy[b]) return "cuts must increase strictly";
  // the pointers are the caller's: the stored description does not keep them
  m.desc.cut_x = nullptr;
  m.desc.cut_y = nullptr;
  const int nsub = d.nsub_x * d.nsub_y;
  m.subs.resize(nsub);
  // owners of every DOF code
  std::unordered_map<int32_t, std::vector<int32_t>> owners;
  owners.reserve((size_t)nsub * 64);
  std::vector<bool> has_dir(nsub, false);
  for (int b = 0; b < d.nsub_y; ++b) {
    for (int a = 0; a < d.nsub_x; ++a) {
      const int sid = b * d.nsub_x + a;
      SubHost& s = m.subs[sid];
      s.sid = sid;
      s.i0 = cx[a]; s.i1 = cx[a + 1]; s.j0 = cy[b]; s.j1 = cy[b + 1];
      if (s.i1 <= s.i0 || s.j1 <= s.j0) return "empty subdomain";
      const bool p0 = cell_poro(d.layout, s.i0, s.j0, n);
      for (int j = s.j0; j < s.j1; ++j)
        for (int i = s.i0; i < s.i1; ++i)
          if (cell_poro(d.layout, i, j, n) != p0) return "a subdomain straddles the interface";
      s.poro = p0;
      for (int J = r * s.j0; J <= r * s.j1; ++J)
        for (int I = r * s.i0; I <= r * s.i1; ++I) {
          if (on_sides(I, J, nu, d.dirichlet_u)) { has_dir[sid] = true; continue; }
          const int32_t node = J * m.mu + I;
          s.codes.push_back(8 * node + K_UX);
          s.codes.push_back(8 * node + K_UY);
        }
      for (int j = s.j0; j <= s.j1; ++j)
        for (int i = s.i0; i <= s.i1; ++i) {
          const int32_t node = j * m.n1 + i;
          if (s.poro) {
            // decoupled: eta and p are not unknowns of the subdomain problems
            if (!decoupled) s.codes.push_back(8 * node + K_ETA);
            s.codes.push_back(8 * node + K_XIP);
            if (!decoupled && !on_sides(i, j, n, d.dirichlet_p)) s.codes.push_back(8 * node + K_P);
          } else {
            s.codes.push_back(8 * node + K_XIE);
          }
        }
      for (int32_t c : s.codes) owners[c].push_back(sid);
    }
  }
  // dual-primal coupling: a shared code is primal when its kind is xi_P, p or xi_E, or when
  // its node lies on a vertical and a horizontal cut line (outer sides included)
  std::vector<uint8_t> xcut(n + 1, 0), ycut(n + 1, 0);
  for (int a = 0; a <= d.nsub_x; ++a) xcut[cx[a]] = 1;
  for (int b = 0; b <= d.nsub_y; ++b) ycut[cy[b]] = 1;
  auto is_primal = [&](int32_t c) -> bool {
    const int node = c / 8, kind = c % 8;
    if (kind == K_XIP || kind == K_P || kind == K_XIE) return true;
    if (kind == K_ETA) return xcut[node % m.n1] && ycut[node / m.n1];
    const int I = node % m.mu, J = node / m.mu;
    return I % r == 0 && J % r == 0 && xcut[I / r] && ycut[J / r];
  };
  std::vector<std::unordered_map<int32_t, int32_t>> pos;
  {
    auto fixed_codes = [&](const SubHost& sh, int32_t& fa, int32_t& fb, int32_t& fc) {
      const int32_t A = (r * sh.j0) * m.mu + r * sh.i0;
      const int32_t C = (r * sh.j1) * m.mu + r * sh.i1;
      fa = 8 * A + K_UX; fb = 8 * A + K_UY; fc = 8 * C + K_UX;
    };
    auto rigid_ok = [](const std::vector<int32_t>& un) { return un.size() >= 2; };
    const std::string err = finish_interface(m, owners, has_dir, dp, is_primal, fixed_codes, rigid_ok, pos);
    if (!err.empty()) return err;
  }
  // coarse space: rigid modes of floating subdomains
  m.sub_float.assign(nsub, -1);
  m.rb.assign(3 * m.sum_nb, 0.0);
  m.rfull.assign(3 * m.sum_ns, 0.0);
  const double hs = 1.0 / (double)nu;
  for (SubHost& s : m.subs) {
    if (!s.floating) continue;
    m.sub_float[s.sid] = (int32_t)m.float_sub.size();
    m.float_sub.push_back(s.sid);
    const double xc = 0.5 * (s.i0 + s.i1) / (double)n, yc = 0.5 * (s.j0 + s.j1) / (double)n;
    for (int i = 0; i < s.ns; ++i) {
      const int32_t c = s.codes[i];
      const int kind = c % 8, node = c / 8;
      if (kind > K_UY) continue;
      const double x = (node % m.mu) * hs, y = (node / m.mu) * hs;
      double* R = &m.rfull[3 * (s.off + i)];
      R[kind] = 1.0;
      R[2] = kind == K_UX ? -(y - yc) : (x - xc);
      if (i >= s.nI) {
        double* Rb = &m.rb[3 * (s.boff + (i - s.nI))];
        Rb[0] = R[0]; Rb[1] = R[1]; Rb[2] = R[2];
      }
    }
  }
  m.n_float = (int)m.float_sub.size();
  // element tables
  const int nloc = d.order_u == 2 ? 6 : 3;
  m.edof = 2 * nloc + 9;  // u, then xi, eta, p (elastic: u, xi_E, unused)
  m.sub_el_off.assign(nsub + 1, 0);
  for (SubHost& s : m.subs) {
    const auto& P = pos[s.sid];
    for (int j = s.j0; j < s.j1; ++j)
      for (int i = s.i0; i < s.i1; ++i)
        for (int t = 0; t < 2; ++t) {
          // vertices on the P1 lattice (counter-clockwise)
          int vi[3], vj[3];
          if (t == 0) { vi[0] = i; vj[0] = j; vi[1] = i + 1; vj[1] = j; vi[2] = i + 1; vj[2] = j + 1; }
          else { vi[0] = i; vj[0] = j; vi[1] = i + 1; vj[1] = j + 1; vi[2] = i; vj[2] = j + 1; }
          int32_t un[6];
          for (int v = 0; v < 3; ++v) un[v] = (r * vj[v]) * m.mu + r * vi[v];
          if (nloc == 6) {
            const int pa[3] = {0, 1, 2}, pb[3] = {1, 2, 0};
            for (int e = 0; e < 3; ++e) {
              const int I = (r * vi[pa[e]] + r * vi[pb[e]]) / 2, J = (r * vj[pa[e]] + r * vj[pb[e]]) / 2;
              un[3 + e] = J * m.mu + I;
            }
          }
          m.el_sub.push_back(s.sid);
          m.el_cell.push_back(j * n + i);
          m.el_type.push_back(t);
          std::vector<int32_t> codes(m.edof, -1);
          for (int a = 0; a < nloc; ++a) {
            codes[2 * a] = 8 * un[a] + K_UX;
            codes[2 * a + 1] = 8 * un[a] + K_UY;
          }
          for (int v = 0; v < 3; ++v) {
            const int32_t node = vj[v] * m.n1 + vi[v];
            if (s.poro) {
              codes[2 * nloc + v] = 8 * node + K_XIP;
              codes[2 * nloc + 3 + v] = 8 * node + K_ETA;
              codes[2 * nloc + 6 + v] = 8 * node + K_P;
            } else {
              codes[2 * nloc + v] = 8 * node + K_XIE;
            }
          }
          for (int a = 0; a < m.edof; ++a) {
            int32_t li = -1;
            if (codes[a] >= 0) {
              auto it = P.find(codes[a]);
              if (it != P.end()) li = it->second;
            }
            m.el_ldof.push_back(li);
            m.el_code.push_back(codes[a]);
          }
        }
    m.sub_el_off[s.sid + 1] = (int32_t)m.el_sub.size();
  }
  // decoupled scheme: the fluid nodes and their element entries
  if (decoupled) {
    const int n1n = m.n1 * m.n1;
    std::vector<int32_t> cntn(n1n, 0), dec_index(n1n, -1);
    const int64_t nel0 = (int64_t)m.el_sub.size();
    for (int64_t e = 0; e < nel0; ++e) {
      if (!m.subs[m.el_sub[e]].poro) continue;
      for (int v = 0; v < 3; ++v) ++cntn[m.el_code[e * m.edof + 2 * nloc + v] >> 3];
    }
    for (int node = 0; node < n1n; ++node)
      if (cntn[node] > 0) {
        dec_index[node] = (int32_t)m.dec_node.size();
        m.dec_node.push_back(node);
        const int i = node % m.n1, j = node / m.n1;
        m.dec_pdir.push_back(on_sides(i, j, n, d.dirichlet_p) ? 1 : 0);
      }
    const int nd = (int)m.dec_node.size();
    m.dec_ptr.assign(nd + 1, 0);
    for (int k = 0; k < nd; ++k) m.dec_ptr[k + 1] = m.dec_ptr[k] + cntn[m.dec_node[k]];
    m.dec_ent.assign(m.dec_ptr[nd], 0);
    std::vector<int32_t> fillp(m.dec_ptr.begin(), m.dec_ptr.end() - 1);
    for (int64_t e = 0; e < nel0; ++e) {
      if (!m.subs[m.el_sub[e]].poro) continue;
      for (int v = 0; v < 3; ++v) {
        const int k = dec_index[m.el_code[e * m.edof + 2 * nloc + v] >> 3];
        m.dec_ent[fillp[k]++] = (int32_t)(e * 3 + v);
      }
    }
    m.dec_xi.assign(nd, -1);
    for (const SubHost& s : m.subs) {
      if (!s.poro) continue;
      for (int i = 0; i < s.ns; ++i) {
        const int32_t c = s.codes[i];
        if (c % 8 != K_XIP) continue;
        const int k = dec_index[c / 8];
        if (k >= 0 && m.dec_xi[k] < 0) m.dec_xi[k] = (int32_t)(s.off + i);
      }
    }
    for (int k = 0; k < nd; ++k)
      if (m.dec_xi[k] < 0) return "a poroelastic node without a xi_P unknown";
  }
  build_adjacency(m);
  if (dp) build_deflation(m);
  return "";
}

}  // namespace feti