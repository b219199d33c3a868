"""A second, independent reference at 50 significant digits (mpmath) for tiny
axisymmetric grids: one global step of the scheme (Sec. 3.1-3.5) written
again from the paper and the readings the FP64 reference documents, in plain
Python, sharing no code with it.  It serves only to show that the FP64
reference's result is its arithmetic's rounding of the same computation.

Scope: the 2D axisymmetric wedge (theta over [0, pi], one phi zone), a
specular inner boundary and an outflow outer boundary, Gauss-Legendre or
Gauss-Lobatto mu nodes, the linear or the direction-preserving Phi split, any
number of species and groups.
"""

import mpmath as mp

mp.mp.dps = 50
PI = mp.pi


def mpf(x):
    return mp.mpf(float(x)) if not isinstance(x, mp.mpf) else x


def legendre(n):
    xs, ws = [], []
    for k in range(1, n + 1):
        x = mp.cos(PI * (k - mp.mpf(1) / 4) / (n + mp.mpf(1) / 2))
        for _ in range(100):
            p0, p1 = mp.mpf(1), x
            for m in range(2, n + 1):
                p0, p1 = p1, ((2 * m - 1) * x * p1 - (m - 1) * p0) / m
            dp = n * (x * p1 - p0) / (x * x - 1)
            dx = p1 / dp
            x -= dx
            if abs(dx) < mp.mpf(10) ** -45:
                break
        p0, p1 = mp.mpf(1), x
        for m in range(2, n + 1):
            p0, p1 = p1, ((2 * m - 1) * x * p1 - (m - 1) * p0) / m
        dp = n * (x * p1 - p0) / (x * x - 1)
        xs.append(x)
        ws.append(2 / ((1 - x * x) * dp * dp))
    order = sorted(range(n), key=lambda i: xs[i])
    return [xs[i] for i in order], [ws[i] for i in order]


def lobatto(n):
    """Gauss-Lobatto nodes (-1, +1 and the zeros of the derivative of P_{n-1},
    found by Newton's method from Chebyshev-Gauss-Lobatto guesses) and weights
    2 / (n (n-1) P_{n-1}(x)^2)"""
    m = n - 1

    def P_and_dP(x):
        p0, p1 = mp.mpf(1), x
        for k in range(2, m + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        # P_m'(x) = m (x P_m - P_{m-1}) / (x^2 - 1), and P_m'' from the Legendre equation
        d1 = m * (x * p1 - p0) / (x * x - 1)
        d2 = (2 * x * d1 - m * (m + 1) * p1) / (1 - x * x)
        return p1, d1, d2

    xs = [mp.mpf(-1)]
    for k in range(1, m):
        x = -mp.cos(PI * k / m)
        for _ in range(100):
            _, d1, d2 = P_and_dP(x)
            dx = d1 / d2
            x -= dx
            if abs(dx) < mp.mpf(10) ** -45:
                break
        xs.append(x)
    xs.append(mp.mpf(1))
    xs.sort()
    ws = []
    for x in xs:
        p0, p1 = mp.mpf(1), x
        for k in range(2, m + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        ws.append(mp.mpf(2) / (n * (n - 1) * p1 * p1))
    return xs, ws


def point(r, t, p):
    return [r * mp.sin(t) * mp.cos(p), r * mp.sin(t) * mp.sin(p), r * mp.cos(t)]


def cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def quad(p1, p2, p3, p4):
    """flat quadrilateral: half the cross product of the diagonals"""
    n = cross([p3[i] - p1[i] for i in range(3)], [p4[i] - p2[i] for i in range(3)])
    return mp.sqrt(sum(x * x for x in n)) / 2, n


def dist(r1, t1, p1, r2, t2, p2):
    a, b = point(r1, t1, p1), point(r2, t2, p2)
    return mp.sqrt(sum((a[i] - b[i]) ** 2 for i in range(3)))


def basis(t, p):
    """columns e_r, e_theta, e_phi at (t, p), as rows of the transposed matrix"""
    st, ct, sp, cp = mp.sin(t), mp.cos(t), mp.sin(p), mp.cos(p)
    return [[st * cp, st * sp, ct], [ct * cp, ct * sp, -st], [-sp, cp, mp.mpf(0)]]


def to_basis(ta, pa, tb, pb, x):
    if ta == tb and pa == pb:
        return list(x)
    A, B = basis(ta, pa), basis(tb, pb)
    cart = [sum(A[j][i] * x[j] for j in range(3)) for i in range(3)]
    return [sum(B[j][i] * cart[i] for i in range(3)) for j in range(3)]


def lorentz(v, u):
    """boost of the four-vector u by the 3-velocity v"""
    g = gamma(v)
    k = g * g / (g + 1)                      # (gamma - 1) / v^2
    vu = sum(v[i] * u[i + 1] for i in range(3))
    return [g * (u[0] + vu)] + [u[i + 1] + (k * vu + g * u[0]) * v[i] for i in range(3)]


class Frame:
    def __init__(self, v, alpha, psi, th, ph):
        self.v, self.alpha, self.psi, self.th, self.ph = list(v), alpha, psi, th, ph

    def key(self):
        return tuple(self.v) + (self.alpha, self.psi, self.th, self.ph)


def gamma(v):
    return 1 / mp.sqrt(1 - sum(x * x for x in v))


def transform(S, D, axis, u):
    """comoving(S) -> comoving(D): boost out of S, to covariant components,
    kick on the axis of motion when the metric changes, rotate the basis,
    back with the metric of D, boost into D"""
    e = lorentz(S.v, u)
    low0 = -S.alpha * e[0]
    low = [S.psi ** 2 * e[i + 1] for i in range(3)]
    if S.alpha != D.alpha or S.psi != D.psi:
        perp = sum(low[i] ** 2 for i in range(3) if i != axis)
        rad = D.psi ** 4 * low0 ** 2 / D.alpha ** 2 - perp
        if rad >= 0:
            low[axis] = (1 if low[axis] >= 0 else -1) * mp.sqrt(rad)
        else:
            sc = D.psi ** 2 * abs(low0) / D.alpha / mp.sqrt(perp)
            low = [mp.mpf(0) if i == axis else low[i] * sc for i in range(3)]
    lowD = to_basis(S.th, S.ph, D.th, D.ph, low)
    eD = [-low0 / D.alpha] + [x / D.psi ** 2 for x in lowD]
    return lorentz([-x for x in D.v], eD)


class Grid:
    def __init__(self, w):
        self.w = w
        self.nr, self.nth, self.ne = w.n_r, w.n_theta, w.n_eps
        self.nmu, self.nphi, self.ns = w.n_mu, w.n_phi, w.n_species
        self.nd = self.nmu * self.nphi
        self.nz = self.nr * self.nth
        e = [mpf(x) for x in w.eps_edges]
        self.eps = [mp.sqrt(e[i] * e[i + 1]) for i in range(self.ne)]
        self.G = [(e[i + 1] ** 3 - e[i] ** 3) / 3 for i in range(self.ne)]
        self.mu, wmu = lobatto(self.nmu) if w.mu_rule == "lobatto" else legendre(self.nmu)
        self.phi_sin = w.phi_rule == 0        # Phi split keeping the direction (else linear)
        self.Phi = [(k + mp.mpf(1) / 2) * 2 * PI / self.nphi for k in range(self.nphi)]
        self.dOm, self.n = [], []
        for j in range(self.nmu):
            for k in range(self.nphi):
                self.dOm.append(wmu[j] * 2 * PI / self.nphi)
                st = mp.sqrt(1 - self.mu[j] ** 2)
                self.n.append([self.mu[j], st * mp.cos(self.Phi[k]), st * mp.sin(self.Phi[k])])
        self.re = [mpf(x) for x in w.r_edges]
        self.te = [mpf(x) for x in w.theta_edges]
        self.dphi = mpf(w.dphi)
        self.rc, self.thc, self.vol = [], [], []
        for b in range(self.nth):
            p0, p1 = -self.dphi / 2, self.dphi / 2
            A1, nrm = quad(point(1, self.te[b], p0), point(1, self.te[b + 1], p0),
                           point(1, self.te[b + 1], p1), point(1, self.te[b], p1))
            V1 = point(1, self.te[b], p0)
            h1 = abs(sum(nrm[i] * V1[i] for i in range(3))) / mp.sqrt(sum(x * x for x in nrm))
            for a in range(self.nr):
                lo, hi = self.re[a], self.re[a + 1]
                self.rc.append((lo + hi) / 2)
                self.thc.append((self.te[b] + self.te[b + 1]) / 2)
                self.vol.append((hi ** 3 - lo ** 3) * A1 * h1 / 3)
        self.bg = {k: [mpf(x) for x in getattr(w, k).ravel()] for k in
                   ("v_r", "v_theta", "alpha", "psi", "kappa_a", "kappa_s", "f_eq")}
        self.faces = self._faces()

    # ------------------------------------------------------------- frames
    def frame(self, z, th, ph, mirror=False):
        v = [self.bg["v_r"][z], self.bg["v_theta"][z], mp.mpf(0)]
        if mirror:
            v[0] = -v[0]
        return Frame(v, self.bg["alpha"][z], self.bg["psi"][z], th, ph)

    def side(self, z, th, ph):
        return {"kind": "zone", "z": z, "slope": True, "fr": self.frame(z, th, ph)}

    def ghost(self, z, inner):
        return {"kind": "mirror" if inner else "zero", "z": z, "slope": False,
                "fr": self.frame(z, self.thc[z], mp.mpf(0), mirror=inner)}

    def interface(self, L, R, th, ph):
        vl = to_basis(L.th, L.ph, th, ph, L.v)
        vr = to_basis(R.th, R.ph, th, ph, R.v)
        return Frame([(vl[i] + vr[i]) / 2 for i in range(3)], (L.alpha + R.alpha) / 2,
                     (L.psi + R.psi) / 2, th, ph)

    def _faces(self):
        """faces in the order radial (per row), theta, phi; each with its two
        sides, geometry and interface frame"""
        F, zero = [], mp.mpf(0)
        p0, p1 = -self.dphi / 2, self.dphi / 2
        for b in range(self.nth):
            th = (self.te[b] + self.te[b + 1]) / 2
            A1 = quad(point(1, self.te[b], p0), point(1, self.te[b + 1], p0),
                      point(1, self.te[b + 1], p1), point(1, self.te[b], p1))[0]
            for a in range(-1, self.nr):
                R = self.re[a + 1]
                zL, zR = b * self.nr + a, b * self.nr + a + 1
                f = {"axis": 0, "area": R * R * A1, "active": R != 0}
                f["L"] = self.side(zL, th, zero) if a >= 0 else self.ghost(zR, True)
                f["R"] = self.side(zR, th, zero) if a + 1 < self.nr else self.ghost(zL, False)
                if a >= 0 and a + 1 < self.nr:
                    f["h"] = self.rc[zR] - self.rc[zL]
                elif a < 0:
                    f["h"] = 2 * (self.rc[zR] - R)
                else:
                    f["h"] = 2 * (R - self.rc[zL])
                f["dL"] = R - self.rc[zL] if a >= 0 else f["h"] / 2
                f["dR"] = -(self.rc[zR] - R) if a + 1 < self.nr else -f["h"] / 2
                f["s"] = self.interface(f["L"]["fr"], f["R"]["fr"], th, zero)
                f["zero_opacity"] = "zero" in (f["L"]["kind"], f["R"]["kind"])
                F.append(f)
        for b in range(self.nth - 1):
            for a in range(self.nr):
                zL, zR = b * self.nr + a, (b + 1) * self.nr + a
                tf = self.te[b + 1]
                f = {"axis": 1, "active": True, "zero_opacity": False}
                f["area"] = quad(point(self.re[a], tf, p0), point(self.re[a + 1], tf, p0),
                                 point(self.re[a + 1], tf, p1), point(self.re[a], tf, p1))[0]
                f["L"] = self.side(zL, self.thc[zL], zero)
                f["R"] = self.side(zR, self.thc[zR], zero)
                f["h"] = dist(self.rc[zL], self.thc[zL], zero, self.rc[zR], self.thc[zR], zero)
                f["dL"], f["dR"] = f["h"] / 2, -f["h"] / 2
                f["s"] = self.interface(f["L"]["fr"], f["R"]["fr"], tf, zero)
                F.append(f)
        for z in range(self.nz):
            a, b = z % self.nr, z // self.nr
            tlo, thi, w = self.te[b], self.te[b + 1], self.dphi
            pf, th = w / 2, self.thc[z]
            f = {"axis": 2, "active": True, "zero_opacity": False, "self": True}
            f["area"] = quad(point(self.re[a], tlo, pf), point(self.re[a + 1], tlo, pf),
                             point(self.re[a + 1], thi, pf), point(self.re[a], thi, pf))[0]
            f["L"] = self.side(z, th, zero)
            f["R"] = self.side(z, th, w)
            f["h"] = dist(self.rc[z], th, zero, self.rc[z], th, w)
            f["dL"], f["dR"] = f["h"] / 2, -f["h"] / 2
            f["s"] = self.interface(f["L"]["fr"], f["R"]["fr"], th, pf)
            F.append(f)
        return F

    def zone_faces(self, z):
        """(face, +1 if the zone is R else -1), in the reference's order"""
        a, b = z % self.nr, z // self.nr
        nfr = self.nth * (self.nr + 1)
        out = [(b * (self.nr + 1) + a, 1), (b * (self.nr + 1) + a + 1, -1)]
        if b > 0:
            out.append((nfr + (b - 1) * self.nr + a, 1))
        if b < self.nth - 1:
            out.append((nfr + b * self.nr + a, -1))
        nft = (self.nth - 1) * self.nr
        out += [(nfr + nft + z, -1), (nfr + nft + z, 1)]
        return out

    # -------------------------------------------------------------- remap
    def u0(self, fr, d):
        return gamma(fr.v) * (1 + sum(fr.v[i] * self.n[d][i] for i in range(3)))

    @staticmethod
    def bracket(xs, x):
        if len(xs) == 1 or x <= xs[0]:
            return 0, 0, mp.mpf(0)
        if x >= xs[-1]:
            return len(xs) - 1, len(xs) - 1, mp.mpf(0)
        l = max(i for i in range(len(xs) - 1) if xs[i] <= x)
        return l, l + 1, (x - xs[l]) / (xs[l + 1] - xs[l])

    def remap(self, S, D, axis, density, X):
        """number content of every source bin split over the 2x2x2 bracketing
        destination bins (linear weights in energy, mu and Phi)"""
        if S.key() == D.key():
            return [list(row) for row in X]
        ne, nd, nphi = self.ne, self.nd, self.nphi
        acc = [[mp.mpf(0)] * nd for _ in range(ne)]
        for d in range(nd):
            o = transform(S, D, axis, [mp.mpf(1)] + self.n[d])
            rho, mus = o[0], min(max(o[1] / o[0], mp.mpf(-1)), mp.mpf(1))
            if o[2] ** 2 + o[3] ** 2 <= mp.mpf("1e-12") * o[0] ** 2:
                P = self.Phi[d % nphi]
            else:
                P = mp.atan2(o[3], o[2])
                if P < 0:
                    P += 2 * PI
            jL, jR, wj = self.bracket(self.mu, mus)
            if nphi == 1:
                kL = kR = 0
                wk = mp.mpf(0)
            else:
                dP = 2 * PI / nphi
                kl = int(mp.floor(P / dP - mp.mpf(1) / 2))
                PL = (kl + mp.mpf(1) / 2) * dP
                if self.phi_sin:
                    # weights proportional to the sines of the angular distances to the
                    # far node: the split keeps the direction of the transverse momentum
                    a, b = mp.sin(PL + dP - P), mp.sin(P - PL)
                    wk = b / (a + b)
                else:
                    wk = (P - PL) / dP
                kL, kR = kl % nphi, (kl + 1) % nphi
            Wsd = S.psi ** 6 * self.u0(S, d) * self.dOm[d] if density else 1
            for i in range(ne):
                n = X[i][d] * (Wsd * self.G[i] if density else 1)
                if n == 0:
                    continue
                iL, iR, wi = self.bracket(self.eps, rho * self.eps[i])
                for ii, wI in ((iL, 1 - wi), (iR, wi)):
                    for jj, wJ in ((jL, 1 - wj), (jR, wj)):
                        for kk, wK in ((kL, 1 - wk), (kR, wk)):
                            acc[ii][jj * nphi + kk] += n * wI * wJ * wK
        out = [[mp.mpf(0)] * nd for _ in range(ne)]
        for i in range(ne):
            for d in range(nd):
                W = D.psi ** 6 * self.u0(D, d) * self.G[i] * self.dOm[d] if density else 1
                out[i][d] = acc[i][d] / W
        return out

    # ----------------------------------------------------------- the step
    def data(self, f, sd, s):
        z = sd["z"]
        if sd["kind"] == "zone":
            return [list(row) for row in f[z][s]]
        if sd["kind"] == "zero":
            return [[mp.mpf(0)] * self.nd for _ in range(self.ne)]
        return [[f[z][s][i][(self.nmu - 1 - d // self.nphi) * self.nphi + d % self.nphi]
                 for d in range(self.nd)] for i in range(self.ne)]

    def neighbours(self, z, axis):
        a, b = z % self.nr, z // self.nr
        th, zero = self.thc[z], mp.mpf(0)
        if axis == 0:
            m = (self.side(z - 1, th, zero), self.rc[z] - self.rc[z - 1]) if a > 0 else \
                (self.ghost(z, True), 2 * (self.rc[z] - self.re[0]))
            p = (self.side(z + 1, th, zero), self.rc[z + 1] - self.rc[z]) if a < self.nr - 1 else \
                (self.ghost(z, False), 2 * (self.re[-1] - self.rc[z]))
            return m, p
        if axis == 1:
            zm = z - self.nr if b > 0 else z
            zp = z + self.nr if b < self.nth - 1 else z

            def nb(y):
                h = mp.mpf(1) if y == z else dist(self.rc[y], self.thc[y], zero, self.rc[z], self.thc[z], zero)
                return self.side(y, self.thc[y], zero), h
            return nb(zm), nb(zp)
        h = dist(self.rc[z], th, zero, self.rc[z], th, self.dphi)
        return (self.side(z, th, -self.dphi), h), (self.side(z, th, self.dphi), h)

    def slope(self, f, z, axis):
        (m, hm), (p, hp) = self.neighbours(z, axis)
        me = self.frame(z, self.thc[z], mp.mpf(0))
        out = []
        for s in range(self.ns):
            Ym = self.remap(m["fr"], me, axis, True, self.data(f, m, s))
            Yp = self.remap(p["fr"], me, axis, True, self.data(f, p, s))
            sl = []
            for i in range(self.ne):
                row = []
                for d in range(self.nd):
                    dm, dp = (f[z][s][i][d] - Ym[i][d]) / hm, (Yp[i][d] - f[z][s][i][d]) / hp
                    A, B, M = 2 * dm, 2 * dp, (dm + dp) / 2
                    if A > 0 and B > 0 and M > 0:
                        row.append(min(A, B, M))
                    elif A < 0 and B < 0 and M < 0:
                        row.append(max(A, B, M))
                    else:
                        row.append(mp.mpf(0))
                sl.append(row)
            out.append(sl)
        return out

    def collide(self, S, tau, ka, ks, feq):
        avg = sum(S[d] * self.dOm[d] for d in range(self.nd)) / (4 * PI)
        fav = avg / (1 + tau * ka)
        return [(S[d] + tau * ks * fav) / (1 + tau * (ka + ks)) for d in range(self.nd)]

    def face(self, f, F, dt):
        """content changes of the two sides of face F (all species)"""
        ax, s_fr = F["axis"], F["s"]
        L, R = F["L"], F["R"]
        g = gamma(s_fr.v)
        ap4 = s_fr.alpha * s_fr.psi ** 4
        vn = s_fr.v[ax]
        Uadv = ap4 * g * vn
        Ur, Vn, UL, UR = [], [], [], []
        for d in range(self.nd):
            nv = self.n[d]
            # the direction boosted out of the interface frame: u^0, its normal
            # component, and the radiative part of the normal speed
            e = lorentz(s_fr.v, [mp.mpf(1)] + nv)
            k = g * g / (g + 1)
            vdn = sum(s_fr.v[i] * nv[i] for i in range(3))
            Ur.append(ap4 * (nv[ax] + k * vdn * vn))
            Vn.append(s_fr.alpha * e[1 + ax] / (s_fr.psi ** 2 * e[0]))
            for side, lst in ((L, UL), (R, UR)):
                e = lorentz(side["fr"].v, [mp.mpf(1)] + nv)
                y = to_basis(side["fr"].th, side["fr"].ph, s_fr.th, s_fr.ph, e[1:])
                lst.append(ap4 * y[ax])
        slL = self.slope(f, L["z"], ax) if L["slope"] else None
        slR = self.slope(f, R["z"], ax) if R["slope"] else None
        tau = s_fr.alpha * dt / g / 2
        cA = dt * F["area"]
        dNL, dNR = [], []
        for sp in range(self.ns):
            XL, XR = self.data(f, L, sp), self.data(f, R, sp)
            A = self.remap(L["fr"], s_fr, ax, True, XL)
            B = self.remap(R["fr"], s_fr, ax, True, XR)
            EL = [[XL[i][d] + (F["dL"] * slL[sp][i][d] if slL else 0) for d in range(self.nd)]
                  for i in range(self.ne)]
            ER = [[XR[i][d] + (F["dR"] * slR[sp][i][d] if slR else 0) for d in range(self.nd)]
                  for i in range(self.ne)]
            FL = [[mp.mpf(0)] * self.nd for _ in range(self.ne)]
            for i in range(self.ne):
                if F["zero_opacity"]:
                    ka = ks = fe = mp.mpf(0)
                else:
                    kl = (L["z"] * self.ns + sp) * self.ne + i
                    kr = (R["z"] * self.ns + sp) * self.ne + i
                    ka = (self.bg["kappa_a"][kl] + self.bg["kappa_a"][kr]) / 2
                    ks = (self.bg["kappa_s"][kl] + self.bg["kappa_s"][kr]) / 2
                    fe = (self.bg["f_eq"][kl] + self.bg["f_eq"][kr]) / 2
                Sv = [(A[i][d] + B[i][d]) / 2 - dt * Vn[d] * (B[i][d] - A[i][d]) / (2 * F["h"]) + tau * ka * fe
                      for d in range(self.nd)]
                flw = self.collide(Sv, tau, ka, ks, fe)
                w = mp.exp(-(ka + ks) * F["h"])
                for d in range(self.nd):
                    dG = self.G[i] * self.dOm[d]
                    FL[i][d] = cA * (1 - w) * Ur[d] * flw[d] * dG
                    eL = w * max(UL[d], 0) + (1 - w) * max(Uadv, 0)
                    eR = w * max(-UR[d], 0) + (1 - w) * max(-Uadv, 0)
                    EL[i][d] = cA * eL * EL[i][d] * dG
                    ER[i][d] = cA * eR * ER[i][d] * dG
            YL = self.remap(s_fr, L["fr"], ax, False, FL)
            YR = self.remap(s_fr, R["fr"], ax, False, FL)
            RL = self.remap(R["fr"], L["fr"], ax, False, ER)
            LR = self.remap(L["fr"], R["fr"], ax, False, EL)
            dNL.append([[-YL[i][d] - EL[i][d] + RL[i][d] for d in range(self.nd)] for i in range(self.ne)])
            dNR.append([[YR[i][d] - ER[i][d] + LR[i][d] for d in range(self.nd)] for i in range(self.ne)])
        return dNL, dNR

    def step(self, f, dt):
        dt = mpf(dt)
        contrib = [self.face(f, F, dt) if F["active"] else None for F in self.faces]
        out = []
        for z in range(self.nz):
            me = self.frame(z, self.thc[z], mp.mpf(0))
            g = gamma(me.v)
            tau = me.alpha * dt / g
            new_z = []
            for s in range(self.ns):
                blk = []
                for i in range(self.ne):
                    dN = [mp.mpf(0)] * self.nd
                    for fid, sg in self.zone_faces(z):
                        if contrib[fid] is None:
                            continue
                        src = contrib[fid][1 if sg > 0 else 0][s][i]
                        dN = [dN[d] + src[d] for d in range(self.nd)]
                    k = (z * self.ns + s) * self.ne + i
                    ka, ks, fe = self.bg["kappa_a"][k], self.bg["kappa_s"][k], self.bg["f_eq"][k]
                    S = [f[z][s][i][d] + tau * ka * fe +
                         dN[d] / (me.psi ** 6 * self.vol[z] * self.u0(me, d) * self.G[i] * self.dOm[d])
                         for d in range(self.nd)]
                    blk.append(self.collide(S, tau, ka, ks, fe))
                new_z.append(blk)
            out.append(new_z)
        return out


def run(w, dt, steps):
    """the state after `steps` global steps of size dt, as nested lists of mpf"""
    grid = Grid(w)
    f = [[[[mpf(w.f0[z, s, i, d]) for d in range(grid.nd)] for i in range(grid.ne)]
          for s in range(grid.ns)] for z in range(grid.nz)]
    for _ in range(steps):
        f = grid.step(f, dt)
    return f
