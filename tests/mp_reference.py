"""Brute-force reference with mpmath (30 digits) for single P0 pairs.

Polar coordinates about the particle: the radial integral is exact (a
polynomial antiderivative), the angular one uses mpmath.quad split at the
vertex directions and circle crossings.  Independent of the oracle's C code;
used to pin the oracle on geometries where the particle is almost on an edge
line or near a vertex.
"""
import mpmath as mp
def mp_pair(v, kid=0, dps=30):
    """I*, G*x, G*y (without C_d) for a unit field, Wendland C2, support 1."""
    mp.mp.dps = dps
    V = [(mp.mpf(x), mp.mpf(y)) for x, y in v]
    area2 = (V[1][0]-V[0][0])*(V[2][1]-V[0][1]) - (V[2][0]-V[0][0])*(V[1][1]-V[0][1])
    o = 1 if area2 > 0 else -1
    k = lambda r: (1-r)**4*(1+4*r)
    dk = lambda r: -20*r*(1-r)**3
    # antiderivatives of k(r) r and dk(r) r
    def rng(th):
        c, s = mp.cos(th), mp.sin(th); lo, hi = mp.mpf(0), mp.inf
        for e in range(3):
            a, b = V[e], V[(e+1) % 3]; ex, ey = b[0]-a[0], b[1]-a[1]
            al = o*(ex*s-ey*c); be = o*(ex*a[1]-ey*a[0])
            if al > 0: lo = max(lo, be/al)
            elif al < 0: hi = min(hi, be/al)
            elif be > 0: return None
        hi = min(hi, 1)
        return (lo, hi) if hi > lo else None
    def P(poly, a, b):  # int_a^b poly(r) dr, poly as coefficient list
        return sum(c*(b**(i+1)-a**(i+1))/(i+1) for i, c in enumerate(poly))
    kr = [0, 1, 0, -10, 20, -15, 4]          # k(r) r
    dkr = [0, 0, -20, 60, -60, 20]            # k'(r) r = -20 r^2 (1-r)^3
    def f(th, comp):
        ab = rng(th)
        if ab is None: return 0
        a, b = ab
        if comp == 0: return P(kr, a, b)
        g = -P(dkr, a, b)
        return g*mp.cos(th) if comp == 1 else g*mp.sin(th)
    br = [-mp.pi, mp.pi]
    for x, y in V: br.append(mp.atan2(y, x))
    for e in range(3):
        a, b = V[e], V[(e+1) % 3]; dx, dy = b[0]-a[0], b[1]-a[1]
        A = dx*dx+dy*dy; B = 2*(a[0]*dx+a[1]*dy); C = a[0]**2+a[1]**2-1; D = B*B-4*A*C
        if D > 0:
            for sg in (-1, 1):
                t = (-B+sg*mp.sqrt(D))/(2*A)
                if 0 < t < 1: br.append(mp.atan2(a[1]+t*dy, a[0]+t*dx))
    br = sorted(br)
    return [mp.quad(lambda th: f(th, c), br) for c in range(3)]


# ---------------------------------------------------------------------------
# any field order (P0, P1, P3 Lagrange) and any of the four kernels
# ---------------------------------------------------------------------------

def _kernel_pieces(kid):
    """[(radius, [b_0..b_d]) ] with exact mpf coefficients of k(q) = sum b_k q^k."""
    import sympy as sp
    from tests.exact import KERNELS, q
    out = []
    for k, R in KERNELS[kid]:
        p = sp.Poly(sp.expand(k), q)
        coef = [p.coeff_monomial(q ** i) for i in range(p.degree() + 1)]
        out.append((mp.mpf(sp.Rational(R).p) / sp.Rational(R).q,
                    [mp.mpf(sp.Rational(c).p) / sp.Rational(c).q for c in coef]))
    return out


def _pmul(a, b):
    out = {}
    for (i, j), u in a.items():
        for (k, l), v in b.items():
            out[(i + k, j + l)] = out.get((i + k, j + l), 0) + u * v
    return out


def _padd(a, b, w=1):
    out = dict(a)
    for key, v in b.items():
        out[key] = out.get(key, 0) + w * v
    return out


def field_polynomial(V, A):
    """Monomial coefficients {(i, j): c} of the element's field in (x, y):
    P0 (1 value), P1 (3, barycentric), P3 (10, cubic Lagrange; node order v0,
    v1, v2, edge v0v1 at 1/3 and 2/3, edge v1v2, edge v2v0, centroid)."""
    A = [mp.mpf(a) for a in A]
    if len(A) == 1:
        return {(0, 0): A[0]}
    (x0, y0), (x1, y1), (x2, y2) = V
    D = (y1 - y2) * (x0 - x2) + (x2 - x1) * (y0 - y2)
    # lambda_k = a + b x + c y
    l0 = {(0, 0): ((y1 - y2) * (-x2) + (x2 - x1) * (-y2)) / D, (1, 0): (y1 - y2) / D, (0, 1): (x2 - x1) / D}
    l1 = {(0, 0): ((y2 - y0) * (-x2) + (x0 - x2) * (-y2)) / D, (1, 0): (y2 - y0) / D, (0, 1): (x0 - x2) / D}
    l2 = _padd(_padd({(0, 0): mp.mpf(1)}, l0, -1), l1, -1)
    lam = [l0, l1, l2]
    if len(A) == 3:
        out = {}
        for k in range(3):
            out = _padd(out, lam[k], A[k])
        return out
    one = {(0, 0): mp.mpf(1)}

    def lin(l, s, t):                       # s l - t
        return _padd({key: s * v for key, v in l.items()}, one, -t)
    out = {}
    for i in range(3):
        b = _pmul(_pmul(lam[i], lin(lam[i], 3, 1)), lin(lam[i], 3, 2))
        out = _padd(out, b, A[i] / 2)
    for e in range(3):
        a, bb = e, (e + 1) % 3
        base = _pmul(lam[a], lam[bb])
        out = _padd(out, _pmul(base, lin(lam[a], 3, 1)), A[3 + 2 * e] * mp.mpf(9) / 2)
        out = _padd(out, _pmul(base, lin(lam[bb], 3, 1)), A[4 + 2 * e] * mp.mpf(9) / 2)
    out = _padd(out, _pmul(_pmul(lam[0], lam[1]), lam[2]), A[9] * 27)
    return out


def mp_pair_field(v, A, kid, dps=32, check=None):
    """(I, Gx, Gy) of one pair with C_d, support 1, particle at the origin.

    v: three vertices; A: nodal values (1, 3 or 10).  Polar coordinates about
    the particle: the field times the kernel piece is a polynomial in r along
    each ray, integrated exactly; the angle by mpmath.quad between
    breakpoints (vertex directions, edge directions, feet of perpendiculars,
    circle crossings of every kernel piece, and a geometric grading towards
    the directions of edge lines passing close to the particle), by fixed
    Gauss-Legendre rules of 24 and 48 points, bisecting an interval until the
    two agree to `check` per unit angle (default 10^(8-dps)); raises if that
    does not happen within 40 bisections."""
    import sympy as sp
    from tests.exact import c_d
    mp.mp.dps = dps
    V = [(mp.mpf(x), mp.mpf(y)) for x, y in v]
    area2 = (V[1][0] - V[0][0]) * (V[2][1] - V[0][1]) - (V[2][0] - V[0][0]) * (V[1][1] - V[0][1])
    if area2 == 0:
        return [mp.mpf(0)] * 3
    o = 1 if area2 > 0 else -1
    F = field_polynomial(V, A)
    pieces = _kernel_pieces(kid)
    deg = max(i + j for i, j in F)

    def rng(th):
        c, s = mp.cos(th), mp.sin(th)
        lo, hi = mp.mpf(0), mp.inf
        for e in range(3):
            a, b = V[e], V[(e + 1) % 3]
            ex, ey = b[0] - a[0], b[1] - a[1]
            al = o * (ex * s - ey * c)
            be = o * (ex * a[1] - ey * a[0])
            if al > 0:
                lo = max(lo, be / al)
            elif al < 0:
                hi = min(hi, be / al)
            elif be > 0:
                return None
        return (lo, hi) if hi > lo else None

    def f(th):
        ab = rng(th)
        if ab is None:
            return [mp.mpf(0)] * 3
        a, b = ab
        c, s = mp.cos(th), mp.sin(th)
        d = [sum(cf * c ** i * s ** j for (i, j), cf in F.items() if i + j == m) for m in range(deg + 1)]
        val = grad = mp.mpf(0)
        for R, bk in pieces:
            hb = min(b, R)
            if not hb > a:
                continue
            for m in range(deg + 1):
                for k, bb in enumerate(bk):
                    # int r^m (b_k (r/R)^k ... ) with q = r: the pieces are in q = r/h, h = 1
                    n = m + k + 2
                    val += d[m] * bb * (hb ** n - a ** n) / n
                    if k >= 1:
                        n1 = m + k + 1
                        grad += d[m] * k * bb * (hb ** n1 - a ** n1) / n1
        return [val, -grad * c, -grad * s]

    br = [-mp.pi, mp.pi]
    for x, y in V:
        if x != 0 or y != 0:
            br.append(mp.atan2(y, x))
    for e in range(3):
        a, b = V[e], V[(e + 1) % 3]
        dx, dy = b[0] - a[0], b[1] - a[1]
        L2 = dx * dx + dy * dy
        if L2 == 0:
            continue
        ang = mp.atan2(dy, dx)
        p = abs(dx * a[1] - dy * a[0]) / mp.sqrt(L2)
        for base in (ang, ang + mp.pi):
            br.append(base)
            if 0 < p < mp.mpf("0.05"):
                off = p / 4
                while off < mp.mpf("0.2"):
                    br += [base + off, base - off]
                    off *= 2
        t = -(a[0] * dx + a[1] * dy) / L2          # foot of the perpendicular
        br.append(mp.atan2(a[1] + t * dy, a[0] + t * dx))
        for R, _ in pieces:
            A2 = L2
            B = 2 * (a[0] * dx + a[1] * dy)
            C = a[0] ** 2 + a[1] ** 2 - R * R
            D = B * B - 4 * A2 * C
            if D > 0:
                for sg in (-1, 1):
                    t = (-B + sg * mp.sqrt(D)) / (2 * A2)
                    if 0 < t < 1:
                        br.append(mp.atan2(a[1] + t * dy, a[0] + t * dx))
    wrapped = []
    for b in br:
        while b > mp.pi:
            b -= 2 * mp.pi
        while b < -mp.pi:
            b += 2 * mp.pi
        wrapped.append(b)
    br = sorted(set(wrapped))
    cd = mp.mpf(sp.Rational(c_d(kid) * sp.pi).p) / sp.Rational(c_d(kid) * sp.pi).q / mp.pi
    # fixed Gauss-Legendre rules of 24 and 48 points on every interval (the
    # integrand is analytic inside each one); their difference bounds the
    # error, checked against `check`
    lo_rule, hi_rule = _gl_rule(4), _gl_rule(5)
    tol = mp.mpf(check) if check is not None else mp.mpf(10) ** (-dps + 8)

    def rule(rl, lo, hi):
        h2, m = (hi - lo) / 2, (hi + lo) / 2
        a = [mp.mpf(0)] * 3
        for x, w in rl:
            v = f(m + h2 * x)
            for comp in range(3):
                a[comp] += w * h2 * v[comp]
        return a

    def integrate(lo, hi, depth):
        a, b = rule(lo_rule, lo, hi), rule(hi_rule, lo, hi)
        d = max(abs(b[c] - a[c]) for c in range(3))
        if d <= tol * (hi - lo) or depth >= 40:
            if d > tol * (hi - lo):
                raise ArithmeticError(f"mp reference not converged on [{lo}, {hi}]: {d}")
            return b
        mid = (lo + hi) / 2
        l, r = integrate(lo, mid, depth + 1), integrate(mid, hi, depth + 1)
        return [l[c] + r[c] for c in range(3)]

    out = [mp.mpf(0)] * 3
    for lo, hi in zip(br[:-1], br[1:]):
        if hi > lo:
            v = integrate(lo, hi, 0)
            for comp in range(3):
                out[comp] += v[comp]
    return [cd * x for x in out]


_GL_CACHE = {}


def _gl_rule(degree):
    """(node, weight) pairs on [-1, 1] of mpmath's Gauss-Legendre rule of
    3 * 2^(degree-1) points at the working precision."""
    key = (degree, mp.mp.prec)
    if key not in _GL_CACHE:
        gl = mp.calculus.quadrature.GaussLegendre(mp.mp)
        _GL_CACHE[key] = gl.calc_nodes(degree, mp.mp.prec)
    return _GL_CACHE[key]
