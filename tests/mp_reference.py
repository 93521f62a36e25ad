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
