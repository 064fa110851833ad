"""An arbitrary-precision (50-digit) model of the colour conversions, written
from the published definitions (IEC 61966-2-1 sRGB with its chromaticities
and transfer function, CIE 1976 L*a*b* with the D65 white).  It shares no
code with the FP64 oracle or the HIP library; the oracle's pins use it as an
independent brute force."""
from __future__ import annotations

from decimal import ROUND_HALF_EVEN, Decimal, getcontext

getcontext().prec = 50
D = Decimal

def _solve3(A, b):
    """Gauss-Jordan elimination with partial pivoting (Decimal)."""
    m = [list(A[r]) + [b[r]] for r in range(3)]
    for c in range(3):
        piv = max(range(c, 3), key=lambda r: abs(m[r][c]))
        m[c], m[piv] = m[piv], m[c]
        for r in range(3):
            if r != c:
                f = m[r][c] / m[c][c]
                m[r] = [m[r][k] - f * m[c][k] for k in range(4)]
    return [m[r][3] / m[r][r] for r in range(3)]


def _dec_space():
    prim = [(D("0.64"), D("0.33")), (D("0.30"), D("0.60")), (D("0.15"), D("0.06"))]
    wx, wy = D("0.3127"), D("0.3290")
    P = [[x / y for x, y in prim], [D(1)] * 3, [(1 - x - y) / y for x, y in prim]]
    Wv = [wx / wy, D(1), (1 - wx - wy) / wy]
    S = _solve3(P, Wv)
    M = [[P[r][c] * S[c] for c in range(3)] for r in range(3)]
    # columns of the inverse: solve M x = e_k
    cols = [_solve3(M, [D(int(k == r)) for r in range(3)]) for k in range(3)]
    Minv = [[cols[c][r] for c in range(3)] for r in range(3)]
    return M, Minv, Wv


DM, DMINV, DW = _dec_space()
DELTA = D(6) / D(29)


def d_decode(c):
    return c / D("12.92") if c <= D("0.04045") else ((c + D("0.055")) / D("1.055")) ** D("2.4")


def d_encode(l):
    return D("12.92") * l if l <= D("0.0031308") else D("1.055") * l ** (D(1) / D("2.4")) - D("0.055")


def d_f(t):
    return t ** (D(1) / D(3)) if t > DELTA ** 3 else t / (3 * DELTA ** 2) + D(4) / D(29)


def d_finv(u):
    return u ** 3 if u > DELTA else 3 * DELTA ** 2 * (u - D(4) / D(29))


def d_rgb8_to_lab(rgb):
    lin = [d_decode(D(int(v)) / D(255)) for v in rgb]
    xyz = [sum(DM[r][k] * lin[k] for k in range(3)) for r in range(3)]
    f = [d_f(xyz[r] / DW[r]) for r in range(3)]
    return [116 * f[1] - 16, 500 * (f[0] - f[1]), 200 * (f[1] - f[2])]


def d_lab_to_linear(lab):
    L, a, b = lab
    fy = (L + 16) / 116
    xyz = [DW[0] * d_finv(fy + a / 500), DW[1] * d_finv(fy), DW[2] * d_finv(fy - b / 200)]
    return [sum(DMINV[r][k] * xyz[k] for k in range(3)) for r in range(3)]


def d_round(v):
    return int(v.quantize(D(1), rounding=ROUND_HALF_EVEN))


# pi to 60 digits, and sine / cosine of an angle in degrees by their Taylor
# series after reduction to [-180, 180]; multiples of 90 degrees are exact.
PI = D("3.14159265358979323846264338327950288419716939937510582097494")


def d_sincos_deg(deg):
    deg = D(deg) % 360
    exact = {D(0): (D(0), D(1)), D(90): (D(1), D(0)), D(180): (D(0), D(-1)), D(270): (D(-1), D(0))}
    if deg in exact:
        return exact[deg]
    if deg > 180:
        deg -= 360
    x = deg * PI / 180
    s, c, term_s, term_c = D(0), D(0), x, D(1)
    for k in range(60):
        s += term_s
        c += term_c
        term_s = -term_s * x * x / ((2 * k + 2) * (2 * k + 3))
        term_c = -term_c * x * x / ((2 * k + 1) * (2 * k + 2))
    return s, c
