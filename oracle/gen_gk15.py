"""Generate the 7-point Gauss / 15-point Kronrod rule on [-1, 1] for the oracle.

TEST INFRASTRUCTURE: part of the CPU oracle. Nothing in the product path reads it.

The Kronrod extension of the n=7 Gauss-Legendre rule adds the n+1=8 zeros of the
Stieltjes polynomial E_8, which is the monic degree-8 polynomial orthogonal to every
polynomial of degree < 8 under the sign-changing weight P_7(x) on [-1, 1]
(Kronrod 1965; Monegato 1982). E_8 is even, so only the odd moments k = 1, 3, 5, 7
give conditions: four linear equations for its four lower coefficients.
The 15 weights then follow from exactness on the even monomials x^0 .. x^14
(odd monomials integrate to zero by symmetry). Everything runs in mpmath at
60 significant digits and is printed with 36, far beyond long double.

Run:  python oracle/gen_gk15.py > oracle/gk15_table.h
"""
import mpmath as mp

mp.mp.dps = 60


def legendre_coeffs(n):
    """Coefficients (ascending powers) of P_n by Bonnet's recursion."""
    p0, p1 = [mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]
    if n == 0:
        return p0
    for k in range(1, n):
        nxt = [mp.mpf(0)] * (k + 2)
        for i, c in enumerate(p1):
            nxt[i + 1] += mp.mpf(2 * k + 1) * c / (k + 1)
        for i, c in enumerate(p0):
            nxt[i] -= mp.mpf(k) * c / (k + 1)
        p0, p1 = p1, nxt
    return p1


def moment(j):
    """Integral of x^j over [-1, 1]."""
    return mp.mpf(0) if j % 2 else mp.mpf(2) / (j + 1)


def poly_eval(c, x):
    return mp.fsum(ci * x ** i for i, ci in enumerate(c))


def main():
    p7 = legendre_coeffs(7)
    # E_8(x) = x^8 + a6 x^6 + a4 x^4 + a2 x^2 + a0 ; unknowns (a0, a2, a4, a6)
    # condition_k: sum_i p7_i * [ mu(i+8+k) + a6 mu(i+6+k) + a4 mu(i+4+k) + a2 mu(i+2+k) + a0 mu(i+k) ] = 0
    A = mp.matrix(4, 4)
    b = mp.matrix(4, 1)
    for r, k in enumerate((1, 3, 5, 7)):
        for cidx, e in enumerate((0, 2, 4, 6)):
            A[r, cidx] = mp.fsum(p7[i] * moment(i + e + k) for i in range(8))
        b[r] = -mp.fsum(p7[i] * moment(i + 8 + k) for i in range(8))
    a = mp.lu_solve(A, b)
    # quartic in y = x^2 : y^4 + a6 y^3 + a4 y^2 + a2 y + a0
    ys = mp.polyroots([1, a[3], a[2], a[1], a[0]], maxsteps=200, extraprec=200)
    ys = sorted(mp.re(y) for y in ys)
    kron_pos = [mp.sqrt(y) for y in ys]
    # Gauss nodes: positive zeros of P_7 (0 is also a zero)
    gz = mp.polyroots(list(reversed(p7)), maxsteps=200, extraprec=200)
    gauss_pos = sorted(mp.re(z) for z in gz if mp.re(z) > mp.mpf("1e-40"))
    # all nonnegative nodes of the 15-point rule, descending like published tables
    nodes = sorted(kron_pos + gauss_pos + [mp.mpf(0)], reverse=True)
    assert len(nodes) == 8
    # weights: exactness on x^(2k), k=0..7; node 0 counted once, others twice
    V = mp.matrix(8, 8)
    rhs = mp.matrix(8, 1)
    for k in range(8):
        for j, xn in enumerate(nodes):
            mult = 1 if xn == 0 else 2
            V[k, j] = mult * xn ** (2 * k)
        rhs[k] = moment(2 * k)
    wk = mp.lu_solve(V, rhs)
    # Gauss weights: 2 / ((1 - x^2) P7'(x)^2)
    dp7 = [i * p7[i] for i in range(1, 8)]
    gw = {}
    for xn in gauss_pos + [mp.mpf(0)]:
        gw[xn] = 2 / ((1 - xn ** 2) * poly_eval(dp7, xn) ** 2)

    out = []
    out.append("/* 7-point Gauss / 15-point Kronrod rule on [-1,1]: nonnegative nodes, descending.")
    out.append(" * Written by oracle/gen_gk15.py (mpmath, 60 digits). TEST INFRASTRUCTURE ONLY. */")
    out.append("#ifndef GK15_TABLE_H")
    out.append("#define GK15_TABLE_H")
    out.append("static const long double GK15_X[8] = {")
    out += ["  %sL," % mp.nstr(xn, 36, min_fixed=-1, max_fixed=1) for xn in nodes]
    out.append("};")
    out.append("static const long double GK15_WK[8] = {")
    out += ["  %sL," % mp.nstr(wk[j], 36, min_fixed=-1, max_fixed=1) for j in range(8)]
    out.append("};")
    out.append("/* Gauss weight of node j, zero where node j is a Kronrod-only node */")
    out.append("static const long double GK15_WG[8] = {")
    for xn in nodes:
        w = gw.get(xn, mp.mpf(0))
        out.append("  %sL," % mp.nstr(w, 36, min_fixed=-1, max_fixed=1))
    out.append("};")
    out.append("#endif")
    print("\n".join(out))


if __name__ == "__main__":
    main()
