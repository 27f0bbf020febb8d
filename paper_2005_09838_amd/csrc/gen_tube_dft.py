#!/usr/bin/env python3
"""Generate straight-line device code for the tube transforms of one thread's tube.

Forward (eq. (bar BA-k)):  X[b] = sum_k x[k] exp(+2 pi i b k / N),  b = 0 .. N/2
Inverse (eq. (barAAk)):    x[k] = (1/N) sum_b X[b] exp(-2 pi i b k / N), with the
                           bins above N/2 taken as conjugates (eq. (rcm_3-k+2)); the
                           imaginary parts of bin 0 (and of bin N/2 for even N) are
                           treated as 0.

Long even tubes use the half-length complex transform of the interleaved samples
(x[2m] + i x[2m+1]) and a final split into even and odd parts; all transforms are
mixed-radix decimation-in-time FFTs evaluated symbolically: every
value is a pair of real terms that are either the constant 0 or a named register, so
real inputs, conjugate-symmetric inputs and unused outputs prune work automatically
(a final liveness pass drops every statement no output depends on).  Radix-4 and
radix-2 butterflies are used where they divide N, then odd radices through the
conjugate-pair form of the small DFT.

Usage: python gen_tube_dft.py OUT.h  (writes specialisations tube_fwd<N> / tube_inv<N>
for every N in SIZES).
"""
import math
import sys

SIZES = list(range(1, 17)) + [20, 24, 28, 32, 40, 48, 56, 64, 84, 96, 112, 128]
SNAP = 1e-14


def snap(c):
    for v in (0.0, 1.0, -1.0, 0.5, -0.5):
        if abs(c - v) < SNAP:
            return v
    return c


class Gen:
    """Emits SSA statements `float tN = expr;` and tracks their inputs for pruning."""

    def __init__(self):
        self.stmts = []   # (name, expr, deps)
        self.n = 0

    def new(self, expr, deps):
        name = f"t{self.n}"
        self.n += 1
        self.stmts.append((name, expr, tuple(deps)))
        return name

    # a term is None (zero) or (sign, name)
    @staticmethod
    def neg(a):
        return None if a is None else (-a[0], a[1])

    def lin(self, pairs):
        """Linear combination sum c_i * a_i of terms with float constants c_i."""
        items = []
        for c, a in pairs:
            if a is None:
                continue
            c = snap(c * a[0])
            if c == 0.0:
                continue
            items.append((c, a[1]))
        if not items:
            return None
        if len(items) == 1:
            c, n = items[0]
            if c == 1.0:
                return (1, n)
            if c == -1.0:
                return (-1, n)
            return (1, self.new(f"{c!r}f * {n}", [n]))
        # unit coefficients first become adds / subtracts; others fold into fmaf chains
        units = [(c, n) for c, n in items if c in (1.0, -1.0)]
        others = [(c, n) for c, n in items if c not in (1.0, -1.0)]
        acc = None   # (sign, name)
        for c, n in units:
            if acc is None:
                acc = (1 if c > 0 else -1, n)
                continue
            sa, na = acc
            if sa > 0 and c > 0:
                acc = (1, self.new(f"{na} + {n}", [na, n]))
            elif sa > 0 and c < 0:
                acc = (1, self.new(f"{na} - {n}", [na, n]))
            elif sa < 0 and c > 0:
                acc = (1, self.new(f"{n} - {na}", [na, n]))
            else:
                acc = (-1, self.new(f"{na} + {n}", [na, n]))
        for c, n in others:
            if acc is None:
                acc = (1, self.new(f"{c!r}f * {n}", [n]))
                continue
            sa, na = acc
            if sa > 0:
                acc = (1, self.new(f"fmaf({c!r}f, {n}, {na})", [n, na]))
            else:
                acc = (-1, self.new(f"fmaf({-c!r}f, {n}, {na})", [n, na]))
        return acc

    def add(self, a, b):
        return self.lin([(1.0, a), (1.0, b)])

    def sub(self, a, b):
        return self.lin([(1.0, a), (-1.0, b)])

    # complex helpers: values are (re_term, im_term)
    def cadd(self, x, y):
        return (self.add(x[0], y[0]), self.add(x[1], y[1]))

    def csub(self, x, y):
        return (self.sub(x[0], y[0]), self.sub(x[1], y[1]))

    def cmul_const(self, x, c, s):
        """(x_re + i x_im)(c + i s)."""
        c, s = snap(c), snap(s)
        if s == 0.0:
            return (self.lin([(c, x[0])]), self.lin([(c, x[1])]))
        if c == 0.0:
            return (self.lin([(-s, x[1])]), self.lin([(s, x[0])]))
        return (self.lin([(c, x[0]), (-s, x[1])]), self.lin([(s, x[0]), (c, x[1])]))

    def ctimes_i(self, x, sigma):
        """(sigma * i) * x."""
        return self.cmul_const(x, 0.0, float(sigma))

    def small_dft(self, xs, sigma):
        p = len(xs)
        if p == 1:
            return list(xs)
        if p == 2:
            return [self.cadd(xs[0], xs[1]), self.csub(xs[0], xs[1])]
        if p == 4:
            a = self.cadd(xs[0], xs[2])
            b = self.csub(xs[0], xs[2])
            c = self.cadd(xs[1], xs[3])
            d = self.csub(xs[1], xs[3])
            id_ = self.ctimes_i(d, sigma)
            return [self.cadd(a, c), self.cadd(b, id_), self.csub(a, c), self.csub(b, id_)]
        assert p % 2 == 1
        h = (p - 1) // 2
        S = [self.cadd(xs[q], xs[p - q]) for q in range(1, h + 1)]
        D = [self.csub(xs[q], xs[p - q]) for q in range(1, h + 1)]
        out = [None] * p
        out[0] = (self.lin([(1.0, xs[0][0])] + [(1.0, s[0]) for s in S]),
                  self.lin([(1.0, xs[0][1])] + [(1.0, s[1]) for s in S]))
        for s in range(1, h + 1):
            cs = [math.cos(2 * math.pi * s * q / p) for q in range(1, h + 1)]
            sn = [sigma * math.sin(2 * math.pi * s * q / p) for q in range(1, h + 1)]
            a_re = self.lin([(1.0, xs[0][0])] + [(cs[q], S[q][0]) for q in range(h)])
            a_im = self.lin([(1.0, xs[0][1])] + [(cs[q], S[q][1]) for q in range(h)])
            b_re = self.lin([(sn[q], D[q][0]) for q in range(h)])
            b_im = self.lin([(sn[q], D[q][1]) for q in range(h)])
            # Y_s = A + i B,  Y_{p-s} = A - i B,  with i B = (-b_im, b_re)
            out[s] = (self.sub(a_re, b_im), self.add(a_im, b_re))
            out[p - s] = (self.add(a_re, b_im), self.sub(a_im, b_re))
        return out

    def fft(self, xs, sigma):
        n = len(xs)
        if n == 1:
            return list(xs)
        if n % 4 == 0 and n != 8:
            p = 4
        elif n % 2 == 0:
            p = 2
        else:
            p = next(f for f in range(3, n + 1) if n % f == 0)
        if p == n:
            return self.small_dft(xs, sigma)
        m = n // p
        subs = [self.fft(xs[q::p], sigma) for q in range(p)]
        out = [None] * n
        for b0 in range(m):
            tw = []
            for q in range(p):
                ang = sigma * 2 * math.pi * b0 * q / n
                tw.append(self.cmul_const(subs[q][b0], math.cos(ang), math.sin(ang)))
            y = self.small_dft(tw, sigma)
            for s in range(p):
                out[b0 + s * m] = y[s]
        return out


def emit_function(signature, gen, outputs):
    """outputs: list of (lvalue, term).  Prunes dead statements."""
    live = set()
    for _, t in outputs:
        if t is not None:
            live.add(t[1])
    keep = []
    for name, expr, deps in reversed(gen.stmts):
        if name in live:
            keep.append((name, expr))
            live.update(deps)
    keep.reverse()
    lines = [signature + " {"]
    for name, expr in keep:
        lines.append(f"  const float {name} = {expr};")
    for lv, t in outputs:
        if t is None:
            lines.append(f"  {lv} = 0.0f;")
        elif t[0] > 0:
            lines.append(f"  {lv} = {t[1]};")
        else:
            lines.append(f"  {lv} = -{t[1]};")
    lines.append("}")
    return "\n".join(lines), len(keep)


def use_half_length(n):
    """Long even tubes go through a half-length complex transform: it keeps the live set
    at about n registers (the direct form holds n complex values between stages)."""
    return n % 2 == 0 and n >= 64


def half_length_forward(g, n):
    """Real length-n transform through a complex length-n/2 one: c[m] = x[2m] + i x[2m+1],
    C = DFT(c); E[b] = (C[b] + conj C[M-b]) / 2, O[b] = (C[b] - conj C[M-b]) / (2i),
    X[b] = E[b] + w^b O[b] for b = 0..M."""
    m = n // 2
    cs = [((1, f"x[{2 * q}]"), (1, f"x[{2 * q + 1}]")) for q in range(m)]
    cc = g.fft(cs, +1)
    out = []
    for b in range(m + 1):
        c1 = cc[b % m]
        c2 = cc[(m - b) % m]
        c2c = (c2[0], g.neg(c2[1]))                       # conj C[M-b]
        e = (g.lin([(0.5, c1[0]), (0.5, c2c[0])]), g.lin([(0.5, c1[1]), (0.5, c2c[1])]))
        dlt = (g.lin([(0.5, c1[0]), (-0.5, c2c[0])]), g.lin([(0.5, c1[1]), (-0.5, c2c[1])]))
        o = (dlt[1], g.neg(dlt[0]))                        # dlt / i
        ang = 2 * math.pi * b / n
        wo = g.cmul_const(o, math.cos(ang), math.sin(ang))
        out.append(g.cadd(e, wo))
    return out


def half_length_inverse(g, n, spec):
    """Inverse of half_length_forward: E[b] = (X[b] + conj X[M-b]) / 2,
    O[b] = (X[b] - conj X[M-b]) conj(w)^b / 2, C = E + i O, c = (1/M) IDFT(C),
    x[2m] = Re c[m], x[2m+1] = Im c[m]."""
    m = n // 2
    cs = []
    for b in range(m):
        x1 = spec[b]
        x2 = spec[m - b]
        x2c = (x2[0], g.neg(x2[1]))
        e = (g.lin([(0.5, x1[0]), (0.5, x2c[0])]), g.lin([(0.5, x1[1]), (0.5, x2c[1])]))
        dlt = (g.lin([(0.5, x1[0]), (-0.5, x2c[0])]), g.lin([(0.5, x1[1]), (-0.5, x2c[1])]))
        ang = -2 * math.pi * b / n
        o = g.cmul_const(dlt, math.cos(ang), math.sin(ang))
        io = (g.neg(o[1]), o[0])                           # i * O
        cs.append(g.cadd(e, io))
    cc = g.fft(cs, -1)
    xs = []
    for q in range(m):
        xs.append(g.lin([(1.0 / m, cc[q][0])]))
        xs.append(g.lin([(1.0 / m, cc[q][1])]))
    return xs


def gen_forward(n):
    g = Gen()
    nb = n // 2 + 1
    if use_half_length(n):
        ys = half_length_forward(g, n)
    else:
        xs = [((1, f"x[{k}]"), None) for k in range(n)]
        ys = g.fft(xs, +1)
    outs = []
    for b in range(nb):
        outs.append((f"re[{b}]", ys[b][0]))
        im = ys[b][1]
        if b == 0 or (n % 2 == 0 and b == n // 2):
            im = None
        outs.append((f"im[{b}]", im))
    sig = (f"template <> TUBE_DFT_QUAL void tube_fwd<{n}>(const float (&x)[{n}], "
           f"float (&re)[{nb}], float (&im)[{nb}])")
    return emit_function(sig, g, outs)


def gen_inverse(n):
    g = Gen()
    nb = n // 2 + 1
    if use_half_length(n):
        spec = []
        for b in range(nb):
            re = (1, f"re[{b}]")
            im = None if (b == 0 or b == n // 2) else (1, f"im[{b}]")
            spec.append((re, im))
        xr = half_length_inverse(g, n, spec)
        outs = [(f"x[{k}]", xr[k]) for k in range(n)]
        sig = (f"template <> TUBE_DFT_QUAL void tube_inv<{n}>(const float (&re)[{nb}], "
               f"const float (&im)[{nb}], float (&x)[{n}])")
        return emit_function(sig, g, outs)
    xs = []
    for b in range(n):
        if b < nb:
            re = (1, f"re[{b}]")
            im = None if (b == 0 or (n % 2 == 0 and b == n // 2)) else (1, f"im[{b}]")
        else:
            re = (1, f"re[{n - b}]")
            im = (-1, f"im[{n - b}]")
        xs.append((re, im))
    ys = g.fft(xs, -1)
    outs = []
    inv_n = 1.0 / n
    for k in range(n):
        outs.append((f"x[{k}]", g.lin([(inv_n, ys[k][0])])))
    sig = (f"template <> TUBE_DFT_QUAL void tube_inv<{n}>(const float (&re)[{nb}], "
           f"const float (&im)[{nb}], float (&x)[{n}])")
    return emit_function(sig, g, outs)


# ---------------------------------------------------------------- LDS four-step plans

def lds_factor(n):
    """(M1, M2) with M1 * M2 = n/2 and both <= 16 for the LDS four-step transform, or None."""
    if n % 2 or n < 16:
        return None
    m = n // 2
    best = None
    for m1 in range(2, 17):
        if m % m1 == 0 and 2 <= m // m1 <= 16:
            cand = (abs(m1 - m // m1), -m1, m1, m // m1)
            best = cand if best is None or cand < best else best
    return None if best is None else (best[2], best[3])


def gen_small_complex(p, sigma):
    """In-place complex DFT of length p: y[k] = sum_n x[n] exp(sigma 2 pi i n k / p)."""
    g = Gen()
    xs = [((1, f"re[{q}]"), (1, f"im[{q}]")) for q in range(p)]
    ys = g.fft(xs, sigma)
    outs = []
    for k in range(p):
        outs.append((f"o_re[{k}]", ys[k][0]))
        outs.append((f"o_im[{k}]", ys[k][1]))
    tag = "p" if sigma > 0 else "n"
    sig = f"template <> TUBE_DFT_QUAL void dftc<{p}, {sigma}>(float (&re)[{p}], float (&im)[{p}])"
    body, cnt = emit_function(sig, g, outs)
    # write through temporaries so the outputs may alias the inputs
    body = body.replace(sig + " {", sig + " {\n  float o_re[%d], o_im[%d];" % (p, p), 1)
    body = body[:-1] + "  for (int k = 0; k < %d; ++k) { re[k] = o_re[k]; im[k] = o_im[k]; }\n}" % p
    return body, cnt


def main(path):
    parts = [
        "// Generated by gen_tube_dft.py: straight-line tube transforms (do not edit).",
        "// tube_fwd<N>: X[b] = sum_k x[k] exp(+2 pi i b k / N), b = 0..N/2 (eq. (bar BA-k)).",
        "// tube_inv<N>: x[k] = (1/N) sum_b X[b] exp(-2 pi i b k / N) over the conjugate-",
        "//              symmetric extension of bins 0..N/2 (eq. (barAAk), eq. (rcm_3-k+2)).",
        "#pragma once",
        "#ifndef TUBE_DFT_QUAL",
        "#define TUBE_DFT_QUAL __device__ __forceinline__",
        "#endif",
        "template <int N> TUBE_DFT_QUAL void tube_fwd(const float (&x)[N], float (&re)[N / 2 + 1], float (&im)[N / 2 + 1]);",
        "template <int N> TUBE_DFT_QUAL void tube_inv(const float (&re)[N / 2 + 1], const float (&im)[N / 2 + 1], float (&x)[N]);",
        "#define TUBE_DFT_SIZES(X) " + " ".join(f"X({n})" for n in SIZES),
    ]
    parts.append("template <int P, int S> TUBE_DFT_QUAL void dftc(float (&re)[P], float (&im)[P]);")
    plans = {n: lds_factor(n) for n in SIZES}
    smalls = sorted({f for pl in plans.values() if pl for f in pl})
    for q in smalls:
        for sg in (+1, -1):
            parts.append(gen_small_complex(q, sg)[0])
    parts.append("// Four-step plan of each tube length that runs through LDS: N/2 = M1 * M2 (0 = registers).")
    parts.append("template <int N> struct TubePlan { static constexpr int M1 = 0, M2 = 0; };")
    for n, pl in plans.items():
        if pl:
            parts.append(f"template <> struct TubePlan<{n}> {{ static constexpr int M1 = {pl[0]}, M2 = {pl[1]}; }};")
    stats = []
    for n in SIZES:
        f, cf = gen_forward(n)
        i, ci = gen_inverse(n)
        parts += [f, i]
        stats.append(f"//   N={n}: forward {cf} ops, inverse {ci} ops")
    parts.insert(4, "// Operation counts (add/sub/mul/fma statements):\n" + "\n".join(stats))
    with open(path, "w") as fh:
        fh.write("\n".join(parts) + "\n")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "tube_dft_gen.h")
