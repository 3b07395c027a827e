#!/usr/bin/env python3
"""Generates bitslice_sbox.h: the AES S-box and inverse S-box (FIPS-197 5.1.1,
5.3.2) as straight-line Boolean circuits for the bitsliced kernels, derived
here in a tower field.

The multiplicative inverse in GF(2^8) = GF(2)[x]/(x^8+x^4+x^3+x+1) is computed
in the isomorphic composite field GF((2^4)^2): GF(16) = GF(2)[y]/(y^4+y+1),
and GF(256) = GF(16)[X]/(X^2+X+lam) for the first lam that makes X^2+X+lam
irreducible.  For a = hX + l:
    d = lam*h^2 + h*l + l^2,   a^-1 = (h*d^-1) X + ((h+l)*d^-1).
The change of basis maps x -> b, where b is a root of the AES polynomial in the
composite field (found by search); the output basis change is merged with the
S-box affine map.  The inverse S-box runs the same inversion between the inverse
affine map (merged with the input basis change, its constant 0x63 included)
and the plain output basis change.  Linear maps are emitted as XOR networks (greedy pair
sharing), GF(16) products as AND/XOR terms, and d^-1 (four 4-input functions)
by Shannon expansion into three-input lookups, which the kernel evaluates
with v_bitop3_b32.

The script checks the emitted circuits on all 256 inputs against an S-box it
computes directly (inverse by search, then the affine map) and against that
S-box's inverse permutation before writing.

Run: python gen_bitslice_sbox.py   (rewrites bitslice_sbox.h beside it)
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "bitslice_sbox.h")


# ----------------------------------------------------------------- fields

def gf256_mul(a, b):
    p = 0
    while b:
        if b & 1:
            p ^= a
        a = ((a << 1) ^ 0x11B) if a & 0x80 else (a << 1)
        b >>= 1
    return p


def gf16_mul(a, b):
    p = 0
    for i in range(4):
        if (b >> i) & 1:
            p ^= a << i
    for i in (6, 5, 4):  # reduce by y^4 + y + 1
        if (p >> i) & 1:
            p ^= 0b10011 << (i - 4)
    return p


def gf16_inv(a):
    if a == 0:
        return 0
    return next(c for c in range(1, 16) if gf16_mul(a, c) == 1)


def pick_lambda():
    for lam in range(1, 16):
        if all(gf16_mul(x, x) ^ x ^ lam for x in range(16)):
            return lam
    raise AssertionError


LAM = pick_lambda()


def comp_mul(a, b):
    h1, l1, h2, l2 = a >> 4, a & 15, b >> 4, b & 15
    hh = gf16_mul(h1, h2)
    h = hh ^ gf16_mul(h1, l2) ^ gf16_mul(l1, h2)
    l = gf16_mul(l1, l2) ^ gf16_mul(LAM, hh)
    return (h << 4) | l


def comp_pow(a, n):
    r = 1
    for _ in range(n):
        r = comp_mul(r, a)
    return r


def find_root():
    # root of x^8 + x^4 + x^3 + x + 1 in the composite field
    for b in range(2, 256):
        v = comp_pow(b, 8) ^ comp_pow(b, 4) ^ comp_pow(b, 3) ^ b ^ 1
        if v == 0:
            return b
    raise AssertionError


BETA = find_root()
# M: AES polynomial basis -> composite (column i = beta^i)
M_COLS = [comp_pow(BETA, i) for i in range(8)]


def to_comp(a):
    r = 0
    for i in range(8):
        if (a >> i) & 1:
            r ^= M_COLS[i]
    return r


def invert_matrix(cols):
    # cols: 8 ints (column i); returns columns of the inverse (GF(2))
    rows = [[(cols[c] >> r) & 1 for c in range(8)] + [1 if r == k else 0 for k in range(8)]
            for r in range(8)]
    for c in range(8):
        p = next(r for r in range(c, 8) if rows[r][c])
        rows[c], rows[p] = rows[p], rows[c]
        for r in range(8):
            if r != c and rows[r][c]:
                rows[r] = [x ^ y for x, y in zip(rows[r], rows[c])]
    inv_rows = [row[8:] for row in rows]
    return [sum(inv_rows[r][c] << r for r in range(8)) for c in range(8)]


MINV_COLS = invert_matrix(M_COLS)


def from_comp(a):
    r = 0
    for i in range(8):
        if (a >> i) & 1:
            r ^= MINV_COLS[i]
    return r


def affine(b):
    s = b
    for k in range(1, 5):
        s ^= ((b << k) | (b >> (8 - k))) & 0xFF
    return s ^ 0x63


def sbox_direct(a):
    inv = 0 if a == 0 else next(c for c in range(1, 256) if gf256_mul(a, c) == 1)
    return affine(inv)


# The linear part of the affine map and its inverse (columns).
AFF_COLS = [affine(1 << i) ^ 0x63 for i in range(8)]
AFF_INV_COLS = invert_matrix(AFF_COLS)


def apply_cols(cols, a):
    r = 0
    for i in range(8):
        if (a >> i) & 1:
            r ^= cols[i]
    return r


# Sanity: the map is a field isomorphism and the tower inverse is right.
for a in range(256):
    for b in range(0, 256, 37):
        assert to_comp(gf256_mul(a, b)) == comp_mul(to_comp(a), to_comp(b))
    assert from_comp(to_comp(a)) == a


# ---------------------------------------------------------------- circuit

class Circuit:
    def __init__(self):
        self.ops = []  # (kind, dst, args)
        self.n = 0

    def new(self):
        self.n += 1
        return f"t{self.n}"

    def op(self, kind, *args):
        d = self.new()
        self.ops.append((kind, d, args))
        return d


def linear(c, inputs, rows, consts=None):
    """Outputs row_i = XOR of inputs[j] for bit j of rows[i] (then NOT if the
    constant bit is set), sharing frequent pairs first."""
    sig = list(inputs)
    sets = [set(j for j in range(len(inputs)) if (r >> j) & 1) for r in rows]
    while True:
        count = {}
        for s in sets:
            lst = sorted(s)
            for i in range(len(lst)):
                for j in range(i + 1, len(lst)):
                    count[(lst[i], lst[j])] = count.get((lst[i], lst[j]), 0) + 1
        if not count:
            break
        (a, b), k = max(count.items(), key=lambda kv: (kv[1], -kv[0][0], -kv[0][1]))
        if k < 2:
            break
        sig.append(c.op("xor2", sig[a], sig[b]))
        idx = len(sig) - 1
        for s in sets:
            if a in s and b in s:
                s.discard(a)
                s.discard(b)
                s.add(idx)
    outs = []
    for i, s in enumerate(sets):
        lst = [sig[j] for j in sorted(s)]
        neg = bool(consts and (consts >> i) & 1)
        if not lst:
            raise AssertionError("zero row")
        while len(lst) > 3:
            lst = [c.op("xor3", lst[0], lst[1], lst[2])] + lst[3:]
        if len(lst) == 1:
            outs.append(c.op("not", lst[0]) if neg else lst[0])
        elif len(lst) == 2:
            outs.append(c.op("xnor2" if neg else "xor2", lst[0], lst[1]))
        else:
            outs.append(c.op("xnor3" if neg else "xor3", *lst))
    return outs


def gf16_mult(c, a, b):
    """Bitsliced GF(16) product of nibbles a, b (4 signals each, LSB first)."""
    p = {}
    for k in range(7):
        terms = [(i, k - i) for i in range(4) if 0 <= k - i < 4]
        p[k] = terms
    # c0 = p0+p4, c1 = p1+p4+p5, c2 = p2+p5+p6, c3 = p3+p6
    def sum_terms(terms, acc=None):
        for (i, j) in terms:
            acc = c.op("and2", a[i], b[j]) if acc is None else c.op("andxor", a[i], b[j], acc)
        return acc
    p4 = sum_terms(p[4])
    p5 = sum_terms(p[5])
    p6 = sum_terms(p[6])
    c0 = sum_terms(p[0], p4)
    c1 = sum_terms(p[1], c.op("xor2", p4, p5))
    c2 = sum_terms(p[2], c.op("xor2", p5, p6))
    c3 = sum_terms(p[3], p6)
    return [c0, c1, c2, c3]


def gf16_linear_rows(f):
    """Rows of the GF(2) matrix of a linear map on nibbles."""
    cols = [f(1 << i) for i in range(4)]
    return [sum(((cols[i] >> r) & 1) << i for i in range(4)) for r in range(4)]


def build(inverse=False):
    """The S-box circuit, or with inverse=True the inverse S-box circuit."""
    c = Circuit()
    u = [f"u{i}" for i in range(8)]
    if inverse:
        # x = affine^-1(u) = L^-1(u) ^ L^-1(0x63), then into the composite basis
        cols = [to_comp(AFF_INV_COLS[i]) for i in range(8)]
        const = to_comp(apply_cols(AFF_INV_COLS, 0x63))
        v = linear(c, u, [sum(((cols[i] >> r) & 1) << i for i in range(8)) for r in range(8)],
                   consts=const)
    else:
        v = linear(c, u, [sum(((M_COLS[i] >> r) & 1) << i for i in range(8)) for r in range(8)])
    l, h = v[0:4], v[4:8]
    # lam*h^2 + l^2 (linear in h and l) plus h*l
    lin_h = gf16_linear_rows(lambda x: gf16_mul(LAM, gf16_mul(x, x)))
    lin_l = gf16_linear_rows(lambda x: gf16_mul(x, x))
    rows = [lin_h[r] << 4 | lin_l[r] for r in range(4)]
    sq = linear(c, l + h, rows)
    hl = gf16_mult(c, h, l)
    d = [c.op("xor2", sq[i], hl[i]) for i in range(4)]
    # d^-1: each output bit a 4-input function, Shannon-expanded on d3
    di = []
    for bit in range(4):
        tt = [(gf16_inv(x) >> bit) & 1 for x in range(16)]
        lo = sum(tt[x] << x for x in range(8))       # d3 = 0, index = d2 d1 d0
        hi = sum(tt[8 + x] << x for x in range(8))   # d3 = 1
        f0 = c.op("lut3", d[2], d[1], d[0], lo)
        f1 = c.op("lut3", d[2], d[1], d[0], hi)
        di.append(c.op("mux", d[3], f1, f0))
    hx = [c.op("xor2", h[i], l[i]) for i in range(4)]
    oh = gf16_mult(c, h, di)
    ol = gf16_mult(c, hx, di)
    if inverse:
        # output: from_comp(oh:ol)
        lin_out = [from_comp(1 << i) for i in range(8)]
        rows = [sum(((lin_out[i] >> r) & 1) << i for i in range(8)) for r in range(8)]
        y = linear(c, ol + oh, rows)
    else:
        # output: affine(from_comp(oh:ol)) -- linear part and constant 0x63
        lin_out = [affine(from_comp(1 << i)) ^ 0x63 for i in range(8)]
        rows = [sum(((lin_out[i] >> r) & 1) << i for i in range(8)) for r in range(8)]
        y = linear(c, ol + oh, rows, consts=0x63)
    return c, y


def lut3_tt(x, y, z, tt):
    return (tt >> ((x << 2) | (y << 1) | z)) & 1


def simulate(c, outs, a):
    val = {f"u{i}": (a >> i) & 1 for i in range(8)}
    for kind, d, args in c.ops:
        g = [val[x] if isinstance(x, str) else x for x in args]
        if kind == "xor2":
            val[d] = g[0] ^ g[1]
        elif kind == "xnor2":
            val[d] = 1 ^ g[0] ^ g[1]
        elif kind == "xor3":
            val[d] = g[0] ^ g[1] ^ g[2]
        elif kind == "xnor3":
            val[d] = 1 ^ g[0] ^ g[1] ^ g[2]
        elif kind == "not":
            val[d] = 1 ^ g[0]
        elif kind == "and2":
            val[d] = g[0] & g[1]
        elif kind == "andxor":
            val[d] = (g[0] & g[1]) ^ g[2]
        elif kind == "lut3":
            val[d] = lut3_tt(g[0], g[1], g[2], g[3])
        elif kind == "mux":
            val[d] = g[1] if g[0] else g[2]
        else:
            raise AssertionError(kind)
    return sum(val[o] << i for i, o in enumerate(outs))


# bitop3 truth tables: index = (S0 << 2) | (S1 << 1) | S2
TT = {"xor2": None, "xnor2": None, "xor3": 0x96, "xnor3": 0x69, "and2": None,
      "andxor": 0x6A, "mux": 0xCA}


def emit(c, outs):
    lines = []
    for kind, d, args in c.ops:
        a = list(args)
        if kind == "xor2":
            e = f"{a[0]} ^ {a[1]}"
        elif kind == "xnor2":
            e = f"~({a[0]} ^ {a[1]})"
        elif kind == "not":
            e = f"~{a[0]}"
        elif kind == "and2":
            e = f"{a[0]} & {a[1]}"
        elif kind == "lut3":
            e = f"__builtin_amdgcn_bitop3_b32({a[0]}, {a[1]}, {a[2]}, 0x{a[3]:02X})"
        else:
            e = f"__builtin_amdgcn_bitop3_b32({a[0]}, {a[1]}, {a[2]}, 0x{TT[kind]:02X})"
        lines.append(f"    const uint32_t {d} = {e};")
    for i, o in enumerate(outs):
        lines.append(f"    s{i} = {o};")
    return lines


def function(name, what, c, outs):
    body = emit(c, outs)
    return (f"""// {what}: {len(c.ops)} operations.
__device__ __forceinline__ void {name}(uint32_t u0, uint32_t u1, uint32_t u2,
""" + " " * (len(name) + 33) + """uint32_t u3, uint32_t u4, uint32_t u5,
""" + " " * (len(name) + 33) + """uint32_t u6, uint32_t u7, uint32_t &s0,
""" + " " * (len(name) + 33) + """uint32_t &s1, uint32_t &s2, uint32_t &s3,
""" + " " * (len(name) + 33) + """uint32_t &s4, uint32_t &s5, uint32_t &s6,
""" + " " * (len(name) + 33) + """uint32_t &s7) {
""" + "\n".join(body) + "\n}\n")


def main():
    c, outs = build()
    ci, outs_i = build(inverse=True)
    sbox = [sbox_direct(a) for a in range(256)]
    assert sorted(sbox) == list(range(256))
    inv = [0] * 256
    for a in range(256):
        inv[sbox[a]] = a
    for a in range(256):
        assert simulate(c, outs, a) == sbox[a], a
        assert simulate(ci, outs_i, a) == inv[a], a
    # the and-xor and mux tables follow the index convention above
    assert all(lut3_tt(x, y, z, 0x6A) == ((x & y) ^ z) for x in (0, 1) for y in (0, 1)
               for z in (0, 1))
    assert all(lut3_tt(x, y, z, 0xCA) == (y if x else z) for x in (0, 1) for y in (0, 1)
               for z in (0, 1))
    hdr = f"""// bitslice_sbox.h -- generated by gen_bitslice_sbox.py; do not edit.
//
// The AES S-box and inverse S-box (FIPS-197 5.1.1, 5.3.2) as straight-line
// circuits on bit planes: bit i of each input byte is in u<i> (one bit per
// lane bit, so 32 blocks at once), output bit i is written to s<i>.  Derived
// in the tower field GF((2^4)^2) with GF(16) = GF(2)[y]/(y^4+y+1) and
// X^2 + X + {LAM} (root of the AES polynomial: 0x{BETA:02X} in that field); each
// operation is one VALU instruction (three-input functions use v_bitop3_b32
// with index (S0 << 2) | (S1 << 1) | S2).  Both checked on all 256 inputs
// when generated.
#pragma once

#include <stdint.h>

"""
    text = hdr + function("bitslice_sbox", "S-box", c, outs) + "\n" + \
        function("bitslice_inv_sbox", "Inverse S-box", ci, outs_i)
    with open(OUT, "w") as f:
        f.write(text)
    print(f"wrote {OUT}: {len(c.ops)} + {len(ci.ops)} ops, lambda={LAM}, beta=0x{BETA:02X}")


if __name__ == "__main__":
    main()
