"""The FP64 quotient by 6 of the kernels' pointwise solve (the relaxation of
Sec. 3.2, (h^2 f + sum of neighbours) / 6 in 3D) is formed as
fma(y, C_hi, RN(y * C_lo)) with C_hi = RN(1/6), C_lo = RN(1/6 - C_hi).
These CPU tests pin that form to the correctly rounded quotient y / 6:

- the two constants written in the kernel header are those roundings,
  computed here in exact rational arithmetic;
- in exact rational arithmetic, the form equals y / 6 rounded to nearest
  for a sample of doubles;
- compiled C (gcc, no contraction, libm's fma) gives y / 6 bit for bit on
  tens of millions of doubles over the whole exponent range the argument
  covers, on integers and on small multiples of a power of two.

Why it holds for every such y: y / 3 is a 53-bit integer over 3, so it sits
at least 1/6 ulp away from every rounding midpoint, while the value the FMA
rounds differs from y / 6 by at most 2^-108 |y|.
"""
import os
import random
import re
import shutil
import subprocess
import tempfile
from fractions import Fraction

import pytest

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "paper_1208_4247_amd", "csrc", "gmg_internal.h")


def header_constants():
    src = open(HEADER).read()
    body = src[src.index("point_solve(T h2, T f, T nb)"):]
    body = body[:body.index("\n}\n")]
    hexes = re.findall(r"T\((0x1\.[0-9a-f]+p-?\d+)\)", body)
    assert len(hexes) == 2, hexes
    return float.fromhex(hexes[0]), float.fromhex(hexes[1])


def exact_form(y, ch, cl):
    t = float(Fraction(y) * Fraction(cl))  # RN(y * C_lo)
    return float(Fraction(y) * Fraction(ch) + Fraction(t))  # one rounding (the FMA)


def test_header_constants_are_the_split_reciprocal():
    ch, cl = header_constants()
    assert ch == float(Fraction(1, 6))
    assert cl == float(Fraction(1, 6) - Fraction(ch))
    assert cl != 0.0


def test_form_equals_the_rounded_quotient_exactly():
    ch, cl = header_constants()
    rng = random.Random(20121)
    ys = [rng.uniform(-1e3, 1e3) for _ in range(3000)]
    ys += [rng.uniform(0.5, 1.0) * 2.0 ** rng.randint(-960, 1000) for _ in range(3000)]
    ys += [float(k) for k in range(-300, 301)] + [k * 2.0 ** -40 for k in range(1, 300)]
    for y in ys:
        want = float(Fraction(y) / 6)
        assert exact_form(y, ch, cl) == want, y.hex()


C_SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
int main(void) {
  const double ch = %s, cl = %s;
  uint64_t s = 0x2545F4914F6CDD1Dull;
  long bad = 0, n = 0;
  for (long i = 0; i < 40000000L; i++) {
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    uint64_t e = 60 + (s >> 11) %% 1980;   /* biased exponents 60 .. 2039 */
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    uint64_t b = (s & 0x800FFFFFFFFFFFFFull) | (e << 52);
    double y; memcpy(&y, &b, 8);
    double want = y / 6.0, got = fma(y, ch, y * cl);
    n++; if (memcmp(&want, &got, 8)) bad++;
  }
  for (long k = -3000000; k <= 3000000; k++) {
    double y = (double)k, want = y / 6.0, got = fma(y, ch, y * cl);
    n++; if (memcmp(&want, &got, 8)) bad++;
    y = (double)k * 0x1p-40; want = y / 6.0; got = fma(y, ch, y * cl);
    n++; if (memcmp(&want, &got, 8)) bad++;
  }
  printf("%%ld %%ld\n", n, bad);
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_form_equals_division_on_many_doubles():
    ch, cl = header_constants()
    with tempfile.TemporaryDirectory() as tmp:
        c = os.path.join(tmp, "q6.c")
        exe = os.path.join(tmp, "q6")
        open(c, "w").write(C_SRC % (ch.hex(), cl.hex()))
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", c, "-o", exe, "-lm"],
                       check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    n, bad = int(out[0]), int(out[1])
    assert n == 40000000 + 2 * 6000001
    assert bad == 0
