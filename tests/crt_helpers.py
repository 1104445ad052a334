"""Plain-Python number theory shared by the dual-exponent tests (no library
and no oracle code): the combined exponent of the footnote on CRT exponents."""
import math


def combined_exponent(p, q, ep, eq):
    """The smallest e >= 1 with e = ep mod (p - 1) and e = eq mod (q - 1), by
    the Chinese remainder theorem on the exponents (it exists when ep = eq mod
    gcd(p - 1, q - 1))."""
    a, b = p - 1, q - 1
    g = math.gcd(a, b)
    assert (ep - eq) % g == 0
    t = ((eq - ep) // g * pow(a // g, -1, b // g)) % (b // g)
    lcm = a // g * b
    return (ep + a * t) % lcm or lcm
