"""The addresses whose hashed form equals the LDS tables' empty marker.

The library hashes every source with one 32-bit bijection and every
destination with another (in its entity outputs destinations use the source
one), and keeps the one address per view whose hash is 0xFFFFFFFF outside
its tables.  Tests use these addresses to reach that path; they are computed
here from the published form of the two mixers (xor-shift / odd-multiply
rounds), inverted step by step.
"""
M32 = 0xFFFFFFFF


def _inv_odd(m):
    return pow(m, -1, 1 << 32)


def _unmix(x, key, m1, m2):
    # undo: x ^= key; x ^= x >> 16; x *= m1; x ^= x >> 15; x *= m2; x ^= x >> 16
    x ^= x >> 16
    x = (x * _inv_odd(m2)) & M32
    x ^= (x >> 15) ^ (x >> 30)
    x = (x * _inv_odd(m1)) & M32
    x ^= x >> 16
    x ^= key
    return x & M32


def _mix(x, key, m1, m2):
    x ^= key
    x ^= x >> 16
    x = (x * m1) & M32
    x ^= x >> 15
    x = (x * m2) & M32
    x ^= x >> 16
    return x


ROW = (0x421E9A93, 0x897EA68D, 0x3EA9E261)
COL = (0x3F4760C9, 0xE8F25BB3, 0xA84F7BAF)

SOURCE_MARKER = _unmix(M32, *ROW)        # row_hash(SOURCE_MARKER) == 0xFFFFFFFF
DESTINATION_MARKER = _unmix(M32, *COL)   # col_hash(DESTINATION_MARKER) == 0xFFFFFFFF
assert _mix(SOURCE_MARKER, *ROW) == M32 and _mix(DESTINATION_MARKER, *COL) == M32
