"""Host-side logic of the library checked exhaustively on the CPU.

The network's SiLU for BF16 pre-activations is read from a table of bf16(fp32(silu(z))) over
2^-13 <= |z| < 2^7 with closed forms outside (z/2 below, z above for z > 0, -0 for z < 0); this
checks that rule against the direct rounding for every finite BF16 value."""
import numpy as np


def bf16_rne(x32):
    u = x32.view(np.uint32).astype(np.uint64)
    return ((u + 0x7fff + ((u >> 16) & 1)) >> 16).astype(np.uint32) & 0xffff


def test_silu_table_rule_is_exact_for_every_bf16():
    b = np.arange(65536, dtype=np.uint32)
    z32 = (b << 16).view(np.float32)
    finite = np.isfinite(z32)
    z = z32.astype(np.float64)
    with np.errstate(over="ignore", invalid="ignore"):
        ref = bf16_rne((z / (1.0 + np.exp(-z))).astype(np.float32))
    E0, NE = 114, 20                           # the table's exponent range
    rel = ((b >> 7) & 0xff).astype(np.int64) - E0
    inr = (rel >= 0) & (rel < NE)
    tiny = bf16_rne((z32 * np.float32(0.5)).astype(np.float32))
    big = np.where((b >> 15) == 1, 0x8000, b)
    rule = np.where(inr, ref, np.where(rel < 0, tiny, big))
    assert np.array_equal(rule[finite], ref[finite])
