"""Lane layouts of the low-precision matrix-core instructions used by the split
path, recovered from raw registers: the test packs small-integer operands under
each candidate input layout, runs one instruction, and checks every accumulator
register against the exact product under each candidate output layout.  The
kernels assume the "blocked" input layout (lane l holds row l % R and the V
consecutive k values starting at (l // R) * V) and the "standard" output layout."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1706_10086_amd as mg  # noqa: E402

# kind: (R rows, K depth, V values per lane, element type)
KINDS = {0: (32, 16, 8, "bf16"), 1: (32, 32, 16, "int8"), 2: (16, 32, 8, "bf16"),
         3: (16, 64, 16, "int8"), 4: (32, 64, 32, "e4m3")}


def e4m3_bits(q: int, bias: int) -> int:
    """An integer |q| <= 16 as an FP8 byte with 4 exponent bits (bias 7: the OCP
    e4m3 format; bias 8: the variant without negative zero), 3 mantissa bits."""
    if q == 0:
        return 0
    a, sign = abs(q), 0x80 if q < 0 else 0
    e = a.bit_length() - 1                      # a = 1.m * 2^e, at most 4 significant bits
    m = (a << 3 >> e) & 7
    return sign | ((e + bias) << 3) | m


def in_layouts(R, K, V):
    G = 64 // R
    return {
        "blocked": lambda l, v: (l % R, (l // R) * V + v),
        "strided": lambda l, v: (l % R, v * G + (l // R)),
    }


def out_layouts(R):
    if R == 32:
        return {"standard": lambda l, r: (8 * (r // 4) + 4 * (l // 32) + r % 4, l % 32),
                "interleaved": lambda l, r: ((l // 32) + 2 * r, l % 32)}
    return {"standard": lambda l, r: (4 * (l // 16) + r, l % 16),
            "interleaved": lambda l, r: ((l // 16) + 4 * r, l % 16)}


def pack(M, layout, V, elem, rows_first=True, bias=7):
    """Registers (64 x 16 bytes, 64 x 32 for e4m3) holding matrix M (R x K if
    rows_first else K x R)."""
    out = np.zeros((64, 32 if elem == "e4m3" else 16), dtype=np.uint8)
    for l in range(64):
        vals = []
        for v in range(V):
            r, k = layout(l, v)
            vals.append(M[r, k] if rows_first else M[k, r])
        if elem == "int8":
            out[l, :V] = np.array(vals, dtype=np.int8).view(np.uint8)
        elif elem == "e4m3":
            out[l, :V] = [e4m3_bits(int(x), bias) for x in vals]
        else:
            bits = (np.array(vals, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)
            out[l, :2 * V] = bits.view(np.uint8)
    return out


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_lowp_mfma_layout(kind):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    R, K, V, elem = KINDS[kind]
    print(f"probe raw kind={kind} R={R} K={K}", flush=True)
    A = synth.integer_valued((R, K), 10 + kind, 8)
    B = synth.integer_valued((K, R), 20 + kind, 8)
    P = (A.astype(np.int64) @ B.astype(np.int64))
    dev = torch.device("cuda:0")
    found = []
    nreg = 16 if R == 32 else 4
    # e4m3: both exponent biases are tried; the split path encodes with bias 7
    for bias in ((7, 8) if elem == "e4m3" else (7,)):
        for hname, h in in_layouts(R, K, V).items():
            ta = torch.from_numpy(pack(A, h, V, elem, True, bias)).to(dev)
            tb = torch.from_numpy(pack(B, h, V, elem, False, bias)).to(dev)
            td = torch.zeros((64, 16), dtype=torch.int32, device=dev)
            mg.probe_mfma_raw(kind, ta, tb, td)
            torch.cuda.synchronize()
            raw = td.cpu().numpy()
            vals = raw.view(np.int32) if elem == "int8" else raw.view(np.float32)
            for oname, o in out_layouts(R).items():
                ok = all(vals[l, r] == P[o(l, r)] for l in range(64) for r in range(nreg))
                if ok:
                    found.append((hname, oname) if bias == 7 else (hname, oname, bias))
    print(f"  kind {kind}: matching layouts {found}", flush=True)
    assert ("blocked", "standard") in found
