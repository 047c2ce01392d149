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

# kind: (R rows, K depth, V values per lane, integer kind)
KINDS = {0: (32, 16, 8, False), 1: (32, 32, 16, True), 2: (16, 32, 8, False), 3: (16, 64, 16, True)}


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


def pack(M, layout, V, is_int, rows_first=True):
    """Registers (64 x 16 bytes) holding matrix M (R x K if rows_first else K x R)."""
    out = np.zeros((64, 16), dtype=np.uint8)
    for l in range(64):
        vals = []
        for v in range(V):
            r, k = layout(l, v)
            vals.append(M[r, k] if rows_first else M[k, r])
        if is_int:
            out[l, :V] = np.array(vals, dtype=np.int8).view(np.uint8)
        else:
            bits = (np.array(vals, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)
            out[l, :2 * V] = bits.view(np.uint8)
    return out


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_lowp_mfma_layout(kind):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    R, K, V, is_int = KINDS[kind]
    print(f"probe raw kind={kind} R={R} K={K}", flush=True)
    A = synth.integer_valued((R, K), 10 + kind, 8)
    B = synth.integer_valued((K, R), 20 + kind, 8)
    P = (A.astype(np.int64) @ B.astype(np.int64))
    dev = torch.device("cuda:0")
    found = []
    nreg = 16 if R == 32 else 4
    for hname, h in in_layouts(R, K, V).items():
        ta = torch.from_numpy(pack(A, h, V, is_int, True)).to(dev)
        tb = torch.from_numpy(pack(B, h, V, is_int, False)).to(dev)
        td = torch.zeros((64, 16), dtype=torch.int32, device=dev)
        mg.probe_mfma_raw(kind, ta, tb, td)
        torch.cuda.synchronize()
        raw = td.cpu().numpy()
        vals = raw.view(np.int32) if is_int else raw.view(np.float32)
        for oname, o in out_layouts(R).items():
            ok = all(vals[l, r] == P[o(l, r)] for l in range(64) for r in range(nreg))
            if ok:
                found.append((hname, oname))
    print(f"  kind {kind}: matching layouts {found}", flush=True)
    assert ("blocked", "standard") in found
