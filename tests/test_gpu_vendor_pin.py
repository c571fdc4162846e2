"""Opaque external pin of the oracle's Philox4x32-10 (constants and round
structure): the installed rocRAND generator, run only through its public
host API, must produce the same word sequence as the oracle for the same
64-bit seed: words 0 .. N-1 of the key (lo32(seed), hi32(seed)) in counter
order, which pins the multipliers, the round structure, the counter layout
(R3) and the word order within a block (R5).  The vendor library is not a dependency of the GPU
path: this test checks the oracle only.  It needs the HIP runtime (the
vendor's generators allocate device memory), hence the GPU mark."""
import ctypes
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

LIB = "/opt/rocm/lib/librocrand.so"
PHILOX = 404      # ROCRAND_RNG_PSEUDO_PHILOX4_32_10 (public rocrand.h)


def _vendor_words(seed: int, n: int) -> np.ndarray:
    import torch   # binds the vendor library to the same HIP runtime
    torch.cuda.init()
    L = ctypes.CDLL(LIB)
    gen = ctypes.c_void_p()
    assert L.rocrand_create_generator(ctypes.byref(gen), PHILOX) == 0
    try:
        assert L.rocrand_set_seed(gen, ctypes.c_ulonglong(seed)) == 0
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        assert L.rocrand_generate(gen, ctypes.c_void_p(out.data_ptr()), ctypes.c_size_t(n)) == 0
        torch.cuda.synchronize()
        return out.cpu().numpy().view(np.uint32).copy()
    finally:
        L.rocrand_destroy_generator(gen)


@pytest.mark.skipif(not os.path.exists(LIB), reason="vendor generator not installed")
@pytest.mark.parametrize("seed", [0x0123456789ABCDEF, 42, 0xFFFFFFFF00000001])
def test_oracle_philox_words_equal_vendor_words(seed):
    n = 1 << 14
    v = _vendor_words(seed, n)
    ours = oracle.philox_words(seed, 0, n)
    exact = bool(np.array_equal(v, ours))
    vb = {tuple(int(x) for x in v[i:i + 4]) for i in range(0, n, 4)}
    ob = {tuple(int(x) for x in ours[i:i + 4]) for i in range(0, n, 4)}
    print(f"seed {seed:#x}: exact sequence match {exact}, common blocks {len(vb & ob)} of {len(ob)}")
    assert vb == ob
    assert exact, "same blocks in another order: the counter layout or word order differs"
