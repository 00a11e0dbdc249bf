"""A join past 2^31 input tuples on one MI355X: |R| = |S| = 1.2·10^9 (R keys a
permutation of 1..|R|, S keys uniform over 1..2^31 - 1, so ~56% of S
matches), HJ_AUTO parameters (two
radix passes of 9 + 9 bits, ~4.6K R tuples per partition, one-pass output).
R's keys are unique, so the result is fixed by three checks made on the
device: the count equals #{s.key <= |R|}, every pair joins equal keys, and no
S row appears twice."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1307_1955_amd.hj as hj  # noqa: E402
from paper_1307_1955_amd.gen import device as dgen  # noqa: E402

N = 1_200_000_000


def test_join_past_2_31_tuples():
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < (120 << 30):
        pytest.skip("needs ~110 GB of free device memory (%.0f GB free)" % (free / 2 ** 30))
    p = hj.params("auto", one_pass=True)
    q = hj.hj_resolve_params(p, N, N)
    assert (q.passes, tuple(q.bits)) == (2, (9, 9))
    rk, rr, sk, sr = dgen.unique_uniform(61, N, N, (1 << 31) - 1)
    want = int((sk <= N).sum().item())
    o_r, o_s, cnt = hj.join(rk, rr, sk, sr, p=p)
    assert cnt == want
    assert int(o_r.min()) >= 0 and int(o_r.max()) < N
    assert int(o_s.min()) >= 0 and int(o_s.max()) < N
    # every pair joins equal keys (rid = row index on both sides)
    for a in range(0, cnt, 1 << 28):
        b = min(cnt, a + (1 << 28))
        assert torch.equal(rk[o_r[a:b].long()], sk[o_s[a:b].long()])
    # no S row twice
    mark = torch.zeros(N, dtype=torch.uint8, device=o_s.device)
    mark[o_s.long()] = 1
    assert int(mark.sum(dtype=torch.int64).item()) == cnt
    del rk, rr, sk, sr, o_r, o_s, mark
    torch.cuda.empty_cache()
