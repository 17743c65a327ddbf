"""Argument checks of the Python binding, on the host: a buffer that is not a contiguous
GPU tensor of 64-bit integers, or that holds too few elements for the call, is rejected
before any pointer reaches the C ABI.  A duck-typed stand-in plays the GPU tensor, so no
GPU is needed; every rejection happens before the library is called."""
import pytest

torch = pytest.importorskip("torch")
ntt = pytest.importorskip("paper_2012_01968_amd")


class FakePlan:
    handle = 0x1000   # never dereferenced: every call below fails its argument checks first
    N = 16
    L = 3


class FakeGpuTensor:
    def __init__(self, numel, dtype=torch.int64, contiguous=True, cuda=True):
        self._numel, self.dtype, self._contig, self.is_cuda = numel, dtype, contiguous, cuda

    def numel(self):
        return self._numel

    def element_size(self):
        return torch.empty(0, dtype=self.dtype).element_size()

    def is_contiguous(self):
        return self._contig

    def data_ptr(self):
        return 0x7F0000000000   # an operand that passes; the call still fails on a later one


PER = FakePlan.N * FakePlan.L


def test_host_tensor_rejected():
    with pytest.raises(ValueError, match="GPU memory"):
        ntt.ntt_forward(FakePlan(), torch.zeros(PER, dtype=torch.int64))


@pytest.mark.parametrize("dtype", [torch.int32, torch.float64, torch.uint8, torch.complex64])
def test_wrong_element_type_rejected(dtype):
    with pytest.raises(ValueError, match="64-bit integers"):
        ntt.ntt_inverse(FakePlan(), FakeGpuTensor(PER, dtype=dtype), n_polys=1)


def test_strided_view_rejected():
    with pytest.raises(ValueError, match="contiguous"):
        ntt.ntt_forward(FakePlan(), FakeGpuTensor(PER, contiguous=False), n_polys=1)


def test_short_operands_rejected():
    plan = FakePlan()
    a, short = FakeGpuTensor(2 * PER), FakeGpuTensor(2 * PER - 1)
    with pytest.raises(ValueError, match="holds"):
        ntt.ntt_forward(plan, FakeGpuTensor(PER), n_polys=2)
    with pytest.raises(ValueError, match="b holds"):
        ntt.ntt_pointwise_mul(plan, a, short, a)
    with pytest.raises(ValueError, match="c holds"):
        ntt.ntt_polymul_negacyclic(plan, a, a, short)
    with pytest.raises(ValueError, match="whole number"):
        ntt.ntt_forward(plan, FakeGpuTensor(PER + 1))
    with pytest.raises(ValueError, match="at least 1"):
        ntt.ntt_forward(plan, FakeGpuTensor(PER), n_polys=0)


def test_raw_address_needs_count():
    with pytest.raises(ValueError, match="raw address"):
        ntt.ntt_forward(FakePlan(), 0x7F0000000000)


def test_batch_job_sizes_checked():
    plan = FakePlan()
    data = FakeGpuTensor(2 * 2 * plan.N)   # 2 polys of 2 limbs
    key_short = FakeGpuTensor(2 * plan.N - 1)
    with pytest.raises(ValueError, match="job 0 data holds"):
        ntt._jobs_array([(plan, data, 3, 2, ntt.OP_FORWARD)])
    with pytest.raises(ValueError, match="job 0 key holds"):
        ntt._jobs_array([(plan, data, 2, 2, ntt.OP_FORWARD | ntt.OP_MULKEY, key_short)])
    with pytest.raises(ValueError, match="GPU memory"):
        ntt._jobs_array([(plan, torch.zeros(4 * plan.N, dtype=torch.int64), 2, 2, ntt.OP_FORWARD)])
