"""The bucket dictionary on the GPU against the FP64 oracle: lookups through
a codebook, an index map and gains (a two-level gather), and Lloyd's steps
that build the codebook (the assignment on the matrix cores, the update by a
counting sort and fixed-order sums).

Tolerances.  Dictionary lookups: 1e-5 absolute, the forward's bound (the
decoded texel is one binary32 product of a gain and an entry).  Assignment:
the GPU ranks entries by |c|^2 - 2 x . c in binary32 (matrix-core products
accumulated over D terms), so each value is within
eps_k = 2 D 2^-24 (|c_k|^2 + 2 sum_i |x_i c_ki|) of the exact one: the chosen
entry must be within eps of the best in exact squared distance, and must be
the best wherever the runner-up is more than the two eps away.  Update:
counts exact; each mean within (64 + pieces) 2^-24 max|x| of the exact mean
(binary32 sums of at most 64 rows, then of the pieces); empty entries
untouched bit for bit; two runs bitwise equal.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import check_fwd, host
from paper_2301_01719_amd import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
U = 2.0 ** -24


@pytest.fixture(scope="module")
def rt():
    from paper_2301_01719_amd import radtex
    return radtex


def _frames_up(g, N):
    z = torch.rand(N, generator=g, dtype=torch.float64) * (1 - 0.7) + 0.7
    phi = torch.rand(N, generator=g, dtype=torch.float64) * 2 * np.pi
    r = torch.sqrt(1 - z * z)
    Nv = torch.stack([r * torch.cos(phi), r * torch.sin(phi), z], 1)
    a = torch.randn((N, 3), generator=g, dtype=torch.float64)
    T = a - (a * Nv).sum(1, keepdim=True) * Nv
    T = T / torch.linalg.vector_norm(T, dim=1, keepdim=True)
    return torch.stack([T, torch.linalg.cross(Nv, T, dim=1), Nv], 1).to(torch.float32)


def _frags(seed, N):
    g = torch.Generator().manual_seed(seed)
    uv = (torch.rand((N, 2), generator=g, dtype=torch.float64) * 5 - 2).to(torch.float32)
    tbn = _frames_up(g, N)
    # views on the cap I_z >= -0.3 of each fragment's texture space
    z = torch.rand(N, generator=g, dtype=torch.float64) * 1.3 - 0.3
    phi = torch.rand(N, generator=g, dtype=torch.float64) * 2 * np.pi
    rr = torch.sqrt(torch.clamp(1 - z * z, min=0))
    vt = torch.stack([rr * torch.cos(phi), rr * torch.sin(phi), z], 1)
    view = torch.einsum("nkm,nk->nm", tbn.to(torch.float64), vt).to(torch.float32)
    return uv.contiguous(), tbn.contiguous(), view.contiguous()


def _index(g, H, W, K, dtype):
    idx = torch.randint(0, K, (H, W), generator=g, dtype=torch.int64)
    if dtype == "u8":
        return idx.to(torch.uint8), idx.to(torch.int32)
    if dtype == "u16":  # stored in int16, read as unsigned
        return idx.to(torch.int32).to(torch.int16), idx.to(torch.int32)
    return idx.to(torch.int32), idx.to(torch.int32)


@pytest.mark.parametrize("W,H,n,C,K,idx_t", [(5, 3, 4, 3, 7, "u8"), (16, 9, 8, 4, 200, "u8"),
                                             (7, 6, 16, 4, 1000, "u16"), (3, 2, 5, 1, 6, "i32"),
                                             (33, 17, 16, 2, 256, "u8"), (1, 1, 32, 4, 3, "u16"),
                                             (3, 2, 64, 4, 5, "u8")])
@pytest.mark.parametrize("fmt", ["f32", "bf16"])
@pytest.mark.parametrize("with_gains", [False, True])
def test_dictionary_lookup_vs_oracle(rt, W, H, n, C, K, idx_t, fmt, with_gains):
    g = torch.Generator().manual_seed(W * 13 + K + len(fmt))
    cb = torch.rand((K, n, n, C), generator=g)
    if fmt == "bf16":
        cb_dev = cb.to(torch.bfloat16).view(torch.int16)
        cb_host = cb_dev.numpy().view(np.uint16)
        of = oracle.FMT_BF16
    else:
        cb_dev, cb_host, of = cb, cb.numpy(), oracle.FMT_F32
    idx_dev, idx_host = _index(g, H, W, K, idx_t)
    gains = (torch.rand((H, W), generator=g) * 1.5 + 0.25) if with_gains else None
    tex = rt.DictionaryTexture(cb_dev.contiguous().to(DEV), idx_dev.to(DEV), W, H, n, C, fmt,
                               None if gains is None else gains.to(DEV))
    N = 3001
    uv, tbn, view = _frags(W + K, N)
    for mode, om in (("nearest", oracle.MODE_NEAREST), ("bilinear", oracle.MODE_BILINEAR)):
        out = rt.lookup_fwd(tex, uv.to(DEV), tbn.to(DEV), view.to(DEV), mode=mode)
        torch.cuda.synchronize()
        ref = oracle.lookup_fwd_dict(cb_host, K, idx_host.numpy(),
                                     None if gains is None else gains.numpy(), W, H, n, C,
                                     uv.numpy(), tbn.numpy(), view.numpy(), fmt=of, mode=om)
        if mode == "nearest":
            from helpers import bucket_edge_mask
            keep = bucket_edge_mask(uv.numpy(), tbn.numpy(), view.numpy(), W, H, n)
        else:
            keep = None
        check_fwd(host(out), ref, keep)


def test_dictionary_entry_numbers_past_the_codebook_read_its_last_entry(rt):
    W, H, n, C, K = 6, 5, 8, 3, 10
    g = torch.Generator().manual_seed(3)
    cb = torch.rand((K, n, n, C), generator=g)
    idx = torch.randint(0, 40, (H, W), generator=g, dtype=torch.int32)
    tex = rt.DictionaryTexture(cb.to(DEV), idx.to(DEV), W, H, n, C)
    uv, tbn, view = _frags(4, 2000)
    out = rt.lookup_fwd(tex, uv.to(DEV), tbn.to(DEV), view.to(DEV), mode="bilinear")
    torch.cuda.synchronize()
    ref = oracle.lookup_fwd_dict(cb.numpy(), K, np.minimum(idx.numpy(), K - 1), None, W, H, n, C,
                                 uv.numpy(), tbn.numpy(), view.numpy(), mode=oracle.MODE_BILINEAR)
    check_fwd(host(out), ref)


def test_dictionary_light_lookup(rt):
    # the light lookup reads a dictionary like any texture: against the
    # oracle's light lookup of the matrix decoded by numpy
    W, H, n, C, K = 8, 4, 16, 4, 12
    g = torch.Generator().manual_seed(5)
    cb = torch.rand((K, n, n, C), generator=g)
    idx = torch.randint(0, K, (H, W), generator=g, dtype=torch.int64).to(torch.uint8)
    gains = torch.rand((H, W), generator=g) + 0.5
    tex = rt.DictionaryTexture(cb.to(DEV), idx.to(DEV), W, H, n, C, gains=gains.to(DEV))
    uv, tbn, _ = _frags(6, 1500)
    sun = wl.sun_light(9, elevation_deg=70.0, radius_deg=10.0)
    out = rt.lookup_light(tex, uv.to(DEV), tbn.to(DEV), rt.make_light(sun.numpy()),
                          mode="bilinear")
    torch.cuda.synchronize()
    dec = cb.numpy().astype(np.float64)[idx.numpy().astype(np.int64)]
    dec = dec * gains.numpy().astype(np.float64)[:, :, None, None, None]
    ref = oracle.lookup_light(oracle.Tex(dec, W, H, n, C, oracle.FMT_F64), uv.numpy(), tbn.numpy(),
                              sun.numpy(), mode=oracle.MODE_BILINEAR)
    check_fwd(host(out), ref)


# ---------------------------------------------------------------------------
# Lloyd's steps
# ---------------------------------------------------------------------------

def _eps(X, cb):
    """eps [M, K] of the module docstring."""
    X64, c64 = X.astype(np.float64), cb.astype(np.float64)
    D = X.shape[1]
    return 2 * D * U * ((c64 * c64).sum(1)[None, :] + 2 * np.abs(X64) @ np.abs(c64).T)


def _check_assign(X, cb, a_gpu, d_gpu=None):
    """Validity of a GPU assignment against exact squared distances."""
    from scipy.spatial.distance import cdist
    X64, c64 = X.astype(np.float64), cb.astype(np.float64)
    d = cdist(X64, c64, "sqeuclidean")
    eps = _eps(X, cb)
    a_o, _ = oracle.vq_assign(X, cb)
    rows = np.arange(X.shape[0])
    best = d[rows, a_o]
    chosen = d[rows, a_gpu]
    assert np.all(chosen <= best + eps[rows, a_gpu] + eps[rows, a_o]), \
        np.max(chosen - best - eps[rows, a_gpu] - eps[rows, a_o])
    # where no other entry comes within the two eps of the best, the choice is exact
    slack = d - best[:, None] - eps - eps[rows, a_o][:, None]
    slack[rows, a_o] = np.inf
    clear = np.all(slack > 0, axis=1)
    np.testing.assert_array_equal(a_gpu[clear], a_o[clear])
    if d_gpu is not None:
        xsq = (X64 * X64).sum(1)
        tol = eps[rows, a_gpu] + 2 * X.shape[1] * U * xsq + 1e-30
        assert np.all(np.abs(d_gpu - chosen) <= tol), np.max(np.abs(d_gpu - chosen) - tol)
    return clear.mean()


@pytest.mark.parametrize("M,D,K", [(1000, 48, 37), (4097, 8, 5), (70, 1024, 256), (513, 7, 300),
                                   (257, 1, 2), (64, 1024, 1), (3000, 256, 1000), (129, 20, 256)])
def test_vq_assign_vs_oracle(rt, M, D, K):
    g = torch.Generator().manual_seed(M + D + K)
    X = torch.randn((M, D), generator=g)
    cb = torch.randn((K, D), generator=g)
    if K > 4:
        cb[3] = cb[1]  # an exact duplicate: either is right, both at the same distance
    a, d = rt.vq_assign(X.to(DEV), cb.to(DEV), want_dist=True)
    torch.cuda.synchronize()
    frac = _check_assign(X.numpy(), cb.numpy(), host(a), host(d))
    assert frac > 0.5, frac  # the exact-match check covers most rows (not the duplicate's)
    assert host(a).min() >= 0 and host(a).max() < K


def test_vq_update_vs_oracle_and_deterministic(rt):
    M, D, K = 20000, 96, 300
    g = torch.Generator().manual_seed(8)
    X = torch.randn((M, D), generator=g)
    a = torch.randint(0, K - 20, (M,), generator=g, dtype=torch.int32)  # 20 empty entries
    a[:5000] = 7  # one large entry: many pieces
    prev = torch.randn((K, D), generator=g)
    cb1 = prev.clone().to(DEV)
    cnt1 = rt.vq_update(X.to(DEV), a.to(DEV), cb1)
    cb2 = prev.clone().to(DEV)
    cnt2 = rt.vq_update(X.to(DEV), a.to(DEV), cb2)
    torch.cuda.synchronize()
    assert torch.equal(cb1, cb2) and torch.equal(cnt1, cnt2)
    ref, cnt = oracle.vq_update(X.numpy(), a.numpy(), prev.numpy())
    np.testing.assert_array_equal(host(cnt1), cnt)
    got = host(cb1)
    empty = cnt == 0
    np.testing.assert_array_equal(got[empty], prev.numpy()[empty])
    pieces = np.ceil(cnt / 64.0)
    tol = (64 + pieces + 2)[:, None] * U * np.abs(X.numpy()).max()
    assert np.all(np.abs(got - ref) <= tol)


def _repetitive(seed, P, M, D, sigma, device="cpu"):
    """M rows drawn from P prototypes U[0,1)^D plus N(0, sigma^2) noise."""
    g = torch.Generator(device=device).manual_seed(seed)
    protos = torch.rand((P, D), generator=g, device=device)
    labels = torch.randint(0, P, (M,), generator=g, device=device)
    X = protos[labels] + sigma * torch.randn((M, D), generator=g, device=device)
    return protos.cpu(), labels.cpu(), X.contiguous()


def test_lloyd_on_repetitive_buckets_recovers_them_and_the_lookup(rt):
    """Buckets drawn from 24 prototypes plus noise (the 'highly repetitive'
    case): from one member of each group, one assignment and one update find
    the groups and their means; the dictionary built from them renders within
    the noise of the original texture."""
    W, H, n, C, P = 32, 16, 8, 4, 24
    D = n * n * C
    protos, labels, X = _repetitive(9, P, W * H, D, 0.01)
    init = torch.stack([X[int(torch.nonzero(labels == k)[0])] for k in range(P)])
    cb = init.clone().to(DEV)
    a = rt.vq_assign(X.to(DEV), cb)
    counts = rt.vq_update(X.to(DEV), a, cb)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(a), labels.numpy())
    np.testing.assert_array_equal(host(counts), np.bincount(labels.numpy(), minlength=P))
    a_o, _ = oracle.vq_assign(X.numpy(), init.numpy())
    ref, _ = oracle.vq_update(X.numpy(), a_o, init.numpy())
    assert np.max(np.abs(host(cb) - ref)) <= 80 * U * 1.1
    tex = rt.DictionaryTexture(cb.reshape(P, n, n, C), a.to(torch.int32).reshape(H, W), W, H, n, C)
    plain = rt.Texture(X.reshape(H, W, n, n, C).to(DEV), W, H, n, C)
    uv, tbn, view = _frags(10, 4000)
    o1 = rt.lookup_fwd(tex, uv.to(DEV), tbn.to(DEV), view.to(DEV))
    o2 = rt.lookup_fwd(plain, uv.to(DEV), tbn.to(DEV), view.to(DEV))
    torch.cuda.synchronize()
    assert np.abs(host(o1) - host(o2)).max() < 0.06  # a few sigma of the noise


def test_full_size_assignment_and_update(rt):
    """The single-view matrix as a repetitive texture (1024 x 1024 buckets of
    16 x 16 RGBA = 1M rows of D = 1024) against K = 256 entries, in the launch
    the bench times: assignment checked on 4096 sampled rows; the update's
    counts and a sample of entries against the oracle's own full assignment
    and update."""
    W = H = 1024
    D = 16 * 16 * 4
    P = K = 256
    M = W * H
    protos, labels, Xd = _repetitive(11, P, M, D, 0.02, device=DEV)
    first = [int(torch.nonzero(labels == k)[0]) for k in range(K)]
    init = Xd[first].cpu()
    X = Xd.cpu()
    cb = init.clone().to(DEV)
    a, d = rt.vq_assign(Xd, cb, want_dist=True)
    counts = rt.vq_update(Xd, a, cb)
    torch.cuda.synchronize()
    ah, dh = host(a), host(d)
    rows = np.unique(np.concatenate([np.linspace(0, M - 1, 4000).astype(np.int64),
                                     np.arange(M - 96, M)]))
    Xs = X.numpy()[rows]
    _check_assign(Xs, init.numpy(), ah[rows], dh[rows])
    a_o, _ = oracle.vq_assign(X.numpy(), init.numpy())
    np.testing.assert_array_equal(ah, a_o)  # separated groups: no near-ties
    ref, cnt = oracle.vq_update(X.numpy(), a_o, init.numpy())
    np.testing.assert_array_equal(host(counts), cnt)
    pieces = np.ceil(cnt / 64.0)
    tol = (64 + pieces + 2)[:, None] * U * np.abs(X.numpy()).max()
    sel = np.arange(0, K, 7)
    assert np.all(np.abs(host(cb)[sel] - ref[sel]) <= tol[sel])
