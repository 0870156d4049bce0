"""Learned rank proposal (not in the paper): the network's kernels against the
FP64 oracle (forward, gradient, one Adam step), and the construction with a
proposer against the plain construction and the exact kernel."""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_1809_10573_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_1809_10573_amd import binding as B  # noqa: E402

DEV = "cuda:0"
NI = B.MLP_INPUTS


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (n, NI)).astype(np.float32)
    y = (np.sin(3 * X[:, 0]) + X[:, 2] * X[:, 3] + 0.5 * X[:, 4]).astype(np.float32)
    return X, y


@pytest.mark.parametrize("hidden", [16, 128])
def test_forward_and_gradient_match_oracle(hidden):
    p = B.mlp_init(hidden, seed=hidden)
    p[NI * hidden:NI * hidden + hidden] = 0.05          # nonzero biases exercise every term
    X, y = _data(300, 1)                                 # 300: several forward tiles, a ragged tail
    net = B.RankProposer(hidden, params=p)
    Xd, yd = torch.as_tensor(X, device=DEV), torch.as_tensor(y, device=DEV)
    out = net.forward(Xd).cpu().numpy()
    ref = omlp.forward(p.astype(np.float64), X.astype(np.float64), NI, hidden)
    assert np.max(np.abs(out - ref)) <= 1e-5 * max(1.0, np.abs(ref).max())
    loss, g = net.loss_grad(Xd, yd)
    rloss, rg = omlp.loss_and_grad(p.astype(np.float64), X.astype(np.float64), y.astype(np.float64), NI, hidden)
    assert abs(loss - rloss) <= 1e-5 * rloss
    assert np.linalg.norm(g.cpu().numpy() - rg) <= 1e-4 * np.linalg.norm(rg)


def test_one_adam_step_matches_oracle():
    hidden = 32
    p = B.mlp_init(hidden, seed=3)
    X, y = _data(256, 2)
    net = B.RankProposer(hidden, params=p)
    net.train(torch.as_tensor(X, device=DEV), torch.as_tensor(y, device=DEV), epochs=1, batch=256, lr=1e-2)
    _, rg = omlp.loss_and_grad(p.astype(np.float64), X.astype(np.float64), y.astype(np.float64), NI, hidden)
    zero = np.zeros_like(rg)
    rp, _, _ = omlp.adam_step(p.astype(np.float64), rg, zero, zero, step=1, lr=1e-2)
    got = net.params()
    # the first Adam step moves every weight by about lr sign(g); compare where |g| is not tiny
    big = np.abs(rg) > 1e-4 * np.abs(rg).max()
    assert np.max(np.abs(got - rp)[big]) <= 1e-5


def test_training_on_construction_ranks_reduces_the_loss():
    feats, targ = [], []
    for (a, m) in I.family_draws(6, seed=9):
        X, O = I.uniform_grid(4096)
        fac = B.construct(I.fio_phase(a, float(m)), X, O, 1e-6, 16, oversample=2, device=DEV)
        for side in (B.SIDE_U, B.SIDE_V):
            for t in range(1, fac.info()["H"] + 1):
                F, tg = B.rank_samples(fac, side, t, device=DEV)
                feats.append(F)
                targ.append(tg)
    F, tg = torch.cat(feats), torch.cat(targ)
    assert torch.all((tg * 16 >= 1) & (tg * 16 <= 64))
    net = B.RankProposer(64, seed=1)
    before = net.loss_grad(F, tg)[0]
    losses = net.train(F, tg, epochs=60, batch=256, lr=3e-3, seed=2)
    assert losses[-1] < 0.1 * before
    pred = net.forward(F) * 16
    print("rank MAE", float(torch.mean(torch.abs(pred - tg * 16))), "losses", before, losses[0], losses[-1])
    assert float(torch.mean(torch.abs(pred - tg * 16))) < 3.0   # ranks within a few on average


def _rows_error(fac, ph, X, O, seed):
    N = len(X)
    g = I.gaussian_vectors(N, None, seed)
    y = fac.apply(torch.as_tensor(g, device=DEV)).cpu().numpy()
    rows = np.sort(np.random.default_rng(seed).choice(N, 64, replace=False))
    return oracle.relative_error(y[rows], oracle.matvec_rows(ph, X, O, g, rows))


def test_proposal_that_keeps_plain_counts_reproduces_the_plain_construction():
    ph = I.fio_phase(0.6, 2.0)
    X, O = I.uniform_grid(4096)
    plain = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV)
    p = B.mlp_init(16, seed=4)
    p[-1] = 4.0                                           # output bias: every proposed rank is large
    net = B.RankProposer(16, params=p)
    prop = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV, proposer=net, proposal_margin=64)
    info = prop.info()
    assert info["proposed"] == info["n_ids"] and info["rejected"] == 0
    for side in (B.SIDE_U, B.SIDE_V):
        for t in range(1, info["H"] + 1):
            a, b = plain.batch(side, t), prop.batch(side, t)
            assert np.array_equal(a.rank, b.rank) and np.array_equal(a.skel, b.skel)


def test_wrong_proposals_fall_back_and_keep_accuracy():
    ph = I.fio_phase(1.0, 3.0)
    X, O = I.uniform_grid(4096)
    p = B.mlp_init(16, seed=5)
    p[:] = 0.0                                            # predicts rank 1 everywhere: s' = t (1 + 0)
    net = B.RankProposer(16, params=p)
    fac = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV, proposer=net, proposal_margin=0, seed=7)
    info = fac.info()
    assert info["rejected"] > 0.5 * info["proposed"]
    plain = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV)
    e_prop, e_plain = _rows_error(fac, ph, X, O, 3), _rows_error(plain, ph, X, O, 3)
    assert e_prop <= max(2 * e_plain, 1e-4)


def test_trained_proposer_saves_samples_at_equal_accuracy():
    feats, targ = [], []
    for (a, m) in I.family_draws(8, seed=11):
        X, O = I.uniform_grid(4096)
        fac = B.construct(I.fio_phase(a, float(m)), X, O, 1e-6, 16, oversample=2, device=DEV)
        for side in (B.SIDE_U, B.SIDE_V):
            for t in range(1, fac.info()["H"] + 1):
                F, tg = B.rank_samples(fac, side, t, device=DEV)
                feats.append(F)
                targ.append(tg)
    net = B.RankProposer(64, seed=3)
    net.train(torch.cat(feats), torch.cat(targ), epochs=60, batch=256, lr=3e-3, seed=4)
    for (a, m) in I.family_draws(3, seed=12):             # held-out family members
        ph = I.fio_phase(a, float(m))
        X, O = I.uniform_grid(4096)
        plain = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV)
        prop = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV, proposer=net, proposal_margin=4,
                           seed=1)
        ip, iq = plain.info(), prop.info()
        assert iq["sampled_entries"] < ip["sampled_entries"]
        assert _rows_error(prop, ph, X, O, 5) <= max(2 * _rows_error(plain, ph, X, O, 5), 1e-5)


def test_accepted_proposals_match_the_oracle():
    """Every ID of a construction with a proposer, judged by the oracle on the
    GPU's own candidate and allowed sets: an accepted proposal is the oracle's
    column_id of the proposal's s' Mock-Chebyshev samples (same skeleton, T to
    the parity bound) and passes oracle.mlp.residual_ok on the same check
    rows; a rejected one fails that test and is stored as the plain ID.  The
    network only chooses s' (passed to the oracle as an input)."""
    ph = I.fio_phase(1.0, 1.0)
    N, leaf, tol, t_os, seed = 4096, 16, 1e-6, 2, 5
    X, O = I.uniform_grid(N)
    counts = {"accepted": 0, "rejected": 0, "kept": 0}
    # a proposal of rank 12 (+2) that the test mostly accepts, and one of rank 3
    # that it mostly rejects
    for k_hat, margin in ((12, 2), (3, 0)):
        p = np.zeros(B.load().idbf_mlp_param_count(16), np.float32)
        p[-1] = k_hat / 16.0                              # proposes rank k_hat everywhere
        net = B.RankProposer(16, params=p)
        fac = B.construct(ph, X, O, tol, leaf, oversample=t_os, device=DEV, proposer=net,
                          proposal_margin=margin, seed=seed)
        _judge_proposals(fac, ph, X, O, tol, t_os, seed, k_hat + margin, counts)
        print(k_hat, margin, counts, flush=True)
    assert counts["accepted"] > 0 and counts["rejected"] > 0


def _judge_proposals(fac, ph, X, O, tol, t_os, seed, k_prop, counts):
    from gpu_export import GpuLevels
    G = GpuLevels(fac)
    for t in range(1, G.H + 1):
        for side in (B.SIDE_U, B.SIDE_V):
            proposed, used, rejected = fac.proposal(side, t)
            b, offs = G.batches[(side, t)]
            for q in range(len(b.rank)):
                cand, allowed = G.sets(side, t, q)
                coords = X[allowed] if side == B.SIDE_V else O[allowed]
                s_plain = oracle.sample_count(len(cand), len(allowed), t_os)
                sp = int(proposed[q])
                assert sp == min(s_plain, t_os * k_prop), (t, side, q)
                samp = allowed[oracle.mock_chebyshev(coords, sp)]
                Bm = (oracle.entries(ph, X, O, samp, cand) if side == B.SIDE_V
                      else oracle.entries(ph, X, O, cand, samp).T)
                cid = oracle.column_id(Bm, tol)
                pos = omlp.check_positions(seed, t, side, q, len(allowed))
                rows = allowed[pos]
                A = (oracle.entries(ph, X, O, rows, cand) if side == B.SIDE_V
                     else oracle.entries(ph, X, O, cand, rows).T)
                ok = sp == s_plain or omlp.residual_ok(A, cid.skel, cid.red, cid.T, tol)
                assert bool(rejected[q]) == (not ok), (t, side, q)
                rec = G.record(side, t, q)
                if ok:
                    counts["kept" if sp == s_plain else "accepted"] += 1
                    assert int(used[q]) == sp
                else:
                    counts["rejected"] += 1
                    assert int(used[q]) == s_plain
                    samp = allowed[oracle.mock_chebyshev(coords, s_plain)]
                    Bm = (oracle.entries(ph, X, O, samp, cand) if side == B.SIDE_V
                          else oracle.entries(ph, X, O, cand, samp).T)
                    cid = oracle.column_id(Bm, tol)
                assert np.array_equal(rec.skel, cand[cid.skel]), (t, side, q)
                kappa = cid.rdiag[0] / cid.rdiag[-1]
                scale = max(1.0, np.abs(cid.T).max(initial=0.0))
                assert np.max(np.abs(rec.T - cid.T), initial=0.0) <= 1e-12 * kappa * scale, (t, side, q)


def test_force_reject_gives_the_plain_factors_bit_for_bit():
    """IDBF_FLAG_PROPOSER_FORCE_REJECT: every proposal is rejected and
    recomputed by the plain ID, so ranks, skeletons, T and S equal those of a
    construction without a proposer exactly."""
    ph = I.fio_phase(0.8, 3.0)
    X, O = I.uniform_grid(4096)
    plain = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV)
    p = B.mlp_init(16, seed=4)
    net = B.RankProposer(16, params=p)
    forced = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV, proposer=net, proposal_margin=2,
                         force_reject=True)
    st = forced.stats()
    assert sum(L[s]["rejected"] for L in st["per_level"] for s in "UV") == forced.info()["n_ids"]
    assert sum(L[s]["accepted"] for L in st["per_level"] for s in "UV") == 0
    from gpu_export import same_factors
    same_factors(plain, forced)


def _train_nets(members, N=4096, epochs=40):
    """Rank and skeleton networks trained on the GPU on plain constructions."""
    fr, tr, fs, ts = [], [], [], []
    for (a, m) in members:
        X, O = I.uniform_grid(N)
        fac = B.construct(I.fio_phase(a, float(m)), X, O, 1e-6, 16, oversample=2, device=DEV)
        for side in (B.SIDE_U, B.SIDE_V):
            for t in range(1, fac.info()["H"] + 1):
                F, tg = B.rank_samples(fac, side, t, device=DEV)
                fr.append(F)
                tr.append(tg)
                F, tg = B.skeleton_samples(fac, side, t, device=DEV)
                fs.append(F)
                ts.append(tg)
    rank = B.RankProposer(64, seed=3)
    rank.train(torch.cat(fr), torch.cat(tr), epochs=epochs, batch=256, lr=3e-3, seed=4)
    skel = B.RankProposer(64, seed=5)
    losses = skel.train(torch.cat(fs), torch.cat(ts), epochs=epochs // 2, batch=1024, lr=3e-3, seed=6)
    return rank, skel, losses


def test_skeleton_samples_label_the_plain_skeletons():
    ph = I.fio_phase(0.5, 2.0)
    X, O = I.uniform_grid(2048)
    fac = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV)
    for side in (B.SIDE_U, B.SIDE_V):
        for t in range(1, fac.info()["H"] + 1):
            F, tg = B.skeleton_samples(fac, side, t, device=DEV)
            b = fac.batch(side, t)
            assert F.shape == (int(b.cand_len.sum()), B.MLP_INPUTS)
            assert int(tg.sum().item()) == int(b.rank.sum())        # one label per skeleton
            rel = F[:, 6].cpu().numpy()                               # l / c in [0, 1)
            assert rel.min() >= 0 and rel.max() < 1


def _judge_skeleton_proposals(fac, ph, X, O, tol, t_os, seed, counts):
    """Every ID of a construction with rank and skeleton proposers, judged by
    the oracle on the GPU's own sets: an accepted proposal is
    oracle.column_id on the s' Mock-Chebyshev samples with the pivot search
    restricted to the proposed set (same skeleton, T to the parity bound)
    and passes oracle.mlp.residual_ok on the same check rows; a rejected one
    fails it (or keeps no column) and is stored as the plain pivoted ID."""
    from gpu_export import GpuLevels
    G = GpuLevels(fac)
    for t in range(1, G.H + 1):
        for side in (B.SIDE_U, B.SIDE_V):
            proposed, used, rejected = fac.proposal(side, t)
            n_prop, order = fac.skeleton_proposal(side, t)
            b, offs = G.batches[(side, t)]
            for q in range(len(b.rank)):
                cand, allowed = G.sets(side, t, q)
                coords = X[allowed] if side == B.SIDE_V else O[allowed]
                s_plain = oracle.sample_count(len(cand), len(allowed), t_os)
                sp = int(proposed[q])
                assert 1 <= n_prop[q] <= min(len(cand), B.MAX_RANK)
                among = order[q, :n_prop[q]].astype(np.int64)
                assert len(np.unique(among)) == n_prop[q] and among.max() < len(cand)
                samp = allowed[oracle.mock_chebyshev(coords, sp)]
                Bm = (oracle.entries(ph, X, O, samp, cand) if side == B.SIDE_V
                      else oracle.entries(ph, X, O, cand, samp).T)
                cid = oracle.column_id(Bm, tol, among=among)
                ok = False
                if cid is not None:
                    pos = omlp.check_positions(seed, t, side, q, len(allowed))
                    rows = allowed[pos]
                    A = (oracle.entries(ph, X, O, rows, cand) if side == B.SIDE_V
                         else oracle.entries(ph, X, O, cand, rows).T)
                    ok = omlp.residual_ok(A, cid.skel, cid.red, cid.T, tol)
                assert bool(rejected[q]) == (not ok), (t, side, q)
                rec = G.record(side, t, q)
                if ok:
                    counts["accepted"] += 1
                    counts["tall"] += sp > 128
                    assert int(used[q]) == sp
                else:
                    counts["rejected"] += 1
                    assert int(used[q]) == s_plain
                    samp = allowed[oracle.mock_chebyshev(coords, s_plain)]
                    Bm = (oracle.entries(ph, X, O, samp, cand) if side == B.SIDE_V
                          else oracle.entries(ph, X, O, cand, samp).T)
                    cid = oracle.column_id(Bm, tol)
                assert np.array_equal(rec.skel, cand[cid.skel]), (t, side, q)
                kappa = cid.rdiag[0] / cid.rdiag[-1]
                scale = max(1.0, np.abs(cid.T).max(initial=0.0))
                assert np.max(np.abs(rec.T - cid.T), initial=0.0) <= 1e-12 * kappa * scale, (t, side, q)
            print(t, side, counts, flush=True)


def test_skeleton_proposals_match_the_oracle():
    rank, skel, _ = _train_nets(I.family_draws(4, seed=31))
    (a, m), = I.family_draws(1, seed=32)
    ph = I.fio_phase(a, float(m))
    N, leaf, tol, t_os, seed, margin = 4096, 16, 1e-6, 2, 9, 3
    X, O = I.uniform_grid(N)
    fac = B.construct(ph, X, O, tol, leaf, oversample=t_os, device=DEV, proposer=rank, proposal_margin=margin,
                      skeleton_proposer=skel, seed=seed)
    counts = {"accepted": 0, "rejected": 0, "tall": 0}
    _judge_skeleton_proposals(fac, ph, X, O, tol, t_os, seed, counts)
    assert counts["accepted"] > 0 and counts["rejected"] > 0


def test_skeleton_proposals_on_tall_samples_match_the_oracle():
    """Proposals of more than 128 sampled rows: the restricted pivot search
    runs on the tall sample's reduced triangular factor.  Fixed networks: a
    rank of 24 (+4) everywhere, so s' = 5 * 28 = 140 rows, and equal scores,
    so the proposed set is the first 32 candidates."""
    nz = B.load().idbf_mlp_param_count(16)
    p = np.zeros(nz, np.float32)
    p[-1] = 24 / 16.0
    rank = B.RankProposer(16, params=p)
    q = np.zeros(nz, np.float32)
    q[-1] = 0.5
    skel = B.RankProposer(16, params=q)
    ph = I.dft_phase()
    N, leaf, tol, t_os, seed = 1024, 32, 1e-10, 5, 4
    X, O = I.uniform_grid(N)
    fac = B.construct(ph, X, O, tol, leaf, oversample=t_os, device=DEV, proposer=rank, proposal_margin=4,
                      skeleton_proposer=skel, seed=seed)
    counts = {"accepted": 0, "rejected": 0, "tall": 0}
    _judge_skeleton_proposals(fac, ph, X, O, tol, t_os, seed, counts)
    assert counts["accepted"] > 0 and counts["rejected"] > 0 and counts["tall"] > 0


def test_trained_skeleton_proposer_keeps_accuracy():
    rank, skel, losses = _train_nets(I.family_draws(8, seed=41))
    assert losses[-1] < losses[0]
    for (a, m) in I.family_draws(3, seed=42):             # held-out family members
        ph = I.fio_phase(a, float(m))
        X, O = I.uniform_grid(4096)
        plain = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV)
        prop = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV, proposer=rank, proposal_margin=4,
                           skeleton_proposer=skel, seed=1)
        ip, iq = plain.info(), prop.info()
        st = prop.stats()
        acc = sum(L[s]["accepted"] for L in st["per_level"] for s in "UV")
        print(a, m, "accepted", acc, "of", iq["n_ids"], "sampled", iq["sampled_entries"], ip["sampled_entries"],
              flush=True)
        assert acc > 0
        assert _rows_error(prop, ph, X, O, 5) <= max(2 * _rows_error(plain, ph, X, O, 5), 1e-5)
