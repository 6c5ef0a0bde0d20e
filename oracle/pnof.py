"""Definitional FP64 oracle (test infrastructure only; see the package docstring).

Notation (arXiv:2004.06142):
  nbf        number of AO basis functions N_B (Section 3.5, Eq. lcao)
  C[mu, p]   NO coefficients, phi_p = sum_mu C[mu,p] zeta_mu (Eq. lcao); S = I
  n[p]       per-spin occupation numbers, 0 <= n <= 1 (Section 2)
  npairs     number of electron pairs N_II/2; ncwo = N_g, weak orbitals per pair
  nsingle    N_I singly occupied orbitals (Omega_I, n = 1/2 each); 0 for singlets
  nact       npairs * (ncwo + 1) + nsingle active orbitals; orbitals >= nact have n = 0
  ERI[m,n,l,s] = (mn|ls) in chemists' notation; the paper's <mu eta|nu delta> = (mu nu|eta delta)
  B[P,m,n]   density-fitting factor, (mn|ls) = sum_P B[P,m,n] B[P,l,s]
Multiplets of highest multiplicity (Section 2, S = N_I / 2) add N_I singly occupied orbitals;
every function takes nsingle (default 0, the singlet case).
"""
from __future__ import annotations

import math

import numpy as np

PNOF5, PNOF7, PNOF7S = 5, 7, 8


# --------------------------------------------------------------------------- layout
def layout(npairs: int, ncwo: int, nbf: int | None = None, nsingle: int = 0):
    """Subspace membership of every orbital (Section 2, Eqs. OmegaG and sum1).

    Strong orbital of pair g (0-based) is orbital g.  The nsingle singly occupied orbitals of
    Omega_I (each its own subspace, n = 1/2) follow: orbitals npairs .. npairs+nsingle-1, so
    that the N_Omega = npairs + nsingle subspace-defining orbitals come first, as in the sums of
    Eqs. EPNOF7 and HFL.  The ncwo weak orbitals of pair g form one consecutive block, the
    blocks taken in reverse pair order: weak k of pair g is npairs + nsingle + ncwo*(npairs-1-g) + k.
    This is the coupling that makes every subspace of the water occupation tables (Tables 1 and
    2) sum to two electrons.

    Returns (pair, strong): pair[p] = subspace id (g for pair g, npairs + t for the t-th single
    orbital) or -1 for inactive p; strong[p] bool.
    """
    nact = npairs * (ncwo + 1) + nsingle
    nbf = nact if nbf is None else nbf
    pair = np.full(nbf, -1, dtype=np.int64)
    strong = np.zeros(nbf, dtype=bool)
    for g in range(npairs):
        pair[g] = g
        strong[g] = True
        for k in range(ncwo):
            pair[npairs + nsingle + ncwo * (npairs - 1 - g) + k] = g
    for t in range(nsingle):
        pair[npairs + t] = npairs + t
    return pair, strong


def single_orbitals(npairs: int, nsingle: int):
    """Orbitals of Omega_I (one electron each, n = 1/2)."""
    return list(range(npairs, npairs + nsingle))


def weak_orbitals(g: int, npairs: int, ncwo: int, nsingle: int = 0):
    return [npairs + nsingle + ncwo * (npairs - 1 - g) + k for k in range(ncwo)]


# --------------------------------------------------------------------------- ON maps
def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def on_sigmoid(gamma, npairs: int, ncwo: int, nsingle: int = 0):
    """n_p = s(gamma_p) / sum_{r in Omega(p)} s(gamma_r): one gamma per active orbital.

    Satisfies 0 < n < 1 and the pairing sum rule (Eq. sum1) by construction.  Orbitals of
    Omega_I have n = 1/2 whatever their gamma.
    """
    pair, _ = layout(npairs, ncwo, nsingle=nsingle)
    s = _sigmoid(np.asarray(gamma, dtype=np.float64))
    tot = np.zeros(npairs + nsingle)
    for p in range(len(s)):
        tot[pair[p]] += s[p]
    singles = set(single_orbitals(npairs, nsingle))
    return np.array([0.5 if p in singles else s[p] / tot[pair[p]] for p in range(len(s))])


def on_sigmoid_jac(gamma, npairs: int, ncwo: int, nsingle: int = 0):
    """dn_p/dgamma_r for the sigmoid-normalised map (quotient rule, block-diagonal)."""
    pair, _ = layout(npairs, ncwo, nsingle=nsingle)
    s = _sigmoid(np.asarray(gamma, dtype=np.float64))
    ds = s * (1.0 - s)
    tot = np.zeros(npairs + nsingle)
    for p in range(len(s)):
        tot[pair[p]] += s[p]
    nact = len(s)
    singles = set(single_orbitals(npairs, nsingle))
    jac = np.zeros((nact, nact))
    for p in range(nact):
        if p in singles:
            continue
        for r in range(nact):
            if pair[p] != pair[r]:
                continue
            S = tot[pair[p]]
            jac[p, r] = ((ds[p] if p == r else 0.0) * S - s[p] * ds[r]) / (S * S)
    return jac


def _trig_gammas(gamma, npairs: int, ncwo: int, g: int):
    """gamma of the strong orbital of pair g, and its ncwo-1 weak-orbital gammas.

    Storage: gamma[g] for g < npairs, then gamma[npairs + g*(ncwo-1) + i], i < ncwo-1.
    """
    gs = gamma[g]
    gw = [gamma[npairs + g * (ncwo - 1) + i] for i in range(ncwo - 1)]
    return gs, gw


def on_trig(gamma, npairs: int, ncwo: int, nsingle: int = 0):
    """Trigonometric ON map of Section 3.1 (Eqs. soo, sum1-h, woo).

    n_g = (1 + cos^2 gamma_g)/2, hole h_g = sin^2(gamma_g)/2; the i-th weak orbital
    (i = 1..N_g) gets h_g * prod_{j<i} cos^2 gamma_{p_j} * sin^2 gamma_{p_i}, the last one
    h_g * prod_{j<N_g} cos^2 gamma_{p_j}.  Orbitals of Omega_I have n = 1/2 (no variable).
    """
    gamma = np.asarray(gamma, dtype=np.float64)
    nact = npairs * (ncwo + 1) + nsingle
    n = np.zeros(nact)
    for t in single_orbitals(npairs, nsingle):
        n[t] = 0.5
    for g in range(npairs):
        gs, gw = _trig_gammas(gamma, npairs, ncwo, g)
        n[g] = 0.5 * (1.0 + math.cos(gs) ** 2)
        h = 0.5 * math.sin(gs) ** 2
        prod = 1.0
        for i, p in enumerate(weak_orbitals(g, npairs, ncwo, nsingle)):
            if i < ncwo - 1:
                n[p] = h * prod * math.sin(gw[i]) ** 2
                prod *= math.cos(gw[i]) ** 2
            else:
                n[p] = h * prod
    return n


def on_trig_jac(gamma, npairs: int, ncwo: int, nsingle: int = 0):
    """dn/dgamma of the trigonometric map (nact x npairs*ncwo), by the product rule."""
    gamma = np.asarray(gamma, dtype=np.float64)
    nact = npairs * (ncwo + 1) + nsingle
    jac = np.zeros((nact, npairs * ncwo))
    for g in range(npairs):
        gs, gw = _trig_gammas(gamma, npairs, ncwo, g)
        col_g = g
        col_w = [npairs + g * (ncwo - 1) + i for i in range(ncwo - 1)]
        jac[g, col_g] = -math.cos(gs) * math.sin(gs)          # d/dx (1+cos^2 x)/2
        h = 0.5 * math.sin(gs) ** 2
        dh = math.sin(gs) * math.cos(gs)
        weak = weak_orbitals(g, npairs, ncwo, nsingle)
        for i, p in enumerate(weak):
            # factors f_j of n_p = h * prod_j f_j, and their derivatives
            factors = [math.cos(gw[j]) ** 2 for j in range(min(i, ncwo - 1))]
            dfactors = [-2.0 * math.cos(gw[j]) * math.sin(gw[j]) for j in range(min(i, ncwo - 1))]
            cols = [col_w[j] for j in range(min(i, ncwo - 1))]
            if i < ncwo - 1:
                factors.append(math.sin(gw[i]) ** 2)
                dfactors.append(2.0 * math.sin(gw[i]) * math.cos(gw[i]))
                cols.append(col_w[i])
            prod = 1.0
            for f in factors:
                prod *= f
            jac[p, col_g] = dh * prod
            for a, c in enumerate(cols):
                other = 1.0
                for b, f in enumerate(factors):
                    if b != a:
                        other *= f
                jac[p, c] += h * other * dfactors[a]
    return jac


# --------------------------------------------------------------------------- coefficients
def phi(n):
    """Phi_p = sqrt(n_p (1 - n_p)) (Section 2, after Eq. interab)."""
    n = np.asarray(n, dtype=np.float64)
    return np.sqrt(n * (1.0 - n))


def coefficients(n, npairs: int, ncwo: int, functional: int = PNOF7, nsingle: int = 0):
    """alpha, beta with E_2 = sum_{p,q in A} (alpha_pq J_pq + beta_pq K_pq).

    Same subspace (Eq. Eg with Pi of Eq. intra): alpha = 0, beta_pp = n_p,
    beta_pq = +sqrt(n_p n_q) for two weak orbitals, -sqrt(n_p n_q) when one is strong.
    Different subspaces (Eq. Efg, counted once per ordered pair (f, g), f != g):
    alpha = 2 n_p n_q; beta = -n_p n_q - Phi_p Phi_q (PNOF7), -n_p n_q (PNOF5, Phi = 0),
    -n_p n_q - 4 Phi_p^2 Phi_q^2 (PNOF7s, Eq. Efg_s).
    A singly occupied orbital has no intra-subspace term (no opposite-spin partner in its own
    orbital, Eq. intra): beta_pp = 0; its interactions with other subspaces follow Eq. Efg with
    n = 1/2 (Eq. interab takes K for real orbitals in both of its cases).
    """
    pair, strong = layout(npairs, ncwo, nsingle=nsingle)
    singles = set(single_orbitals(npairs, nsingle))
    n = np.asarray(n, dtype=np.float64)
    nact = len(pair)
    ph = phi(n)
    alpha = np.zeros((nact, nact))
    beta = np.zeros((nact, nact))
    for p in range(nact):
        for q in range(nact):
            if pair[p] == pair[q]:
                if p == q:
                    beta[p, q] = 0.0 if p in singles else n[p]
                elif strong[p] or strong[q]:
                    beta[p, q] = -math.sqrt(n[p] * n[q])
                else:
                    beta[p, q] = math.sqrt(n[p] * n[q])
            else:
                alpha[p, q] = 2.0 * n[p] * n[q]
                if functional == PNOF5:
                    beta[p, q] = -n[p] * n[q]
                elif functional == PNOF7:
                    beta[p, q] = -n[p] * n[q] - ph[p] * ph[q]
                elif functional == PNOF7S:
                    beta[p, q] = -n[p] * n[q] - 4.0 * ph[p] ** 2 * ph[q] ** 2
                else:
                    raise ValueError(f"unknown functional {functional}")
    return alpha, beta


# --------------------------------------------------------------------------- integrals
def eri_from_df(B):
    """(mn|ls) = sum_P B[P,m,n] B[P,l,s]."""
    naux, nbf, _ = B.shape
    Bm = B.reshape(naux, nbf * nbf)
    return (Bm.T @ Bm).reshape(nbf, nbf, nbf, nbf)


def gamma_ao(C, p):
    """Gamma^p_{mu nu} = C_{mu p} C_{nu p} (Section 3.5)."""
    return np.outer(C[:, p], C[:, p])


def jk_ao_eri(ERI, C, q):
    """J^q, K^q of Eq. Gpmn from the explicit 4-index integrals.

    J^q_{mu nu} = sum_{eta delta} Gamma^q_{eta delta} (mu nu|eta delta)
    K^q_{mu nu} = sum_{eta delta} Gamma^q_{eta delta} (mu delta|eta nu)
    """
    G = gamma_ao(C, q)
    Jq = np.einsum("mnls,ls->mn", ERI, G)
    Kq = np.einsum("msln,ls->mn", ERI, G)
    return Jq, Kq


def jk_ao_df(B, C, q):
    """J^q, K^q of Eq. Gpmn with (mn|ls) = sum_P B_P B_P written out."""
    c = C[:, q]
    x = np.einsum("Pmn,n->Pm", B, c)          # (B_P c_q)_mu
    d = x @ c                                 # c_q^T B_P c_q
    Jq = np.einsum("P,Pmn->mn", d, B)
    Kq = x.T @ x
    return Jq, Kq


def jk_ao(ints, C, q, kind: str):
    return jk_ao_eri(ints, C, q) if kind == "eri" else jk_ao_df(ints, C, q)


def jk_no(ints, C, nact: int, kind: str):
    """J_pq = <Gamma^p, J^q>, K_pq = <Gamma^p, K^q> (Eq. JKpq), p, q < nact."""
    J = np.zeros((nact, nact))
    K = np.zeros((nact, nact))
    for q in range(nact):
        Jq, Kq = jk_ao(ints, C, q, kind)
        for p in range(nact):
            G = gamma_ao(C, p)
            J[p, q] = np.sum(G * Jq)
            K[p, q] = np.sum(G * Kq)
    return J, K


def h_no(C, H, nact: int):
    """H_pp = c_p^T H c_p."""
    return np.array([C[:, p] @ H @ C[:, p] for p in range(nact)])


# --------------------------------------------------------------------------- energy
def energy_from_jk(n, Hpp, J, K, npairs: int, ncwo: int, functional: int = PNOF7, nsingle: int = 0):
    """Singlet PNOF energy, Eqs. EPNOF7, Eg, Efg (and Efg_s / PNOF5 variants).

    E = 2 sum_p n_p H_pp + sum_{p,q in A} (alpha_pq J_pq + beta_pq K_pq); summed with fsum.
    For multiplets the singly occupied orbitals contribute 2 (1/2) H_gg = H_gg (Eq. EPNOF7).
    """
    alpha, beta = coefficients(n, npairs, ncwo, functional, nsingle)
    nact = len(n)
    terms = [2.0 * n[p] * Hpp[p] for p in range(nact)]
    for p in range(nact):
        for q in range(nact):
            terms.append(alpha[p, q] * J[p, q])
            terms.append(beta[p, q] * K[p, q])
    return math.fsum(terms)


def energy(C, n, H, ints, npairs: int, ncwo: int, functional: int = PNOF7, kind: str = "df", nsingle: int = 0):
    nact = npairs * (ncwo + 1) + nsingle
    J, K = jk_no(ints, C, nact, kind)
    return energy_from_jk(n, h_no(C, H, nact), J, K, npairs, ncwo, functional, nsingle)


# --------------------------------------------------------------------------- Fock / Lagrangian
def fock_ao(C, n, H, ints, npairs: int, ncwo: int, functional: int = PNOF7, kind: str = "df", nsingle: int = 0):
    """F^q = n_q H + sum_{r in A} (alpha_qr J^r + beta_qr K^r), q in A.

    This is Eq. lowdin divided by 4: the one-particle part 4 n_p H and the
    Coulomb/exchange operators of Eqs. Vee-s and Vee-d, whose weights are the
    derivative of Eqs. Eg/Efg with respect to the orbital.
    """
    nact = npairs * (ncwo + 1) + nsingle
    alpha, beta = coefficients(n, npairs, ncwo, functional, nsingle)
    Jr, Kr = [], []
    for r in range(nact):
        a, b = jk_ao(ints, C, r, kind)
        Jr.append(a)
        Kr.append(b)
    F = []
    for q in range(nact):
        Fq = n[q] * H.copy()
        for r in range(nact):
            Fq = Fq + alpha[q, r] * Jr[r] + beta[q, r] * Kr[r]
        F.append(Fq)
    return F


def fock_vectors(C, F):
    """Y[:, q] = F^q c_q, the AO 'Fock times orbital' columns."""
    return np.stack([F[q] @ C[:, q] for q in range(len(F))], axis=1)


def lagrangian(C, F):
    """lambda_pq = c_p^T F^q c_q for all p, q in A (Eq. lag with Eq. gval); zero columns q >= nact."""
    nbf = C.shape[0]
    lam = np.zeros((nbf, nbf))
    for q in range(len(F)):
        for p in range(nbf):
            lam[p, q] = C[:, p] @ F[q] @ C[:, q]
    return lam


def max_asym(lam):
    """max |lambda_pq - lambda_qp|, the symmetry criterion of Section 3.4."""
    return float(np.max(np.abs(lam - lam.T)))


def grad_C(C, F):
    """dE/dC[:, q] = 4 F^q c_q for q in A, zero for inactive q (Eq. lowdin)."""
    g = np.zeros_like(C)
    for q in range(len(F)):
        g[:, q] = 4.0 * (F[q] @ C[:, q])
    return g


def grad_n(n, Hpp, J, K, npairs: int, ncwo: int, functional: int = PNOF7, nsingle: int = 0):
    """dE/dn_p: the derivative of Eqs. EPNOF7/Eg/Efg with J, K, H_pp held fixed.

    Same subspace:   2 H_pp + K_pp + sum_{q != p} s_pq sqrt(n_q / n_p) K_pq,
                     s_pq = -1 if p or q is strong, +1 otherwise.
    Other subspaces: sum_q [4 n_q J_pq - 2 n_q K_pq + kappa_pq K_pq],
                     kappa = -Phi_q (1-2n_p)/Phi_p (PNOF7), 0 (PNOF5),
                     -8 (1-2n_p) n_q (1-n_q) (PNOF7s).
    A singly occupied orbital has no K_pp term (beta_pp = 0); its occupation is fixed at 1/2,
    so its entry is the partial derivative only.
    """
    pair, strong = layout(npairs, ncwo, nsingle=nsingle)
    singles = set(single_orbitals(npairs, nsingle))
    n = np.asarray(n, dtype=np.float64)
    nact = len(n)
    ph = phi(n)
    g = np.zeros(nact)
    for p in range(nact):
        terms = [2.0 * Hpp[p], 0.0 if p in singles else K[p, p]]
        for q in range(nact):
            if q == p:
                continue
            if pair[p] == pair[q]:
                s = -1.0 if (strong[p] or strong[q]) else 1.0
                terms.append(s * math.sqrt(n[q] / n[p]) * K[p, q])
            else:
                terms.append(4.0 * n[q] * J[p, q] - 2.0 * n[q] * K[p, q])
                if functional == PNOF7:
                    terms.append(-ph[q] * (1.0 - 2.0 * n[p]) / ph[p] * K[p, q])
                elif functional == PNOF7S:
                    terms.append(-8.0 * (1.0 - 2.0 * n[p]) * n[q] * (1.0 - n[q]) * K[p, q])
        g[p] = math.fsum(terms)
    return g


# --------------------------------------------------------------------------- orbital step
def fockian_offdiag(lam):
    """Off-diagonal part of the symmetric matrix of Eq. Fockian.

    Its elements are differences of the two Lagrange multipliers of a pair; the orientation
    is the one for which the first-order energy change of Eq. ene1 is negative when the diagonal
    increases with the orbital index (the aufbau choice of Section 3.2).  With
    lambda_pq = c_p^T F^q c_q (bra p, operator of orbital q, as in Eqs. lowdin and lag) that is,
    for q < p: F_qp = F_pq = lambda_pq - lambda_qp (the multiplier whose operator belongs to the
    lower orbital is subtracted).
    """
    nbf = lam.shape[0]
    F = np.zeros_like(lam)
    for q in range(nbf):
        for p in range(q + 1, nbf):
            F[q, p] = lam[p, q] - lam[q, p]
            F[p, q] = F[q, p]
    return F


def scale_zeta(F, zeta: float):
    """Divide every off-diagonal element with |F_pq| > zeta by ten until it is <= zeta."""
    F = F.copy()
    nbf = F.shape[0]
    for p in range(nbf):
        for q in range(nbf):
            if p == q:
                continue
            while abs(F[p, q]) > zeta:
                F[p, q] /= 10.0
    return F


def sign_fix(U):
    """Make the largest-|.| entry of each column positive (lowest index on ties)."""
    U = U.copy()
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
    return U


def orbital_step(lam, C, diag_prev=None, zeta: float = 0.0):
    """One diagonalisation step of Section 3.2 / 3.4.

    diag_prev is None: S = (lambda + lambda^T)/2 (the initial step).
    Otherwise S = matrix of Eq. Fockian with S_pp = diag_prev (aufbau diagonal kept from the
    previous diagonalisation) and, if zeta > 0, the off-diagonal scaling by powers of ten.
    (eps, U) = eigh(S), eps ascending; C_new = C U.
    """
    if diag_prev is None:
        S = 0.5 * (lam + lam.T)
    else:
        S = fockian_offdiag(lam)
        if zeta > 0:
            S = scale_zeta(S, zeta)
        S[np.diag_indices(S.shape[0])] = diag_prev
    eps, U = np.linalg.eigh(S)
    U = sign_fix(U)
    return C @ U, eps, S


# --------------------------------------------------------------------------- NOF-MP2 reference terms
def nofmp2_reference(n, Hpp, J, K, npairs: int, ncwo: int, nsingle: int = 0):
    """HF-like energy with the natural orbitals (Eq. HFL) and static correlation (Eq. Esta).

    The HF-like density occupies the N_Omega = npairs + nsingle subspace-defining orbitals, the
    strong ones doubly (A_g = 1) and those of Omega_I singly (A_g = 1/2); the term J_gg/4 of
    Eq. HFL removes the self-interaction A_g^2 (2 J_gg - K_gg) = J_gg/4 of a singly occupied orbital:
        E_hf  = sum_g 2 A_g H_gg + sum_{f,g} A_f A_g (2 J_fg - K_fg) - sum_{g in Omega_I} J_gg / 4.
    Static correlation, with Lambda_p = 1 - |1 - 2 n_p| and Phi_p^2 = n_p (1 - n_p):
        E_sta = sum_g sum_{p != q in Omega_g} sqrt(Lambda_p Lambda_q) Pi_qp K_pq
                - 4 sum_{f != g} sum_{p in Omega_f, q in Omega_g} Phi_q^2 Phi_p^2 K_pq,
    Pi_qp = +sqrt(n_q n_p) for two weak orbitals, -sqrt(n_q n_p) when one is strong (Eq. intra).
    Both sums use math.fsum.
    """
    pair, strong = layout(npairs, ncwo, nsingle=nsingle)
    nact = npairs * (ncwo + 1) + nsingle
    nom = npairs + nsingle
    A = [1.0 if g < npairs else 0.5 for g in range(nom)]
    hf = [2.0 * A[g] * Hpp[g] for g in range(nom)]
    for f in range(nom):
        for g in range(nom):
            hf.append(A[f] * A[g] * (2.0 * J[f, g] - K[f, g]))
    for g in range(npairs, nom):
        hf.append(-0.25 * J[g, g])
    lam = [1.0 - abs(1.0 - 2.0 * n[p]) for p in range(nact)]
    ph2 = [n[p] * (1.0 - n[p]) for p in range(nact)]
    sta = []
    for p in range(nact):
        for q in range(nact):
            if p == q:
                continue
            if pair[p] == pair[q]:
                s = -1.0 if (strong[p] or strong[q]) else 1.0
                sta.append(math.sqrt(lam[p] * lam[q]) * s * math.sqrt(n[p] * n[q]) * K[p, q])
            else:
                sta.append(-4.0 * ph2[q] * ph2[p] * K[p, q])
    return math.fsum(hf), math.fsum(sta)
