"""Oracle: a plain, slow, FP64 CPU reference for the orbital-free DFT hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The product library (``paper_2002_02985_amd``) never imports, links or calls
it, and the oracle never imports the product.

What it computes follows the paper (Shao, Jiang, Mi, Genova, Pavanello,
"DFTpy: An efficient and object-oriented platform for orbital-free DFT
simulations", arXiv:2002.02985):

* the energy functional E[rho] = T_s + E_H + E_xc + int v_ext rho
  (Introduction, eq. "efunc"; E_xc the LDA of Perdew and Zunger, optional),
* its functional derivative v = dE/drho and the Euler-Lagrange residual
  (Introduction, eqs. "euler", "euler2a"; Section "Density optimization
  strategies", eq. "euler2"),
* the Thomas-Fermi and von Weizsaecker kinetic terms, Hartree, and a local
  pseudopotential through the ionic structure factor,
* the Wang-Teter nonlocal kinetic functional (Section "New-generation nonlocal
  KEDFs", eqs. "nl2" and "WT" and the Lindhard function G_NL),
* the density-dependent-kernel (LWT) functional evaluated with linear splines
  over k_F knots (steps s1-s4 of the same section),
* Hellmann-Feynman forces and the ion-ion Ewald energy,
* the smooth particle-mesh Ewald structure factor the paper uses for large
  cells (``oracle.pme``),
* the constrained minimisation over psi = sqrt(rho) with the orthogonal
  rotation update (Section "Density optimization strategies"), and the
  coarse-to-fine interpolation of the multi-step scheme (``oracle.multistep``),
* real-time TD-OFDFT: Crank-Nicolson propagation of the collective orbital
  with exact linear solves (Section "Time-Dependent OFDFT",
  ``oracle.tdofdft``).

Conventions used by every module here (and, independently, by the GPU path):

* grid N = N0*N1*N2, C order (i2 fastest), r = sum_d (i_d / N_d) a_d;
* int f = (V/N) sum_r f(r);
* f(G) = (1/N) sum_r f(r) exp(-i G.r); the inverse of a half spectrum X is
  f(r) = Re sum_{half} c(m2) X(m) exp(i G.r) with c = 1 on the m2 = 0 and
  m2 = N2/2 planes and 2 elsewhere;
* G = sum_d m_d b_d, a_i.b_j = 2 pi delta_ij, m_d in [-floor(N_d/2),
  ceil(N_d/2) - 1] (the Nyquist index takes the negative sign);
* every reciprocal-space sum runs over the half spectrum with the weights c;
* Hartree atomic units (Ha, Bohr).
"""
