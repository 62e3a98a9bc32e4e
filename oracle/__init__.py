"""FP64 CPU oracle for the asynchrony-tolerant (AT) compressible-flow solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports, links or
calls it, and shares no code with it.

The oracle is a plain, slow, readable restatement of the method of
arXiv 2506.03027 (Arumugam, Goswami, Vadlamani, Aditya):

* ``rk``      -- classical RK4 and the 2N-storage LSERK2/LSERK4 schemes
                 (Sec. 2, Eq. 3, App. B Table 4) and their stage polynomials.
* ``at``      -- asynchrony-tolerant coefficients: PE-boundary extrapolation
                 (Eq. 7, Eqs. 14-15), buffer temporal derivatives (Eqs. 8-13,
                 App. C Table 5) and the per-stage halo weights W.
* ``delays``  -- delay schedules of the communication-avoiding (Alg. 2) and
                 synchronization-avoiding (Alg. 3) algorithms.
* ``flow``    -- Euler / Navier-Stokes fluxes (Eq. 1, App. A) and the explicit
                 CD4 and CD2 derivatives (Eq. 2, App. B).
* ``solver``  -- blocks (processing elements), delayed history, halo filling
                 in SA / AS / AT modes and the RK step (Sec. 3.2, Alg. 1-3).
* ``diagnostics`` -- conserved totals, kinetic energy and enstrophy (Sec. 5.2).
* ``mlp``     -- FP64 reference of the learned-halo MLP (forward, backward).
* ``filter``  -- the tenth-order Pade low-pass filter (Sec. 2, Sec. 5.2) and
                 its block-local application with synchronous, AT or AS
                 halos (a reading; the paper does not define it across PEs).

Everything is float64 numpy or exact ``fractions.Fraction`` arithmetic.

What pins it (tests/test_oracle_*.py, all on the CPU):

* coefficients -- Table 4 and Table 5 values, Eqs. 14-15 (with the AT4
  k^2 coefficient read as 26), RK4/LSERK order conditions, observed temporal
  order on an ODE, exactness of the extrapolation for polynomials, the
  literal buffer recursion equal to the closed form;
* flow -- the CD4 and CD2 modified wavenumbers, fourth- and second-order
  convergence, CD2 exact on quadratics, closed-form
  viscous solutions (shear wave, heat conduction, compression wave),
  rotation covariance, the translating vortex, TGV initial kinetic energy and
  enstrophy in closed form;
* solver -- decomposed SA equal to one block bit for bit, Table 1 orders for
  SA/AT/AS (cases 4-6 with RK4/LSERK4-CD4-AT4, cases 1-3 with
  LSERK2-CD2-AT2), AT with zero delay converging to SA, conservation under SA,
  a brute-force pointwise halo rule, the delay patterns of Alg. 2 and
  Alg. 3 and SplitMix64's published outputs;
* mlp -- central-difference gradients, BF16 rounding, the fallback rule;
* filter -- the coefficients at alpha = 0 (binomial closed form of
  1 - sin^10(w/2)) and alpha = 1/2 (identity), affine in between; the
  transfer function on Fourier modes of the periodic filter; exactness of
  the block filter on degree-9 polynomials and not on degree 10; agreement
  with the periodic filter far from block faces; one axis per pass; the AT
  halo exact for time polynomials of degree C-1; alpha = 1/2 steps equal to
  unfiltered steps.

Parity unpinned: the TGV kinetic-energy and enstrophy time series beyond
t = 0 (the paper shows them only as plots, without data), and the
flux-level form of the stage-0 extrapolation (the solver extrapolates the
conserved variables and computes fluxes from them; see ``solver``).
"""
