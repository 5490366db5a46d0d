"""Plain FP64 CPU oracle for the one- and two-level AS / RAS / ORAS-preconditioned (weighted)
GMRES solve of the lowest- and second-order Nedelec discretisations of
curl curl E - (k^2 + i xi) E = F.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library and its Python
binding) imports, links or runs anything here; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark do.  The oracle shares no code with the GPU path.

Every function is written from the paper (Bonazzoli, Dolean, Graham, Spence, Tournier,
"Domain decomposition preconditioning for the high-frequency time-harmonic Maxwell equations
with absorption", Math. Comp. 2019 / arXiv:1711.03789):

* mesh.py      structured box mesh, Kuhn 6-tetrahedra split, edge numbering (Sec. 2.2)
* fem.py       Whitney element matrices, Galerkin matrix A_xi and load f (Sec. 2.2,
               eq:Helmholtzvf_intro, impedance condition eq:imp)
* order2.py    second-order Nedelec elements (first family) in a hierarchical basis: exact element
               integrals, assembly, order-2 local DOF sets, owners and local problems, the
               weight D_k and the coarse restriction of the order-2 space
* dd.py        non-overlapping boxes, overlap by tetrahedron layers (Sec. 6.1), local DOF
               sets and restriction (eq:restriction1), minors (eq:minor), Boolean partition
               of unity (eq:algebPartUnity), local impedance problems (ImpRAS, Sec. 6.3),
               AS / RAS / ORAS application (eq:defAS without the coarse term, RAS_1, ImpRAS_1)
* coarse.py    nested or non-nested coarse mesh, restriction R^0 (eq:restriction; exact on nested
               meshes, by a Gauss rule along each fine edge otherwise), coarse Galerkin matrix and
               the two-level AS / RAS / ImpRAS preconditioners in additive (eq:defAS,
               eq:RAS2), hybrid (eq:HRAS) and deflated (eq:ADEF1ras) form
* rcm.py       reverse Cuthill-McKee ordering of a local matrix graph (not in the paper: the
               paper's local solves are sparse direct; the ordering is only compared
               integer-for-integer with the library's own)
* pool.py      the same Schwarz preconditioner with its local factorisations and solves on a
               pool of host processes, one subdomain per task (bitwise equal to dd.Schwarz)
* gmres.py     restarted right-preconditioned (F)GMRES with classical Gram-Schmidt twice and
               complex Givens rotations (Sec. 5.2 minimal-residual definition, Sec. 6.1
               stopping rule), also in the D_k-weighted inner product (eq:ip)

Precision: float64 / complex128 throughout.
"""
