"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation of what the GPU path computes
for the OSRC-preconditioned permuted PMCHWT formulation (van 't Wout,
Haqshenas, Gelat, Betcke, Saffari: "Frequency-robust preconditioning of
boundary integral equations for acoustic transmission", J. Comput. Phys. 2022):

  * dense Galerkin P1 matrices of the Helmholtz V, K, K' and Maue-form D
    (Sec. 2.2 boundary operators; Sec. 2.3 P1 Galerkin), regular 6-point rule
    for separated triangles and Sauter-Schwab-type singular quadrature for
    triangles sharing a vertex, an edge or coinciding;
  * the permuted PMCHWT block operator with density scaling (Sec. 2.7);
  * mass matrix / strong form (Sec. 2.4);
  * OSRC DtN/NtD operators with damped wavenumber and rotated Pade
    square root, sparse LU per shift (Sec. 2.6, 2.7);
  * unrestarted MGS GMRES (Sec. 3.1);
  * plane-wave right-hand side, far field, and the Mie series of a penetrable
    sphere used as the end-to-end pin.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in this package.  It shares no code
with the HIP path (``paper_2104_04609_amd``); the only common input is the
seeded mesh/vector generator package ``bem_inputs``.
"""
