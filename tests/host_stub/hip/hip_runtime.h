/* Empty stand-in for the HIP runtime header: lets the host compiler build the
 * device-side stencil header of the library as plain C++ in
 * test_stencil_host.py (the qualifiers are defined away there). */
