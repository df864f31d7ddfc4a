// Host build of the GPU path's spin projector header, so that its table can be
// checked on the CPU against dense (1 +- gamma_mu).
#include "../../paper_0905_3331_amd/csrc/spin.h"

using namespace tmq;

template <int MU, int S>
static void run(const double *in, double *out)
{
    spinor<double> s, acc;
    for (int k = 0; k < 12; k++) {
        s.c[k / 3][k % 3] = cx<double>{in[2 * k], in[2 * k + 1]};
        acc.c[k / 3][k % 3] = cx<double>{0.0, 0.0};
    }
    half<double> h;
    project<MU, S>(s, h);
    reconstruct_add<MU, S>(acc, h);
    for (int k = 0; k < 12; k++) {
        out[2 * k] = acc.c[k / 3][k % 3].re;
        out[2 * k + 1] = acc.c[k / 3][k % 3].im;
    }
}

extern "C" void spin_project_reconstruct(int mu, int sign, const double *in, double *out)
{
    switch (mu * 2 + (sign > 0)) {
    case 0: run<0, -1>(in, out); break;
    case 1: run<0, +1>(in, out); break;
    case 2: run<1, -1>(in, out); break;
    case 3: run<1, +1>(in, out); break;
    case 4: run<2, -1>(in, out); break;
    case 5: run<2, +1>(in, out); break;
    case 6: run<3, -1>(in, out); break;
    case 7: run<3, +1>(in, out); break;
    }
}

extern "C" void su3_reconstruct(const double *two_rows, double *third)
{
    su3<double> u;
    for (int k = 0; k < 6; k++) u.e[k / 3][k % 3] = cx<double>{two_rows[2 * k], two_rows[2 * k + 1]};
    su3_third_row(u);
    for (int c = 0; c < 3; c++) {
        third[2 * c] = u.e[2][c].re;
        third[2 * c + 1] = u.e[2][c].im;
    }
}
