// CPU model of the cooperative sweep's exchange (spread walkers), with threads
// for workgroups.  A toy walker of n atoms on a ring [0, 1) is split into C
// slices, worker g holding atoms [g S, g S + S).  Each micro-update moves atom
// s by delta; every worker forms its slice's part of the change of a pair sum,
// and the move is accepted when the total exceeds ln xi.  The exchange is the
// kernel's: per move, a mailbox row chosen by the parity of the move counter
// holds 4C + 6 words of 32 bits of sequence number (move + 1) over 32 bits of
// payload, written and read with relaxed atomics only.  Words 4g .. 4g + 3
// carry worker g's two partials (high and low halves of two doubles); the
// worker holding the next move's atom, if that is another atom, publishes its
// position in words 4C .. 4C + 5 before it forms its partials.  A worker
// polls (at most cap times) until every word it needs carries the move's
// sequence, then adds the C partials in slice order.  The next move's old
// position is the published one, or for the same atom the trial position if
// accepted and the old one if not.
//
// The model checks every worker's decisions and totals against a sequential
// run of the same arithmetic, bitwise, and the final positions; and that a
// worker that stops publishing makes the others give up, every worker leaving.
//
//   spread_protocol_model C N MOVES CAP STALL_AT
//     STALL_AT < 0: no stall; else worker C-1 stops before move STALL_AT.
// Prints "ok <moves agreed> <accepted>" or "gaveup <moves agreed by all> <workers left>".
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

namespace {

uint64_t mix(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

struct Move {
    int s;
    double delta, lnxi;
};

Move move_of(int k, int n)
{
    const uint64_t a = mix((uint64_t)k * 3 + 0), b = mix((uint64_t)k * 3 + 1), c = mix((uint64_t)k * 3 + 2);
    Move m;
    m.s = (int)(a % (uint64_t)n);
    m.delta = ((double)(b >> 11) * 0x1.0p-53 - 0.5) * 0.2;
    m.lnxi = std::log(((double)(c >> 11) + 0.5) * 0x1.0p-53);
    return m;
}

double wrap(double x) { return x - std::floor(x); }
double pair_f(double d) { return std::cos(6.283185307179586 * d); }
double pair_g(double d) { return 0.3 * std::sin(6.283185307179586 * d); }

// a slice's two partials of a move of atom s from xo to xn
void partials(const double *x, int i0, int ns, int s, double xo, double xn, double &pu, double &pv)
{
    pu = 0.0;
    pv = 0.0;
    for (int q = 0; q < ns; ++q) {
        if (i0 + q == s)
            continue;
        pu += pair_f(xn - x[q]) - pair_f(xo - x[q]);
        pv += pair_g(xn - x[q]) - pair_g(xo - x[q]);
    }
}

uint32_t hi(double v)
{
    uint64_t b;
    memcpy(&b, &v, 8);
    return (uint32_t)(b >> 32);
}
uint32_t lo(double v)
{
    uint64_t b;
    memcpy(&b, &v, 8);
    return (uint32_t)b;
}
double join(uint32_t h, uint32_t l)
{
    const uint64_t b = ((uint64_t)h << 32) | l;
    double v;
    memcpy(&v, &b, 8);
    return v;
}

}   // namespace

int main(int argc, char **argv)
{
    if (argc != 6)
        return 2;
    const int C = atoi(argv[1]), n = atoi(argv[2]), moves = atoi(argv[3]);
    const unsigned long cap = strtoul(argv[4], nullptr, 10);
    const int stall_at = atoi(argv[5]);
    const int S = (n + C - 1) / C, row_words = 4 * C + 8;
    std::vector<double> x0(n);
    for (int i = 0; i < n; ++i)
        x0[i] = wrap((double)(mix(1000003ull + (uint64_t)i) >> 11) * 0x1.0p-53);

    // sequential reference: the same partials, added in slice order
    std::vector<double> xr = x0;
    std::vector<double> want_u(moves);
    std::vector<int> want_acc(moves);
    for (int k = 0; k < moves; ++k) {
        const Move m = move_of(k, n);
        const double xo = xr[m.s], xn = wrap(xo + m.delta);
        double du = 0.0, dv = 0.0;
        for (int g = 0; g < C; ++g) {
            const int i0 = g * S, ns = std::min(S, n - i0);
            double pu, pv;
            partials(xr.data() + i0, i0, ns, m.s, xo, xn, pu, pv);
            du += pu;
            dv += pv;
        }
        want_u[k] = du + dv;
        want_acc[k] = du > m.lnxi;
        if (want_acc[k])
            xr[m.s] = xn;
    }

    std::vector<std::atomic<uint64_t>> mail(2 * (size_t)row_words);
    for (auto &w : mail)
        w.store(0, std::memory_order_relaxed);
    std::atomic<unsigned> status{0}, left{0};
    std::vector<std::vector<double>> seen(C, std::vector<double>(moves, 0.0));
    std::vector<std::vector<int>> acc(C, std::vector<int>(moves, -1));
    std::vector<int> done(C, 0);
    std::vector<double> xfinal(n, -1.0);
    auto put = [&](int par, int idx, uint32_t seq, uint32_t payload) {
        mail[(size_t)par * row_words + idx].store(((uint64_t)seq << 32) | payload, std::memory_order_relaxed);
    };
    auto worker = [&](int g) {
        const int i0 = g * S, ns = std::min(S, n - i0);
        std::vector<double> x(x0.begin() + i0, x0.begin() + i0 + ns);
        double xo = x0[move_of(0, n).s];   // the first move reads the start copy
        for (int k = 0; k < moves; ++k) {
            if (g == C - 1 && stall_at >= 0 && k == stall_at)
                break;   // this worker stops publishing
            const Move m = move_of(k, n);
            const int s_next = k + 1 < moves ? move_of(k + 1, n).s : -1;
            const bool pub = s_next >= 0 && s_next != m.s;
            const uint32_t seq = (uint32_t)k + 1u;
            const int par = k & 1;
            const double xn = wrap(xo + m.delta);
            if (pub && s_next >= i0 && s_next < i0 + ns) {
                const double p = x[s_next - i0];
                put(par, 4 * C, seq, hi(p));
                put(par, 4 * C + 1, seq, lo(p));
            }
            double pu, pv;
            partials(x.data(), i0, ns, m.s, xo, xn, pu, pv);
            put(par, 4 * g, seq, hi(pu));
            put(par, 4 * g + 1, seq, lo(pu));
            put(par, 4 * g + 2, seq, hi(pv));
            put(par, 4 * g + 3, seq, lo(pv));
            const int nw = 4 * C + (pub ? 2 : 0);
            std::vector<uint64_t> word(nw, 0);
            std::vector<char> have(nw, 0);
            unsigned long spins = 0;
            bool gave_up = false;
            for (;;) {
                bool all = true;
                for (int q = 0; q < nw; ++q) {
                    if (!have[q]) {
                        word[q] = mail[(size_t)par * row_words + q].load(std::memory_order_relaxed);
                        have[q] = (uint32_t)(word[q] >> 32) == seq;
                    }
                    all = all && have[q];
                }
                if (all)
                    break;
                if (++spins > cap) {
                    gave_up = true;
                    break;
                }
                std::this_thread::yield();
            }
            if (gave_up) {
                status.fetch_or(1);
                break;
            }
            double DU = 0.0, DV = 0.0;
            for (int q = 0; q < C; ++q) {
                DU += join((uint32_t)word[4 * q], (uint32_t)word[4 * q + 1]);
                DV += join((uint32_t)word[4 * q + 2], (uint32_t)word[4 * q + 3]);
            }
            const bool accept = DU > m.lnxi;
            seen[g][k] = DU + DV;
            acc[g][k] = accept;
            if (accept && m.s >= i0 && m.s < i0 + ns)
                x[m.s - i0] = xn;
            if (!pub) {
                if (accept)
                    xo = xn;
            } else {
                xo = join((uint32_t)word[4 * C], (uint32_t)word[4 * C + 1]);
            }
            done[g] = k + 1;
        }
        if (done[g] == moves)
            for (int q = 0; q < ns; ++q)
                xfinal[i0 + q] = x[q];
        left.fetch_add(1);
    };
    std::vector<std::thread> th;
    for (int g = 0; g < C; ++g)
        th.emplace_back(worker, g);
    for (auto &t : th)
        t.join();
    int agreed = moves;
    for (int g = 0; g < C; ++g)
        agreed = done[g] < agreed ? done[g] : agreed;
    int n_acc = 0;
    for (int k = 0; k < agreed; ++k) {
        for (int g = 0; g < C; ++g)
            if (seen[g][k] != want_u[k] || acc[g][k] != want_acc[k]) {
                printf("mismatch move %d worker %d\n", k, g);
                return 1;
            }
        n_acc += want_acc[k];
    }
    if (status.load()) {
        printf("gaveup %d %u\n", agreed, left.load());
        return 0;
    }
    for (int i = 0; i < n; ++i)
        if (xfinal[i] != xr[i]) {
            printf("position mismatch atom %d\n", i);
            return 1;
        }
    printf("ok %d %d\n", agreed, n_acc);
    return 0;
}
